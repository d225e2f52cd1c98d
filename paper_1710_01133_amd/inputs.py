"""Seeded synthetic workloads for the fractional ABM solver.

This module only describes problems (right-hand side, order, step, length,
initial state, parameters); it holds none of the method's arithmetic, so both
the GPU library's tests and the CPU oracle can take their inputs from here.

Workloads (shapes follow the paper's setting: a forced nonlinear oscillator of
dimension 2 swept over a forcing parameter, as in the LCR experiment of the
"Numerical experiment" section, plus a scalar linear test equation and a
three-dimensional chaotic system):

* ``linear_c``   D^0.8 y = -y, y(0)=1, h=2^-10, N=8192 (exact solution is a
  Mittag-Leffler function).
* ``duffing_single``  forced Duffing-type oscillator, alpha=0.9, x0=(0.1,0),
  delta=0.1, A=0.3, omega=1.2, h=1e-3, N=200000.
* ``duffing_sweep``   B=1024 copies of that oscillator with forcing amplitude
  drawn uniform in [0.1, 0.6] (numpy PCG64, seed 1710), alpha=0.95, h=2^-8,
  N=65536.
* ``lcr_sweep``   the numerical experiment's forced fractional LCR circuit
  (sigma=1.015, omega=0.55, a=-1.02, b=-0.58, x0=(0.1, 0)) at B forcing
  amplitudes F evenly spaced in [0, 0.2] (the bifurcation parameter of its
  figures), orders (0.9, 0.9) or incommensurate (alpha_1, alpha_2), step
  h = T/M with T = 2 pi / omega and M = 1142 (h ~ 0.01), so that writing every
  M-th state gives the stroboscopic (Poincare) section y(kT), N=65536.
* ``serving_stream``  Poisson arrivals (rate 200/s, seed 1710) of requests,
  half Duffing (d=2) and half Lorenz (sigma=10, rho=28, beta=8/3, x0=(1,1,1),
  d=3), alpha uniform in [0.90, 0.99], N log-uniform in [4096, 262144],
  h=2^-8.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple, Union

import numpy as np

SEED = 1710

RHS_NAMES = ("LINEAR", "DUFFING", "LORENZ", "POLY", "LCR", "DIAG")
RHS_DIM = {"LINEAR": 1, "DUFFING": 2, "LORENZ": 3, "POLY": 1, "LCR": 2, "DIAG": 2}


@dataclass
class Problem:
    rhs: str                      # one of RHS_NAMES
    alpha: Union[float, Tuple[float, ...]]   # order in (0, 2], or one per component
    h: float                      # step size
    N: int                        # number of steps
    x0: Tuple[float, ...]         # initial state, length d
    p: Tuple[float, ...] = field(default_factory=tuple)   # rhs parameters
    far_prec: str = "fp64"        # far-field precision: fp64 | fp32 | bf16x3 | bf16x6 | fp16x3 | i8x9 | dd
    x1: Optional[Tuple[float, ...]] = None   # y'(0), for components of order above 1

    @property
    def d(self) -> int:
        return RHS_DIM[self.rhs]

    def history_macs(self) -> int:
        """History MACs of one solve: d * N(N+1)/2 (one predictor plus one
        corrector multiply-add per (step, history index, component))."""
        return self.d * self.N * (self.N + 1) // 2


DUFFING_P = (0.1, 0.3, 1.2)            # delta, A, omega
LORENZ_P = (10.0, 28.0, 8.0 / 3.0)     # sigma, rho, beta
LCR_P = (1.015, 0.55, -1.02, -0.58)    # sigma, omega, a, b (forcing F appended)


def linear_c(N: int = 8192, h: float = 2.0 ** -10, alpha: float = 0.8, lam: float = 1.0) -> Problem:
    return Problem("LINEAR", alpha, h, N, (1.0,), (lam,))


def duffing_single(N: int = 200000, h: float = 1e-3, alpha: float = 0.9, A: float = 0.3) -> Problem:
    return Problem("DUFFING", alpha, h, N, (0.1, 0.0), (DUFFING_P[0], A, DUFFING_P[2]))


LCR_SECTION_STEPS = 1142               # steps per forcing period of the LCR sweep


def sweep_amplitudes(B: int = 1024, seed: int = SEED) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.1, 0.6, B)


def duffing_sweep(B: int = 1024, N: int = 65536, h: float = 2.0 ** -8, alpha: float = 0.95,
                  far_prec: str = "fp64", seed: int = SEED) -> List[Problem]:
    amps = sweep_amplitudes(B, seed)
    return [Problem("DUFFING", alpha, h, N, (0.1, 0.0), (DUFFING_P[0], float(A), DUFFING_P[2]),
                    far_prec) for A in amps]


def lcr_section_step(M: int = LCR_SECTION_STEPS) -> float:
    """Step that puts M steps in one forcing period T = 2 pi / omega."""
    return 2.0 * np.pi / LCR_P[1] / M


def lcr_sweep(B: int = 1024, N: int = 65536, h: float = None, alpha=(0.9, 0.9),
              f_lo: float = 0.0, f_hi: float = 0.2, x0=(0.1, 0.0),
              far_prec: str = "fp64") -> List[Problem]:
    """Forcing sweep of the fractional LCR circuit (eq. sys.LRC), evenly spaced
    F; h defaults to lcr_section_step()."""
    h = lcr_section_step() if h is None else h
    fs = np.linspace(f_lo, f_hi, B) if B > 1 else np.array([f_lo])
    al = tuple(alpha) if isinstance(alpha, (tuple, list)) else alpha
    return [Problem("LCR", al, h, N, tuple(x0), LCR_P + (float(f),), far_prec) for f in fs]


@dataclass
class Request:
    arrival_s: float
    problem: Problem


def serving_stream(n_req: int = 2000, rate: float = 200.0, seed: int = SEED,
                   n_lo: int = 4096, n_hi: int = 262144, h: float = 2.0 ** -8,
                   far_prec: str = "fp32") -> List[Request]:
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_req)
    t = np.cumsum(gaps) - gaps[0]
    kinds = rng.integers(0, 2, n_req)
    alphas = rng.uniform(0.90, 0.99, n_req)
    Ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), n_req)).astype(np.int64)
    out = []
    for i in range(n_req):
        if kinds[i] == 0:
            pr = Problem("DUFFING", float(alphas[i]), h, int(Ns[i]), (0.1, 0.0), DUFFING_P, far_prec)
        else:
            pr = Problem("LORENZ", float(alphas[i]), h, int(Ns[i]), (1.0, 1.0, 1.0), LORENZ_P,
                         far_prec)
        out.append(Request(float(t[i]), pr))
    return out
