"""Python access to the CPU oracle of the fractional ABM scheme.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark load this; the GPU library never does.  The arithmetic lives
in ``abm_oracle.c`` (plain C, FP64, weights from the literal formulas of
Section 2 evaluated in __float128); this module only builds it with gcc and
marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "abm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# right-hand side ids used by the oracle (its own numbering)
RHS_LINEAR, RHS_DUFFING, RHS_LORENZ, RHS_POLY, RHS_LCR, RHS_DIAG = 0, 1, 2, 3, 4, 5
RHS_DIM = {RHS_LINEAR: 1, RHS_DUFFING: 2, RHS_LORENZ: 3, RHS_POLY: 1, RHS_LCR: 2, RHS_DIAG: 2}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/liboracle.so with gcc (-O2, OpenMP,
    libquadmath, no FP contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           _SRC, "-o", tmp, "-lquadmath", "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    c_dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_weights.argtypes = [ctypes.c_double, ctypes.c_int64, c_dp, c_dp, c_dp]
    lib.oracle_weights.restype = ctypes.c_int
    lib.oracle_weights_at.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_int64, c_dp, c_dp,
                                      c_dp]
    lib.oracle_weights_at.restype = ctypes.c_int
    lib.oracle_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int64, c_dp, c_dp, ctypes.c_int64, c_dp, ctypes.c_int]
    lib.oracle_solve.restype = ctypes.c_int
    lib.oracle_solve_gen.argtypes = [ctypes.c_int, ctypes.c_int, c_dp, ctypes.c_double,
                                     ctypes.c_int64, c_dp, c_dp, c_dp, ctypes.c_int64, c_dp,
                                     ctypes.c_int]
    lib.oracle_solve_gen.restype = ctypes.c_int
    lib.oracle_steps_from_states_gen.argtypes = [ctypes.c_int, ctypes.c_int, c_dp,
                                                 ctypes.c_double, c_dp, c_dp, c_dp, c_dp,
                                                 ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                                 c_dp, c_dp, ctypes.c_int]
    lib.oracle_steps_from_states_gen.restype = ctypes.c_int
    lib.oracle_solve_batch_gen.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32), c_dp, c_dp,
                                           ctypes.POINTER(ctypes.c_int64), c_dp, c_dp, c_dp,
                                           ctypes.c_int64, ctypes.POINTER(c_dp),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.c_int]
    lib.oracle_solve_batch_gen.restype = ctypes.c_int
    lib.oracle_solve_quad.argtypes = [ctypes.c_int, ctypes.c_int, c_dp, ctypes.c_double,
                                      ctypes.c_int64, c_dp, c_dp, c_dp, ctypes.c_int64, c_dp]
    lib.oracle_solve_quad.restype = ctypes.c_int
    lib.oracle_steps_from_states_quad.argtypes = [ctypes.c_int, ctypes.c_int, c_dp,
                                                  ctypes.c_double, c_dp, c_dp, c_dp, c_dp,
                                                  ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                                  c_dp]
    lib.oracle_steps_from_states_quad.restype = ctypes.c_int
    lib.oracle_weights_quad.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_int64, c_dp,
                                        c_dp, c_dp]
    lib.oracle_weights_quad.restype = ctypes.c_int
    lib.oracle_history_sum.argtypes = [c_dp, c_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    lib.oracle_history_sum.restype = ctypes.c_double
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def n_out(N: int, out_stride: int) -> int:
    """Number of states written for a run of N steps at the given stride."""
    if out_stride == 0:
        return 1
    return N // out_stride + 1 + (1 if N % out_stride else 0)


def weights(alpha: float, n: int, k0: int = 0):
    """b_k, a_k, c_k for k = k0..k0+n-1 (Section 2), as three float64 arrays."""
    lib = _load()
    b = np.zeros(n, np.float64)
    a = np.zeros(n, np.float64)
    c = np.zeros(n, np.float64)
    rc = lib.oracle_weights_at(float(alpha), int(k0), int(n), _dp(b), _dp(a), _dp(c))
    if rc != 0:
        raise ValueError("oracle_weights failed: %d" % rc)
    return b, a, c


def _params(rhs, d, x0, p):
    x = np.zeros(4, np.float64)
    pp = np.zeros(8, np.float64)
    x0 = np.asarray(x0, np.float64).ravel()
    p = np.asarray(p, np.float64).ravel()
    if x0.size != d or p.size > 8:
        raise ValueError("bad x0/p size")
    x[:d] = x0
    pp[:p.size] = p
    return x, pp


def _orders(alpha, d, x1):
    """Per-component orders (a scalar means one order for all components)
    and the initial first derivative (zeros when not given)."""
    al = np.zeros(4, np.float64)
    a = np.asarray(alpha, np.float64).ravel()
    if a.size == 1:
        al[:d] = a[0]
    elif a.size == d:
        al[:d] = a
    else:
        raise ValueError("alpha must be a scalar or one value per component")
    v = np.zeros(4, np.float64)
    if x1 is not None:
        x1 = np.asarray(x1, np.float64).ravel()
        if x1.size != d:
            raise ValueError("bad x1 size")
        v[:d] = x1
    return al, v


def solve(rhs: int, alpha, h: float, N: int, x0, p, out_stride: int = 1,
          compensated: bool = False, x1=None) -> np.ndarray:
    """One trajectory; returns the written states as an (n_out, d) array.
    alpha: one order, or one per component (incommensurate system), each in
    (0, 2]; x1: y'(0), used by components of order above 1."""
    lib = _load()
    d = RHS_DIM[rhs]
    x, pp = _params(rhs, d, x0, p)
    al, v = _orders(alpha, d, x1)
    y = np.zeros((n_out(N, out_stride), d), np.float64)
    rc = lib.oracle_solve_gen(rhs, d, _dp(al), float(h), int(N), _dp(x), _dp(v), _dp(pp),
                              int(out_stride), _dp(y), 1 if compensated else 0)
    if rc != 0:
        raise ValueError("oracle_solve failed: %d" % rc)
    return y


def steps_from_states(rhs: int, alpha, h: float, x0, p, y_hist: np.ndarray,
                      s_list, x1=None, return_scale: bool = False, compensated: bool = False):
    """y_s recomputed for each s in s_list from the given states y_0..y_{s-1}.
    With return_scale, also the size of each step's history terms per
    component, h^alpha (sum |b_{n-k} F_k| + |c_n F_0| + sum |a_{n-k} F_k|):
    rounding inside the sums moves y_s by a small multiple of eps times it.
    compensated: Neumaier-compensated history sums (nearly free of rounding)."""
    lib = _load()
    d = RHS_DIM[rhs]
    x, pp = _params(rhs, d, x0, p)
    al, v = _orders(alpha, d, x1)
    s_arr = np.ascontiguousarray(np.asarray(s_list, np.int64))
    yh = np.ascontiguousarray(np.asarray(y_hist, np.float64).reshape(-1, d))
    if s_arr.size and (s_arr.min() < 1 or s_arr.max() > yh.shape[0]):
        raise ValueError("s out of range of the given history")
    out = np.zeros((s_arr.size, d), np.float64)
    scale = np.zeros((s_arr.size, d), np.float64) if return_scale else None
    rc = lib.oracle_steps_from_states_gen(rhs, d, _dp(al), float(h), _dp(x), _dp(v), _dp(pp),
                                          _dp(yh),
                                          s_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          int(s_arr.size), _dp(out),
                                          _dp(scale) if return_scale else None,
                                          1 if compensated else 0)
    if rc != 0:
        raise ValueError("oracle_steps_from_states failed: %d" % rc)
    return (out, scale) if return_scale else out


def solve_batch(rhs, alpha, h, N, x0, p, out_stride: int = 0, compensated: bool = False,
                x1=None):
    """Many independent trajectories (OpenMP over trajectories).  Every argument
    is per trajectory (sequence of length B; alpha[i] a scalar or one order per
    component, x1[i] or None); returns a list of (n_out, d) arrays."""
    lib = _load()
    B = len(rhs)
    rhs_a = np.asarray(rhs, np.int32)
    d_a = np.asarray([RHS_DIM[int(r)] for r in rhs_a], np.int32)
    hh = np.asarray(h, np.float64)
    NN = np.asarray(N, np.int64)
    xs = np.zeros((B, 4), np.float64)
    vs = np.zeros((B, 4), np.float64)
    als = np.zeros((B, 4), np.float64)
    ps = np.zeros((B, 8), np.float64)
    for i in range(B):
        xs[i], ps[i] = _params(int(rhs_a[i]), int(d_a[i]), x0[i], p[i])
        als[i], vs[i] = _orders(alpha[i], int(d_a[i]), None if x1 is None else x1[i])
    outs = [np.zeros((n_out(int(NN[i]), out_stride), int(d_a[i])), np.float64) for i in range(B)]
    ptrs = (ctypes.POINTER(ctypes.c_double) * max(B, 1))(*[_dp(o) for o in outs])
    st = np.zeros(B, np.int32)
    i32 = ctypes.POINTER(ctypes.c_int32)
    rc = lib.oracle_solve_batch_gen(B, rhs_a.ctypes.data_as(i32), d_a.ctypes.data_as(i32),
                                    _dp(als), _dp(hh),
                                    NN.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(xs),
                                    _dp(vs), _dp(ps), int(out_stride), ptrs,
                                    st.ctypes.data_as(i32), 1 if compensated else 0)
    if rc != 0:
        raise ValueError("oracle_solve_batch failed: %s" % st)
    return outs


def solve_quad(rhs: int, alpha, h: float, N: int, x0, p, out_stride: int = 1,
               x1=None) -> np.ndarray:
    """One trajectory of the scheme in __float128 (weights, Gamma, h^alpha,
    right-hand side, sums and state); returns (n_out, d, 2): the (hi, lo)
    double pair of every component of every written state."""
    lib = _load()
    d = RHS_DIM[rhs]
    x, pp = _params(rhs, d, x0, p)
    al, v = _orders(alpha, d, x1)
    y = np.zeros((n_out(N, out_stride), d, 2), np.float64)
    rc = lib.oracle_solve_quad(rhs, d, _dp(al), float(h), int(N), _dp(x), _dp(v), _dp(pp),
                               int(out_stride), _dp(y))
    if rc != 0:
        raise ValueError("oracle_solve_quad failed: %d" % rc)
    return y


def steps_from_states_quad(rhs: int, alpha, h: float, x0, p, y_hist: np.ndarray, s_list,
                           x1=None) -> np.ndarray:
    """Quad y_s for each s in s_list from the given states y_0..y_{s-1}, each
    a (hi, lo) pair: y_hist of shape (>= max s, d, 2); returns (len, d, 2)."""
    lib = _load()
    d = RHS_DIM[rhs]
    x, pp = _params(rhs, d, x0, p)
    al, v = _orders(alpha, d, x1)
    s_arr = np.ascontiguousarray(np.asarray(s_list, np.int64))
    yh = np.ascontiguousarray(np.asarray(y_hist, np.float64).reshape(-1, d, 2))
    if s_arr.size and (s_arr.min() < 1 or s_arr.max() > yh.shape[0]):
        raise ValueError("s out of range of the given history")
    out = np.zeros((s_arr.size, d, 2), np.float64)
    rc = lib.oracle_steps_from_states_quad(rhs, d, _dp(al), float(h), _dp(x), _dp(v), _dp(pp),
                                           _dp(yh),
                                           s_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           int(s_arr.size), _dp(out))
    if rc != 0:
        raise ValueError("oracle_steps_from_states_quad failed: %d" % rc)
    return out


def weights_quad(alpha: float, n: int, k0: int = 0):
    """Quad b_k, a_k, c_k for k = k0..k0+n-1 as (n, 2) arrays of (hi, lo)."""
    lib = _load()
    out = [np.zeros((n, 2), np.float64) for _ in range(3)]
    rc = lib.oracle_weights_quad(float(alpha), int(k0), int(n), *[_dp(o) for o in out])
    if rc != 0:
        raise ValueError("oracle_weights_quad failed: %d" % rc)
    return tuple(out)


def history_sum(w, F, k_lo: int, n: int, compensated: bool) -> float:
    """sum_{k=k_lo..n} w[n-k] F[k] with the solver's summation (plain
    ascending or Neumaier-compensated)."""
    w = np.ascontiguousarray(np.asarray(w, np.float64))
    F = np.ascontiguousarray(np.asarray(F, np.float64))
    if not (0 <= k_lo <= n < F.size and n - k_lo < w.size):
        raise ValueError("index range outside the arrays")
    return float(_load().oracle_history_sum(_dp(w), _dp(F), int(k_lo), int(n),
                                            1 if compensated else 0))


def num_threads() -> int:
    return int(_load().oracle_num_threads())
