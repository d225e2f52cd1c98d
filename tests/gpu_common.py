"""Helpers shared by the GPU parity tests: run the library through the C ABI
and the oracle on the same seeded problems."""
import json
import os

import numpy as np

import oracle as O
from paper_1710_01133_amd import abm

RID = {"LINEAR": O.RHS_LINEAR, "DUFFING": O.RHS_DUFFING, "LORENZ": O.RHS_LORENZ,
       "POLY": O.RHS_POLY, "LCR": O.RHS_LCR, "DIAG": O.RHS_DIAG}

# Parity bar of the double-precision GPU path against the oracle: normwise
# relative error max_s |y_s - yref_s|_inf / max_s |yref_s|_inf.  Both sides
# round differently (fused multiply-adds, summation order, libm vs device
# cos/pow/tgamma), which the oracle's own noise-floor test bounds near 1e-14.
TOL_FP64 = 1e-12

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_fullsize.json")


def oracle_run(p, stride):
    return O.solve(RID[p.rhs], p.alpha, p.h, p.N, p.x0, p.p, out_stride=stride, x1=p.x1)


def normerr(y, ref):
    y = np.asarray(y)
    ref = np.asarray(ref)
    assert y.shape == ref.shape, (y.shape, ref.shape)
    return float(np.max(np.abs(y - ref)) / max(np.max(np.abs(ref)), 1e-300))


def run_plain(ctx, p, stride):
    plan = abm.Plan(ctx, [p], out_stride=stride)
    y = abm.alloc_out(p, stride)
    abm.solve(plan, p, y)
    plan.check()
    out = y.cpu().numpy()
    plan.close()
    return out


def run_batch(ctx, probs, stride):
    plan = abm.Plan(ctx, probs, out_stride=stride)
    ys = [abm.alloc_out(p, stride) for p in probs]
    st = abm.solve_batch(plan, probs, ys)
    plan.check()
    outs = [y.cpu().numpy() for y in ys]
    plan.close()
    return outs, st


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


SWEEP_ALL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "duffing_sweep_all.npy")


def sweep_golden():
    """Stored oracle runs of all 1024 forcing-sweep members, every 1024th
    state: shape (1024, 65, 2) (tests/golden/make_golden.py --parts sweep)."""
    return np.load(SWEEP_ALL, allow_pickle=False)


def sweep_errors(outs):
    """Normwise error of every sweep member against its stored oracle run."""
    g = sweep_golden()
    assert len(outs) == g.shape[0]
    return np.array([normerr(y, g[i]) for i, y in enumerate(outs)])


# Per-step recompute (the oracle takes one predictor-corrector step from the
# GPU's own states y_0..y_{s-1}, with compensated history sums so that its own
# rounding drops out).  Bound for a double far field: rounding inside the two
# history sums moves y_s by at most n eps times the size of its terms,
# h^alpha sum |w_{n-k} f_k|, for a run of n sequential additions (2048 history
# rows per far-field chunk: 4.5e-13); measured up to 56 eps (1.2e-14) where
# every late term has one sign (a trajectory settling on an equilibrium),
# 2-8 eps otherwise.  1e-13 of the term size (450 eps), with the two sides'
# weights within 1.2e-15 relative and 1e-14 of the state's scale for the
# update's own rounding.  A wrong term, index or weight moves y_s by at least
# one term h^alpha w f, ten or more orders of magnitude above this.
EPS_TERMS = 1e-13
EPS_STATE = 1e-14


def sampled_steps(N, L=256, seed=0):
    """Block boundaries of the first blocks, 1024-row chunk and 8192-row slice
    boundaries, the middle, the last blocks and the ragged end, plus 20
    seeded draws."""
    s = {1, 2, 3, L - 1, L, L + 1, 2 * L - 1, 2 * L, 2 * L + 1, 3 * L, 3 * L + 1,
         1023, 1024, 1025, 8191, 8192, 8193, 16385, 65536, 65537, 131073,
         N // 2, N // 2 + 1, N - L - 1, N - L, N - L + 1, N - (N % L) if N % L else N - L,
         N - 64, N - 2, N - 1, N}
    s |= set(int(v) for v in np.random.default_rng(seed).integers(1, N + 1, 20))
    return sorted(v for v in s if 1 <= v <= N)


def recompute_errors(p, y, s_list):
    """|y_s - oracle step from y_0..y_{s-1}| per listed step and component,
    and the size of that step's history terms (y: every state, stride 1)."""
    ys, scale = O.steps_from_states(RID[p.rhs], p.alpha, p.h, p.x0, p.p, y[:-1], s_list,
                                    x1=p.x1, return_scale=True, compensated=True)
    return np.abs(y[s_list] - ys), scale


def check_steps_fp64(p, y, s_list):
    """Every listed step within the double-precision bound; returns the
    largest error relative to its bound."""
    err, scale = recompute_errors(p, y, s_list)
    bound = EPS_TERMS * scale + EPS_STATE * np.max(np.abs(y))
    ratio = np.max(err / bound, axis=1)
    worst = float(np.max(ratio))
    assert worst <= 1.0, (p.rhs, p.N, s_list[int(np.argmax(ratio))], float(np.max(err)))
    return worst
