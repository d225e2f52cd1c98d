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
