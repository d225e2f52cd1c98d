"""Write the stored oracle values used by the full-size GPU parity tests.

Calls only the CPU oracle (oracle/) on the seeded workloads of
paper_1710_01133_amd.inputs; nothing here touches the GPU library.  Run from
the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1710_01133_amd import inputs  # noqa: E402

RID = {"LINEAR": O.RHS_LINEAR, "DUFFING": O.RHS_DUFFING, "LORENZ": O.RHS_LORENZ,
       "POLY": O.RHS_POLY, "LCR": O.RHS_LCR}
HERE = os.path.dirname(os.path.abspath(__file__))


def run(p, stride):
    t = time.time()
    y = O.solve(RID[p.rhs], p.alpha, p.h, p.N, p.x0, p.p, out_stride=stride)
    return y, time.time() - t


def main():
    out = {}
    # forced Duffing oscillator, alpha=0.9, h=1e-3, N=200000: every 1000th state
    p = inputs.duffing_single()
    y, dt = run(p, 1000)
    out["duffing_single"] = {"problem": p.__dict__, "out_stride": 1000, "y": y.tolist(),
                             "oracle_seconds": dt}
    print("duffing_single", dt, flush=True)
    # forcing sweep, alpha=0.95, h=2^-8, N=65536: four members, every 1024th state
    sweep = inputs.duffing_sweep()
    for idx in (0, 1, 511, 1023):
        q = sweep[idx]
        y, dt = run(q, 1024)
        out["duffing_sweep_%d" % idx] = {"problem": q.__dict__, "index": idx, "out_stride": 1024,
                                         "y": y.tolist(), "oracle_seconds": dt}
        print("sweep", idx, dt, flush=True)
    # the LCR forcing sweep (eq. sys.LRC): two members at both order pairs, the
    # Poincare section points (every 1142nd state) of the first 3600 steps
    M = inputs.LCR_SECTION_STEPS
    for al in ((0.9, 0.9), (0.9, 0.8)):
        sweep = inputs.lcr_sweep(alpha=al)
        for idx in (300, 700):
            q = sweep[idx]
            t = time.time()
            y = O.solve(RID["LCR"], q.alpha, q.h, 3600, q.x0, q.p, out_stride=M)
            out["lcr_sweep_%g_%g_%d" % (al[0], al[1], idx)] = {
                "problem": q.__dict__, "index": idx, "steps": 3600, "out_stride": M,
                "y": y.tolist(), "oracle_seconds": time.time() - t}
            print("lcr", al, idx, flush=True)
    # the serving stream (2000 requests, seed 1710): the first 16 Duffing
    # requests of at most 8192 steps, final state and largest |y|
    reqs = inputs.serving_stream()
    picked = [i for i, r in enumerate(reqs) if r.problem.rhs == "DUFFING" and r.problem.N <= 8192][:16]
    for i in picked:
        q = reqs[i].problem
        t = time.time()
        y = O.solve(RID["DUFFING"], q.alpha, q.h, q.N, q.x0, q.p, out_stride=1)
        out["serving_%d" % i] = {"problem": q.__dict__, "index": i, "final": y[-1].tolist(),
                                 "max_abs_y": float(np.max(np.abs(y))),
                                 "oracle_seconds": time.time() - t}
    print("serving", picked, flush=True)
    with open(os.path.join(HERE, "oracle_fullsize.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
