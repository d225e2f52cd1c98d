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
    with open(os.path.join(HERE, "oracle_fullsize.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
