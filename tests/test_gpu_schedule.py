"""The tick schedule of the blocked batch path changes only timing: with the
chain and far-field streams alternating per tick or fixed, with chains spread
one wave per SIMD or packed two per SIMD, and eager or graph-replayed, every
trajectory's result is bitwise the same (each sum keeps its order), and the
double members match the oracle."""
import numpy as np
import pytest

from paper_1710_01133_amd import abm, inputs
from gpu_common import TOL_FP64, normerr, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    c = abm.Context(0)
    yield c
    c.close()


def _mix():
    rng = np.random.default_rng(17)
    probs = []
    precs = ["fp64", "fp16x3", "fp64", "bf16x6", "fp32", "fp64"]
    for i, N in enumerate([2100, 1537, 1800, 999, 2048, 300]):
        A = float(rng.uniform(0.1, 0.6))
        probs.append(inputs.Problem("DUFFING", 0.95, 2 ** -7, N, (0.1, 0.0), (0.1, A, 1.2),
                                    far_prec=precs[i]))
    probs.append(inputs.Problem("LCR", (0.9, 0.8), 0.01, 1700, (0.2, 0.1), inputs.LCR_P + (0.1,)))
    probs.append(inputs.Problem("LORENZ", 0.93, 2 ** -8, 1100, (1.0, 1.0, 1.0), (10.0, 28.0, 8 / 3)))
    return probs


def _run(ctx, probs, stride, monkeypatch, alt, spread, graph):
    monkeypatch.setenv("ABM_CHAIN_SPREAD", str(spread))
    monkeypatch.setenv("ABM_ALT_STREAMS", str(alt))
    plan = abm.Plan(ctx, probs, out_stride=stride)
    plan.graph(graph)
    out = None
    for _ in range(2 if graph else 1):    # capture, then a replay
        ys = [abm.alloc_out(p, stride) for p in probs]
        abm.solve_batch(plan, probs, ys)
        plan.check()
        out = [y.cpu().numpy() for y in ys]
    plan.close()
    return out


def test_schedules_bitwise_equal(ctx, monkeypatch):
    monkeypatch.setenv("ABM_BLOCK_L", "256")
    monkeypatch.setenv("ABM_KCHUNK", "512")
    monkeypatch.setenv("ABM_MAX_SPLIT", "2")
    probs = _mix()
    stride = 7
    ref = _run(ctx, probs, stride, monkeypatch, alt=1, spread=101, graph=False)
    for alt, spread, graph in [(0, 101, False), (1, 0, False), (0, 0, False), (1, 70, False),
                               (1, 101, True), (0, 0, True)]:
        got = _run(ctx, probs, stride, monkeypatch, alt, spread, graph)
        for i, (a, b) in enumerate(zip(ref, got)):
            assert np.array_equal(a, b), (alt, spread, graph, i)
    for i in (0, 2, 5):
        assert normerr(ref[i], oracle_run(probs[i], stride)) <= TOL_FP64
