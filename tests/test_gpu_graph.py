"""Graph replay of the blocked batch path (abm_plan_graph): the launch
sequence captured once per plan and replayed gives bitwise the eager results,
on every replay, with the program's own eager work and synchronisations
between replays, new per-solve parameters and new output buffers."""
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


def _mix(seed, amp_shift=0.0):
    rng = np.random.default_rng(seed)
    probs = []
    for i, N in enumerate([1500, 900, 1333, 257, 1024, 64]):
        A = float(rng.uniform(0.1, 0.6)) + amp_shift
        probs.append(inputs.Problem("DUFFING", 0.95, 2 ** -7, N, (0.1, 0.0), (0.1, A, 1.2),
                                    far_prec="fp64" if i % 2 == 0 else "fp32"))
    probs.append(inputs.Problem("LORENZ", 0.93, 2 ** -8, 1100, (1.0, 1.0, 1.0 + amp_shift),
                                (10.0, 28.0, 8 / 3)))
    probs.append(inputs.Problem("LINEAR", 0.8, 2 ** -7, 700, (1.0,), (1.0 + amp_shift,)))
    return probs


def _solve(plan, probs, stride):
    ys = [abm.alloc_out(p, stride) for p in probs]
    st = abm.solve_batch(plan, probs, ys)
    plan.check()
    return [y.cpu().numpy() for y in ys], st


def _busy_work():
    """Unrelated eager work on torch's stream between graph replays."""
    import torch
    a = torch.randn(512, 512, device="cuda")
    for _ in range(4):
        a = torch.tanh(a @ a.T / 512.0)
    torch.cuda.synchronize()
    return float(a.sum())


@pytest.mark.parametrize("L", [128, 256])
def test_graph_replays_match_eager(ctx, L, monkeypatch):
    monkeypatch.setenv("ABM_BLOCK_L", str(L))
    monkeypatch.setenv("ABM_KCHUNK", "512")
    monkeypatch.setenv("ABM_MAX_SPLIT", "2")
    stride = 3
    p0, p1 = _mix(5), _mix(6, amp_shift=0.05)
    eager = abm.Plan(ctx, p0, out_stride=stride)
    ref0, st_e = _solve(eager, p0, stride)
    ref1, _ = _solve(eager, p1, stride)
    eager.close()

    plan = abm.Plan(ctx, p0, out_stride=stride)
    plan.graph(True)
    for rep, (probs, ref) in enumerate([(p0, ref0), (p1, ref1), (p0, ref0), (p1, ref1)]):
        _busy_work()
        out, st = _solve(plan, probs, stride)        # fresh output buffers every replay
        assert st["far_launches"] == st_e["far_launches"]
        assert st["chain_launches"] == st_e["chain_launches"]
        for i, (y, r) in enumerate(zip(out, ref)):
            assert np.array_equal(y, r), (L, rep, i, float(np.max(np.abs(y - r))))
    plan.close()
    # and the eager results themselves are the method's
    tol = {"fp64": TOL_FP64, "fp32": 1e-6}
    for p, y in zip(p1, ref1):
        assert normerr(y, oracle_run(p, stride)) <= tol[p.far_prec], (p.rhs, p.N)


def test_graph_off_after_on_and_timing_runs_eagerly(ctx):
    probs = _mix(9)
    plan = abm.Plan(ctx, probs, out_stride=0)
    plan.graph(True)
    a, _ = _solve(plan, probs, 0)
    plan.timing(True)                       # timed solves bypass the graph
    b, st = _solve(plan, probs, 0)
    assert st["far_ms"] > 0 and st["chain_ms"] > 0
    plan.timing(False)
    plan.graph(False)
    c, _ = _solve(plan, probs, 0)
    plan.graph(True)                        # the captured graph is reused
    d, _ = _solve(plan, probs, 0)
    plan.close()
    for x in (b, c, d):
        for y, r in zip(x, a):
            assert np.array_equal(y, r)
