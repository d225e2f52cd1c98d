"""GPU parity of the weight kernel and the plain per-step path (abm_solve)
against the CPU oracle, through the C ABI."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1710_01133_amd import abm, inputs
from gpu_common import TOL_FP64, golden, normerr, oracle_run, run_plain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    c = abm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("alpha", [0.3, 0.8, 0.9, 0.95, 1.0])
def test_device_weights_match_quad_oracle(ctx, alpha):
    N = 300000
    p = inputs.Problem("LINEAR", alpha, 0.01, N, (1.0,), (1.0,))
    plan = abm.Plan(ctx, [p])
    b, a, c = plan.weights(0, N)
    for lo, n in ((0, 4000), (N - 2000, 2000)):
        ob, oa, oc = O.weights(alpha, n, k0=lo)
        for dev, ref in ((b, ob), (a, oa), (c, oc)):
            rel = np.max(np.abs(dev[lo:lo + n] - ref) / np.abs(ref))
            if alpha == 1.0:
                # series collapse to 1, 1, 1/2; only the device Gamma can round
                assert rel <= 2.3e-16
            else:
                assert rel <= 1.2e-15, (alpha, lo, rel)
    plan.close()


def test_linear_mittag_leffler_workload(ctx):
    p = inputs.linear_c()
    y = run_plain(ctx, p, 1)
    ref = oracle_run(p, 1)
    assert normerr(y, ref) <= TOL_FP64


CASES = [
    ("LINEAR", 0.7, 0.01, (1.0,), (1.3,)),
    ("DUFFING", 0.9, 1e-2, (0.1, 0.0), (0.1, 0.3, 1.2)),
    ("LORENZ", 0.95, 2 ** -8, (1.0, 1.0, 1.0), (10.0, 28.0, 8 / 3)),
    ("POLY", 0.55, 1 / 64, (0.25,), (0.7, -0.3)),
    ("LCR", 0.9, 0.05, (1.2, -0.4), (1.015, 0.55, -1.02, -0.58, 0.117)),
]


@pytest.mark.parametrize("N", [1, 2, 255, 256, 257, 1000, 3001])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_plain_small_vs_oracle(ctx, case, N):
    rhs, alpha, h, x0, pp = case
    p = inputs.Problem(rhs, alpha, h, N, x0, pp)
    for stride in (1, 0, 7):
        y = run_plain(ctx, p, stride)
        assert normerr(y, oracle_run(p, stride)) <= TOL_FP64, (rhs, N, stride)


@pytest.mark.parametrize("G,N", [(1, 4000), (3, 4000), (64, 4000), (256, 4000),
                                 (1, 8192), (2, 8192), (5, 9000), (1, 300)])
def test_plain_workgroup_counts(ctx, G, N, monkeypatch):
    """Workgroup counts from one (no cross-workgroup synchronisation) to more
    than there are history chunks, so that each register-prefetch size
    (1..16 local chunks) and the in-step loads of more than 16 local chunks
    (G = 1 at N = 8192: 32 chunks) all run."""
    monkeypatch.setenv("ABM_PLAIN_G", str(G))
    p = inputs.duffing_single(N=N)
    y = run_plain(ctx, p, 1)
    assert normerr(y, oracle_run(p, 1)) <= TOL_FP64


@pytest.mark.parametrize("G", [1, 2, 65])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 9, 12])
def test_plain_pipeline_start_and_end(ctx, G, N, monkeypatch):
    """The cooperative kernel's all-reduce runs four steps ahead of the
    update: runs shorter than twice that cover steps with no published
    partials, the first published ones and the last; 65 workgroups put two
    of them on some lanes of the synchronising wave."""
    monkeypatch.setenv("ABM_PLAIN_G", str(G))
    p = inputs.duffing_single(N=N)
    for stride in (1, 0):
        y = run_plain(ctx, p, stride)
        assert normerr(y, oracle_run(p, stride)) <= TOL_FP64, (G, N, stride)


@pytest.mark.parametrize("G", [1, 2, 7])
def test_plain_workgroup_counts_per_component_orders(ctx, G, monkeypatch):
    """Two weight tables (incommensurate orders) halve the register prefetch:
    local chunk counts of 3, 8 and 15 (in-step loads) at N = 3600 (t = 36,
    inside the span where the chaotic circuit's rounding noise stays below
    1e-13)."""
    monkeypatch.setenv("ABM_PLAIN_G", str(G))
    p = inputs.Problem("LCR", (0.9, 0.8), 0.01, 3600, (1.2, -0.4),
                       (1.015, 0.55, -1.02, -0.58, 0.117))
    y = run_plain(ctx, p, 1)
    assert normerr(y, oracle_run(p, 1)) <= TOL_FP64


def test_plain_is_deterministic(ctx):
    p = inputs.duffing_single(N=5000)
    y1 = run_plain(ctx, p, 1)
    y2 = run_plain(ctx, p, 1)
    assert np.array_equal(y1, y2)


def test_plain_duffing_20000_steps(ctx):
    p = inputs.duffing_single(N=20000)
    y = run_plain(ctx, p, 1)
    assert normerr(y, oracle_run(p, 1)) <= TOL_FP64


def test_plain_duffing_full_size(ctx):
    """N = 200000 at the launch shape the benchmark times: every 1000th state
    against the stored oracle run, and single steps recomputed by the oracle
    from the GPU's own history at sampled s (including the ragged end)."""
    p = inputs.duffing_single()
    y = run_plain(ctx, p, 1)
    g = golden()["duffing_single"]
    assert normerr(y[::1000], np.array(g["y"])) <= TOL_FP64
    s_list = [1, 2, 255, 256, 257, 65535, 65536, 123457, 199999, 200000]
    ys = O.steps_from_states(O.RHS_DUFFING, p.alpha, p.h, p.x0, p.p, y[:-1], s_list)
    assert normerr(y[s_list], ys) <= 1e-13


def test_plain_rejects_mismatched_problem(ctx):
    p = inputs.duffing_single(N=100)
    plan = abm.Plan(ctx, [p], out_stride=1)
    y = abm.alloc_out(p, 1)
    q = inputs.duffing_single(N=101)
    with pytest.raises(abm.AbmError) as e:
        abm.solve(plan, q, y)
    assert e.value.code == abm.ABM_EINVAL
    bad = inputs.Problem("DUFFING", 2.5, 0.01, 100, (0.1, 0.0), (0.1, 0.3, 1.2))
    with pytest.raises(abm.AbmError) as e:
        abm.Plan(ctx, [bad])
    assert e.value.code == abm.ABM_EINVAL
    plan.close()
