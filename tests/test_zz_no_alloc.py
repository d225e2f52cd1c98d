"""abm_solve_noalloc, the plain solve for callers that cannot allocate device
memory, through the C ABI: bitwise equal to abm_solve (same kernels, same
launch shape) and within the oracle bar, on calls in a row where the later
call is smaller (the workspace keeps the earlier call's contents), in the
one-workgroup and the cooperative form, with per-component orders; and a
problem larger than the workspace refused."""
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
    torch.cuda.set_device(0)
    c = abm.Context(0)
    yield c
    c.close()


def _plan_solve(ctx, p, stride):
    plan = abm.Plan(ctx, [p], out_stride=stride)
    y = abm.alloc_out(p, stride)
    abm.solve(plan, p, y)
    plan.check()
    out = y.cpu().numpy()
    plan.close()
    return out


def _noalloc(p, stride):
    import torch
    y = abm.alloc_out(p, stride)
    torch.cuda.synchronize()
    abm.solve_noalloc(p, y, stride)
    torch.cuda.synchronize()
    return y.cpu().numpy()


LCR = (1.015, 0.55, -1.02, -0.58, 0.117)


@pytest.mark.parametrize("seq", ["single", "cooperative"])
def test_noalloc_equals_abm_solve_on_calls_in_a_row(ctx, seq):
    if seq == "single":
        # one-workgroup form: 3000 steps of the oscillator, then 1700 steps of
        # the circuit with two orders (two weight tables)
        calls = [(inputs.duffing_single(N=3000, h=1e-2), 1),
                 (inputs.Problem("LCR", (0.9, 0.8), 0.01, 1700, (1.2, -0.4), LCR), 7)]
    else:
        # cooperative form (history larger than one CU), then a smaller one
        calls = [(inputs.duffing_single(N=20000), 1),
                 (inputs.duffing_single(N=12001, h=2e-3, A=0.45), 3)]
    for p, stride in calls:
        y = _noalloc(p, stride)
        ref = _plan_solve(ctx, p, stride)
        assert np.array_equal(y, ref), (p.rhs, p.N)
        assert normerr(y, oracle_run(p, stride)) <= TOL_FP64


def test_noalloc_refuses_a_problem_larger_than_its_workspace(ctx):
    """The stated limit, exactly: with one order the 8 MiB workspace holds
    N = 341952 steps ((N + 2048) 8-byte weights in three tables, 256-byte
    aligned, after the status word, the flags and 8 partial slots of 256
    workgroups); one step more is refused."""
    p = inputs.Problem("LINEAR", 0.8, 1e-3, 341953, (1.0,), (1.0,))
    y = abm.alloc_out(p, 0)
    with pytest.raises(abm.AbmError) as e:
        abm.solve_noalloc(p, y, 0)
    assert e.value.code == abm.ABM_EINVAL
    p = inputs.Problem("LINEAR", 0.8, 1e-3, 341952, (1.0,), (1.0,))
    y = abm.alloc_out(p, 0)
    abm.solve_noalloc(p, y, 0)
    assert np.array_equal(y.cpu().numpy(), _plan_solve(ctx, p, 0))
