"""The double-double mode (ABM_FAR_DD: every weight, sum, state and
right-hand side in double-double, the counterpart of the paper's long-double
runs) on the GPU, through the C ABI, against the quad oracle and 50-digit
values.

Bounds: double-double carries about 106 bits (2^-104 ~ 5e-32 per operation);
the quad oracle 113 bits, with weights good to about 1e-33 (k+2).  The
comparisons allow 1e-25 of the state's scale for whole trajectories (N up to
8192) and, for the sampled steps of the 200000-step run, 1e-26 of the size of
each step's history terms: about nine orders of magnitude tighter than the
double path's bar (1e-12), so a double-rounded weight, Gamma factor, h^alpha,
forcing or history value (1e-16) fails them."""
import mpmath as mp
import numpy as np
import pytest

import oracle as O
from paper_1710_01133_amd import abm, inputs
from gpu_common import RID, sampled_steps

pytestmark = pytest.mark.gpu

TOL_DD = 1e-25          # normwise, whole trajectories
TOL_DD_TERMS = 1e-26    # per step, of h^alpha sum |w f|
LCR = (1.015, 0.55, -1.02, -0.58, 0.117)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    c = abm.Context(0)
    yield c
    c.close()


def dd_problem(p):
    return inputs.Problem(p.rhs, p.alpha, p.h, p.N, p.x0, p.p, "dd", p.x1)


def run_dd(ctx, p, stride):
    p = dd_problem(p)
    plan = abm.Plan(ctx, [p], out_stride=stride)
    y = abm.alloc_out(p, stride)
    abm.solve(plan, p, y)
    plan.check()
    out = y.cpu().numpy()
    plan.close()
    return out


def err_pairs(y, q):
    """max |y - q| over max |q| for (.., 2) arrays of (hi, lo) pairs."""
    diff = (y[..., 0] - q[..., 0]) + (y[..., 1] - q[..., 1])
    return float(np.max(np.abs(diff)) / max(np.max(np.abs(q[..., 0])), 1e-300))


def quad_run(p, stride):
    return O.solve_quad(RID[p.rhs], p.alpha, p.h, p.N, p.x0, p.p, out_stride=stride, x1=p.x1)


@pytest.mark.parametrize("alpha", [0.3, 0.9, 1.0, 1.5, 2.0])
def test_dd_weights_match_50_digits(ctx, alpha):
    """The device series (double-double) against 50-digit evaluations of the
    literal formulas of Section 2, including Gamma(alpha+1) and Gamma(alpha+2)
    (through b_0 = 1/Gamma(alpha+1) and a_0 = (2^(alpha+1) - 2)/Gamma(alpha+2)).
    Bound 1e-29: Gamma comes from Stirling's series after a shift by 40, about
    a hundred double-double operations of 2^-104 each (3e-30 measured), while
    a weight rounded to double anywhere is off by about 1e-16."""
    N = 200000
    p = inputs.Problem("LINEAR", alpha, 0.01, N, (1.0,), (1.0,), "dd",
                       x1=(0.0,) if alpha > 1 else None)
    plan = abm.Plan(ctx, [p])
    b, a, c = plan.weights(0, N)
    plan.close()
    with mp.workdps(50):
        al = mp.mpf(alpha)
        g1, g2 = mp.gamma(al + 1), mp.gamma(al + 2)
        worst = 0.0
        for k in (0, 1, 2, 3, 5, 17, 1000, 65535, 199000, 199999):
            km = mp.mpf(k)
            rb = ((km + 1) ** al - (km ** al if k else 0)) / g1
            ra = ((km + 2) ** (al + 1) - 2 * (km + 1) ** (al + 1) + (km ** (al + 1) if k else 0)) / g2
            rc = ((km ** (al + 1) if k else 0) - (km - al) * (km + 1) ** al) / g2
            for got, ref in ((b[k], rb), (a[k], ra), (c[k], rc)):
                v = mp.mpf(float(got[0])) + mp.mpf(float(got[1]))
                worst = max(worst, float(abs(v - ref) / abs(ref)))
    print("alpha", alpha, "largest relative weight error %.3g" % worst)
    assert worst <= 1e-29


CASES = [
    ("LINEAR", 0.7, 0.01, (1.0,), (1.3,), None),
    ("DUFFING", 0.9, 1e-2, (0.1, 0.0), (0.1, 0.3, 1.2), None),
    ("LORENZ", 0.95, 2 ** -8, (1.0, 1.0, 1.0), (10.0, 28.0, 8 / 3), None),
    ("POLY", 0.55, 1 / 64, (0.25,), (0.7, -0.3), None),
    ("LCR", 0.9, 0.05, (1.2, -0.4), LCR, None),
    ("LCR", (0.9, 0.8), 0.05, (1.2, -0.4), LCR, None),
    ("DIAG", (0.6, 0.95), 1 / 64, (1.0, -0.5), (1.3, 0.7, 0.2, -0.1), None),
    ("LINEAR", 1.5, 1 / 64, (1.0,), (1.0,), (0.5,)),
]


@pytest.mark.parametrize("N", [1, 2, 257, 1000, 3001])
@pytest.mark.parametrize("case", CASES, ids=["%s-%s" % (c[0], c[1]) for c in CASES])
def test_dd_small_vs_quad_oracle(ctx, case, N):
    rhs, alpha, h, x0, pp, x1 = case
    p = inputs.Problem(rhs, alpha, h, N, x0, pp, x1=x1)
    q1 = quad_run(p, 1)                     # every state; the strides below subsample it
    for stride in (1, 0, 7):
        if stride == 1:
            q = q1
        elif stride == 0:
            q = q1[-1:]
        else:
            q = q1[::stride] if N % stride == 0 else np.concatenate([q1[::stride], q1[-1:]])
        e = err_pairs(run_dd(ctx, p, stride), q)
        assert e <= TOL_DD, (rhs, N, stride, e)


@pytest.mark.parametrize("G", [1, 2, 3, 50])
def test_dd_cooperative_workgroup_counts(ctx, G, monkeypatch):
    """The cooperative double-double kernel at forced workgroup counts (the
    history of 3000 steps would otherwise run in one workgroup): 12 local
    chunks in one workgroup (no flags: the sums come from its own LDS), 6
    (weights loaded in the step), 4 (weights prefetched) and 1."""
    monkeypatch.setenv("ABM_PLAIN_G", str(G))
    p = inputs.duffing_single(N=3000, h=1e-2)
    assert err_pairs(run_dd(ctx, p, 1), quad_run(p, 1)) <= TOL_DD


@pytest.mark.parametrize("G", [1, 2, 65])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 9, 12])
def test_dd_pipeline_start_and_end(ctx, G, N, monkeypatch):
    """The cooperative kernel's all-reduce runs four steps ahead of the
    update: runs shorter than twice that cover steps with no published
    partials, the first published ones and the last; 65 workgroups put two
    of them on some lanes of the synchronising wave."""
    monkeypatch.setenv("ABM_PLAIN_G", str(G))
    p = inputs.duffing_single(N=N, h=1e-2)
    for stride in (1, 0):
        assert err_pairs(run_dd(ctx, p, stride), quad_run(p, stride)) <= TOL_DD, (G, N, stride)


COOP_CASES = [c for c in CASES if c[0] in ("LORENZ", "DIAG") or c[1] == (0.9, 0.8)]


@pytest.mark.parametrize("case", COOP_CASES, ids=["%s-%s" % (c[0], c[1]) for c in COOP_CASES])
def test_dd_cooperative_systems(ctx, case, monkeypatch):
    """Three components and per-component orders (a weight table each) in the
    cooperative kernel: 5 workgroups over 2000 steps."""
    rhs, alpha, h, x0, pp, x1 = case
    monkeypatch.setenv("ABM_PLAIN_G", "5")
    p = inputs.Problem(rhs, alpha, h, 2000, x0, pp, x1=x1)
    assert err_pairs(run_dd(ctx, p, 1), quad_run(p, 1)) <= TOL_DD, rhs


def test_dd_scalar_linear_workload(ctx):
    """D^0.8 y = -y, N = 8192, h = 2^-10, every state."""
    p = inputs.linear_c()
    e = err_pairs(run_dd(ctx, p, 1), quad_run(p, 1))
    print("linear N=8192: double-double vs quad %.3g" % e)
    assert e <= TOL_DD


def test_dd_single_oscillator_full_length_steps(ctx):
    """The 200000-step oscillator in double-double: sampled steps recomputed
    in quad from the GPU's own states, each within 1e-26 of its history
    terms' size (the double recompute supplies that size)."""
    p = inputs.duffing_single()
    y = run_dd(ctx, p, 1)
    assert np.all(np.isfinite(y))
    s_list = sampled_steps(p.N, seed=3)
    q = O.steps_from_states_quad(O.RHS_DUFFING, p.alpha, p.h, p.x0, p.p, y[:-1], s_list)
    _, scale = O.steps_from_states(O.RHS_DUFFING, p.alpha, p.h, p.x0, p.p, y[:-1, :, 0], s_list,
                                   return_scale=True)
    err = np.abs((y[s_list, :, 0] - q[..., 0]) + (y[s_list, :, 1] - q[..., 1]))
    # a floor of 1e-30 of the state's scale: the corrector's f(t, y^P) term and
    # the update itself round too, and a step whose history terms vanish (the
    # first velocity step from rest) has no term size to measure against
    bound = TOL_DD_TERMS * scale + 1e-30 * np.max(np.abs(y[..., 0]))
    ratio = float(np.max(err / bound))
    print("oscillator N=200000: largest step error over its bound %.3g" % ratio)
    assert ratio <= 1.0


def test_dd_nonfinite_reports_edevice(ctx):
    p = inputs.Problem("LINEAR", 0.9, 0.01, 2000, (1.0,), (-50.0,), "dd")
    plan = abm.Plan(ctx, [p], out_stride=0)
    y = abm.alloc_out(p, 0)
    abm.solve(plan, p, y)
    with pytest.raises(abm.AbmError) as e:
        plan.check()
    assert e.value.code == abm.ABM_EDEVICE
    plan.close()


def test_dd_is_refused_where_it_does_not_run(ctx):
    p = dd_problem(inputs.duffing_single(N=500))
    y = abm.alloc_out(p, 0)
    with pytest.raises(abm.AbmError) as e:
        abm.Plan(ctx, [p, p])                       # one trajectory per plan
    assert e.value.code == abm.ABM_EINVAL
    plan = abm.Plan(ctx, [p])
    with pytest.raises(abm.AbmError) as e:
        abm.solve_batch(plan, [p], [y])             # no blocked path
    assert e.value.code == abm.ABM_EINVAL
    plan.close()
    with pytest.raises(abm.AbmError) as e:
        abm.submit(ctx, p, y)                       # not served
    assert e.value.code == abm.ABM_EINVAL
    with pytest.raises(abm.AbmError) as e:
        abm.solve_noalloc(p, y)
    assert e.value.code == abm.ABM_EINVAL
