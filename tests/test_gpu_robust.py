"""Failure isolation and thread safety of the boundary, on the GPU.

* A trajectory whose state overflows (finite arithmetic reaching +-inf / NaN,
  nothing faults) fails on its own: in a batch abm_plan_check reports
  ABM_EDEVICE while every other member still matches the oracle; in the
  serving loop only that request's result carries ABM_EDEVICE.
* abm_submit / abm_poll from many threads on a fresh context: unique tickets,
  every result equal to the oracle.
* Destroying a context with queued and running requests, and a server whose
  arena cannot be allocated, end without touching freed requests.
* A device-side wait of the cooperative plain kernels that cannot be met
  (forced from the host) gives up within its bound in every workgroup.
"""
import threading
import time

import numpy as np
import pytest

from paper_1710_01133_amd import abm, inputs
from gpu_common import TOL_FP64, normerr, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_ready():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch


def _wait(ctx, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            r = abm.poll(ctx, t)
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.002)
    return out


# Overflowing problems: D^0.9 y = 50 y grows like E_0.9(50 t^0.9) and reaches
# +inf near t = 10; the oscillator started at x0 = 1000 has a cubic restoring
# force of 1e9 that the explicit predictor overshoots, NaN within 10 steps.
def _overflow_linear(N=3000, prec="fp64"):
    return inputs.Problem("LINEAR", 0.9, 0.01, N, (1.0,), (-50.0,), prec)


def _overflow_duffing(N=3000, prec="fp64"):
    return inputs.Problem("DUFFING", 0.95, 2 ** -8, N, (1e3, 0.0), inputs.DUFFING_P, prec)


def _good_duffing(A, N=3000, prec="fp64"):
    return inputs.Problem("DUFFING", 0.95, 2 ** -8, N, (0.1, 0.0), (0.1, A, 1.2), prec)


@pytest.mark.parametrize("prec,tol", [("fp64", TOL_FP64), ("fp16x3", 1e-6)])
def test_nonfinite_member_fails_alone_in_batch(torch_ready, prec, tol):
    """The overflowing oscillator shares its group (same order, system and
    precision) with three good ones, so their columns meet in the same
    far-field products; the overflowing linear equation is a group of its own."""
    good = [_good_duffing(A, prec=prec) for A in (0.15, 0.3, 0.55)]
    probs = good[:2] + [_overflow_duffing(prec=prec)] + good[2:] + [_overflow_linear(prec=prec)]
    ctx = abm.Context(0)
    plan = abm.Plan(ctx, probs, out_stride=1)
    ys = [abm.alloc_out(p, 1) for p in probs]
    abm.solve_batch(plan, probs, ys)
    with pytest.raises(abm.AbmError) as e:
        plan.check()
    assert e.value.code == abm.ABM_EDEVICE
    for p, y in zip(probs, ys):
        out = y.cpu().numpy()
        if p.x0[0] == 1e3 or p.rhs == "LINEAR":
            assert not np.all(np.isfinite(out))
        else:
            assert normerr(out, oracle_run(p, 1)) <= tol, p.p
    # the status was cleared by the check: the same plan with benign
    # parameters for the two overflowing members runs clean
    fixed = list(probs)
    fixed[2] = _good_duffing(0.4, prec=prec)
    fixed[4] = inputs.Problem("LINEAR", 0.9, 0.01, 3000, (1.0,), (1.0,), prec)
    abm.solve_batch(plan, fixed, ys)
    plan.check()
    for p, y in zip(fixed, ys):
        assert normerr(y.cpu().numpy(), oracle_run(p, 1)) <= tol
    plan.close()
    ctx.close()


def test_nonfinite_plain_path_reports_edevice(torch_ready):
    p = _overflow_linear(N=2000)
    ctx = abm.Context(0)
    plan = abm.Plan(ctx, [p], out_stride=0)
    y = abm.alloc_out(p, 0)
    abm.solve(plan, p, y)
    with pytest.raises(abm.AbmError) as e:
        plan.check()
    assert e.value.code == abm.ABM_EDEVICE
    assert not np.isfinite(y.cpu().numpy()).all()
    plan.close()
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "dd"])
def test_cooperative_wait_that_cannot_be_met_gives_up(torch_ready, prec, monkeypatch):
    """The cooperative plain kernels' bounded waits, forced from the host to
    fail: the ABM_WAIT_BIAS test hook raises every awaited step number by 2^30
    (no flag reaches it) and ABM_SPIN_LIMIT bounds each wait at 64 polls.
    Every workgroup gives up and exits, abm_plan_check reports ABM_EDEVICE,
    the final state reads NaN, and the next solve on the same context (hooks
    cleared) matches the oracle."""
    monkeypatch.setenv("ABM_PLAIN_G", "3")
    monkeypatch.setenv("ABM_SPIN_LIMIT", "64")
    monkeypatch.setenv("ABM_WAIT_BIAS", str(1 << 30))
    base = inputs.duffing_single(N=3000, h=1e-2)
    p = inputs.Problem(base.rhs, base.alpha, base.h, base.N, base.x0, base.p, prec)
    ctx = abm.Context(0)
    plan = abm.Plan(ctx, [p], out_stride=0)
    y = abm.alloc_out(p, 0)
    abm.solve(plan, p, y)
    with pytest.raises(abm.AbmError) as e:
        plan.check()
    assert e.value.code == abm.ABM_EDEVICE
    assert np.isnan(y.cpu().numpy()).all()
    monkeypatch.delenv("ABM_WAIT_BIAS")
    monkeypatch.delenv("ABM_SPIN_LIMIT")
    plan.close()
    plan = abm.Plan(ctx, [p], out_stride=0)
    abm.solve(plan, p, y)
    plan.check()
    out = y.cpu().numpy()
    if prec == "dd":
        out = out[..., 0] + out[..., 1]
    assert normerr(out, oracle_run(base, 0)) <= TOL_FP64
    plan.close()
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_request_fails_alone_in_serving(torch_ready, prec):
    probs = [_good_duffing(0.2, N=2500, prec=prec), _overflow_duffing(N=2200, prec=prec),
             inputs.Problem("LORENZ", 0.95, 2 ** -8, 1800, (1.0, 1.0, 1.0), inputs.LORENZ_P, prec),
             _overflow_linear(N=2600, prec=prec), _good_duffing(0.5, N=3100, prec=prec)]
    tol = TOL_FP64 if prec == "fp64" else 1e-6
    ctx = abm.Context(0, arena_bytes=256 << 20)
    ys = [abm.alloc_out(p, 1) for p in probs]
    tickets = [abm.submit(ctx, p, y, out_stride=1) for p, y in zip(probs, ys)]
    res = _wait(ctx, tickets)
    torch_ready.cuda.synchronize()
    for p, y, t in zip(probs, ys, tickets):
        overflow = p.x0[0] == 1e3 or p.rhs == "LINEAR"
        if overflow:
            assert res[t]["status"] == abm.ABM_EDEVICE, (p.rhs, res[t])
        else:
            assert res[t]["status"] == abm.ABM_OK, (p.rhs, res[t])
            assert normerr(y.cpu().numpy(), oracle_run(p, 1)) <= tol
    # the server keeps serving after a failed request
    q = _good_duffing(0.33, N=1500, prec=prec)
    yq = abm.alloc_out(q, 1)
    r = _wait(ctx, [abm.submit(ctx, q, yq, out_stride=1)])
    assert list(r.values())[0]["status"] == abm.ABM_OK
    assert normerr(yq.cpu().numpy(), oracle_run(q, 1)) <= tol
    ctx.close()


def test_concurrent_submits_on_a_fresh_context(torch_ready):
    """8 threads submit 4 requests each at once (ctypes releases the GIL
    around every call), then poll their own tickets."""
    n_thr, per = 8, 4
    rng = np.random.default_rng(5)
    probs = []
    for i in range(n_thr * per):
        N = int(rng.integers(300, 2500))
        if i % 3 == 2:
            probs.append(inputs.Problem("LORENZ", float(rng.uniform(0.9, 0.99)), 2 ** -8, N,
                                        (1.0, 1.0, 1.0), inputs.LORENZ_P))
        else:
            probs.append(_good_duffing(float(rng.uniform(0.1, 0.6)), N=N))
    ys = [abm.alloc_out(p, 1) for p in probs]
    torch_ready.cuda.synchronize()
    ctx = abm.Context(0, arena_bytes=512 << 20)
    start = threading.Barrier(n_thr)
    tickets = [None] * len(probs)
    results = [None] * len(probs)
    errors = []

    def worker(w):
        try:
            mine = list(range(w * per, (w + 1) * per))
            start.wait()
            for i in mine:
                tickets[i] = abm.submit(ctx, probs[i], ys[i], out_stride=1)
            got = _wait(ctx, [tickets[i] for i in mine])
            for i in mine:
                results[i] = got[tickets[i]]
        except Exception as exc:   # reported by the main thread
            errors.append(repr(exc))

    threads = [threading.Thread(target=worker, args=(w,)) for w in range(n_thr)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=180)
    assert not errors, errors
    assert len(set(tickets)) == len(tickets)
    torch_ready.cuda.synchronize()
    for p, y, r in zip(probs, ys, results):
        assert r["status"] == abm.ABM_OK
        assert normerr(y.cpu().numpy(), oracle_run(p, 1)) <= TOL_FP64
    # every ticket was collected exactly once
    for t in tickets:
        with pytest.raises(abm.AbmError) as e:
            abm.poll(ctx, t)
        assert e.value.code == abm.ABM_ENOENT
    ctx.close()


def test_destroy_context_with_queued_and_running_requests(torch_ready):
    """A context destroyed right after its submits (some requests running,
    the rest queued behind a small arena), and one destroyed after a poll
    collected part of them; a fresh context then serves normally."""
    probs = [_good_duffing(0.1 + 0.05 * i, N=4000 + 500 * i) for i in range(8)]
    ys = [abm.alloc_out(p, 1) for p in probs]
    sizer = abm.Context(0)
    need = max(abm.request_bytes(sizer, p, 1) for p in probs)
    sizer.close()
    for collect_first in (False, True):
        ctx = abm.Context(0, arena_bytes=2 * need)      # two at a time: the rest queue
        tickets = [abm.submit(ctx, p, y, out_stride=1) for p, y in zip(probs, ys)]
        if collect_first:
            _wait(ctx, tickets[:1])
        ctx.close()
    torch_ready.cuda.synchronize()
    ctx = abm.Context(0)
    r = _wait(ctx, [abm.submit(ctx, probs[0], ys[0], out_stride=1)])
    assert list(r.values())[0]["status"] == abm.ABM_OK
    assert normerr(ys[0].cpu().numpy(), oracle_run(probs[0], 1)) <= TOL_FP64
    ctx.close()


def test_server_whose_arena_cannot_be_allocated(torch_ready):
    """An arena of 2^50 bytes passes abm_submit's size check but not the
    server's allocation: the queued request completes with ABM_EDEVICE, later
    submits are refused, and the context is destroyed cleanly."""
    ctx = abm.Context(0, arena_bytes=1 << 50)
    p = _good_duffing(0.2, N=500)
    y = abm.alloc_out(p, 0)
    t = abm.submit(ctx, p, y)
    res = _wait(ctx, [t], timeout=30)
    assert res[t]["status"] == abm.ABM_EDEVICE
    with pytest.raises(abm.AbmError) as e:
        abm.submit(ctx, p, y)
    assert e.value.code == abm.ABM_EDEVICE
    ctx.close()
