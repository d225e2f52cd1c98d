"""The paper's LCR circuit (eq. sys.LRC) on the GPU at zero forcing, started
on its equilibria: E0 = (0, 0) and E+- = (+-sigma(a-b)/(1+sigma b),
+-(b-a)/(1+sigma b)) as given in the "Numerical experiment" section.  An
equilibrium is a fixed point of the fractional system for any orders, so
every path and every far-field precision must keep the state on it: the
right-hand side there is zero up to rounding (about 1e-16), and so is every
history term.  A wrong coefficient in f, a history term that should vanish,
or a start term other than x0 moves the state by order one.  This checks
the library against the paper's own closed form, not against the oracle."""
import numpy as np
import pytest

from paper_1710_01133_amd import abm, inputs
from gpu_common import run_batch, run_plain

pytestmark = pytest.mark.gpu

SIGMA, OMEGA, A, B = inputs.LCR_P


def equilibria():
    den = 1 + SIGMA * B
    return {"E0": (0.0, 0.0), "E+": (SIGMA * (A - B) / den, (B - A) / den),
            "E-": (-SIGMA * (A - B) / den, -(B - A) / den)}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    c = abm.Context(0)
    yield c
    c.close()


def _problems(prec, alpha):
    return [inputs.Problem("LCR", alpha, 0.01, 1500, E, (SIGMA, OMEGA, A, B, 0.0), prec)
            for E in equilibria().values()]


def _dev(y, x0):
    return float(np.max(np.abs(y - np.asarray(x0)[None, :])))


@pytest.mark.parametrize("alpha", [0.9, (0.9, 0.75)])
def test_equilibria_stay_put_plain(ctx, alpha):
    for p in _problems("fp64", alpha):
        y = run_plain(ctx, p, 1)
        assert _dev(y, p.x0) <= 1e-12 * max(1.0, max(abs(v) for v in p.x0)), (p.x0, _dev(y, p.x0))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "fp16x3", "i8x9"])
@pytest.mark.parametrize("alpha", [0.9, (0.9, 0.75)])
def test_equilibria_stay_put_blocked(ctx, prec, alpha):
    probs = _problems(prec, alpha)
    outs, _ = run_batch(ctx, probs, 1)
    for p, y in zip(probs, outs):
        assert _dev(y, p.x0) <= 1e-12 * max(1.0, max(abs(v) for v in p.x0)), (prec, p.x0, _dev(y, p.x0))


def test_equilibria_stay_put_served(ctx):
    probs = _problems("fp32", 0.9) + _problems("i8x9", (0.9, 0.75))
    ys = [abm.alloc_out(p, 1) for p in probs]
    tickets = [abm.submit(ctx, p, y, out_stride=1) for p, y in zip(probs, ys)]
    import time
    deadline = time.time() + 60
    for tk in tickets:
        res = abm.poll(ctx, tk)
        while res is None:
            assert time.time() < deadline
            time.sleep(0.002)
            res = abm.poll(ctx, tk)
        assert res["status"] == 0, res
    for p, y in zip(probs, ys):
        d = _dev(y.cpu().numpy(), p.x0)
        assert d <= 1e-12 * max(1.0, max(abs(v) for v in p.x0)), (p.far_prec, p.x0, d)
