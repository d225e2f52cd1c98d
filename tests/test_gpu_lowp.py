"""Reduced-precision far field (float, bf16 split x3 / x6, scaled fp16 split
x3, int8 limbs x9) of the blocked path
against the double oracle, through the C ABI.  Here the error is the quantity
measured: each precision has a stated bound on the normwise relative error
max_s |y_s - yref_s|_inf / max_s |yref_s|_inf."""
import numpy as np
import pytest

from paper_1710_01133_amd import abm, inputs
from gpu_common import golden, normerr, oracle_run, run_batch, sweep_errors

pytestmark = pytest.mark.gpu

# stated error bounds of the far-field precisions (near band and state stay double)
# Largest normwise error over all 1024 members of the forcing sweep against the
# double oracle, per far-field precision.  fp32 and bf16x6 carry 24 significant
# bits of every operand and meet 1e-6 (measured 6.7e-7, 4.9e-7); fp16x3 keeps
# about 22 (11 + 11 bits per operand, the lo*lo product dropped): measured
# 1.1e-6 on its worst member, so its bound is 2e-6; bf16x3 keeps 16 (1.0e-4).
# i8x9 carries 30 bits of every weight and 21-22 of the history (relative to
# their window's and block's largest value) and sums its products exactly: a
# CPU model of its arithmetic put the sweep's worst member near 5e-8, against
# 3e-7 for the same model of bf16x6; measured 7.9e-8 over the sweep and 2.25e-7
# on the LCR case of the mixed test, so its bound is 3e-7.
BOUND = {"fp32": 1e-6, "bf16x3": 2e-4, "bf16x6": 1e-6, "fp16x3": 2e-6, "i8x9": 3e-7}
LOWP = ["fp32", "bf16x3", "bf16x6", "fp16x3", "i8x9"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    c = abm.Context(0)
    yield c
    c.close()


def _sweep(Ns, prec, alpha=0.95, h=2 ** -6, seed=5):
    amps = np.random.default_rng(seed).uniform(0.1, 0.6, len(Ns))
    return [inputs.Problem("DUFFING", alpha, h, int(N), (0.1, 0.0), (0.1, float(A), 1.2), prec)
            for N, A in zip(Ns, amps)]


@pytest.mark.parametrize("prec", LOWP)
@pytest.mark.parametrize("L", [128, 256, 512])
def test_lowp_ragged_vs_oracle(ctx, prec, L, monkeypatch):
    if prec == "i8x9" and L == 512:
        pytest.skip("the int8 far field runs at block lengths 128 and 256 (refusal tested below)")
    monkeypatch.setenv("ABM_BLOCK_L", str(L))
    monkeypatch.setenv("ABM_KCHUNK", "1024")
    monkeypatch.setenv("ABM_MAX_SPLIT", "2")   # workgroups walk several chunks
    probs = _sweep([4000, 2 * L + 1, 1, 3 * L, 2500, 100], prec)
    outs, _ = run_batch(ctx, probs, 1)
    errs = [normerr(y, oracle_run(p, 1)) for p, y in zip(probs, outs)]
    print(prec, L, "max err %.3e" % max(errs))
    assert max(errs) <= BOUND[prec], errs


@pytest.mark.parametrize("prec", LOWP)
def test_lowp_mixed_rhs(ctx, prec):
    probs = [
        inputs.Problem("LORENZ", 0.97, 2 ** -8, 3000, (1.0, 1.0, 1.0), (10.0, 28.0, 8 / 3), prec),
        inputs.Problem("LCR", 0.9, 0.02, 3000, (1.2, -0.4), (1.015, 0.55, -1.02, -0.58, 0.117), prec),
        inputs.Problem("LINEAR", 0.8, 2 ** -9, 4096, (1.0,), (1.0,), prec),
    ]
    outs, _ = run_batch(ctx, probs, 1)
    for p, y in zip(probs, outs):
        e = normerr(y, oracle_run(p, 1))
        print(prec, p.rhs, "err %.3e" % e)
        assert e <= BOUND[prec], (p.rhs, e)


def test_lowp_needs_block_128(ctx, monkeypatch):
    monkeypatch.setenv("ABM_BLOCK_L", "64")
    with pytest.raises(abm.AbmError) as e:
        abm.Plan(ctx, _sweep([500], "fp32"))
    assert e.value.code == abm.ABM_EINVAL


def test_int8_needs_block_at_most_256(ctx, monkeypatch):
    monkeypatch.setenv("ABM_BLOCK_L", "512")
    with pytest.raises(abm.AbmError) as e:
        abm.Plan(ctx, _sweep([1500], "i8x9"))
    assert e.value.code == abm.ABM_EINVAL


@pytest.mark.parametrize("prec", LOWP)
def test_lowp_batch_invariance(ctx, prec, monkeypatch):
    # column tiles for the lone trajectory too (a narrow float group would
    # take the blocked convolution, the same sums in another order)
    monkeypatch.setenv("ABM_NARROW", "0")
    probs = _sweep([3000, 2200, 3000], prec, seed=9)
    outs, _ = run_batch(ctx, probs, 1)
    alone, _ = run_batch(ctx, [probs[1]], 1)
    assert np.array_equal(alone[0], outs[1])
    again, _ = run_batch(ctx, probs, 1)
    for a, b in zip(outs, again):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", LOWP)
def test_lowp_sweep_full_size(ctx, prec):
    """B = 1024, N = 65536: error of every member against its stored double
    oracle run, at the library's default blocking."""
    probs = inputs.duffing_sweep(far_prec=prec)
    outs, _ = run_batch(ctx, probs, 1024)
    errs = sweep_errors(outs)
    print(prec, "full-size max error %.3g (member %d)" % (errs.max(), errs.argmax()))
    assert errs.max() <= BOUND[prec], int(errs.argmax())


@pytest.mark.parametrize("prec", ["bf16x6", "fp16x3", "i8x9"])
@pytest.mark.parametrize("blocking", [(256, 2048, 2), (256, 1024, 8), (256, 2048, 4), (512, 2048, 4),
                                      (128, 1024, 16), (256, 4096, 2)])
def test_split_sweep_full_size_at_tuned_blockings(ctx, blocking, prec):
    """The full sweep in the split far precisions at blockings the autotuner
    chooses between (the benchmark times the one it picks): every member
    against its stored double oracle run."""
    L, kchunk, split = blocking
    if prec == "i8x9" and L == 512:
        pytest.skip("the int8 far field runs at block lengths 128 and 256")
    probs = inputs.duffing_sweep(far_prec=prec)
    tuning = dict(block_L=L, kchunk=kchunk, max_split=split, column_tiles_only=0)
    plan = abm.Plan(ctx, probs, out_stride=1024, tuning=tuning)
    assert plan.config() == tuning
    ys = [abm.alloc_out(p, 1024) for p in probs]
    abm.solve_batch(plan, probs, ys)
    plan.check()
    plan.close()
    errs = sweep_errors([y.cpu().numpy() for y in ys])
    print(prec, blocking, "max error %.3g (member %d)" % (errs.max(), errs.argmax()))
    assert errs.max() <= BOUND[prec], (blocking, int(errs.argmax()), errs.max())


@pytest.mark.parametrize("prec", ["fp16x3", "i8x9"])
@pytest.mark.parametrize("scale", [1e-6, 1e4, 1e-200, 1e150])
def test_scaled_splits_far_from_unit_magnitudes(ctx, scale, prec):
    """The fp16 split scales the history per 32 rows and column and the
    weights per window, the int8 limbs the history per block and column and
    the weights per window: a linear problem whose state and right-hand side
    are of order 1e-6 .. 1e150 (far outside fp16's normal range of about
    6e-5 .. 6.5e4, and outside float's) keeps the same error, and so do orders
    0.3 and 1.5 (weights decreasing and increasing along the window)."""
    if prec == "fp16x3" and not 1e-30 < scale < 1e30:
        pytest.skip("the fp16 split takes float copies of the history: |f| within float's range")
    probs = [inputs.Problem("LINEAR", 0.8, 2 ** -9, 3000, (scale,), (1.0,), prec),
             inputs.Problem("DUFFING", 0.3, 2 ** -6, 3000, (0.1, 0.0), (0.1, 0.45, 1.2), prec),
             inputs.Problem("LCR", 1.5, 0.01, 3000, (1.2, -0.4), (1.015, 0.55, -1.02, -0.58, 0.117),
                            prec, x1=(0.0, 0.0))]
    outs, _ = run_batch(ctx, probs, 1)
    for p, y in zip(probs, outs):
        e = normerr(y, oracle_run(p, 1))
        print(prec, p.rhs, p.alpha, "err %.3e" % e)
        assert e <= BOUND[prec], (p.rhs, e)
