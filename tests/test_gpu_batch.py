"""GPU parity of the blocked batch path (abm_solve_batch, double far field)
against the CPU oracle, through the C ABI: several tiles and ragged tails,
every block length, mixed groups, batch invariance and the full-size sweep."""
import numpy as np
import pytest

from paper_1710_01133_amd import abm, inputs
from gpu_common import sweep_errors, TOL_FP64, golden, normerr, oracle_run, run_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    c = abm.Context(0)
    yield c
    c.close()


def _sweep(Ns, alpha=0.95, h=2 ** -6, seed=7):
    amps = np.random.default_rng(seed).uniform(0.1, 0.6, len(Ns))
    return [inputs.Problem("DUFFING", alpha, h, int(N), (0.1, 0.0), (0.1, float(A), 1.2))
            for N, A in zip(Ns, amps)]


@pytest.mark.parametrize("L", [64, 128, 256, 512])
def test_batch_ragged_vs_oracle(ctx, L, monkeypatch):
    monkeypatch.setenv("ABM_BLOCK_L", str(L))
    monkeypatch.setenv("ABM_KCHUNK", "1024")
    monkeypatch.setenv("ABM_MAX_SPLIT", "2")   # workgroups walk several chunks
    probs = _sweep([3000, 2 * L, 777, 1, 2 * L + 1, 64, 1500, 40])
    outs, st = run_batch(ctx, probs, 1)
    assert st["block_L"] == L
    for p, y in zip(probs, outs):
        assert normerr(y, oracle_run(p, 1)) <= TOL_FP64, (L, p.N)


def test_batch_many_columns_several_tiles(ctx, monkeypatch):
    monkeypatch.setenv("ABM_BLOCK_L", "128")
    monkeypatch.setenv("ABM_KCHUNK", "512")
    Ns = [2100] * 40 + [1900, 333]
    probs = _sweep(Ns, seed=11)
    outs, _ = run_batch(ctx, probs, 10)
    for p, y in zip(probs, outs):
        assert normerr(y, oracle_run(p, 10)) <= TOL_FP64


def test_batch_mixed_groups(ctx):
    probs = [
        inputs.Problem("LORENZ", 0.93, 2 ** -8, 1200, (1.0, 1.0, 1.0), (10.0, 28.0, 8 / 3)),
        inputs.Problem("LCR", 0.9, 0.05, 900, (1.2, -0.4), (1.015, 0.55, -1.02, -0.58, 0.117)),
        inputs.Problem("DUFFING", 0.93, 2 ** -8, 1100, (0.1, 0.0), (0.1, 0.5, 1.2)),
        inputs.Problem("LINEAR", 0.8, 2 ** -7, 1024, (1.0,), (1.0,)),
        inputs.Problem("POLY", 0.5, 1 / 64, 700, (0.25,), (0.7, -0.3)),
        inputs.Problem("LORENZ", 0.99, 2 ** -8, 300, (1.0, 1.0, 1.0), (10.0, 28.0, 8 / 3)),
    ]
    outs, st = run_batch(ctx, probs, 1)
    assert st["n_groups"] == 6
    for p, y in zip(probs, outs):
        assert normerr(y, oracle_run(p, 1)) <= TOL_FP64, p.rhs


def test_batch_invariance_and_determinism(ctx, monkeypatch):
    probs = _sweep([2500, 1700, 2500, 900], seed=3)
    outs1, _ = run_batch(ctx, probs, 1)
    outs2, _ = run_batch(ctx, probs, 1)
    for a, b in zip(outs1, outs2):
        assert np.array_equal(a, b)
    for i in (0, 3):
        # alone, a trajectory is a narrow group (blocked convolution): the
        # same sums in another order
        alone, st = run_batch(ctx, [probs[i]], 1)
        assert st["narrow_groups"] == 1
        assert normerr(alone[0], outs1[i]) <= 1e-13
    # with the same far-field kernel the batch does not change a trajectory's bits
    monkeypatch.setenv("ABM_NARROW", "0")
    for i in (0, 3):
        alone, st = run_batch(ctx, [probs[i]], 1)
        assert st["narrow_groups"] == 0
        assert np.array_equal(alone[0], outs1[i])


def test_batch_single_trajectory_long(ctx):
    p = inputs.duffing_single(N=20000)
    outs, _ = run_batch(ctx, [p], 1)
    assert normerr(outs[0], oracle_run(p, 1)) <= TOL_FP64


def test_sweep_full_size_fp64(ctx, monkeypatch):
    """B = 1024, N = 65536 forcing sweep at the benchmark's launch shape:
    every member against its stored oracle run, and one member alone equal
    bit for bit to its column in the full batch."""
    probs = inputs.duffing_sweep()
    outs, st = run_batch(ctx, probs, 1024)
    errs = sweep_errors(outs)
    print("fp64 sweep: max error %.3g (member %d)" % (errs.max(), errs.argmax()))
    assert errs.max() <= TOL_FP64, int(errs.argmax())
    alone, _ = run_batch(ctx, [probs[511]], 1024)           # narrow group: other sum order
    assert normerr(alone[0], outs[511]) <= 1e-13
    monkeypatch.setenv("ABM_NARROW", "0")                    # same kernel: same bits
    alone, _ = run_batch(ctx, [probs[511]], 1024)
    assert np.array_equal(alone[0], outs[511])


def test_batch_partial_slices_bounded_over_all_blocks(ctx):
    """With N = 20000 and block length 256 a middle block needs more far
    partial slices (6) than the last one (5); three groups (three alphas) sit
    next to each other in memory, so an undersized partial buffer would spill
    into a neighbour.  Every member must still match the oracle."""
    probs = [inputs.Problem("DUFFING", al, 2 ** -8, 20000, (0.1, 0.0), (0.1, 0.3, 1.2))
             for al in (0.9, 0.91, 0.92)]
    outs, st = run_batch(ctx, probs, 100)
    assert st["n_groups"] == 3
    for p, y in zip(probs, outs):
        assert normerr(y, oracle_run(p, 100)) <= TOL_FP64
