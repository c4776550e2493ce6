"""Logical values on the GPU against the oracle: the pairs that have a true
triplet, their order, the slots (-1 for pairs with no true triplet) and the
true values, bit for bit in every bin mode, with the capacity retry, bytes
other than 0/1 read as true, and the degenerate cases."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_1066_amd as fs
    fs.set_tuning(reset=True)
    yield fs
    fs.set_tuning(reset=True)


def check_logical(fs, ii, jj, sl, m=None, n=None, **kw):
    ref = oracle.assemble_logical(ii, jj, sl, m, n)
    res = fs.sparse_logical(to_dev(ii), to_dev(jj), to_dev(sl), m, n,
                            keep_slot=True, **kw)
    assert (res.m, res.n, res.nnz) == (ref.m, ref.n, ref.nnz)
    np.testing.assert_array_equal(res.jcS.cpu().numpy(), ref.jcS)
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    np.testing.assert_array_equal(res.slot.cpu().numpy(), ref.slot)
    assert res.prS.dtype == torch.bool
    np.testing.assert_array_equal(res.prS.cpu().numpy().view(np.uint8), ref.prS)
    return res, ref


def test_hand_example(fs):
    ii = np.array([1, 2, 1, 1, 1], np.int32)
    jj = np.array([1, 1, 2, 1, 2], np.int32)
    sl = np.array([False, False, True, True, True])
    res, _ = check_logical(fs, ii, jj, sl)
    assert res.slot.cpu().tolist() == [0, -1, 1, 0, 1]


@pytest.mark.parametrize("mode", ["auto", "dense", "slot", "claim"])
def test_random_and_mesh_all_modes(fs, mode):
    fs.set_tuning(bin_mode=mode)
    try:
        rng = np.random.default_rng(90)
        L, m, n = 300_007, 2000, 500
        ii = rng.integers(1, m + 1, L).astype(np.int32)
        jj = rng.integers(1, n + 1, L).astype(np.int32)
        for frac in (0.05, 0.4, 0.9):
            check_logical(fs, ii, jj, rng.random(L) < frac, m, n)
        t = W.fem3d(11, 0.15, seed=91)
        check_logical(fs, t.ii, t.jj, rng.random(t.L) < 0.3, t.m, t.n)
    finally:
        fs.set_tuning(reset=True)


def test_all_true_all_false_empty(fs):
    t = W.fem2d(30, 0.2, seed=92)
    res, _ = check_logical(fs, t.ii, t.jj, np.ones(t.L, bool))
    real = fs.sparse(to_dev(t.ii), to_dev(t.jj), to_dev(t.ss))
    assert torch.equal(res.jcS, real.jcS) and torch.equal(res.irS, real.irS)
    res, _ = check_logical(fs, t.ii, t.jj, np.zeros(t.L, bool))
    assert res.nnz == 0 and (res.m, res.n) == (t.m, t.n)
    e = np.zeros(0, np.int32)
    res, _ = check_logical(fs, e, e, np.zeros(0, bool), 3, 2)
    assert res.jcS.cpu().tolist() == [0, 0, 0]


def test_bytes_and_capacity_retry(fs):
    # uint8 values other than 0/1 are true; a small cap is grown by the
    # binding from the reported count
    rng = np.random.default_rng(93)
    t = W.uniform(80_000, 300, 200, seed=94)
    b = rng.choice(np.array([0, 1, 2, 255], np.uint8), t.L)
    ref = oracle.assemble_logical(t.ii, t.jj, b != 0, t.m, t.n)
    res = fs.sparse_logical(to_dev(t.ii), to_dev(t.jj), to_dev(b), t.m, t.n,
                            keep_slot=True, cap=10)
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    np.testing.assert_array_equal(res.jcS.cpu().numpy(), ref.jcS)
    np.testing.assert_array_equal(res.slot.cpu().numpy(), ref.slot)
    assert bool(res.prS.all())


def test_fem3d_50_full_size(fs):
    t = W.fem3d(50, 0.15, seed=1070)
    sl = np.random.default_rng(95).random(t.L) < 0.5
    check_logical(fs, t.ii, t.jj, sl, t.m, t.n)


def test_argument_errors(fs):
    ii = to_dev(np.array([1, 2], np.int32))
    with pytest.raises(TypeError):
        fs.sparse_logical(ii, ii, to_dev(np.array([1.0, 0.0])))
    with pytest.raises(fs.FsparseIndexError):
        fs.sparse_logical(ii, ii, to_dev(np.array([True, True])), 1, 1)
