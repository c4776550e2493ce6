"""Complex values (split real and imaginary arrays) on the GPU against the
oracle: pattern, slots and both value arrays bit for bit in every bin mode
and value type, the order-free sums within tolerance, zeros dropped only
where both parts are zero, and re-assembly of each part through a plan.
"""
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


def same_bits(got, want, name):
    got = got.cpu().numpy()
    assert got.dtype == want.dtype, name
    if got.tobytes() != want.tobytes():
        d = np.nonzero(got != want)[0]
        raise AssertionError("%s differs at %d positions, first %s: %r vs %r"
                             % (name, d.size, d[:5], got[d[:5]], want[d[:5]]))


def check_complex(fs, ii, jj, sr, si, m=None, n=None, drop=False, **kw):
    ref = oracle.assemble_complex(ii, jj, sr, si, m, n)
    if drop:
        ref = oracle.drop_zeros_complex(ref)
    res = fs.sparse_complex(to_dev(ii), to_dev(jj), to_dev(sr), to_dev(si),
                            m, n, keep_slot=True, drop_zeros=drop, **kw)
    assert (res.m, res.n, res.nnz) == (ref.m, ref.n, ref.nnz)
    np.testing.assert_array_equal(res.jcS.cpu().numpy(), ref.jcS)
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    np.testing.assert_array_equal(res.slot.cpu().numpy(), ref.slot)
    if not kw.get("atomic"):
        same_bits(res.prS, ref.prS, "prS")
        same_bits(res.piS, ref.piS, "piS")
    return res, ref


def spread(L, seed, dtype):
    # magnitudes 1e-8..1e8 and -0.0: the result depends on the fold order
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(L) * 10.0 ** rng.integers(-8, 9, L)
    v[rng.random(L) < 0.03] = -0.0
    return v.astype(dtype)


@pytest.mark.parametrize("mode", ["auto", "dense", "slot", "claim"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_random_and_mesh_all_modes(fs, mode, dtype):
    fs.set_tuning(bin_mode=mode)
    try:
        # several tiles and a ragged tail; about 3 triplets per pair
        L, m, n = 300_007, 2000, 500
        rng = np.random.default_rng(70)
        ii = rng.integers(1, m + 1, L).astype(np.int32)
        jj = rng.integers(1, n + 1, L).astype(np.int32)
        check_complex(fs, ii, jj, spread(L, 71, dtype), spread(L, 72, dtype),
                      m, n)
        t = W.fem3d(11, 0.15, seed=73, dtype=dtype)
        check_complex(fs, t.ii, t.jj, t.ss, spread(t.L, 74, dtype), t.m, t.n)
    finally:
        fs.set_tuning(reset=True)


def test_default_dims_and_empty(fs):
    t = W.uniform(50_000, 700, 300, seed=75)
    check_complex(fs, t.ii, t.jj, t.ss, spread(t.L, 76, np.float64))
    e = np.zeros(0, np.int32)
    res, _ = check_complex(fs, e, e, np.zeros(0), np.zeros(0), 4, 3)
    assert res.nnz == 0 and res.jcS.cpu().tolist() == [0, 0, 0, 0]


def test_zero_imaginary_parts_equal_the_real_call(fs):
    t = W.fem2d(40, 0.2, seed=77)
    res, _ = check_complex(fs, t.ii, t.jj, t.ss, np.zeros(t.L), t.m, t.n)
    real = fs.sparse(to_dev(t.ii), to_dev(t.jj), to_dev(t.ss), t.m, t.n)
    assert torch.equal(res.prS, real.prS)
    assert not bool(torch.signbit(res.piS).any())


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-14), (np.float32, 1e-6)])
def test_atomic_tolerance(fs, dtype, tol):
    t = W.fem3d(12, 0.15, seed=78, dtype=dtype)
    si = spread(t.L, 79, dtype)
    res, ref = check_complex(fs, t.ii, t.jj, t.ss, si, t.m, t.n, atomic=True)
    for got, want, s in ((res.prS, ref.prS, t.ss), (res.piS, ref.piS, si)):
        scale = oracle.assemble(t.ii, t.jj, np.abs(s).astype(np.float64),
                                t.m, t.n).prS
        err = np.abs(got.cpu().numpy().astype(np.float64)
                     - want.astype(np.float64))
        assert np.all(err <= tol * np.maximum(scale, 1e-300)), err.max()


def test_drop_zeros_hand_example(fs):
    ii = np.array([1, 2, 1, 1, 1, 2, 2], np.int32)
    jj = np.array([1, 1, 2, 1, 2, 2, 2], np.int32)
    sr = np.array([1.0, 0.0, 3.0, -1.0, 0.0, 1.0, -1.0])
    si = np.array([2.0, -0.0, 1.0, 0.0, -1.0, 1.0, -1.0])
    res, _ = check_complex(fs, ii, jj, sr, si, 2, 2, drop=True)
    assert res.slot.cpu().tolist() == [0, -1, 1, 0, 1, -1, -1]


@pytest.mark.parametrize("mode", ["auto", "slot", "claim"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_drop_zeros_cancelling(fs, mode, dtype):
    # small integers: many real sums, fewer complex sums, are exactly zero
    fs.set_tuning(bin_mode=mode)
    try:
        rng = np.random.default_rng(80)
        L, m, n = 200_000, 1000, 300
        ii = rng.integers(1, m + 1, L).astype(np.int32)
        jj = rng.integers(1, n + 1, L).astype(np.int32)
        sr = rng.integers(-1, 2, L).astype(dtype)
        si = np.where(rng.random(L) < 0.7, 0, rng.integers(-1, 2, L)).astype(dtype)
        res, ref = check_complex(fs, ii, jj, sr, si, m, n, drop=True)
        full = oracle.assemble_complex(ii, jj, sr, si, m, n)
        assert 0 < ref.nnz < full.nnz
        assert ref.nnz > int(np.count_nonzero(full.prS))
        res, ref = check_complex(fs, ii, jj, sr, si, m, n, drop=True,
                                 atomic=True)
        same_bits(res.prS, ref.prS, "prS")        # integer sums are exact
        same_bits(res.piS, ref.piS, "piS")
    finally:
        fs.set_tuning(reset=True)


def test_plan_reassembles_each_part(fs):
    t = W.fem3d(10, 0.15, seed=81)
    si = spread(t.L, 82, np.float64)
    res, _ = check_complex(fs, t.ii, t.jj, t.ss, si, t.m, t.n, plan=True)
    sr2 = t.ss * np.random.default_rng(83).uniform(0.5, 2.0, t.L)
    si2 = spread(t.L, 84, np.float64)
    ref2 = oracle.assemble_complex(t.ii, t.jj, sr2, si2, t.m, t.n)
    same_bits(fs.reassemble(res, to_dev(sr2)), ref2.prS, "prS")
    same_bits(fs.reassemble(res, to_dev(si2)), ref2.piS, "piS")


def test_fem3d_50_full_size(fs):
    # the 11.3M-triplet mesh, every output compared
    t = W.fem3d(50, 0.15, seed=1070)
    check_complex(fs, t.ii, t.jj, t.ss, spread(t.L, 85, np.float64), t.m, t.n)


def test_argument_errors(fs):
    ii = to_dev(np.array([1, 2], np.int32))
    sr = to_dev(np.array([1.0, 2.0]))
    with pytest.raises(ValueError):
        fs.sparse_complex(ii, ii, sr, sr.float())
    with pytest.raises(ValueError):
        fs.sparse_complex(ii, ii, sr, sr, plan=True, drop_zeros=True)
    with pytest.raises(fs.FsparseIndexError):
        fs.sparse_complex(ii, ii, sr, sr, 1, 1)


def test_to_dense_carries_both_parts(fs):
    t = W.fem2d(6, 0.2, seed=86)
    si = spread(t.L, 87, np.float64)
    res, ref = check_complex(fs, t.ii, t.jj, t.ss, si, t.m, t.n)
    D = np.zeros((t.m, t.n), dtype=np.complex128)
    cols = np.repeat(np.arange(t.n), np.diff(ref.jcS))
    D[ref.irS, cols] = ref.prS + 1j * ref.piS
    got = res.to_dense().cpu().numpy()
    assert got.dtype == np.complex128
    np.testing.assert_array_equal(got, D)
