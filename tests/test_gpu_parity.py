"""HIP path against the CPU oracle, element by element (bit-exact).

Sizes span many LDS chunks and ragged tails; the chunk capacity is lowered
in some cases so that the multi-batch and long-column paths run on inputs
the oracle handles in seconds.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from golden.load import load
from gpu_util import assert_same, check, run, to_dev

pytestmark = pytest.mark.gpu

EX = load("worked_example.txt")


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_1066_amd as fs
    fs.set_tuning(reset=True)
    yield fs
    fs.set_tuning(reset=True)


@pytest.fixture
def cap(fs):
    def set_cap(c):
        fs.set_tuning(chunk_cap=c)
    yield set_cap
    fs.set_tuning(reset=True)


def i32(a):
    return np.asarray(a, dtype=np.int32)


def test_worked_example(fs):
    res, ref = check(fs, i32(EX["example_i"]), i32(EX["example_j"]),
                     EX["example_s"])
    np.testing.assert_array_equal(res.prS.cpu().numpy(), EX["prS"])
    np.testing.assert_array_equal(res.slot.cpu().numpy(), EX["example_irank"])


def test_worked_example_sorted(fs):
    check(fs, i32(EX["sorted_i"]), i32(EX["sorted_j"]), EX["sorted_s"])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_tiny_random(fs, dtype):
    rng = np.random.default_rng(77)
    for case in range(60):
        m = int(rng.integers(1, 13))
        n = int(rng.integers(1, 13))
        L = int(rng.integers(1, 80))
        ii = rng.integers(1, m + 1, size=L).astype(np.int32)
        jj = rng.integers(1, n + 1, size=L).astype(np.int32)
        ss = (rng.standard_normal(L) * 10.0 ** rng.integers(-6, 7, size=L)
              ).astype(dtype)
        check(fs, ii, jj, ss, m, n)


def test_fold_order_and_signed_zero(fs):
    check(fs, i32([2, 2, 2, 1, 1]), i32([1, 1, 1, 2, 2]),
          np.array([1.0, 1e16, -1e16, -0.0, -0.0]), 2, 2)


@pytest.mark.parametrize("c", [1024, 2048, 4096])
def test_fem2d_100_all_caps(fs, cap, c):
    cap(c)
    t = W.config("fem2d_100")
    check(fs, t.ii, t.jj, t.ss, t.m, t.n)


def test_fem3d_small(fs):
    t = W.fem3d(14, 0.15, seed=3)
    check(fs, t.ii, t.jj, t.ss, t.m, t.n)


def test_fem3d_fp32(fs):
    t = W.fem3d(11, 0.15, seed=4, dtype=np.float32)
    check(fs, t.ii, t.jj, t.ss, t.m, t.n)


def test_uniform_medium(fs):
    t = W.uniform(300_000, 20_000, 7_000, seed=5)
    check(fs, t.ii, t.jj, t.ss, t.m, t.n)


def test_ransparse_counts(fs):
    t = W.ransparse(3000, 30, 20, seed=8)
    res, ref = check(fs, t.ii, t.jj, t.ss, t.m, t.n)
    assert float(res.prS.sum().item()) == t.L


@pytest.mark.parametrize("c", [8, 16, 64, 256])
def test_small_capacity_forces_slow_paths(fs, cap, c):
    cap(c)
    rng = np.random.default_rng(c)
    # mixed column lengths: many short, some far longer than the capacity
    t = W.uniform(6000, 40, 30, seed=c)
    check(fs, t.ii, t.jj, t.ss, t.m, t.n)
    t = W.fem2d(9, 0.2, seed=c)
    check(fs, t.ii, t.jj, t.ss, t.m, t.n)
    ii = rng.integers(1, 500, size=3000).astype(np.int32)
    jj = np.full(3000, 3, dtype=np.int32)
    check(fs, ii, jj, rng.standard_normal(3000), 600, 5)


def test_single_column_and_single_pair(fs, cap):
    rng = np.random.default_rng(2)
    for c in (2048, 64):
        cap(c)
        L = 20000
        ii = rng.integers(1, 3000, size=L).astype(np.int32)
        check(fs, ii, np.ones(L, dtype=np.int32), rng.standard_normal(L))
        check(fs, np.full(L, 7, dtype=np.int32), np.full(L, 2, dtype=np.int32),
              rng.standard_normal(L), 9, 4)


def test_empty_columns_and_given_dims(fs):
    check(fs, i32([1, 3]), i32([2, 9]), np.array([1.0, 2.0]), 5, 200000)
    check(fs, i32([4]), i32([1]), np.array([1.5]), 10, 1)


def test_len_zero(fs):
    res = run(fs, i32([]), i32([]), np.array([]), 3, 4)
    assert res.nnz == 0 and res.jcS.cpu().tolist() == [0] * 5
    res = run(fs, i32([]), i32([]), np.array([]))
    assert (res.m, res.n, res.nnz) == (0, 0, 0)


def test_default_dims(fs):
    t = W.uniform(5000, 300, 200, seed=1)
    ref = oracle.assemble(t.ii, t.jj, t.ss)
    res = run(fs, t.ii, t.jj, t.ss, keep_slot=True)
    assert (res.m, res.n) == (ref.m, ref.n)
    assert_same(res, ref)


@pytest.mark.parametrize("ii,jj,m,n", [
    ([0, 1], [1, 1], None, None), ([1, 1], [1, -2], None, None),
    ([3, 1], [1, 1], 2, 2), ([1, 1], [1, 3], 2, 2)])
def test_bad_index(fs, ii, jj, m, n):
    with pytest.raises(fs.FsparseIndexError):
        run(fs, i32(ii), i32(jj), np.ones(2), m, n)


def test_capacity_retry(fs):
    t = W.fem2d(30, 0.2, seed=2)
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    res = run(fs, t.ii, t.jj, t.ss, t.m, t.n, cap=10, keep_slot=True)
    assert_same(res, ref)


def test_deterministic_bytes(fs, cap):
    t = W.fem3d(12, 0.15, seed=9)
    outs = []
    for c in (1024, 2048, 4096, 1024):
        cap(c)
        r = run(fs, t.ii, t.jj, t.ss, t.m, t.n, keep_slot=True)
        outs.append((r.jcS.cpu().numpy().tobytes(),
                     r.irS.cpu().numpy().tobytes(),
                     r.prS.cpu().numpy().tobytes(),
                     r.slot.cpu().numpy().tobytes()))
    assert all(o == outs[0] for o in outs)


def test_stream_copy(fs):
    a = torch.arange(1 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    fs.stream_copy(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("mode", ["dense", "slot", "claim"])
@pytest.mark.parametrize("c", [64, 2048])
def test_bin_modes(fs, mode, c):
    fs.set_tuning(chunk_cap=c, bin_mode=mode)
    try:
        t = W.uniform(400_000, 3000, 40_000, seed=12)
        check(fs, t.ii, t.jj, t.ss, t.m, t.n)
        t = W.fem3d(16, 0.15, seed=13)
        check(fs, t.ii, t.jj, t.ss, t.m, t.n)
        t = W.fem2d(120, 0.2, seed=14, dtype=np.float32)
        check(fs, t.ii, t.jj, t.ss, t.m, t.n)
    finally:
        fs.set_tuning(reset=True)


def test_slot_overflow_falls_back(fs):
    # one column far heavier than a fixed-capacity bin: the one-pass
    # placement overflows and the call redoes the placement in two passes
    fs.set_tuning(chunk_cap=64, bin_mode="slot")
    try:
        t = W.uniform(400_000, 3000, 40_000, seed=15)
        t.jj[:700] = 7
        check(fs, t.ii, t.jj, t.ss, t.m, t.n)
    finally:
        fs.set_tuning(reset=True)


def test_huge_row_indices(fs):
    # rows near 2^31 do not fit a packed (row, column) word
    rng = np.random.default_rng(16)
    m = 2**31 - 2
    ii = rng.integers(m - 50, m + 1, size=5000).astype(np.int32)
    jj = rng.integers(1, 301, size=5000).astype(np.int32)
    check(fs, ii, jj, rng.standard_normal(5000), m, 300)


@pytest.mark.parametrize("c,n,L", [(2048, 1000, 60_000), (2048, 3000, 100_000),
                                   (64, 997, 20_000), (64, 300, 5_000),
                                   (2048, 12_345, 9_000)])
def test_bin_widths(fs, cap, c, n, L):
    # average bin fill fixes the bin width: these give widths that are and
    # are not powers of two, with a ragged last bin, and repeated pairs
    cap(c)
    t = W.uniform(L, 5000, n, seed=17 + n)
    k = L // 5
    ii = np.concatenate([t.ii, t.ii[:k]])
    jj = np.concatenate([t.jj, t.jj[:k]])
    ss = np.concatenate([t.ss, np.arange(k, dtype=np.float64) * 0.25])
    check(fs, ii, jj, ss, t.m, t.n)


@pytest.mark.parametrize("m", [2**30 - 1, 2**30])
def test_packed_word_limit(fs, cap, m):
    # with a 64-entry capacity, 300 columns and 5000 triplets the bins are 3
    # columns wide (2 bits): rows below 2^30 share a word with the column (the
    # largest such word is just below the hash table's empty mark), 2^30 rows
    # do not
    cap(64)
    rng = np.random.default_rng(18)
    ii = rng.integers(m - 40, m + 1, size=5000).astype(np.int32)
    jj = rng.integers(1, 301, size=5000).astype(np.int32)
    ii[:100] = m
    jj[:100] = 300
    check(fs, ii, jj, rng.standard_normal(5000), m, 300)


@pytest.mark.parametrize("mode", ["slot", "claim"])
def test_forced_modes_on_dense_geometry(fs, mode):
    # 3M triplets over few bins: the dense passes would use tiles larger than
    # the claim kernels' (one round of resident blocks); a forced claim or
    # slot mode must still cover every triplet with its own tiles
    fs.set_tuning(chunk_cap=2048, stream_block=512, bin_mode=mode)
    try:
        t = W.uniform(3_000_000, 20_000, 30_000, seed=19)
        check(fs, t.ii, t.jj, t.ss, t.m, t.n)
    finally:
        fs.set_tuning(reset=True)


def test_uneven_column_density_refit(fs, cap):
    # the second half of the columns is ten times denser than the first:
    # fixed-capacity bins sized for the average density overflow in the
    # dense half, and the call redoes the placement counted, in bins of half
    # the average fill
    cap(64)
    rng = np.random.default_rng(20)
    n, m = 100_000, 5000
    jj = np.concatenate([rng.integers(1, n // 2 + 1, 100_000),
                         rng.integers(n // 2 + 1, n + 1, 1_000_000)])
    p = rng.permutation(jj.size)
    jj = jj[p].astype(np.int32)
    ii = rng.integers(1, m + 1, jj.size).astype(np.int32)
    ss = rng.standard_normal(jj.size)
    check(fs, ii, jj, ss, m, n)


@pytest.mark.parametrize("sv", ["binned", "by_k"])
def test_uneven_density_refit_at_4096(fs, sv):
    # the shipped shape of the mesh inputs (4096-entry fixed-capacity bins,
    # 1024 threads), with values binned or read by k: bins sized for the
    # average density overflow where the columns are ten times denser, and
    # the call redoes the placement counted
    fs.set_tuning(chunk_cap=4096, chunk_block=1024, bin_mode="slot",
                  slot_values=sv)
    try:
        rng = np.random.default_rng(21)
        n, m = 100_000, 5000
        jj = np.concatenate([rng.integers(1, n // 2 + 1, 100_000),
                             rng.integers(n // 2 + 1, n + 1, 1_000_000)])
        jj = jj[rng.permutation(jj.size)].astype(np.int32)
        ii = rng.integers(1, m + 1, jj.size).astype(np.int32)
        ss = rng.standard_normal(jj.size)
        check(fs, ii, jj, ss, m, n)
    finally:
        fs.set_tuning(reset=True)
