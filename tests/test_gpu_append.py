"""Delayed assembly on the GPU: chained appends against the oracle.

Appending triplets to an assembled matrix must give, bit for bit, the
oracle's assembly of all the triplets at once (and the oracle's own chained
append, slots included), in every bin mode and value type, with growing
dimensions, empty parts and re-assembly from a plan.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import assert_same, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_1066_amd as fs
    fs.set_tuning(reset=True)
    yield fs
    fs.set_tuning(reset=True)


def chain(fs, ii, jj, ss, cuts, m=None, n=None):
    parts = np.split(np.arange(ii.size), cuts)
    p = parts[0]
    ref = oracle.assemble(ii[p], jj[p], ss[p], m, n)
    res = fs.sparse(to_dev(ii[p]), to_dev(jj[p]), to_dev(ss[p]), m, n,
                    keep_slot=True)
    assert_same(res, ref)
    for p in parts[1:]:
        ref = oracle.append(ref, ii[p], jj[p], ss[p], m, n)
        res = fs.sparse_append(res, to_dev(ii[p]), to_dev(jj[p]),
                               to_dev(ss[p]), m, n, keep_slot=True)
        assert (res.m, res.n) == (ref.m, ref.n)
        assert_same(res, ref)
    return res, ref


@pytest.mark.parametrize("mode", ["auto", "dense", "slot", "claim"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_chained_appends_equal_one_assembly(fs, mode, dtype):
    fs.set_tuning(bin_mode=mode)
    try:
        rng = np.random.default_rng(70)
        L, m, n = 400_000, 3000, 2000
        ii = rng.integers(1, m + 1, L).astype(np.int32)
        jj = rng.integers(1, n + 1, L).astype(np.int32)
        ss = (rng.standard_normal(L) * 10.0 ** rng.integers(-6, 7, L)).astype(dtype)
        ss[rng.random(L) < 0.03] = -0.0
        res, _ = chain(fs, ii, jj, ss, [50_000, 51_000, 300_000], m, n)
        one = oracle.assemble(ii, jj, ss, m, n)
        assert res.prS.cpu().numpy().tobytes() == one.prS.tobytes()
        np.testing.assert_array_equal(res.irS.cpu().numpy(), one.irS)
    finally:
        fs.set_tuning(reset=True)


def test_mesh_in_element_chunks_and_growing_dims(fs):
    t = W.fem3d(12, 0.15, seed=71)
    per = t.per_elem
    ne = t.L // per
    cuts = [per * (ne // 5), per * (ne // 2), per * (ne - 7)]
    res, _ = chain(fs, t.ii, t.jj, t.ss, cuts)        # default dims grow
    one = oracle.assemble(t.ii, t.jj, t.ss)
    assert (res.m, res.n) == (one.m, one.n)
    assert res.prS.cpu().numpy().tobytes() == one.prS.tobytes()


def test_empty_parts_and_small_capacity(fs):
    fs.set_tuning(chunk_cap=16)
    try:
        rng = np.random.default_rng(72)
        ii = rng.integers(1, 60, 5000).astype(np.int32)
        jj = rng.integers(1, 8, 5000).astype(np.int32)
        ss = rng.integers(-3, 4, 5000).astype(np.float64)
        chain(fs, ii, jj, ss, [0, 0, 2500, 5000, 5000], 60, 8)
    finally:
        fs.set_tuning(reset=True)


def test_plan_from_append_and_drop_zeros(fs):
    rng = np.random.default_rng(73)
    ii = rng.integers(1, 200, 60_000).astype(np.int32)
    jj = rng.integers(1, 100, 60_000).astype(np.int32)
    ss = rng.integers(-2, 3, 60_000).astype(np.float64)
    a = fs.sparse(to_dev(ii[:20_000]), to_dev(jj[:20_000]),
                  to_dev(ss[:20_000]), 200, 100)
    ra = oracle.assemble(ii[:20_000], jj[:20_000], ss[:20_000], 200, 100)
    res = fs.sparse_append(a, to_dev(ii[20_000:]), to_dev(jj[20_000:]),
                           to_dev(ss[20_000:]), plan=True, keep_slot=True)
    ref = oracle.append(ra, ii[20_000:], jj[20_000:], ss[20_000:])
    assert_same(res, ref)
    # the plan covers the old sums, then the new values
    v = np.concatenate([ra.prS * 2.0, ss[20_000:] * 2.0])
    pr2 = fs.reassemble(res, to_dev(v)).cpu().numpy()[:ref.nnz]
    assert pr2.tobytes() == (ref.prS * 2.0).tobytes()
    # Matlab's convention on the appended result
    d = fs.sparse_append(a, to_dev(ii[20_000:]), to_dev(jj[20_000:]),
                         to_dev(ss[20_000:]), keep_slot=True, drop_zeros=True)
    assert_same(d, oracle.drop_zeros(ref))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_stored_pairs_between_empty_column_runs(fs, dtype):
    # 40 non-empty columns among 200000: most blocks of stored pairs span
    # runs of empty columns too long for their LDS window and search the
    # column pointers in global memory, the others use the window
    rng = np.random.default_rng(97)
    m, n, L = 3000, 200_000, 120_000
    cols = rng.choice(np.arange(1, n + 1), 40, replace=False)
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.choice(cols, L).astype(np.int32)
    ss = (rng.standard_normal(L) * 10.0 ** rng.integers(-6, 7, L)).astype(dtype)
    res, ref = chain(fs, ii, jj, ss, [L // 2], m, n)
    want = oracle.assemble(ii, jj, ss, m, n)
    assert ref.prS.tobytes() == want.prS.tobytes()
    assert np.array_equal(ref.jcS, want.jcS)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_merge_with_stored_negative_zeros_and_bad_rows(fs, dtype):
    # a stored matrix given by the caller (not assembled here) whose sums
    # include -0.0: the merge starts every stored pair's fold from +0.0, as
    # one assembly of the stored pairs as triplets would
    rng = np.random.default_rng(98)
    m, n = 50, 30
    ii = rng.integers(1, m + 1, 3000).astype(np.int32)
    jj = rng.integers(1, n + 1, 3000).astype(np.int32)
    ss = rng.integers(-2, 3, 3000).astype(dtype)
    ss[rng.random(3000) < 0.2] = -0.0
    a = oracle.assemble(ii[:1000], jj[:1000], ss[:1000], m, n)
    pr = a.prS.copy()
    pr[rng.random(pr.size) < 0.3] = -0.0
    a.prS[:] = pr
    A = fs.Assembled(to_dev(a.jcS), to_dev(a.irS), to_dev(a.prS), m, n, a.nnz,
                     a.nnz, None, None)
    res = fs.sparse_append(A, to_dev(ii[1000:]), to_dev(jj[1000:]),
                           to_dev(ss[1000:]), m, n, keep_slot=True)
    ref = oracle.append(a, ii[1000:], jj[1000:], ss[1000:], m, n)
    assert_same(res, ref)
    # a stored row beyond the given m is an index error
    with pytest.raises(fs.FsparseIndexError):
        fs.sparse_append(A, to_dev(ii[1000:]), to_dev(jj[1000:]),
                         to_dev(ss[1000:]), int(a.irS.max()), n)


def test_merge_of_columns_longer_than_a_merge_block(fs):
    # three columns with thousands of rows among short ones: the merge
    # blocks holding them cannot stage their runs and the call takes the
    # whole re-assembly instead; the result is the same
    rng = np.random.default_rng(99)
    m, n, L = 20_000, 64, 200_000
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = np.where(rng.random(L) < 0.9, rng.choice([5, 6, 40], L),
                  rng.integers(1, n + 1, L)).astype(np.int32)
    ss = rng.standard_normal(L)
    res, ref = chain(fs, ii, jj, ss, [L // 3], m, n)
    assert res.prS.cpu().numpy().tobytes() == \
        oracle.assemble(ii, jj, ss, m, n).prS.tobytes()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_stream_of_host_chunks(fs, dtype):
    # a mesh streamed from host memory in uneven element chunks: the result
    # is one assembly of everything
    t = W.fem3d(16, 0.15, seed=74, dtype=dtype)
    per = t.per_elem
    ne = t.L // per
    cuts = [0, per * 3, per * (ne // 3), per * (ne // 2), per * (ne - 1), t.L]

    def chunks():
        for a, b in zip(cuts[:-1], cuts[1:]):
            yield t.ii[a:b], t.jj[a:b], t.ss[a:b]
    res = fs.sparse_stream(chunks(), dtype=torch.float64
                           if dtype == np.float64 else torch.float32)
    ref = oracle.assemble(t.ii, t.jj, t.ss)
    assert (res.m, res.n) == (ref.m, ref.n)
    assert_same(res, ref, slot=False)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_merge_edges(fs, dtype):
    rng = np.random.default_rng(100)
    ii = rng.integers(1, 40, 2000).astype(np.int32)
    jj = rng.integers(1, 30, 2000).astype(np.int32)
    ss = rng.standard_normal(2000).astype(dtype)
    e32 = np.zeros(0, np.int32)
    # appending to an empty matrix (no stored pairs, no columns)
    A0 = fs.sparse(to_dev(e32), to_dev(e32), to_dev(np.zeros(0, dtype)), 0, 0)
    r = fs.sparse_append(A0, to_dev(ii), to_dev(jj), to_dev(ss), keep_slot=True)
    ref = oracle.append(oracle.assemble(e32, e32, np.zeros(0, dtype), 0, 0),
                        ii, jj, ss)
    assert_same(r, ref)
    # appending nothing
    A = fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), 40, 30)
    r = fs.sparse_append(A, to_dev(e32), to_dev(e32),
                         to_dev(np.zeros(0, dtype)), keep_slot=True)
    assert_same(r, oracle.assemble(ii, jj, ss, 40, 30), slot=False)
    assert r.slot.cpu().numpy().tolist() == list(range(A.nnz))
    # new triplets only in columns past the stored ones, with a given and
    # with default dimensions (the new part is assembled over its own
    # column range)
    i2 = rng.integers(1, 60, 500).astype(np.int32)
    j2 = rng.integers(45, 52, 500).astype(np.int32)
    s2 = rng.standard_normal(500).astype(dtype)
    ra = oracle.assemble(ii, jj, ss, 40, 30)
    for m, n in ((60, 55), (None, None)):
        r = fs.sparse_append(A, to_dev(i2), to_dev(j2), to_dev(s2), m, n,
                             keep_slot=True)
        assert_same(r, oracle.append(ra, i2, j2, s2, m, n))
    # a new column index past a given n is an index error
    with pytest.raises(fs.FsparseIndexError):
        fs.sparse_append(A, to_dev(i2), to_dev(j2), to_dev(s2), 60, 50)
