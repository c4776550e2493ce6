"""The boundary on the GPU: buffers the binding checks before anything is
queued, wide integer indices narrowed by the library, calls queued without a
wait (FSPARSE_NO_SYNC) against the waiting call and the oracle, and the
backward of results whose dropped pairs have slot -1."""
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


def small(seed=0, L=5000, m=300, n=200, dtype=np.float64):
    rng = np.random.default_rng(seed)
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.integers(1, n + 1, L).astype(np.int32)
    ss = rng.standard_normal(L).astype(dtype)
    return ii, jj, ss, m, n


def sentinel(n, dtype):
    return torch.full((n,), -7, dtype=dtype, device="cuda")


def test_reassemble_out_checked_before_launch(fs):
    ii, jj, ss, m, n = small(1)
    res = fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), m, n, plan=True)
    s = to_dev(ss)
    short = sentinel(res.nnz - 1, torch.float64)
    with pytest.raises(ValueError):
        fs.reassemble(res, s, out=short)
    wrong = sentinel(res.nnz, torch.float32)
    with pytest.raises(TypeError):
        fs.reassemble(res, s, out=wrong)
    torch.cuda.synchronize()
    assert bool((short == -7).all()) and bool((wrong == -7).all())
    with pytest.raises(ValueError):
        fs.reassemble(res, s.cpu())
    ok = sentinel(res.nnz, torch.float64)
    fs.reassemble(res, s, out=ok)
    assert ok.cpu().numpy().tobytes() == res.prS.cpu().numpy().tobytes()


def test_backward_out_checked_before_launch(fs):
    ii, jj, ss, m, n = small(2)
    res = fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), m, n, keep_slot=True)
    g = torch.randn(res.nnz, dtype=torch.float64, device="cuda")
    short = sentinel(len(ii) - 1, torch.float64)
    with pytest.raises(ValueError):
        fs.backward(res.slot, g, out=short)
    wrong = sentinel(len(ii), torch.float32)
    with pytest.raises(TypeError):
        fs.backward(res.slot, g, out=wrong)
    with pytest.raises(TypeError):
        fs.backward(res.slot.to(torch.int64), g)
    torch.cuda.synchronize()
    assert bool((short == -7).all()) and bool((wrong == -7).all())


def test_sparse_out_checked_before_launch(fs):
    ii, jj, ss, m, n = small(3)
    d = (to_dev(ii), to_dev(jj), to_dev(ss))
    L = len(ii)
    jc = torch.full((n + 1,), -7, dtype=torch.int32, device="cuda")
    ir = torch.full((L,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(TypeError):      # prS of the wrong value type
        fs.sparse(*d, m, n, out=(jc, ir, sentinel(L, torch.float32)))
    with pytest.raises(ValueError):     # slot shorter than len
        fs.sparse(*d, m, n, out=(jc, ir, sentinel(L, torch.float64),
                                 torch.zeros(L - 1, dtype=torch.int32,
                                             device="cuda")))
    with pytest.raises(ValueError):     # jcS shorter than n + 1
        fs.sparse(*d, m, n, out=(jc[:n], ir, sentinel(L, torch.float64)))
    torch.cuda.synchronize()
    assert bool((jc == -7).all()) and bool((ir == -7).all())


def test_batched_offsets_checked(fs):
    ii, jj, ss, m, n = small(4)
    d = (to_dev(ii), to_dev(jj), to_dev(ss))
    L = len(ii)
    with pytest.raises(ValueError):     # last offset short of the arrays
        fs.assemble_batched(*d, [0, 100, L - 1], [m, m], [n, n])
    with pytest.raises(ValueError):     # nb + 1 offsets needed
        fs.assemble_batched(*d, [0, L], [m, m], [n, n])
    with pytest.raises(ValueError):     # decreasing
        fs.assemble_batched(*d, [0, 200, 100, L], [m] * 3, [n] * 3)
    r = fs.assemble_batched(*d, [0, 100, L], [m, m], [n, n])
    assert r.nb == 2


def test_wide_indices_narrowed_by_the_library(fs):
    ii, jj, ss, m, n = small(5)
    ref = oracle.assemble(ii, jj, ss, m, n)
    for dt in (torch.int64, torch.int16):
        res = fs.sparse(torch.from_numpy(ii).to(dt).cuda(),
                        torch.from_numpy(jj).to(dt).cuda(), to_dev(ss), m, n,
                        keep_slot=True)
        assert_same(res, ref)
    # values int32 cannot hold are rejected, never wrapped into range
    for bad in (2**32 + 3, -2**32 + 1, 2**31, 0, -1):
        i64 = torch.from_numpy(ii.astype(np.int64)).cuda()
        i64[17] = bad
        with pytest.raises(fs.FsparseIndexError):
            fs.sparse(i64, to_dev(jj), to_dev(ss), m, n)
        with pytest.raises(fs.FsparseIndexError):
            fs.sparse(i64, to_dev(jj), to_dev(ss))          # default dims


@pytest.mark.parametrize("mode", ["auto", "slot", "claim", "dense"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_no_sync_equals_the_waiting_call(fs, mode, dtype):
    # fixed-capacity bins give way to counted ones without a wait, so the
    # forced slot mode is covered too
    fs.set_tuning(bin_mode=mode)
    try:
        t = W.fem3d(9, 0.15, seed=6, dtype=dtype)
        ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
        d = (to_dev(t.ii), to_dev(t.jj), to_dev(t.ss))
        res = fs.sparse(*d, t.m, t.n, keep_slot=True, plan=True, wait=False)
        assert res.pending and res.nnz == -1
        res.wait()
        assert_same(res, ref)
        assert int(res.jcS[-1]) == ref.nnz
        s2 = W.element_scale(t, 0, seed=7)
        pr = fs.reassemble(res, to_dev(s2))
        assert pr.cpu().numpy().tobytes() == \
            oracle.postprocess(ref.slot, s2, ref.nnz).tobytes()
    finally:
        fs.set_tuning(reset=True)


def test_no_sync_plan_before_wait_and_atomic(fs):
    ii, jj, ss, m, n = small(8, L=40000, m=500, n=400)
    ref = oracle.assemble(ii, jj, ss, m, n)
    d = (to_dev(ii), to_dev(jj), to_dev(ss))
    # a plan used before nnz was ever read back: re-use and atomic re-use
    res = fs.sparse(*d, m, n, plan=True, wait=False)
    out = torch.zeros(len(ii), dtype=torch.float64, device="cuda")
    from paper_1406_1066_amd import _lib as L
    import ctypes
    st = L.fsparse_assemble_reuse(res.plan.handle, ctypes.c_void_p(d[2].data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), L.ORDERED,
                                  None)
    assert st == L.OK
    torch.cuda.synchronize()
    assert out[:ref.nnz].cpu().numpy().tobytes() == ref.prS.tobytes()
    out2 = torch.full((len(ii),), 3.0, dtype=torch.float64, device="cuda")
    st = L.fsparse_assemble_reuse(res.plan.handle, ctypes.c_void_p(d[2].data_ptr()),
                                  ctypes.c_void_p(out2.data_ptr()), L.ATOMIC,
                                  None)
    assert st == L.OK
    torch.cuda.synchronize()
    got = out2[:ref.nnz].cpu().numpy()
    den = np.zeros(ref.nnz)
    np.add.at(den, ref.slot, np.abs(ss))
    assert np.all(np.abs(got - ref.prS) <= 1e-14 * den)
    assert bool((out2[ref.nnz:] == 3.0).all())        # nothing past nnz
    nnz = ctypes.c_int64()
    assert L.fsparse_plan_query(res.plan.handle, None, ctypes.byref(nnz),
                                None) == L.OK
    assert nnz.value == ref.nnz
    # the atomic fresh call without a wait
    r2 = fs.sparse(*d, m, n, atomic=True, wait=False).wait()
    assert r2.nnz == ref.nnz
    assert np.all(np.abs(r2.prS.cpu().numpy() - ref.prS) <= 1e-14 * den)


def test_no_sync_reports_errors_at_wait(fs):
    ii, jj, ss, m, n = small(9)
    ii = ii.copy()
    ii[33] = m + 1
    res = fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), m, n, wait=False)
    with pytest.raises(fs.FsparseIndexError):
        res.wait()
    empty = fs.sparse(torch.zeros(0, dtype=torch.int32, device="cuda"),
                      torch.zeros(0, dtype=torch.int32, device="cuda"),
                      torch.zeros(0, dtype=torch.float64, device="cuda"),
                      4, 5, wait=False).wait()
    assert empty.nnz == 0 and empty.jcS.cpu().tolist() == [0] * 6


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_backward_of_dropped_and_logical_pairs(fs, dtype):
    rng = np.random.default_rng(10)
    L, m, n = 20000, 60, 50
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.integers(1, n + 1, L).astype(np.int32)
    ss = rng.integers(-2, 3, L).astype(dtype)
    ref = oracle.drop_zeros(oracle.assemble(ii, jj, ss, m, n))
    res = fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), m, n, keep_slot=True,
                    drop_zeros=True)
    assert_same(res, ref)
    assert (ref.slot < 0).any()
    w = rng.standard_normal(ref.nnz).astype(dtype)
    g = fs.backward(res.slot, to_dev(w))
    assert g.cpu().numpy().tobytes() == oracle.backward(ref.slot, w).tobytes()
    sl = ss > 0
    lref = oracle.assemble_logical(ii, jj, sl, m, n)
    lres = fs.sparse_logical(to_dev(ii), to_dev(jj), to_dev(sl), m, n,
                             keep_slot=True)
    wl = rng.standard_normal(lref.nnz).astype(dtype)
    g = fs.backward(lres.slot, to_dev(wl))
    assert g.cpu().numpy().tobytes() == oracle.backward(lref.slot, wl).tobytes()


def test_assembler_results_do_not_alias(fs):
    t = W.fem2d(20, 0.2, seed=11)
    A = fs.Assembler(to_dev(t.ii), to_dev(t.jj), to_dev(t.ss), t.m, t.n)
    p1 = A.reassemble(to_dev(t.ss * 2.0))
    keep = p1.clone()
    p2 = A.reassemble(to_dev(t.ss * 3.0))
    assert bool((p1 == keep).all())
    assert p1.data_ptr() != p2.data_ptr()
