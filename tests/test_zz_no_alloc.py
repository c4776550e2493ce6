"""The no-allocation entry point (fsparse_assemble_noalloc) against the
workspace entry point (fsparse_assemble) on the same inputs: every output
array byte for byte, on two calls in a row (the second on a smaller input,
so the library's fixed workspace holds the first call's data when it
starts), and both against the oracle."""
import ctypes

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
    return fs


def _same(a, b, slot=True):
    np.testing.assert_array_equal(a.jcS.cpu().numpy(), b.jcS.cpu().numpy())
    assert a.nnz == b.nnz
    np.testing.assert_array_equal(a.irS.cpu().numpy(), b.irS.cpu().numpy())
    assert a.prS.cpu().numpy().tobytes() == b.prS.cpu().numpy().tobytes()
    if slot:
        np.testing.assert_array_equal(a.slot.cpu().numpy(),
                                      b.slot.cpu().numpy())


def _oracle(res, t):
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    np.testing.assert_array_equal(res.jcS.cpu().numpy(), ref.jcS)
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    assert res.prS.cpu().numpy().tobytes() == ref.prS.tobytes()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_two_calls_second_smaller(fs, dtype):
    big = W.fem2d(120, 0.2, seed=5, dtype=dtype)         # 254k triplets
    small = W.uniform(20_000, 3_000, 3_000, seed=6, dtype=dtype)
    for t in (big, small):
        ii, jj, ss = to_dev(t.ii), to_dev(t.jj), to_dev(t.ss)
        want = fs.sparse(ii, jj, ss, t.m, t.n, keep_slot=True)
        slot = torch.empty(t.L, dtype=torch.int32, device=ii.device)
        out = (torch.empty(t.n + 1, dtype=torch.int32, device=ii.device),
               torch.empty(t.L, dtype=torch.int32, device=ii.device),
               torch.empty(t.L, dtype=ss.dtype, device=ii.device), slot)
        got = fs.sparse_noalloc(ii, jj, ss, t.m, t.n, out=out)
        _same(got, want)
        _oracle(got, t)


def test_atomic_and_repeat(fs):
    # order-free sums within tolerance of the ordered ones, then the ordered
    # call again on the same workspace contents
    t = W.fem2d(60, 0.2, seed=7)
    ii, jj, ss = to_dev(t.ii), to_dev(t.jj), to_dev(t.ss)
    want = fs.sparse(ii, jj, ss, t.m, t.n, keep_slot=True)
    got = fs.sparse_noalloc(ii, jj, ss, t.m, t.n, atomic=True)
    np.testing.assert_array_equal(got.irS.cpu().numpy(), want.irS.cpu().numpy())
    den = oracle.postprocess(want.slot.cpu().numpy(), np.abs(t.ss), want.nnz)
    assert np.all(np.abs(got.prS.cpu().numpy() - want.prS.cpu().numpy())
                  <= 1e-14 * den)
    again = fs.sparse_noalloc(ii, jj, ss, t.m, t.n)
    _same(again, want, slot=False)


def test_limits(fs):
    from paper_1406_1066_amd import _lib as L
    # beyond the fixed workspace: refused before any work is queued
    n = 1000
    Lbig = 4_000_000
    assert fs.workspace_bytes(Lbig, n) > L.NOALLOC_SCRATCH_BYTES
    ii = torch.ones(Lbig, dtype=torch.int32, device="cuda")
    ss = torch.ones(Lbig, dtype=torch.float64, device="cuda")
    with pytest.raises(fs.FsparseError):
        fs.sparse_noalloc(ii, ii, ss, 1, n)
    # indices out of range are reported like fsparse_assemble's
    t = W.uniform(1000, 50, 50, seed=8)
    ii, jj, ss = to_dev(t.ii), to_dev(t.jj), to_dev(t.ss)
    with pytest.raises(fs.FsparseIndexError):
        fs.sparse_noalloc(ii, jj, ss, t.m, int(t.jj.max()) - 1)
    # and an empty input gives an all-zero jcS
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    r = fs.sparse_noalloc(e, e, torch.empty(0, dtype=torch.float64,
                                            device="cuda"), 3, 4)
    assert r.nnz == 0 and r.jcS.cpu().tolist() == [0] * 5
    # the same call through the raw C ABI, capacity below len: E_CAPACITY
    info = L.FsparseInfo()
    jc = torch.empty(t.n + 1, dtype=torch.int32, device="cuda")
    ir = torch.empty(t.L - 1, dtype=torch.int32, device="cuda")
    pr = torch.empty(t.L - 1, dtype=torch.float64, device="cuda")
    st = L.fsparse_assemble_noalloc(
        ctypes.c_void_p(ii.data_ptr()), ctypes.c_void_p(jj.data_ptr()),
        ctypes.c_void_p(ss.data_ptr()), L.F64, t.L, t.m, t.n, 0, 0,
        ctypes.c_void_p(jc.data_ptr()), t.n + 1, ctypes.c_void_p(ir.data_ptr()),
        ctypes.c_void_p(pr.data_ptr()), t.L - 1, None, ctypes.byref(info),
        None)
    assert st == L.E_CAPACITY and info.nnz == t.L
