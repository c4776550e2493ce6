"""Dropping zero sums (Matlab's convention) on the GPU against the oracle.

Values are small integers so that many pairs cancel exactly; the kept pairs,
the renumbered column pointers and the slots (-1 for a dropped pair) must
equal the oracle's bit for bit in every bin mode, for both value types, with
index expansion, double indices and the order-free sums.
"""
import ctypes

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


def check_drop(fs, ii, jj, ss, m=None, n=None, **kw):
    ref = oracle.drop_zeros(oracle.assemble(ii, jj, ss, m, n))
    res = fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), m, n, keep_slot=True,
                    drop_zeros=True, **kw)
    assert (res.m, res.n) == (ref.m, ref.n)
    assert_same(res, ref)
    return res, ref


def cancelling(L, m, n, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.integers(1, n + 1, L).astype(np.int32)
    ss = rng.integers(-2, 3, L).astype(dtype)
    ss[rng.random(L) < 0.05] = -0.0
    return ii, jj, ss


def test_hand_example(fs):
    ii = np.array([1, 2, 3, 1, 1, 3], np.int32)
    jj = np.array([1, 1, 1, 2, 1, 1], np.int32)
    ss = np.array([1.0, -0.0, 0.0, 2.0, -1.0, 5.0])
    res, _ = check_drop(fs, ii, jj, ss, 3, 3)
    assert res.slot.cpu().tolist() == [-1, -1, 0, 1, -1, 0]


@pytest.mark.parametrize("mode", ["auto", "dense", "slot", "claim"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_cancelling_values_all_modes(fs, mode, dtype):
    fs.set_tuning(bin_mode=mode)
    try:
        # about 3 triplets per pair: a good share of the sums is zero
        res, ref = check_drop(fs, *cancelling(300_000, 1000, 300, 60, dtype),
                              1000, 300)
        assert 0 < ref.nnz < oracle.assemble(
            *cancelling(300_000, 1000, 300, 60, dtype), 1000, 300).nnz
        t = W.fem3d(10, 0.15, seed=61)
        ss = np.round(t.ss * 4.0)              # whole numbers: exact sums
        check_drop(fs, t.ii, t.jj, ss.astype(dtype), t.m, t.n)
    finally:
        fs.set_tuning(reset=True)


def test_all_zero_and_no_zero(fs):
    ii, jj, _ = cancelling(50_000, 200, 100, 62)
    res, ref = check_drop(fs, ii, jj, np.zeros(ii.size), 200, 100)
    assert ref.nnz == 0 and res.jcS.cpu().tolist() == [0] * 101
    assert bool((res.slot == -1).all())
    t = W.uniform(100_000, 3000, 2000, seed=63)
    res, ref = check_drop(fs, t.ii, t.jj, t.ss, t.m, t.n)
    assert ref.nnz == oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n).nnz


def test_small_capacity_long_columns(fs):
    fs.set_tuning(chunk_cap=16)
    try:
        ii, jj, ss = cancelling(40_000, 400, 20, 64)
        check_drop(fs, ii, jj, ss, 400, 20)
    finally:
        fs.set_tuning(reset=True)


def test_with_expansion_double_indices_and_atomic(fs):
    t = W.fem2d(30, 0.2, seed=65)
    conn = t.meta["conn"]
    ne, nv = conn.shape
    K = np.round(t.ss * 3.0).reshape(ne, nv, nv)
    ref = oracle.drop_zeros(oracle.assemble(
        *oracle.expand(conn[:, :, None], conn[:, None, :], K), t.m, t.n))
    res = fs.sparse_expand(to_dev(conn[:, :, None]), to_dev(conn[:, None, :]),
                           to_dev(K), t.m, t.n, keep_slot=True,
                           drop_zeros=True)
    assert_same(res, ref)
    ii, jj, ss = cancelling(100_000, 500, 400, 66)
    check_drop(fs, ii.astype(np.float64), jj.astype(np.float64), ss, 500, 400)
    # whole-number sums are exact in any order: the order-free mode agrees
    ref = oracle.drop_zeros(oracle.assemble(ii, jj, ss, 500, 400))
    at = fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), 500, 400, atomic=True,
                   keep_slot=True, drop_zeros=True)
    assert_same(at, ref)


def test_no_plan_with_drop_zeros(fs):
    ii, jj, ss = cancelling(1000, 20, 20, 67)
    with pytest.raises(ValueError):
        fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), 20, 20, plan=True,
                  drop_zeros=True)
    from paper_1406_1066_amd import _lib as L
    dev = torch.device("cuda", 0)
    d = lambda a: torch.from_numpy(a).to(dev)
    ti, tj, ts = d(ii), d(jj), d(ss)
    jc = torch.empty(21, dtype=torch.int32, device=dev)
    ir = torch.empty(1000, dtype=torch.int32, device=dev)
    pr = torch.empty(1000, dtype=torch.float64, device=dev)
    ws = torch.empty(fs.workspace_bytes(1000, 20), dtype=torch.uint8,
                     device=dev)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    ph = ctypes.c_void_p()
    st = L.fsparse_assemble(p(ti), p(tj), p(ts), L.F64, 1000, 20, 20, 0,
                            L.DROP_ZEROS, p(jc), 21, p(ir), p(pr), 1000, None,
                            p(ws), ws.numel(), ctypes.byref(ph), None, None)
    assert st == L.E_ARG
    st = L.fsparse_assemble(p(ti), p(tj), p(ts), L.F64, 1000, 20, 20, 0,
                            8, p(jc), 21, p(ir), p(pr), 1000, None,
                            p(ws), ws.numel(), None, None, None)
    assert st == L.E_ARG                        # unknown flag
