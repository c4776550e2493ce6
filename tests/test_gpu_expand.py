"""Index expansion on the GPU against the oracle (bit-exact).

The expanded call reads ii, jj, ss through a broadcast map and never forms
the expanded index arrays; its result must equal the oracle's assembly of
the written-out triplets, for every bin mode and capacity, with slots,
re-assembly and backward counting all expanded triplets.
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


def check_expand(fs, ii, jj, ss, m=None, n=None, **kw):
    ref = oracle.assemble(*oracle.expand(ii, jj, ss), m, n)
    kw.setdefault("keep_slot", True)
    res = fs.sparse_expand(to_dev(ii), to_dev(jj), to_dev(ss), m, n, **kw)
    assert (res.m, res.n) == (ref.m, ref.n)
    assert_same(res, ref)
    return res, ref


def _fem(dim, s, dtype=np.float64):
    t = (W.fem2d(s, 0.2, seed=s, dtype=dtype) if dim == 2
         else W.fem3d(s, 0.15, seed=s, dtype=dtype))
    conn = t.meta["conn"]
    ne, nv = conn.shape
    return t, conn, t.ss.reshape(ne, nv, nv)


@pytest.mark.parametrize("mode", ["auto", "dense", "slot", "claim"])
@pytest.mark.parametrize("dim,s", [(2, 60), (3, 14)])
def test_fem_connectivity(fs, mode, dim, s):
    fs.set_tuning(bin_mode=mode)
    try:
        t, conn, K = _fem(dim, s)
        res, ref = check_expand(fs, conn[:, :, None], conn[:, None, :], K,
                                t.m, t.n)
        # the same as the plain call on the emitted triplets
        plain = fs.sparse(to_dev(t.ii), to_dev(t.jj), to_dev(t.ss), t.m, t.n,
                          keep_slot=True)
        assert plain.prS.cpu().numpy().tobytes() == \
            res.prS.cpu().numpy().tobytes()
        np.testing.assert_array_equal(plain.slot.cpu().numpy(),
                                      res.slot.cpu().numpy())
    finally:
        fs.set_tuning(reset=True)


@pytest.mark.parametrize("c", [16, 256, 2048])
def test_fem_fp32_default_dims_and_unit_values(fs, c):
    fs.set_tuning(chunk_cap=c)
    try:
        t, conn, K = _fem(3, 9, np.float32)
        check_expand(fs, conn[:, :, None], conn[:, None, :], K)
        one = np.ones((1, 1, 1), np.float32)
        check_expand(fs, conn[:, :, None], conn[:, None, :], one, t.m, t.n)
    finally:
        fs.set_tuning(reset=True)


SHAPES = [
    # (ii, jj, ss) shapes, broadcast to (P, C, R)
    ((5, 1, 7), (5, 3, 1), (5, 3, 7)),
    ((7,), (3, 1), (1,)),
    ((4, 3, 7), (4, 3, 7), (4, 3, 7)),
    ((1, 300, 1), (1, 1, 400), (1, 300, 400)),
    ((2000, 1, 1), (2000, 1, 6), (1, 1, 6)),
    ((1, 1, 1), (9, 50, 20), (9, 1, 20)),
    ((3, 1), (1, 5), (3, 5)),
    ((123457,), (123457,), (1,)),
]


@pytest.mark.parametrize("k", range(len(SHAPES)))
@pytest.mark.parametrize("c", [64, 2048])
def test_broadcast_shapes(fs, k, c):
    fs.set_tuning(chunk_cap=c)
    try:
        rng = np.random.default_rng(40 + k)
        si, sj, sv = SHAPES[k]
        m, n = 700, 900
        ii = rng.integers(1, m + 1, size=si).astype(np.int32)
        jj = rng.integers(1, n + 1, size=sj).astype(np.int32)
        ss = rng.standard_normal(sv)
        ss[rng.random(sv) < 0.1] = -0.0
        check_expand(fs, ii, jj, ss, m, n)
        check_expand(fs, ii, jj, ss.astype(np.float32))
    finally:
        fs.set_tuning(reset=True)


def test_reuse_backward_and_atomic(fs):
    t, conn, K = _fem(3, 10)
    ii, jj = conn[:, :, None], conn[:, None, :]
    res, ref = check_expand(fs, ii, jj, K, t.m, t.n, plan=True)
    # re-assembly takes values for every expanded triplet
    ss2 = W.element_scale(t, 1, seed=3)
    pr2 = fs.reassemble(res, to_dev(ss2)).cpu().numpy()[:ref.nnz]
    want = oracle.assemble(t.ii, t.jj, ss2, t.m, t.n).prS
    assert pr2.tobytes() == want.tobytes()
    g = np.linspace(-1.0, 1.0, ref.nnz)
    gs = fs.backward(res.slot, to_dev(g)).cpu().numpy()
    assert gs.tobytes() == oracle.backward(ref.slot, g).tobytes()
    # order-free sums: full-shape values only
    at = fs.sparse_expand(to_dev(ii), to_dev(jj), to_dev(K), t.m, t.n,
                          atomic=True)
    np.testing.assert_array_equal(at.irS.cpu().numpy(), ref.irS)
    bound = oracle.assemble(t.ii, t.jj, np.abs(t.ss), t.m, t.n).prS
    assert np.all(np.abs(at.prS.cpu().numpy() - ref.prS) <= 1e-14 * bound)
    with pytest.raises(fs.FsparseError):
        fs.sparse_expand(to_dev(ii), to_dev(jj), to_dev(np.ones((1, 1, 1))),
                         t.m, t.n, atomic=True)


def test_empty_grid_and_errors(fs):
    e = np.zeros((0, 1, 3), np.int32)
    res = fs.sparse_expand(to_dev(e), to_dev(np.ones((1, 4, 1), np.int32)),
                           to_dev(np.ones(1)), 5, 6)
    assert res.nnz == 0 and res.jcS.cpu().tolist() == [0] * 7
    res = fs.sparse_expand(to_dev(e), to_dev(np.ones((1, 4, 1), np.int32)),
                           to_dev(np.ones(1)))
    assert (res.m, res.n, res.nnz) == (0, 0, 0)
    ii = np.array([[1], [2], [9]], np.int32)      # 9 > m
    jj = np.array([[1, 2]], np.int32)
    with pytest.raises(fs.FsparseIndexError):
        fs.sparse_expand(to_dev(ii), to_dev(jj), to_dev(np.ones(1)), 4, 2)
    with pytest.raises(fs.FsparseIndexError):
        fs.sparse_expand(to_dev(ii - 1), to_dev(jj), to_dev(np.ones(1)))


def test_abi_rejects_bad_shapes(fs):
    from paper_1406_1066_amd import _lib as L
    dev = torch.device("cuda", 0)
    ii = torch.ones(12, dtype=torch.int32, device=dev)
    ss = torch.ones(12, dtype=torch.float64, device=dev)
    jc = torch.empty(5, dtype=torch.int32, device=dev)
    ir = torch.empty(12, dtype=torch.int32, device=dev)
    pr = torch.empty(12, dtype=torch.float64, device=dev)
    ws = torch.empty(fs.workspace_bytes(12, 4), dtype=torch.uint8, device=dev)

    def call(shape, si, sj, sv, flags=L.ORDERED):
        x = L.FsparseExpand()
        for d in range(3):
            x.shape[d], x.ii_shape[d] = shape[d], si[d]
            x.jj_shape[d], x.ss_shape[d] = sj[d], sv[d]
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        return L.fsparse_assemble_expand(
            p(ii), p(ii), p(ss), L.F64, ctypes.byref(x), 4, 4, 0, flags,
            p(jc), 5, p(ir), p(pr), 12, None, p(ws), ws.numel(), None, None,
            None)
    good = (3, 4, 1)
    assert call(good, (3, 1, 1), (1, 4, 1), good) == L.OK
    assert call(good, (2, 1, 1), (1, 4, 1), good) == L.E_ARG     # 2 != 3, != 1
    assert call(good, (3, 1, 1), (1, 4, 2), good) == L.E_ARG     # P is 1
    assert call((3, 4, -1), (3, 1, 1), (1, 4, 1), (3, 4, 1)) == L.E_ARG
    assert call((1 << 16, 1 << 16, 1), (1, 1, 1), (1, 1, 1),
                (1, 1, 1)) == L.E_ARG                            # 2^32 triplets
    assert call(good, (3, 1, 1), (1, 4, 1), (1, 1, 1),
                flags=L.ATOMIC) == L.E_ARG
