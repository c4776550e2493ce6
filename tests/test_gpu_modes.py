"""Re-assembly, atomic mode, backward / autograd and batched assembly on the
GPU, each against the oracle (bit-exact where the definition fixes the
bits, within the stated tolerance for the atomic mode)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import assert_same, run, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_1066_amd as fs
    fs.set_tuning(reset=True)
    return fs


# ---------------------------------------------------------------------------
# pattern re-use (Section 2.1, repeated assembly)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_reuse_matches_oracle_and_fresh(fs, dtype):
    t = W.fem3d(13, 0.15, seed=21, dtype=dtype)
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    res = run(fs, t.ii, t.jj, t.ss, t.m, t.n, plan=True)
    assert_same(res, ref)
    out = torch.empty(res.nnz, dtype=res.prS.dtype, device="cuda")
    for step in range(4):
        s2 = W.element_scale(t, step, seed=21)
        got = fs.reassemble(res, to_dev(s2), out=out).cpu().numpy()
        want = oracle.reassemble(ref, t.ii, t.jj, s2)
        assert got.tobytes() == want.tobytes()
        fresh = run(fs, t.ii, t.jj, s2, t.m, t.n).prS.cpu().numpy()
        assert fresh.tobytes() == got.tobytes()


def test_reuse_graph_replay_new_buffers(fs):
    # the plan's graph is re-pointed when ss / prS move
    t = W.fem2d(40, 0.2, seed=3)
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    res = run(fs, t.ii, t.jj, t.ss, t.m, t.n, plan=True)
    for step in range(3):
        s2 = W.element_scale(t, step, seed=3)
        got = fs.reassemble(res, to_dev(s2)).cpu().numpy()   # fresh out each
        assert got.tobytes() == oracle.reassemble(ref, t.ii, t.jj,
                                                  s2).tobytes()


def test_reuse_with_long_columns(fs):
    fs.set_tuning(chunk_cap=32)
    try:
        t = W.uniform(5000, 50, 20, seed=4)
        ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
        res = run(fs, t.ii, t.jj, t.ss, t.m, t.n, plan=True, keep_slot=True)
        assert_same(res, ref)
        s2 = t.ss * 3.0 - 1.0
        got = fs.reassemble(res, to_dev(s2)).cpu().numpy()
        assert got.tobytes() == oracle.reassemble(ref, t.ii, t.jj,
                                                  s2).tobytes()
    finally:
        fs.set_tuning(reset=True)


# ---------------------------------------------------------------------------
# fixed-capacity bins with the values binned, or with (row, k) only and the
# values read by k in the bin stage
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_slot_values_binned_and_by_k(fs, dtype):
    cases = [W.fem3d(14, 0.15, seed=31, dtype=dtype),
             W.uniform(60_000, 3000, 2500, seed=32).astype(dtype)]
    try:
        for t in cases:
            ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
            s2 = (t.ss * 1.5 - 0.25).astype(dtype)
            want = oracle.reassemble(ref, t.ii, t.jj, s2)
            for sv in ("binned", "by_k"):
                fs.set_tuning(reset=True)
                fs.set_tuning(bin_mode="slot", slot_values=sv)
                res = run(fs, t.ii, t.jj, t.ss, t.m, t.n, plan=True,
                          keep_slot=True)
                assert_same(res, ref)
                got = fs.reassemble(res, to_dev(s2)).cpu().numpy()
                assert got.tobytes() == want.tobytes()
    finally:
        fs.set_tuning(reset=True)


# ---------------------------------------------------------------------------
# atomic mode: order-free sums within the stated tolerance
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-14), (np.float32, 1e-6)])
def test_atomic_mode_tolerance(fs, dtype, tol):
    t = W.fem3d(12, 0.15, seed=5, dtype=dtype)
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    scale = oracle.assemble(t.ii, t.jj, np.abs(t.ss).astype(np.float64),
                            t.m, t.n).prS
    res = run(fs, t.ii, t.jj, t.ss, t.m, t.n, atomic=True, plan=True)
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    np.testing.assert_array_equal(res.jcS.cpu().numpy(), ref.jcS)
    for got in (res.prS.cpu().numpy(),
                fs.reassemble(res, to_dev(t.ss), atomic=True).cpu().numpy()):
        err = np.abs(got.astype(np.float64) - ref.prS.astype(np.float64))
        assert np.all(err <= tol * np.maximum(scale, 1e-300)), err.max()


def test_atomic_reuse_on_plan_without_slot(fs):
    # a plan made without a slot array derives the slot map from its sorted
    # order on the first atomic re-use; ordered re-use is unaffected
    t = W.fem3d(12, 0.15, seed=9)
    res = run(fs, t.ii, t.jj, t.ss, t.m, t.n, plan=True)
    assert res.slot is None
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    whole = np.round(t.ss * 8.0)               # whole numbers: exact sums
    want = oracle.assemble(t.ii, t.jj, whole, t.m, t.n).prS
    for _ in range(2):
        got = fs.reassemble(res, to_dev(whole), atomic=True).cpu().numpy()
        assert got.tobytes() == want.tobytes()
    scale = oracle.assemble(t.ii, t.jj, np.abs(t.ss), t.m, t.n).prS
    got = fs.reassemble(res, to_dev(t.ss), atomic=True).cpu().numpy()
    assert np.all(np.abs(got - ref.prS) <= 1e-14 * np.maximum(scale, 1e-300))
    got = fs.reassemble(res, to_dev(t.ss)).cpu().numpy()
    assert got.tobytes() == ref.prS.tobytes()


def test_atomic_mode_exact_on_counts(fs):
    t = W.ransparse(2000, 20, 10, seed=6)
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    res = run(fs, t.ii, t.jj, t.ss, t.m, t.n, atomic=True)
    assert res.prS.cpu().numpy().tobytes() == ref.prS.tobytes()


# ---------------------------------------------------------------------------
# backward
# ---------------------------------------------------------------------------
def test_backward_gather_exact(fs):
    t = W.fem2d(25, 0.2, seed=7)
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    res = run(fs, t.ii, t.jj, t.ss, t.m, t.n, keep_slot=True)
    w = np.random.default_rng(1).standard_normal(ref.nnz)
    g = fs.backward(res.slot, to_dev(w)).cpu().numpy()
    assert g.tobytes() == oracle.backward(ref.slot, w).tobytes()


def test_autograd_function(fs):
    t = W.fem2d(10, 0.2, seed=8)
    ii, jj = to_dev(t.ii), to_dev(t.jj)
    s = to_dev(t.ss).requires_grad_(True)
    prS, jcS, irS = fs.SparseAssemble.apply(s, ii, jj, t.m, t.n)
    w = torch.randn(prS.numel(), dtype=torch.float64, device="cuda")
    (w * prS).sum().backward()
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    assert s.grad.cpu().numpy().tobytes() == oracle.backward(
        ref.slot, w.cpu().numpy()).tobytes()


def test_gradcheck_tiny(fs):
    rng = np.random.default_rng(9)
    ii = to_dev(rng.integers(1, 5, size=30).astype(np.int32))
    jj = to_dev(rng.integers(1, 4, size=30).astype(np.int32))
    s = torch.randn(30, dtype=torch.float64, device="cuda",
                    requires_grad=True)
    f = lambda x: fs.SparseAssemble.apply(x, ii, jj, 4, 3)[0]
    assert torch.autograd.gradcheck(f, (s,), eps=1e-6, atol=1e-8)


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------
def _batch_inputs(mats):
    ii = np.concatenate([m[0] for m in mats]).astype(np.int32)
    jj = np.concatenate([m[1] for m in mats]).astype(np.int32)
    ss = np.concatenate([m[2] for m in mats])
    off = np.zeros(len(mats) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(m[0]) for m in mats])
    return ii, jj, ss, off


@pytest.mark.parametrize("cap", [2048, 16])
def test_batched_uneven(fs, cap):
    fs.set_tuning(chunk_cap=cap)
    try:
        rng = np.random.default_rng(10)
        mats = []
        for s in (2, 7, 30, 3, 55, 12):
            t = W.fem2d(s, 0.2, seed=s)
            mats.append((t.ii, t.jj, t.ss, t.m, t.n))
        mats.append((np.zeros(0, np.int32), np.zeros(0, np.int32),
                     np.zeros(0), 4, 3))                    # empty matrix
        u = W.uniform(3000, 90, 60, seed=11)
        mats.append((u.ii, u.jj, u.ss, 100, 70))            # dims > max
        mats.append((np.zeros(0, np.int32), np.zeros(0, np.int32),
                     np.zeros(0), 5, 0))                    # no columns
        ii, jj, ss, off = _batch_inputs(mats)
        res = fs.assemble_batched(to_dev(ii), to_dev(jj), to_dev(ss), off,
                                  [m[3] for m in mats], [m[4] for m in mats],
                                  keep_slot=True)
        for b, (bi, bj, bs, bm, bn) in enumerate(mats):
            ref = oracle.assemble(bi, bj, bs, bm, bn)
            jc, ir, pr = res.matrix(b)
            np.testing.assert_array_equal(jc.cpu().numpy(), ref.jcS)
            np.testing.assert_array_equal(ir.cpu().numpy(), ref.irS)
            assert pr.cpu().numpy().tobytes() == ref.prS.tobytes()
            sl = res.slot[off[b]:off[b + 1]].cpu().numpy() - res.nnz_off[b]
            np.testing.assert_array_equal(sl, ref.slot)
    finally:
        fs.set_tuning(reset=True)


def test_batched_out_buffers(fs):
    # caller-supplied outputs, reused by a second call on other values, and
    # refused when too small
    b = W.batched_fem2d(5, 1e3, 2e4, seed=17)
    bi, bj, bs, bm, bn = b.concat()
    N, L = int(bn.sum()), len(bi)
    out = (torch.empty(N + b.nb, dtype=torch.int32, device="cuda"),
           torch.empty(L, dtype=torch.int32, device="cuda"),
           torch.empty(L, dtype=torch.float64, device="cuda"))
    for scale in (1.0, -0.5):
        s2 = bs * scale
        res = fs.assemble_batched(to_dev(bi), to_dev(bj), to_dev(s2),
                                  b.trip_off, bm, bn, out=out)
        assert res.prS.data_ptr() == out[2].data_ptr()
        for q, tq in enumerate(b.mats):
            ref = oracle.assemble(tq.ii, tq.jj, tq.ss * scale, tq.m, tq.n)
            jc, ir, pr = res.matrix(q)
            np.testing.assert_array_equal(jc.cpu().numpy(), ref.jcS)
            np.testing.assert_array_equal(ir.cpu().numpy(), ref.irS)
            assert pr.cpu().numpy().tobytes() == ref.prS.tobytes()
    with pytest.raises(ValueError):
        fs.assemble_batched(to_dev(bi), to_dev(bj), to_dev(bs), b.trip_off,
                            bm, bn, out=(out[0][:N], out[1], out[2]))


def test_batched_reuse_and_default_dims(fs):
    mats = []
    for s in (5, 20, 9):
        t = W.fem2d(s, 0.2, seed=100 + s)
        mats.append((t.ii, t.jj, t.ss, t.m, t.n))
    ii, jj, ss, off = _batch_inputs(mats)
    res = fs.assemble_batched(to_dev(ii), to_dev(jj), to_dev(ss), off,
                              [-1] * 3, [-1] * 3, plan=True)
    assert res.m == [m[3] for m in mats] and res.n == [m[4] for m in mats]
    ss2 = ss * 0.5 + 0.25
    pr2 = fs.reassemble(res, to_dev(ss2)).cpu().numpy()
    for b, (bi, bj, bs, bm, bn) in enumerate(mats):
        ref = oracle.assemble(bi, bj, ss2[off[b]:off[b + 1]], bm, bn)
        a, e = res.nnz_off[b], res.nnz_off[b + 1]
        assert pr2[a:e].tobytes() == ref.prS.tobytes()


def test_batched_bad_index(fs):
    with pytest.raises(fs.FsparseIndexError):
        fs.assemble_batched(to_dev(np.array([1, 3], np.int32)),
                            to_dev(np.array([1, 1], np.int32)),
                            to_dev(np.ones(2)), [0, 1, 2], [2, 2], [2, 2])


@pytest.mark.parametrize("mode", ["auto", "dense", "slot", "claim"])
def test_batched_modes_fp32(fs, mode):
    # every bin mode on a batch of single-precision matrices, bins spanning
    # matrix boundaries (small capacity)
    fs.set_tuning(chunk_cap=256, bin_mode=mode)
    try:
        mats = []
        for s in (3, 40, 17, 9):
            t = W.fem2d(s, 0.2, seed=200 + s, dtype=np.float32)
            mats.append((t.ii, t.jj, t.ss, t.m, t.n))
        u = W.uniform(20_000, 500, 300, seed=21, dtype=np.float32)
        mats.append((u.ii, u.jj, u.ss, u.m, u.n))
        ii, jj, ss, off = _batch_inputs(mats)
        res = fs.assemble_batched(to_dev(ii), to_dev(jj), to_dev(ss), off,
                                  [m[3] for m in mats], [m[4] for m in mats])
        for b, (bi, bj, bs, bm, bn) in enumerate(mats):
            ref = oracle.assemble(bi, bj, bs, bm, bn)
            jc, ir, pr = res.matrix(b)
            np.testing.assert_array_equal(jc.cpu().numpy(), ref.jcS)
            np.testing.assert_array_equal(ir.cpu().numpy(), ref.irS)
            assert pr.cpu().numpy().tobytes() == ref.prS.tobytes()
    finally:
        fs.set_tuning(reset=True)


def test_host_value_tensors_are_refused(fs):
    # values left on the host raise before any launch
    ii = to_dev(np.array([1, 2], np.int32))
    host = torch.tensor([1.0, 2.0], dtype=torch.float64)
    with pytest.raises(ValueError):
        fs.sparse(ii, ii, host, 2, 2)
    with pytest.raises(ValueError):
        fs.sparse_complex(ii, ii, host, host, 2, 2)
    with pytest.raises(ValueError):
        fs.sparse_logical(ii, ii, torch.tensor([True, False]), 2, 2)
    res = fs.sparse(ii, ii, to_dev(np.array([1.0, 2.0])), 2, 2, plan=True)
    with pytest.raises(ValueError):
        fs.reassemble(res, host)


@pytest.mark.parametrize("mode", ["auto", "slot", "claim"])
def test_batched_capacity_below_nnz(fs, mode):
    # a capacity below the total of distinct pairs is refused with the
    # capacity status (every bin mode), and the same call with room succeeds
    fs.set_tuning(bin_mode=mode)
    try:
        b = W.batched_fem2d(5, 1e3, 2e4, seed=12)
        ii, jj, ss, m, n = b.concat()
        d = [to_dev(a) for a in (ii, jj, ss)]
        full = fs.assemble_batched(*d, b.trip_off, m, n)
        with pytest.raises(fs.FsparseError) as e:
            fs.assemble_batched(*d, b.trip_off, m, n, cap=full.nnz_off[-1] - 1)
        assert e.value.status == 3
        ok = fs.assemble_batched(*d, b.trip_off, m, n, cap=full.nnz_off[-1])
        assert ok.prS.cpu().numpy().tobytes() == full.prS.cpu().numpy().tobytes()
        assert ok.nnz_off == full.nnz_off
    finally:
        fs.set_tuning(reset=True)
