"""Parity at the full workload sizes, in the launch configuration the
benchmark times (default tuning).

Every workload (uniform_1e7; fem3d_100, 93M triplets, plain and index
expanded; batched_64, 64 matrices with 175M triplets; fem3d_50 in both value
types; complex and logical values on uniform_1e7) is compared with the
oracle array by array, every element.  Re-assembly steps are checked, value
by value, against the serial post-processing pass on the oracle's slot map.
Pattern invariants that hold at any size are checked beside them.
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
    return fs


def check_invariants(res, ii_d, jj_d, m, n):
    """Whole-output properties, evaluated on the GPU."""
    jc = res.jcS.to(torch.int64)
    nnz = res.nnz
    assert int(jc[0]) == 0 and int(jc[-1]) == nnz
    assert bool((jc[1:] >= jc[:-1]).all())
    ir = res.irS.to(torch.int64)
    assert int(ir.min()) >= 0 and int(ir.max()) < m
    colof = torch.repeat_interleave(torch.arange(n, device=jc.device),
                                    jc[1:] - jc[:-1])
    same = colof[1:] == colof[:-1]
    assert bool((ir[1:][same] > ir[:-1][same]).all())   # strictly increasing
    sl = res.slot.to(torch.int64)
    assert int(sl.min()) >= 0 and int(sl.max()) < nnz
    assert bool((ir[sl] == ii_d.to(torch.int64) - 1).all())
    jm = jj_d.to(torch.int64) - 1
    assert bool((jc[jm] <= sl).all()) and bool((sl < jc[jm + 1]).all())
    # every slot receives at least one triplet
    hit = torch.zeros(nnz, dtype=torch.bool, device=jc.device)
    hit[sl] = True
    assert bool(hit.all())


def test_uniform_1e7(fs):
    t = W.config("uniform_1e7")
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    ii, jj, ss = to_dev(t.ii), to_dev(t.jj), to_dev(t.ss)
    res = fs.sparse(ii, jj, ss, t.m, t.n, keep_slot=True, plan=True)
    key = (t.jj.astype(np.int64) - 1) * t.m + (t.ii - 1)
    assert res.nnz == np.unique(key).size
    check_invariants(res, ii, jj, t.m, t.n)
    assert_whole(res, ref)
    # re-assembly with new values on the same pattern
    s2 = t.ss * 0.5 - 1.0
    pr = fs.reassemble(res, to_dev(s2)).cpu().numpy()
    assert pr.tobytes() == oracle.postprocess(ref.slot, s2, ref.nnz).tobytes()


@pytest.fixture(scope="module")
def fem3d_100():
    t = W.config("fem3d_100")
    return t, oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)


def assert_whole(res, ref, slot=True):
    """Every output array against the oracle's, byte for byte."""
    np.testing.assert_array_equal(res.jcS.cpu().numpy(), ref.jcS)
    assert res.nnz == ref.nnz
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    got = res.prS.cpu().numpy()
    if got.tobytes() != ref.prS.tobytes():
        bad = np.nonzero(got.view(np.uint64 if got.itemsize == 8 else np.uint32)
                         != ref.prS.view(np.uint64 if got.itemsize == 8
                                         else np.uint32))[0]
        raise AssertionError("prS differs at %d of %d entries, first %s"
                             % (bad.size, got.size, bad[:5]))
    if slot:
        np.testing.assert_array_equal(res.slot.cpu().numpy(), ref.slot)


def test_fem3d_100_whole_output(fs, fem3d_100):
    # every array of the 93M-triplet assembly against the oracle, then the
    # time-stepping shape: re-assembly with per-element factors U[0.5, 2],
    # every value against the serial post-processing pass on the oracle's
    # slot map, the order-free re-assembly within its tolerance, and the
    # backward gather in full
    t, ref = fem3d_100
    L, nnz = W.fem3d_counts(100)
    assert t.L == L and ref.nnz == nnz
    ii, jj, ss = to_dev(t.ii), to_dev(t.jj), to_dev(t.ss)
    res = fs.sparse(ii, jj, ss, t.m, t.n, keep_slot=True, plan=True)
    assert_whole(res, ref)
    del ii, jj
    out = torch.empty(ref.nnz, dtype=ss.dtype, device=ss.device)
    for step in range(3):
        s2 = W.element_scale(t, step, seed=1068)
        pr = fs.reassemble(res, to_dev(s2), out=out).cpu().numpy()
        want = oracle.postprocess(ref.slot, s2, ref.nnz)
        assert pr.tobytes() == want.tobytes(), "re-assembly step %d" % step
    s2 = W.element_scale(t, 3, seed=1068)
    pa = fs.reassemble(res, to_dev(s2), out=out, atomic=True).cpu().numpy()
    want = oracle.postprocess(ref.slot, s2, ref.nnz)
    den = oracle.postprocess(ref.slot, np.abs(s2), ref.nnz)
    assert np.all(np.abs(pa - want) <= 1e-14 * den)
    w = np.random.default_rng(1068).standard_normal(ref.nnz)
    g = fs.backward(res.slot, to_dev(w)).cpu().numpy()
    assert g.tobytes() == oracle.backward(ref.slot, w).tobytes()


def _oracle_many(mats, vals=None):
    # the oracle on every matrix of a batch, on host threads (the C calls
    # release the interpreter lock)
    from concurrent.futures import ThreadPoolExecutor
    vals = vals or [t.ss for t in mats]
    with ThreadPoolExecutor(16) as ex:
        return list(ex.map(lambda a: oracle.assemble(a[0].ii, a[0].jj, a[1],
                                                     a[0].m, a[0].n),
                           zip(mats, vals)))


def test_batched_64_whole_output_and_graph_reuse(fs):
    # all 64 matrices (175M triplets) in one call, every array of every
    # matrix against the oracle; then two graph-replayed re-assemblies with
    # per-element factors, every value of every matrix checked
    batch = W.config("batched_64")
    ii, jj, ss, m, n = batch.concat()
    off = batch.trip_off
    refs = _oracle_many(batch.mats)
    d = (to_dev(ii), to_dev(jj), to_dev(ss))
    res = fs.assemble_batched(*d, off, m, n, keep_slot=True, plan=True)
    sizes = [t.meta["s"] for t in batch.mats]
    jcn, irn, prn = (res.jcS.cpu().numpy(), res.irS.cpu().numpy(),
                     res.prS.cpu().numpy())
    sln = res.slot.cpu().numpy()
    for b, (t, ref) in enumerate(zip(batch.mats, refs)):
        assert ref.nnz == W.fem2d_counts(sizes[b])[1]
        a, e = res.nnz_off[b], res.nnz_off[b + 1]
        assert e - a == ref.nnz, b
        j0 = res.col_off[b] + b
        np.testing.assert_array_equal(jcn[j0:j0 + t.n + 1], ref.jcS)
        np.testing.assert_array_equal(irn[a:e], ref.irS)
        assert prn[a:e].tobytes() == ref.prS.tobytes(), "matrix %d" % b
        np.testing.assert_array_equal(sln[off[b]:off[b + 1]] - a, ref.slot)
    del jcn, irn, prn, sln
    out = torch.empty(res.nnz, dtype=d[2].dtype, device="cuda")
    for step in range(2):
        s2 = [W.element_scale(t, step, seed=1069 + 1000 * (b + 1))
              for b, t in enumerate(batch.mats)]
        pr = fs.reassemble(res, to_dev(np.concatenate(s2)), out=out)
        pr = pr.cpu().numpy()
        for b, ref in enumerate(refs):
            a, e = res.nnz_off[b], res.nnz_off[b + 1]
            want = oracle.postprocess(ref.slot, s2[b], ref.nnz)
            assert pr[a:e].tobytes() == want.tobytes(), (step, b)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_fem3d_50_full_and_backward(fs, dtype):
    t = W.config("fem3d_50", dtype=dtype)
    ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    ii, jj, ss = to_dev(t.ii), to_dev(t.jj), to_dev(t.ss)
    res = fs.sparse(ii, jj, ss, t.m, t.n, keep_slot=True, plan=True)
    np.testing.assert_array_equal(res.jcS.cpu().numpy(), ref.jcS)
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    assert res.prS.cpu().numpy().tobytes() == ref.prS.tobytes()
    np.testing.assert_array_equal(res.slot.cpu().numpy(), ref.slot)

    # loss = sum(w * prS), w ~ N(0,1); backward through the autograd Function
    rng = np.random.default_rng(1070)
    w = rng.standard_normal(ref.nnz)
    wd = torch.from_numpy(w.astype(dtype)).cuda()
    s_req = ss.clone().requires_grad_(True)
    prS, _, _ = fs.SparseAssemble.apply(s_req, ii, jj, t.m, t.n)
    (wd * prS).sum().backward()
    g = s_req.grad.cpu().numpy()
    assert g.tobytes() == oracle.backward(ref.slot, w.astype(dtype)).tobytes()

    # dense-scatter reference gradient (torch autograd on the CPU, fp64):
    # prS = index_add over the inverse of the unique (column,row) keys
    key = torch.from_numpy((t.jj.astype(np.int64) - 1) * t.m + (t.ii - 1))
    _, inv = torch.unique(key, return_inverse=True)
    sc = torch.from_numpy(t.ss.astype(np.float64)).requires_grad_(True)
    p_ref = torch.zeros(ref.nnz, dtype=torch.float64).index_add(0, inv, sc)
    (torch.from_numpy(w) * p_ref).sum().backward()
    np.testing.assert_array_equal(sc.grad.numpy().astype(dtype), g)

    # central finite differences on 1000 entries, through re-assembly
    h_rel, tol = (1e-3, 1e-8) if dtype == np.float64 else (1e-2, 1e-3)
    ks = rng.choice(t.L, size=1000, replace=False)
    wd64 = torch.from_numpy(w).cuda()
    out = torch.empty(ref.nnz, dtype=ss.dtype, device="cuda")

    def loss(s):
        return float((wd64 * fs.reassemble(res, s, out=out).to(torch.float64)
                      ).sum())

    sp = ss.clone()
    worst = 0.0
    for k in ks:
        h = h_rel * max(1.0, abs(float(t.ss[k])))
        x0 = sp[k].item()
        sp[k] = x0 + h
        hp = float(sp[k].item()) - x0
        lp = loss(sp)
        sp[k] = x0 - h
        hm = x0 - float(sp[k].item())
        lm = loss(sp)
        sp[k] = x0
        fd = (lp - lm) / (hp + hm)
        worst = max(worst, abs(fd - float(g[k])) / max(1.0, abs(float(g[k]))))
    assert worst <= tol, worst


def test_fem3d_100_expanded(fs, fem3d_100):
    # index expansion at full size: connectivity and element matrices only
    # (the 93M-triplet index arrays are never formed); every output array
    # against the oracle's assembly of the written-out triplets
    t, ref = fem3d_100
    conn = t.meta["conn"]
    ne, nv = conn.shape
    c = to_dev(conn)
    K = to_dev(t.ss).view(ne, nv, nv)
    res = fs.sparse_expand(c[:, :, None], c[:, None, :], K, t.m, t.n,
                           keep_slot=True)
    assert res.nnz == W.fem3d_counts(100)[1]
    # the written-out expansion is the generator's element-by-element
    # emission (t.ii, t.jj, t.ss), which the oracle assembled
    assert_whole(res, ref)


def test_uniform_1e7_complex_and_logical(fs):
    # the two other value types at the full random size, every output
    # against the oracle: complex parts bit for bit, logical pattern exact
    t = W.config("uniform_1e7")
    ii, jj = to_dev(t.ii), to_dev(t.jj)
    si = np.random.default_rng(1406).standard_normal(t.L)
    ref = oracle.assemble_complex(t.ii, t.jj, t.ss, si, t.m, t.n)
    res = fs.sparse_complex(ii, jj, to_dev(t.ss), to_dev(si), t.m, t.n)
    np.testing.assert_array_equal(res.jcS.cpu().numpy(), ref.jcS)
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    assert res.prS.cpu().numpy().tobytes() == ref.prS.tobytes()
    assert res.piS.cpu().numpy().tobytes() == ref.piS.tobytes()
    del res, ref
    sl = t.ss > 0.5                              # about 31% true
    ref = oracle.assemble_logical(t.ii, t.jj, sl, t.m, t.n)
    res = fs.sparse_logical(ii, jj, to_dev(sl), t.m, t.n, keep_slot=True)
    assert res.nnz == ref.nnz and 0 < ref.nnz < t.L
    np.testing.assert_array_equal(res.jcS.cpu().numpy(), ref.jcS)
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    np.testing.assert_array_equal(res.slot.cpu().numpy(), ref.slot)
    assert bool(res.prS.all())
