"""Parity at the full workload sizes, in the launch configuration the
benchmark times (default tuning).

At these sizes the whole output is checked through properties that hold at
any size (pattern invariants, exact distinct-pair counts, closed-form nnz),
and a sample of columns is checked bit for bit against the oracle, which
computes exactly those columns (keeping only their triplets keeps their k
order, and a pair's sum only involves its own triplets).
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


def check_sampled(res, t, cols, ss=None):
    ss = t.ss if ss is None else ss
    out, kidx, gslot = oracle.assemble_columns(t.ii, t.jj, ss, t.m, t.n, cols,
                                               full_jcS=res.jcS.cpu().numpy())
    jc = res.jcS.cpu().numpy()
    ir = res.irS.cpu().numpy()
    pr = res.prS.cpu().numpy()
    for c, (rows, vals) in out.items():
        a, b = jc[c], jc[c + 1]
        np.testing.assert_array_equal(ir[a:b], rows)
        assert pr[a:b].tobytes() == vals.tobytes(), "column %d" % c
    if res.slot is not None:
        np.testing.assert_array_equal(res.slot.cpu().numpy()[kidx], gslot)


def sample_cols(n, k, seed):
    rng = np.random.default_rng(seed)
    return sorted(set([0, n - 1] + rng.choice(n, size=k, replace=False).tolist()))


def test_uniform_1e7(fs):
    t = W.config("uniform_1e7")
    ii, jj, ss = to_dev(t.ii), to_dev(t.jj), to_dev(t.ss)
    res = fs.sparse(ii, jj, ss, t.m, t.n, keep_slot=True, plan=True)
    key = (t.jj.astype(np.int64) - 1) * t.m + (t.ii - 1)
    assert res.nnz == np.unique(key).size
    check_invariants(res, ii, jj, t.m, t.n)
    check_sampled(res, t, sample_cols(t.n, 300, 1))
    # re-assembly with new values on the same pattern
    s2 = t.ss * 0.5 - 1.0
    res.prS = fs.reassemble(res, to_dev(s2))
    check_sampled(res, t, sample_cols(t.n, 100, 2), ss=s2)


def test_fem3d_100_and_reuse(fs):
    t = W.config("fem3d_100")
    L, nnz = W.fem3d_counts(100)
    ii, jj, ss = to_dev(t.ii), to_dev(t.jj), to_dev(t.ss)
    res = fs.sparse(ii, jj, ss, t.m, t.n, keep_slot=True, plan=True)
    assert t.L == L and res.nnz == nnz
    check_invariants(res, ii, jj, t.m, t.n)
    check_sampled(res, t, sample_cols(t.n, 200, 3))
    del ii, jj
    for step in range(2):
        s2 = W.element_scale(t, step, seed=1068)
        res.prS = fs.reassemble(res, to_dev(s2))
        check_sampled(res, t, sample_cols(t.n, 60, 10 + step), ss=s2)


def test_batched_64(fs):
    batch = W.config("batched_64")
    ii, jj, ss, m, n = batch.concat()
    res = fs.assemble_batched(to_dev(ii), to_dev(jj), to_dev(ss),
                              batch.trip_off, m, n, keep_slot=True)
    off = batch.trip_off
    sizes = [t.meta["s"] for t in batch.mats]
    for b, t in enumerate(batch.mats):
        assert res.nnz_off[b + 1] - res.nnz_off[b] == W.fem2d_counts(sizes[b])[1]
    order = np.argsort([t.L for t in batch.mats])
    for b in list(order[:3]):                 # smallest matrices: everything
        t = batch.mats[b]
        ref = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
        jc, ir, pr = res.matrix(int(b))
        np.testing.assert_array_equal(jc.cpu().numpy(), ref.jcS)
        np.testing.assert_array_equal(ir.cpu().numpy(), ref.irS)
        assert pr.cpu().numpy().tobytes() == ref.prS.tobytes()
        sl = res.slot[off[b]:off[b + 1]].cpu().numpy() - res.nnz_off[b]
        np.testing.assert_array_equal(sl, ref.slot)
    b = int(order[-1])                         # largest: sampled columns
    t = batch.mats[b]
    jc, ir, pr = res.matrix(b)
    out, _, _ = oracle.assemble_columns(t.ii, t.jj, t.ss, t.m, t.n,
                                        sample_cols(t.n, 100, 4))
    jcn, irn, prn = jc.cpu().numpy(), ir.cpu().numpy(), pr.cpu().numpy()
    for c, (rows, vals) in out.items():
        np.testing.assert_array_equal(irn[jcn[c]:jcn[c + 1]], rows)
        assert prn[jcn[c]:jcn[c + 1]].tobytes() == vals.tobytes()


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


def test_fem3d_100_expanded(fs):
    # index expansion at full size: connectivity and element matrices only
    # (the 93M-triplet index arrays are never formed); sampled columns
    # against the oracle, the whole output through the invariants
    t = W.config("fem3d_100")
    conn = t.meta["conn"]
    ne, nv = conn.shape
    c = to_dev(conn)
    K = to_dev(t.ss).view(ne, nv, nv)
    res = fs.sparse_expand(c[:, :, None], c[:, None, :], K, t.m, t.n,
                           keep_slot=True)
    assert res.nnz == W.fem3d_counts(100)[1]
    check_invariants(res, to_dev(t.ii), to_dev(t.jj), t.m, t.n)
    check_sampled(res, t, sample_cols(t.n, 200, 21))


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
