"""Seeded sweep: many random inputs and launch settings against the oracle.

Each case draws a size, index ranges, a column distribution (uniform,
power-law skewed, a few heavy columns, sorted runs, a single column), a
share of repeated pairs with signed zeros and cancelling values, the value
type, whether the dimensions are given, and a tuning (LDS capacity, block
sizes, bin mode) that the library accepts.  Every result is compared with
the oracle bit for bit (pattern, values, slots), then re-assembled from its
plan with new values and differentiated.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, to_dev

pytestmark = pytest.mark.gpu

CAPS = [2, 4, 16, 64, 256, 1024, 2048, 4096]
MODES = ["auto", "dense", "slot", "claim"]


@pytest.fixture(scope="module")
def fs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1406_1066_amd as fs
    fs.set_tuning(reset=True)
    yield fs
    fs.set_tuning(reset=True)


def _logint(rng, lo, hi):
    return int(np.exp(rng.uniform(np.log(lo), np.log(hi + 1))))


def draw_case(seed, lmax=400_000):
    rng = np.random.default_rng(seed)
    L = _logint(rng, 1, lmax) if rng.random() > 0.05 else 0
    m = _logint(rng, 1, 2**31 - 2) if rng.random() < 0.2 else \
        _logint(rng, 1, 200_000)
    n = _logint(rng, 1, 150_000)
    kind = rng.choice(["uniform", "skew", "heavy", "sorted", "single"])
    if kind == "uniform":
        jj = rng.integers(1, n + 1, size=L)
    elif kind == "skew":
        jj = (n * rng.random(L) ** 4).astype(np.int64) + 1
    elif kind == "heavy":
        jj = rng.integers(1, n + 1, size=L)
        h = rng.integers(1, n + 1, size=3)
        sel = rng.random(L) < 0.5
        jj[sel] = h[rng.integers(0, 3, size=int(sel.sum()))]
    elif kind == "sorted":
        jj = np.sort(rng.integers(1, n + 1, size=L))
        # a few shuffled windows keep it mostly, not fully, ordered
        for _ in range(3):
            a = int(rng.integers(0, max(1, L)))
            b = min(L, a + 500)
            jj[a:b] = rng.permutation(jj[a:b])
    else:
        jj = np.full(L, int(rng.integers(1, n + 1)))
    if rng.random() < 0.2:
        ii = rng.integers(max(1, m - 60), m + 1, size=L)
    else:
        ii = rng.integers(1, m + 1, size=L)
    # repeated pairs: copies of earlier triplets at random places
    rep = rng.choice([0.0, 0.3, 2.0, 10.0])
    k = int(L * rep)
    if k and L:
        src = rng.integers(0, L, size=k)
        ii = np.concatenate([ii, ii[src]])
        jj = np.concatenate([jj, jj[src]])
        if rng.random() < 0.5:
            p = rng.permutation(len(ii))
            ii, jj = ii[p], jj[p]
    Lt = len(ii)
    dtype = np.float64 if rng.random() < 0.6 else np.float32
    ss = rng.standard_normal(Lt)
    z = rng.random(Lt)
    ss[z < 0.05] = 0.0
    ss[(z >= 0.05) & (z < 0.1)] = -0.0
    ints = (z >= 0.1) & (z < 0.3)
    ss[ints] = rng.integers(-3, 4, size=int(ints.sum()))
    ss = ss.astype(dtype)
    given = rng.random() < 0.6
    mm = m if given else None
    nn = n if given else None
    if given and rng.random() < 0.3:
        mm, nn = m + int(rng.integers(0, 5)), n + int(rng.integers(0, 5))
    tune = dict(chunk_cap=int(rng.choice(CAPS)),
                chunk_block=int(rng.choice([256, 512, 1024])),
                stream_block=int(rng.choice([64, 256, 512, 1024])),
                reuse_block=int(rng.choice([64, 256, 1024])),
                bin_mode=str(rng.choice(MODES)),
                slot_values=str(rng.choice(["binned", "by_k"])))
    desc = ("seed %d L %d m %d n %d kind %s rep %.1f %s given %s %r"
            % (seed, Lt, m, n, kind, rep, np.dtype(dtype).name, given, tune))
    return (ii.astype(np.int32), jj.astype(np.int32), ss, mm, nn, tune, desc)


@pytest.mark.parametrize("seed", range(1000, 1048))
def test_sweep(fs, seed):
    ii, jj, ss, m, n, tune, desc = draw_case(seed)
    fs.set_tuning(**tune)
    try:
        ref = oracle.assemble(ii, jj, ss, m, n)
        res = fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), m, n,
                        keep_slot=True, plan=True)
        try:
            assert (res.m, res.n) == (ref.m, ref.n)
            assert_same(res, ref)
            # re-assembly from the plan with new values
            ss2 = (np.asarray(ss, dtype=np.float64) * -0.5 + 0.125).astype(
                ss.dtype)
            pr2 = fs.reassemble(res, to_dev(ss2)).cpu().numpy()[:ref.nnz]
            assert pr2.tobytes() == oracle.reassemble(ref, ii, jj,
                                                      ss2).tobytes()
            # backward: a gather through the slots
            g = np.arange(ref.nnz, dtype=ss.dtype) * 0.5 - 1.0
            gs = fs.backward(res.slot, to_dev(g)).cpu().numpy()
            assert gs.tobytes() == oracle.backward(ref.slot, g).tobytes()
        except AssertionError as e:
            raise AssertionError("%s: %s" % (desc, e)) from None
    finally:
        fs.set_tuning(reset=True)


@pytest.mark.parametrize("seed", range(2000, 2012))
def test_sweep_batched(fs, seed):
    rng = np.random.default_rng(seed)
    nb = int(rng.integers(1, 13))
    mats = [draw_case(seed * 100 + b, lmax=60_000) for b in range(nb)]
    tune = mats[0][5]
    ii = np.concatenate([c[0] for c in mats])
    jj = np.concatenate([c[1] for c in mats])
    dtype = mats[0][2].dtype
    ss = np.concatenate([c[2].astype(dtype) for c in mats])
    off = np.zeros(nb + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(c[0]) for c in mats])
    ms = [-1 if c[3] is None else c[3] for c in mats]
    ns = [-1 if c[4] is None else c[4] for c in mats]
    desc = "seed %d nb %d L %d %r" % (seed, nb, len(ii), tune)
    fs.set_tuning(**tune)
    try:
        res = fs.assemble_batched(to_dev(ii), to_dev(jj), to_dev(ss), off,
                                  ms, ns, keep_slot=True, plan=True)
        ss2 = (ss.astype(np.float64) * 0.75 - 2.0).astype(dtype)
        pr2 = fs.reassemble(res, to_dev(ss2)).cpu().numpy()
        for b, c in enumerate(mats):
            bi, bj, bs = c[0], c[1], ss[off[b]:off[b + 1]]
            ref = oracle.assemble(bi, bj, bs, c[3], c[4])
            try:
                assert (res.m[b], res.n[b]) == (ref.m, ref.n)
                jc, ir, pr = res.matrix(b)
                np.testing.assert_array_equal(jc.cpu().numpy(), ref.jcS)
                np.testing.assert_array_equal(ir.cpu().numpy(), ref.irS)
                assert pr.cpu().numpy().tobytes() == ref.prS.tobytes()
                sl = (res.slot[off[b]:off[b + 1]].cpu().numpy()
                      - res.nnz_off[b])
                np.testing.assert_array_equal(sl, ref.slot)
                a, e = res.nnz_off[b], res.nnz_off[b + 1]
                want = oracle.reassemble(ref, bi, bj, ss2[off[b]:off[b + 1]])
                assert pr2[a:e].tobytes() == want.tobytes()
            except AssertionError as e:
                raise AssertionError("%s matrix %d (%s): %s"
                                     % (desc, b, c[6], e)) from None
    finally:
        fs.set_tuning(reset=True)
