"""Double-valued indices on the GPU against the oracle.

The kernels read the double index arrays directly and apply the paper's
pre-processing check as they go; the result must equal the oracle's
assembly of the converted indices bit for bit, and every kind of value the
check rejects must give an index error, in every bin mode and also when the
dimensions are defaulted.
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


def check_f64(fs, di, dj, ss, m=None, n=None, **kw):
    ref = oracle.assemble(oracle.indices_from_double(di),
                          oracle.indices_from_double(dj), ss, m, n)
    kw.setdefault("keep_slot", True)
    res = fs.sparse(to_dev(di), to_dev(dj), to_dev(ss), m, n, **kw)
    assert (res.m, res.n) == (ref.m, ref.n)
    assert_same(res, ref)
    return res, ref


@pytest.mark.parametrize("mode", ["auto", "dense", "slot", "claim"])
def test_double_indices_all_modes(fs, mode):
    fs.set_tuning(bin_mode=mode)
    try:
        t = W.uniform(300_000, 4000, 30_000, seed=50)
        check_f64(fs, t.ii.astype(np.float64), t.jj.astype(np.float64), t.ss,
                  t.m, t.n)
        t = W.fem3d(12, 0.15, seed=51)
        res, _ = check_f64(fs, t.ii.astype(np.float64),
                           t.jj.astype(np.float64), t.ss)
        plain = fs.sparse(to_dev(t.ii), to_dev(t.jj), to_dev(t.ss))
        assert plain.prS.cpu().numpy().tobytes() == \
            res.prS.cpu().numpy().tobytes()
    finally:
        fs.set_tuning(reset=True)


def test_float32_and_large_whole_numbers(fs):
    rng = np.random.default_rng(52)
    m = 2**31 - 2                      # the largest dimension the library takes
    di = rng.integers(m - 1000, m + 1, 20_000).astype(np.float64)
    dj = rng.integers(1, 5000, 20_000).astype(np.float32)    # exact in fp32
    check_f64(fs, di, dj, rng.standard_normal(20_000), m, 5000)
    check_f64(fs, di, dj, rng.standard_normal(20_000))       # default dims


BAD = [0.0, -0.0, -2.0, 0.5, 3.25, float("nan"), float("inf"),
       float("-inf"), 2147483648.0, 1e300]


@pytest.mark.parametrize("mode", ["dense", "claim"])
@pytest.mark.parametrize("bad", BAD)
def test_rejected_values(fs, mode, bad):
    fs.set_tuning(bin_mode=mode)
    try:
        rng = np.random.default_rng(53)
        L = 200_000
        di = rng.integers(1, 1000, L).astype(np.float64)
        dj = rng.integers(1, 3000, L).astype(np.float64)
        ss = rng.standard_normal(L)
        pos = int(rng.integers(0, L))
        for which in ("row", "col"):
            a, b = di.copy(), dj.copy()
            (a if which == "row" else b)[pos] = bad
            with pytest.raises(oracle.OracleIndexError):
                oracle.indices_from_double(a if which == "row" else b)
            with pytest.raises(fs.FsparseIndexError):
                fs.sparse(to_dev(a), to_dev(b), to_dev(ss), 1000, 3000)
            with pytest.raises(fs.FsparseIndexError):
                fs.sparse(to_dev(a), to_dev(b), to_dev(ss))   # default dims
        # the library state is clean afterwards
        check_f64(fs, di, dj, ss, 1000, 3000)
    finally:
        fs.set_tuning(reset=True)


def test_int64_out_of_int32_range_is_an_index_error(fs):
    ii = np.array([1, 2, 2**32 + 1], dtype=np.int64)   # would wrap to 1
    jj = np.array([1, 1, 1], dtype=np.int64)
    with pytest.raises(fs.FsparseIndexError):
        fs.sparse(to_dev(ii), to_dev(jj), to_dev(np.ones(3)), 5, 5)
    ok = fs.sparse(to_dev(ii[:2]), to_dev(jj[:2]), to_dev(np.ones(2)))
    assert (ok.m, ok.n, ok.nnz) == (2, 1, 2)


def test_reuse_and_backward_from_double_indices(fs):
    t = W.fem2d(40, 0.2, seed=54)
    di, dj = t.ii.astype(np.float64), t.jj.astype(np.float64)
    res, ref = check_f64(fs, di, dj, t.ss, t.m, t.n, plan=True)
    s2 = W.element_scale(t, 0, seed=5)
    pr2 = fs.reassemble(res, to_dev(s2)).cpu().numpy()[:ref.nnz]
    assert pr2.tobytes() == oracle.assemble(t.ii, t.jj, s2, t.m,
                                            t.n).prS.tobytes()
    g = np.linspace(-2.0, 2.0, ref.nnz)
    gs = fs.backward(res.slot, to_dev(g)).cpu().numpy()
    assert gs.tobytes() == oracle.backward(ref.slot, g).tobytes()
