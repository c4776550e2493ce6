"""Pins of the CPU oracle against what the paper and the mathematics fix.

These tests never touch the HIP path.  Each pin is chosen so that a
plausible mistake in the oracle (a dropped or reordered term of the fold, a
wrong row/column offset, transposed operands, a wrong pair grouping, a lost
-0.0 / zero-sum entry) fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads as W
from golden.load import load

EX = load("worked_example.txt")


def i32(a):
    return np.asarray(a, dtype=np.int32)


# ---------------------------------------------------------------------------
# worked example printed in the paper (Section 2.1, Section 2.3.4)
# ---------------------------------------------------------------------------
def test_worked_example_unordered_input():
    r = oracle.assemble(i32(EX["example_i"]), i32(EX["example_j"]),
                        EX["example_s"])
    assert (r.m, r.n) == (4, 4)             # implicit size, Section 2.1
    np.testing.assert_array_equal(r.prS, EX["prS"])
    np.testing.assert_array_equal(r.irS, EX["irS"])
    np.testing.assert_array_equal(r.jcS, EX["jcS"])
    np.testing.assert_array_equal(r.slot, EX["example_irank"])
    # JJ[irank[k]] = jj[k] is column sorted and indexed by jcS
    JJ = np.repeat(np.arange(1, 5), np.diff(r.jcS))
    np.testing.assert_array_equal(JJ, EX["example_JJ"])
    np.testing.assert_array_equal(JJ[r.slot], EX["example_j"])


def test_worked_example_sorted_input():
    r = oracle.assemble(i32(EX["sorted_i"]), i32(EX["sorted_j"]),
                        EX["sorted_s"])
    np.testing.assert_array_equal(r.prS, EX["prS"])
    np.testing.assert_array_equal(r.irS, EX["irS"])
    np.testing.assert_array_equal(r.jcS, EX["jcS"])
    np.testing.assert_array_equal(r.slot, EX["sorted_irank"])


def test_worked_example_brute():
    jc, ir, pr, sl = brute.assemble(EX["example_i"], EX["example_j"],
                                    EX["example_s"], 4, 4)
    np.testing.assert_array_equal(pr, EX["prS"])
    np.testing.assert_array_equal(ir, EX["irS"])
    np.testing.assert_array_equal(jc, EX["jcS"])
    np.testing.assert_array_equal(sl, EX["example_irank"])


def test_transposed_operands_differ():
    # swapping rows and columns assembles S^T, which is not S
    r = oracle.assemble(i32(EX["example_j"]), i32(EX["example_i"]),
                        EX["example_s"])
    assert not np.array_equal(r.irS, EX["irS"])


# ---------------------------------------------------------------------------
# brute force on tiny inputs, bit for bit
# ---------------------------------------------------------------------------
def _tiny_case(rng, dtype):
    m = int(rng.integers(1, 13))
    n = int(rng.integers(1, 13))
    L = int(rng.integers(0, 65))
    # heavy duplication: draw from a small sub-range sometimes
    hm = int(rng.integers(1, m + 1))
    hn = int(rng.integers(1, n + 1))
    ii = rng.integers(1, hm + 1, size=L).astype(np.int32)
    jj = rng.integers(1, hn + 1, size=L).astype(np.int32)
    kind = rng.integers(0, 4)
    if kind == 0:
        ss = rng.standard_normal(L)
    elif kind == 1:
        ss = rng.integers(-3, 4, size=L).astype(np.float64)   # cancellations
    elif kind == 2:
        ss = rng.choice([0.0, -0.0, 1e16, -1e16, 1.0, 0.1], size=L)
    else:
        ss = rng.standard_normal(L) * 10.0 ** rng.integers(-8, 9, size=L)
    return ii, jj, ss.astype(dtype), m, n


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_oracle_matches_brute_force(dtype):
    rng = np.random.default_rng(20150101)
    for _ in range(400):
        ii, jj, ss, m, n = _tiny_case(rng, dtype)
        r = oracle.assemble(ii, jj, ss, m, n)
        jc, ir, pr, sl = brute.assemble(ii, jj, ss, m, n)
        np.testing.assert_array_equal(r.jcS, jc)
        np.testing.assert_array_equal(r.irS, ir)
        assert r.prS.dtype == pr.dtype
        assert r.prS.tobytes() == pr.tobytes()      # bit-exact, incl. -0.0
        np.testing.assert_array_equal(r.slot, sl)


# ---------------------------------------------------------------------------
# summation order and zero handling
# ---------------------------------------------------------------------------
def test_fold_is_increasing_k():
    # (0 + 1) + 1e16 rounds to 1e16, then - 1e16 gives 0; any other order
    # that starts from the large terms gives 1
    r = oracle.assemble(i32([2, 2, 2]), i32([1, 1, 1]),
                        np.array([1.0, 1e16, -1e16]), 2, 1)
    assert r.prS.tolist() == [0.0]
    r = oracle.assemble(i32([2, 2, 2]), i32([1, 1, 1]),
                        np.array([1e16, -1e16, 1.0]), 2, 1)
    assert r.prS.tolist() == [1.0]


def test_fold_in_float32():
    # 2^-25 is below half an ulp of 1.0f, so the f32 fold never moves, while
    # rounding the f64 sum to f32 would (8 * 2^-25 = 2^-22 > ulp/2)
    ss = np.array([1.0] + [2.0 ** -25] * 8, dtype=np.float32)
    r = oracle.assemble(i32([1] * 9), i32([1] * 9), ss, 1, 1)
    assert r.prS.dtype == np.float32
    assert r.prS[0] == np.float32(1.0)
    assert np.float32(ss.astype(np.float64).sum()) != np.float32(1.0)


def test_negative_zero_and_cancellation_kept():
    # a pair whose only contribution is -0.0 starts from +0.0 -> +0.0;
    # a pair that cancels exactly keeps its (explicit zero) entry
    r = oracle.assemble(i32([1, 2, 2]), i32([1, 1, 1]),
                        np.array([-0.0, 3.0, -3.0]), 2, 1)
    assert r.nnz == 2
    assert not math.copysign(1.0, r.prS[0]) < 0
    assert r.prS[1] == 0.0


def test_single_pair_serial_sum():
    rng = np.random.default_rng(7)
    ss = rng.standard_normal(1000)
    r = oracle.assemble(i32([5] * 1000), i32([3] * 1000), ss, 9, 4)
    acc = 0.0
    for v in ss:
        acc = acc + v
    assert r.nnz == 1 and r.prS[0] == acc
    assert r.irS.tolist() == [4]
    assert r.jcS.tolist() == [0, 0, 0, 1, 1]


def test_no_duplicates_is_a_permutation():
    rng = np.random.default_rng(3)
    m, n = 50, 40
    keys = rng.permutation(m * n)[:1500]
    ii = (keys % m + 1).astype(np.int32)
    jj = (keys // m + 1).astype(np.int32)
    ss = rng.standard_normal(keys.shape[0])
    r = oracle.assemble(ii, jj, ss, m, n)
    assert r.nnz == keys.shape[0]
    np.testing.assert_array_equal(r.prS[r.slot], ss)


# ---------------------------------------------------------------------------
# dimensions and errors (Section 2.2, appendix pre-processing)
# ---------------------------------------------------------------------------
def test_len_zero():
    r = oracle.assemble(i32([]), i32([]), np.array([]))
    assert (r.m, r.n, r.nnz) == (0, 0, 0) and r.jcS.tolist() == [0]
    r = oracle.assemble(i32([]), i32([]), np.array([]), 2, 3)
    assert r.jcS.tolist() == [0, 0, 0, 0]


def test_given_dims_larger_than_max():
    r = oracle.assemble(i32([1, 2]), i32([2, 2]), np.array([1.0, 2.0]), 5, 4)
    assert r.jcS.tolist() == [0, 0, 2, 2, 2]
    assert r.irS.tolist() == [0, 1]


@pytest.mark.parametrize("ii,jj,m,n", [
    ([0, 1], [1, 1], None, None), ([1, 1], [1, -2], None, None),
    ([3, 1], [1, 1], 2, 2), ([1, 1], [1, 3], 2, 2)])
def test_bad_index_raises(ii, jj, m, n):
    with pytest.raises(oracle.OracleIndexError):
        oracle.assemble(i32(ii), i32(jj), np.ones(2), m, n)


# ---------------------------------------------------------------------------
# library routine and paper generator
# ---------------------------------------------------------------------------
def test_pattern_against_numpy_unique_and_scipy():
    scipy_sparse = pytest.importorskip("scipy.sparse")
    t = W.uniform(20000, 300, 200, seed=5)
    r = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    key = (t.jj.astype(np.int64) - 1) * t.m + (t.ii - 1)
    u, inv = np.unique(key, return_inverse=True)
    np.testing.assert_array_equal(r.irS, u % t.m)
    np.testing.assert_array_equal(r.slot, inv)
    A = scipy_sparse.coo_matrix((t.ss, (t.ii - 1, t.jj - 1)),
                                shape=(t.m, t.n)).tocsc()
    A.sum_duplicates()
    np.testing.assert_array_equal(r.jcS, A.indptr)
    np.testing.assert_array_equal(r.irS, A.indices)
    np.testing.assert_allclose(r.prS, A.data, rtol=1e-12, atol=1e-12)


def test_ransparse_counts_are_exact():
    siz, nzr, rep = 300, 6, 7
    t = W.ransparse(siz, nzr, rep, seed=11)
    assert t.L == siz * nzr * rep
    r = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    assert np.all(r.prS == np.round(r.prS))
    assert r.prS.sum() == t.L
    assert np.all(r.prS % rep == 0)          # every pick is repeated nrep times
    key = (t.jj.astype(np.int64) - 1) * t.m + (t.ii - 1)
    u, cnt = np.unique(key, return_counts=True)
    np.testing.assert_array_equal(r.prS, cnt.astype(np.float64))
    # each row has nnz_row picks, so between 1 and nnz_row entries per row
    per_row = np.bincount(r.irS, minlength=siz)
    assert per_row.min() >= 1 and per_row.max() <= nzr


# ---------------------------------------------------------------------------
# finite-element meshes: closed forms and P1 properties
# ---------------------------------------------------------------------------
def _csc_to_dense_pattern(r):
    P = np.zeros((r.m, r.n), dtype=bool)
    for c in range(r.n):
        P[r.irS[r.jcS[c]:r.jcS[c + 1]], c] = True
    return P


@pytest.mark.parametrize("s", [2, 3, 5, 17])
def test_fem2d_closed_form_and_symmetry(s):
    t = W.fem2d(s, 0.2, seed=s)
    L, nnz = W.fem2d_counts(s)
    assert t.L == L
    r = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    assert r.nnz == nnz
    _check_symmetric(r)


@pytest.mark.parametrize("s", [2, 3, 6])
def test_fem3d_closed_form_and_symmetry(s):
    t = W.fem3d(s, 0.15, seed=s)
    L, nnz = W.fem3d_counts(s)
    assert t.L == L
    r = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    assert r.nnz == nnz
    _check_symmetric(r)
    # 3D interior diagonal collects 24 tetrahedra x 1 = 24 contributions
    cnt = np.bincount(r.slot, minlength=r.nnz)
    assert cnt.max() == (24 if s >= 3 else 6)


def _check_symmetric(r):
    D = np.zeros((r.m, r.n))
    P = np.zeros((r.m, r.n), dtype=bool)
    for c in range(r.n):
        rows = r.irS[r.jcS[c]:r.jcS[c + 1]]
        D[rows, c] = r.prS[r.jcS[c]:r.jcS[c + 1]]
        P[rows, c] = True
    assert np.array_equal(P, P.T)
    # bitwise symmetric: (i,j) and (j,i) get the same terms in the same order
    assert D.tobytes() == np.ascontiguousarray(D.T).tobytes()
    # constants are in the kernel of the Laplacian: row sums vanish
    assert np.abs(D.sum(axis=1)).max() <= 1e-12 * np.abs(D).max()


# ---------------------------------------------------------------------------
# invariants on a larger random input
# ---------------------------------------------------------------------------
def test_invariants_and_sampled_columns():
    t = W.uniform(200000, 3000, 2000, seed=9)
    t.ss = np.round(t.ss * 8)          # small integers: sums are exact
    r = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    jc = r.jcS.astype(np.int64)
    assert jc[0] == 0 and jc[-1] == r.nnz and np.all(np.diff(jc) >= 0)
    for c in range(t.n):
        rows = r.irS[jc[c]:jc[c + 1]]
        assert np.all(np.diff(rows) > 0)
    assert r.irS.min() >= 0 and r.irS.max() < t.m
    assert np.array_equal(np.unique(r.slot), np.arange(r.nnz))
    np.testing.assert_array_equal(r.irS[r.slot], t.ii - 1)
    assert np.all(jc[t.jj - 1] <= r.slot) and np.all(r.slot < jc[t.jj])
    colsum_p = np.add.reduceat(r.prS, jc[:-1][np.diff(jc) > 0])
    colsum_s = np.bincount(t.jj - 1, weights=t.ss, minlength=t.n)
    np.testing.assert_array_equal(colsum_p, colsum_s[np.diff(jc) > 0])
    # sampled columns give exactly the full answer on those columns
    cols = [0, 5, 17, 1999]
    out, kidx, gslot = oracle.assemble_columns(t.ii, t.jj, t.ss, t.m, t.n,
                                               cols, full_jcS=r.jcS)
    for c in cols:
        np.testing.assert_array_equal(out[c][0], r.irS[jc[c]:jc[c + 1]])
        np.testing.assert_array_equal(out[c][1], r.prS[jc[c]:jc[c + 1]])
    np.testing.assert_array_equal(gslot, r.slot[kidx])


# ---------------------------------------------------------------------------
# backward: derivative of the assembled values
# ---------------------------------------------------------------------------
def test_backward_definition_fd_and_scatter():
    torch = pytest.importorskip("torch")
    t = W.fem2d(6, 0.2, seed=4)
    r = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    rng = np.random.default_rng(1)
    w = rng.standard_normal(r.nnz)
    g = oracle.backward(r.slot, w)
    # central finite differences of loss(ss) = sum(w * prS(ss))
    for k in rng.choice(t.L, size=40, replace=False):
        h = 1e-3 * max(1.0, abs(t.ss[k]))
        sp = t.ss.copy(); sp[k] += h
        sm = t.ss.copy(); sm[k] -= h
        lp = float(np.dot(w, oracle.reassemble(r, t.ii, t.jj, sp)))
        lm = float(np.dot(w, oracle.reassemble(r, t.ii, t.jj, sm)))
        assert abs((lp - lm) / (2 * h) - g[k]) <= 1e-8 * max(1.0, abs(g[k]))
    # dense scatter reference gradient through torch autograd (CPU, fp64)
    s = torch.tensor(t.ss, requires_grad=True)
    D = torch.zeros(t.m * t.n, dtype=torch.float64)
    lin = torch.tensor((t.jj.astype(np.int64) - 1) * t.m + (t.ii - 1))
    D = D.index_add(0, lin, s)
    Wd = torch.zeros(t.m * t.n, dtype=torch.float64)
    pos = torch.tensor(np.repeat(np.arange(t.n), np.diff(r.jcS)) * t.m
                       + r.irS)
    Wd[pos] = torch.tensor(w)
    (D * Wd).sum().backward()
    assert s.grad.numpy().tobytes() == g.tobytes()


def test_backward_of_unstored_pairs_is_zero():
    # a triplet whose pair is not stored (slot -1) moves no stored value
    ii = np.array([1, 1, 2, 3], dtype=np.int32)
    jj = np.array([1, 1, 1, 2], dtype=np.int32)
    ss = np.array([1.0, -1.0, 5.0, 2.0])
    r = oracle.drop_zeros(oracle.assemble(ii, jj, ss))
    np.testing.assert_array_equal(r.slot, [-1, -1, 0, 1])
    g = oracle.backward(r.slot, np.array([3.0, 7.0]))
    assert g.tobytes() == np.array([0.0, 0.0, 3.0, 7.0]).tobytes()


@pytest.mark.parametrize("seed", range(3))
def test_backward_with_dropped_pairs_against_autograd(seed):
    # loss = sum(w * kept prS): torch autograd through a scatter into every
    # distinct pair followed by the selection of the kept ones
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(seed)
    L, m, n = 300, 9, 7
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.integers(1, n + 1, L).astype(np.int32)
    ss = rng.integers(-2, 3, L).astype(np.float64)     # many zero sums
    full = oracle.assemble(ii, jj, ss, m, n)
    kept = oracle.drop_zeros(full)
    assert 0 < kept.nnz < full.nnz
    w = rng.standard_normal(kept.nnz)
    s = torch.tensor(ss, requires_grad=True)
    p = torch.zeros(full.nnz, dtype=torch.float64).index_add(
        0, torch.from_numpy(full.slot.astype(np.int64)), s)
    keep = torch.from_numpy(full.prS != 0)
    (torch.from_numpy(w) * p[keep]).sum().backward()
    assert s.grad.numpy().tobytes() == oracle.backward(kept.slot, w).tobytes()


# ---------------------------------------------------------------------------
# post-processing from a slot map (the value pass of the serial code)
# ---------------------------------------------------------------------------
def test_postprocess_worked_example():
    # the printed irank of Section 2.3.4 and the example's values give the
    # printed prS of eq. (2.1)
    pr = oracle.postprocess(i32(EX["example_irank"]), EX["example_s"],
                            len(EX["prS"]))
    np.testing.assert_array_equal(pr, EX["prS"])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("seed", range(6))
def test_postprocess_equals_assembly(dtype, seed):
    # the k loop over a zeroed prS against the sort-and-sweep assembly, for
    # the values of the assembly and for new values on the same pattern;
    # magnitudes from 1e-8 to 1e8 make any other summation order show
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 5000))
    m, n = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.integers(1, n + 1, L).astype(np.int32)
    for _ in range(2):
        ss = (rng.standard_normal(L) * 10.0 ** rng.integers(-8, 9, L)
              ).astype(dtype)
        r = oracle.assemble(ii, jj, ss, m, n)
        assert oracle.postprocess(r.slot, ss, r.nnz).tobytes() == \
            r.prS.tobytes()
        s2 = (ss * dtype(-0.5) + dtype(1.0)).astype(dtype)
        assert oracle.postprocess(r.slot, s2, r.nnz).tobytes() == \
            oracle.reassemble(r, ii, jj, s2).tobytes()


def test_postprocess_rejects_slots_out_of_range():
    with pytest.raises(ValueError):
        oracle.postprocess(np.array([0, 2], dtype=np.int32), np.ones(2), 2)
    with pytest.raises(ValueError):
        oracle.postprocess(np.array([0, -1], dtype=np.int32), np.ones(2), 2)


# ---------------------------------------------------------------------------
# index expansion (Section 2.1 mentions it; the reading is broadcasting)
# ---------------------------------------------------------------------------
def _expand_by_loops(ii, jj, ss):
    """Triplets of a broadcast input, one grid point at a time."""
    ops = [np.asarray(a) for a in (ii, jj, ss)]
    ops = [a.reshape((1,) * (3 - a.ndim) + a.shape) for a in ops]
    P = max(a.shape[0] for a in ops)
    C = max(a.shape[1] for a in ops)
    R = max(a.shape[2] for a in ops)
    out = ([], [], [])
    for p in range(P):
        for c in range(C):
            for r in range(R):          # r varies fastest: k = r + R*(c + C*p)
                for o, a in zip(out, ops):
                    o.append(a[p if a.shape[0] > 1 else 0,
                               c if a.shape[1] > 1 else 0,
                               r if a.shape[2] > 1 else 0])
    return tuple(np.array(o, dtype=a.dtype) for o, a in zip(out, ops))


@pytest.mark.parametrize("seed", range(8))
def test_expand_against_loops_and_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    P, C, R = (int(x) for x in rng.integers(1, 5, size=3))
    shapes = []
    for _ in range(3):
        full = [P, C, R]
        s = [d if rng.random() < 0.6 else 1 for d in full]
        shapes.append(tuple(s[int(rng.integers(0, 3)):]))  # drop leading dims
    ii = rng.integers(1, 5, size=shapes[0]).astype(np.int32)
    jj = rng.integers(1, 4, size=shapes[1]).astype(np.int32)
    ss = rng.integers(-3, 4, size=shapes[2]).astype(np.float64) * 0.5
    try:
        want = _expand_by_loops(ii, jj, ss)
        np.broadcast_shapes(ii.shape, jj.shape, ss.shape)
    except ValueError:
        with pytest.raises(ValueError):
            oracle.expand(ii, jj, ss)
        return
    got = oracle.expand(ii, jj, ss)
    for g, w in zip(got, want):
        assert g.dtype == w.dtype and np.array_equal(g, w)
    r = oracle.assemble(*got, 4, 3)
    jc, ir, pr, sl = brute.assemble(*want, 4, 3)
    assert np.array_equal(r.jcS, jc) and np.array_equal(r.irS, ir)
    assert r.prS.tobytes() == np.asarray(pr).tobytes()
    assert np.array_equal(r.slot, sl)


@pytest.mark.parametrize("dim", [2, 3])
def test_expand_fem_connectivity(dim):
    # connectivity broadcast against itself gives the element-by-element
    # emission of the generators (built with repeat/tile), and unit values
    # count, on the diagonal, the elements around each node
    t = W.fem2d(7, 0.2, seed=4) if dim == 2 else W.fem3d(4, 0.15, seed=4)
    conn = t.meta["conn"]
    ne, nv = conn.shape
    K = t.ss.reshape(ne, nv, nv)
    ii, jj, ss = oracle.expand(conn[:, :, None], conn[:, None, :], K)
    assert np.array_equal(ii, t.ii) and np.array_equal(jj, t.jj)
    assert ss.tobytes() == t.ss.tobytes()
    L, nnz = (W.fem2d_counts if dim == 2 else W.fem3d_counts)(t.meta["s"])
    assert ii.size == L
    one = np.ones((1, 1, 1))
    r = oracle.assemble(*oracle.expand(conn[:, :, None], conn[:, None, :], one),
                        t.m, t.n)
    assert r.nnz == nnz and r.prS.sum() == L
    valence = np.bincount(conn.reshape(-1) - 1, minlength=t.n)
    for c in range(t.n):
        rows = r.irS[r.jcS[c]:r.jcS[c + 1]]
        assert r.prS[r.jcS[c] + np.searchsorted(rows, c)] == valence[c]


def test_expand_shape_errors():
    with pytest.raises(ValueError):
        oracle.expand(np.ones((2, 3), np.int32), np.ones((4,), np.int32),
                      np.ones(1))
    with pytest.raises(ValueError):
        oracle.expand(np.ones((1, 1, 1, 2), np.int32), np.ones(2, np.int32),
                      np.ones(2))


# ---------------------------------------------------------------------------
# double-valued indices (the pre-processing check of Section 2.2)
# ---------------------------------------------------------------------------
def test_indices_from_double_accepts_whole_numbers():
    v = [1.0, 2.0, 7.0, 2147483647.0, 3.0]
    got = oracle.indices_from_double(v)
    assert got.dtype == np.int32
    assert got.tolist() == [1, 2, 7, 2147483647, 3]
    # a float32 array holds the same whole numbers exactly
    f = np.array([1, 5, 16777216], dtype=np.float32)
    assert oracle.indices_from_double(f).tolist() == [1, 5, 16777216]


@pytest.mark.parametrize("bad", [0.0, -0.0, -3.0, 0.999, 1.5, 2.0000000000000004,
                                 float("nan"), float("inf"), float("-inf"),
                                 2147483648.0, 1e300])
def test_indices_from_double_rejects(bad):
    with pytest.raises(oracle.OracleIndexError):
        oracle.indices_from_double([1.0, 2.0, bad, 3.0])


def test_double_indices_assemble_like_integers():
    rng = np.random.default_rng(17)
    ii = rng.integers(1, 50, 3000)
    jj = rng.integers(1, 40, 3000)
    ss = rng.standard_normal(3000)
    a = oracle.assemble(oracle.indices_from_double(ii.astype(np.float64)),
                        oracle.indices_from_double(jj.astype(np.float64)), ss)
    b = oracle.assemble(ii.astype(np.int32), jj.astype(np.int32), ss)
    assert np.array_equal(a.jcS, b.jcS) and np.array_equal(a.irS, b.irS)
    assert a.prS.tobytes() == b.prS.tobytes()


# ---------------------------------------------------------------------------
# dropping zero sums (Matlab stores no zeros)
# ---------------------------------------------------------------------------
def test_drop_zeros_hand_example():
    # (1,1): 1 + -1 = 0 -> dropped; (2,1): -0.0 alone -> dropped;
    # (3,1): 0 + 5 -> kept; (1,2): 2 -> kept; column 3 empty
    ii = i32([1, 2, 3, 1, 1, 3])
    jj = i32([1, 1, 1, 2, 1, 1])
    ss = np.array([1.0, -0.0, 0.0, 2.0, -1.0, 5.0])
    r = oracle.drop_zeros(oracle.assemble(ii, jj, ss, 3, 3))
    assert r.jcS.tolist() == [0, 1, 2, 2]
    assert r.irS.tolist() == [2, 0] and r.prS.tolist() == [5.0, 2.0]
    assert r.slot.tolist() == [-1, -1, 0, 1, -1, 0]


@pytest.mark.parametrize("seed", range(6))
def test_drop_zeros_against_dense_accumulation(seed):
    # small integers cancel often; the dense matrix summed in k order (the
    # brute force) has exactly the kept pairs as its nonzeros, column-major
    rng = np.random.default_rng(400 + seed)
    m, n, L = 6, 5, 120
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.integers(1, n + 1, L).astype(np.int32)
    ss = rng.integers(-2, 3, L).astype(np.float64)
    r = oracle.drop_zeros(oracle.assemble(ii, jj, ss, m, n))
    D = np.zeros((m, n))
    for k in range(L):
        D[ii[k] - 1, jj[k] - 1] += ss[k]
    rows, cols = np.nonzero(D.T)            # column-major order of nonzeros
    assert r.nnz == rows.size
    assert np.array_equal(r.irS, cols) and np.array_equal(r.prS, D.T[rows, cols])
    assert np.array_equal(np.diff(r.jcS), np.count_nonzero(D, axis=0))
    for k in range(L):
        s = r.slot[k]
        if D[ii[k] - 1, jj[k] - 1] == 0:
            assert s == -1
        else:
            assert r.irS[s] == ii[k] - 1 and r.jcS[jj[k] - 1] <= s < r.jcS[jj[k]]


def test_drop_zeros_keeps_everything_without_zero_sums():
    t = W.uniform(5000, 300, 200, seed=3)
    a = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    b = oracle.drop_zeros(a)
    assert np.array_equal(a.jcS, b.jcS) and np.array_equal(a.slot, b.slot)
    assert a.prS.tobytes() == b.prS.tobytes()


# ---------------------------------------------------------------------------
# delayed assembly: continuing from stored sums = one fold over everything
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("seed", range(4))
def test_append_equals_one_assembly(dtype, seed):
    rng = np.random.default_rng(500 + seed)
    L, m, n = 4000, 30, 20
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.integers(1, n + 1, L).astype(np.int32)
    # magnitudes far apart make the fold order visible; -0.0 and exact
    # cancellation check the sign of zero sums
    ss = (rng.standard_normal(L) * 10.0 ** rng.integers(-8, 9, L)).astype(dtype)
    ss[rng.random(L) < 0.05] = -0.0
    ss[:50] = 1e8
    ss[50:100] = -1e8
    cuts = sorted(rng.choice(np.arange(1, L), size=3, replace=False))
    parts = np.split(np.arange(L), cuts)
    r = oracle.assemble(ii[parts[0]], jj[parts[0]], ss[parts[0]], m, n)
    for p in parts[1:]:
        r = oracle.append(r, ii[p], jj[p], ss[p], m, n)
    want = oracle.assemble(ii, jj, ss, m, n)
    assert np.array_equal(r.jcS, want.jcS) and np.array_equal(r.irS, want.irS)
    assert r.prS.tobytes() == want.prS.tobytes()
    # a fold from +0.0 never ends at -0.0
    assert not np.any(np.signbit(want.prS) & (want.prS == 0))


def test_append_grows_dimensions_and_maps_old_pairs():
    a = oracle.assemble(i32([1, 2]), i32([1, 2]), np.array([1.0, 2.0]), 2, 2)
    r = oracle.append(a, i32([5, 1]), i32([1, 3]), np.array([3.0, 4.0]))
    assert (r.m, r.n) == (5, 3)
    assert r.jcS.tolist() == [0, 2, 3, 4]
    assert r.irS.tolist() == [0, 4, 1, 0] and r.prS.tolist() == [1, 3, 2, 4]
    assert r.slot.tolist() == [0, 2, 1, 3]     # old pairs, then new triplets


# ---------------------------------------------------------------------------
# complex values: split real and imaginary arrays on one pattern
# ---------------------------------------------------------------------------
def _dense_complex(ii, jj, sr, si, m, n, f32):
    # Python complex (two doubles) or numpy complex64 scalars, added into a
    # dense table in k order: no slot map, no sorting, no numpy ufunc.at
    ct = np.complex64 if f32 else complex
    D = [[ct(0) for _ in range(n)] for _ in range(m)]
    hit = [[False] * n for _ in range(m)]
    for k in range(len(ii)):
        r, c = int(ii[k]) - 1, int(jj[k]) - 1
        z = ct(complex(float(sr[k]), float(si[k])))
        D[r][c] = ct(D[r][c] + z)
        hit[r][c] = True
    cells = [(r, c) for c in range(n) for r in range(m) if hit[r][c]]
    return cells, [D[r][c] for r, c in cells]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("seed", range(4))
def test_complex_against_dense_brute_force(dtype, seed):
    rng = np.random.default_rng(600 + seed)
    m, n, L = 7, 6, 150
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.integers(1, n + 1, L).astype(np.int32)
    sr = (rng.standard_normal(L) * 10.0 ** rng.integers(-6, 7, L)).astype(dtype)
    si = (rng.standard_normal(L) * 10.0 ** rng.integers(-6, 7, L)).astype(dtype)
    si[rng.random(L) < 0.1] = -0.0
    r = oracle.assemble_complex(ii, jj, sr, si, m, n)
    cells, vals = _dense_complex(ii, jj, sr, si, m, n, dtype == np.float32)
    assert r.nnz == len(cells)
    assert r.irS.tolist() == [c[0] for c in cells]
    assert np.diff(r.jcS).tolist() == [sum(1 for c in cells if c[1] == q)
                                       for q in range(n)]
    assert r.prS.dtype == dtype and r.piS.dtype == dtype
    assert r.prS.tobytes() == np.array([v.real for v in vals], dtype).tobytes()
    assert r.piS.tobytes() == np.array([v.imag for v in vals], dtype).tobytes()


def test_complex_reduces_to_real_parts():
    # with zero imaginary parts the real parts are the real assembly and the
    # imaginary sums are +0; swapping the parts swaps the outputs
    t = W.fem2d(9, 0.2, seed=5)
    z = np.zeros_like(t.ss)
    a = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    c = oracle.assemble_complex(t.ii, t.jj, t.ss, z, t.m, t.n)
    assert np.array_equal(c.jcS, a.jcS) and np.array_equal(c.irS, a.irS)
    assert np.array_equal(c.slot, a.slot)
    assert c.prS.tobytes() == a.prS.tobytes()
    assert c.piS.tobytes() == np.zeros(a.nnz).tobytes()
    d = oracle.assemble_complex(t.ii, t.jj, z, t.ss, t.m, t.n)
    assert d.piS.tobytes() == a.prS.tobytes()
    assert d.prS.tobytes() == np.zeros(a.nnz).tobytes()


def test_complex_times_i():
    # i*(x + iy) = -y + ix: negation is exact, so the sums rotate exactly
    t = W.uniform(3000, 40, 30, seed=8)
    y = np.random.default_rng(9).standard_normal(t.L)
    a = oracle.assemble_complex(t.ii, t.jj, t.ss, y, t.m, t.n)
    b = oracle.assemble_complex(t.ii, t.jj, -y, t.ss, t.m, t.n)
    assert np.array_equal(b.prS, -a.piS) and np.array_equal(b.piS, a.prS)


def test_complex_drop_zeros_hand_example():
    # (1,1): (1+2i) + (-1+0i) = 0+2i -> kept; (2,1): (0-0i) alone -> dropped;
    # (1,2): (3+1i) + (0-1i) = 3+0i -> kept; (2,2): (1+1i) + (-1-1i) -> dropped
    ii = i32([1, 2, 1, 1, 1, 2, 2])
    jj = i32([1, 1, 2, 1, 2, 2, 2])
    sr = np.array([1.0, 0.0, 3.0, -1.0, 0.0, 1.0, -1.0])
    si = np.array([2.0, -0.0, 1.0, 0.0, -1.0, 1.0, -1.0])
    r = oracle.drop_zeros_complex(oracle.assemble_complex(ii, jj, sr, si, 2, 2))
    assert r.jcS.tolist() == [0, 1, 2]
    assert r.irS.tolist() == [0, 0]
    assert r.prS.tolist() == [0.0, 3.0] and r.piS.tolist() == [2.0, 0.0]
    assert r.slot.tolist() == [0, -1, 1, 0, 1, -1, -1]


# ---------------------------------------------------------------------------
# logical values: a pair is stored when any of its triplets is true
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_logical_against_dense_or(seed):
    # a dense boolean table OR-ed in k order, read out column-major; the
    # slots of every triplet of a stored pair point to it, others are -1
    rng = np.random.default_rng(700 + seed)
    m, n, L = 8, 6, 90
    ii = rng.integers(1, m + 1, L).astype(np.int32)
    jj = rng.integers(1, n + 1, L).astype(np.int32)
    sl = rng.random(L) < (0.1 + 0.15 * seed)
    r = oracle.assemble_logical(ii, jj, sl, m, n)
    T = [[False] * n for _ in range(m)]
    for k in range(L):
        T[ii[k] - 1][jj[k] - 1] = T[ii[k] - 1][jj[k] - 1] or bool(sl[k])
    cells = [(a, c) for c in range(n) for a in range(m) if T[a][c]]
    assert r.irS.tolist() == [a for a, _ in cells]
    assert r.jcS.tolist() == [0] + np.cumsum(
        [sum(1 for _, c in cells if c == q) for q in range(n)]).tolist()
    assert r.prS.dtype == np.uint8 and r.prS.tolist() == [1] * len(cells)
    where = {cell: t for t, cell in enumerate(cells)}
    assert r.slot.tolist() == [where.get((ii[k] - 1, jj[k] - 1), -1)
                               for k in range(L)]
    assert (r.m, r.n) == (m, n)


def test_logical_all_true_is_the_real_pattern_and_all_false_is_empty():
    t = W.fem2d(8, 0.2, seed=11)
    a = oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
    b = oracle.assemble_logical(t.ii, t.jj, np.ones(t.L, bool))
    assert np.array_equal(a.jcS, b.jcS) and np.array_equal(a.irS, b.irS)
    assert np.array_equal(a.slot, b.slot) and (b.m, b.n) == (a.m, a.n)
    c = oracle.assemble_logical(t.ii, t.jj, np.zeros(t.L, bool))
    assert c.nnz == 0 and (c.m, c.n) == (a.m, a.n)
    assert np.all(c.slot == -1)


def test_logical_hand_example():
    # (1,1): false, true -> stored; (2,1): false only -> not stored;
    # (1,2): true, true -> stored once
    ii = i32([1, 2, 1, 1, 1])
    jj = i32([1, 1, 2, 1, 2])
    sl = np.array([False, False, True, True, True])
    r = oracle.assemble_logical(ii, jj, sl)
    assert (r.m, r.n) == (2, 2)
    assert r.jcS.tolist() == [0, 1, 2] and r.irS.tolist() == [0, 0]
    assert r.slot.tolist() == [0, -1, 1, 0, 1]


def test_complex_hermitian_elements_assemble_hermitian():
    # symmetric real and antisymmetric imaginary element matrices: (i,j)
    # and (j,i) receive their terms from the same elements in the same
    # order, so the real sums agree bit for bit and the imaginary sums are
    # exact negatives (zero on the diagonal)
    t = W.fem2d(9, 0.2, seed=13)
    ne = t.meta["elements"]
    Wm = np.random.default_rng(14).standard_normal((ne, 3, 3))
    si = (Wm - Wm.transpose(0, 2, 1)).reshape(-1)
    r = oracle.assemble_complex(t.ii, t.jj, t.ss, si, t.m, t.n)
    cols = np.repeat(np.arange(r.n), np.diff(r.jcS))
    where = {(int(i), int(c)): p for p, (i, c) in enumerate(zip(r.irS, cols))}
    for (i, c), p in where.items():
        q = where[(c, i)]
        assert r.prS[p].tobytes() == r.prS[q].tobytes()
        assert r.piS[p] == -r.piS[q]
        if i == c:
            assert r.piS[p] == 0
    assert np.any(r.piS != 0)
