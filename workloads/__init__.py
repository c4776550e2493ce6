"""Seeded synthetic triplet workloads for sparse assembly.

This module only *produces inputs* (1-based int32 row/column indices and
fp64/fp32 values).  It holds none of the assembly arithmetic, so both the CPU
oracle (through the tests) and the HIP path can be fed from it without sharing
any of the method.

Workload families
-----------------
* ``ransparse``   -- the paper's benchmark generator (Section 4.1, listing
  "Benchmark data generator", Table 4.1): every row 1..siz receives
  ``nnz_row`` uniformly random columns, the whole set is repeated ``nrep``
  times and randomly permuted, values are all ones.
* ``uniform``     -- independent uniform row/column indices, N(0,1) values.
* ``fem2d``       -- P1 Laplacian stiffness triplets on a jittered structured
  triangle mesh of the unit square (the finite-element assembly the paper's
  introduction motivates the operation with).
* ``fem3d``       -- the same on a jittered Kuhn-split tetrahedral cube mesh.
* ``batched_fem2d`` -- many 2D meshes with log-uniform node counts.

Mesh conventions: nodes are numbered lexicographically with x fastest,
elements are emitted cell by cell (x fastest), and every element emits its
full dense element matrix row-major, so the triplets of one element are
contiguous in k.  Element matrices are K_ab = |T| grad(l_a).grad(l_b), with
the dot product written out term by term so that K_ab and K_ba are bitwise
equal.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Triplets", "ransparse", "uniform", "fem2d", "fem3d", "batched_fem2d",
    "Batch", "element_scale", "fem2d_counts", "fem3d_counts", "config",
    "CONFIG_NAMES",
]


@dataclass
class Triplets:
    """One assembly input: 1-based int32 ``ii``/``jj``, values ``ss``."""
    ii: np.ndarray
    jj: np.ndarray
    ss: np.ndarray
    m: int
    n: int
    name: str = ""
    # triplets emitted per element (FEM inputs), used to scale values per
    # element for time-stepping style re-assembly
    per_elem: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        return int(self.ii.shape[0])

    def astype(self, dtype) -> "Triplets":
        return Triplets(self.ii, self.jj, self.ss.astype(dtype), self.m,
                        self.n, self.name, self.per_elem, dict(self.meta))


# ----------------------------------------------------------------------------
# paper generator
# ----------------------------------------------------------------------------
def ransparse(siz: int, nnz_row: int, nrep: int, seed: int = 0) -> Triplets:
    """Random-structure data of the paper's benchmark (Section 4.1).

    Each row index 1..siz appears ``nnz_row`` times with a uniform random
    column in 1..siz; that list is repeated ``nrep`` times (so every final
    entry collects about ``nrep`` contributions) and the whole is randomly
    permuted.  All values are one, so every assembled value is an exact
    integer count.
    """
    rng = np.random.default_rng(seed)
    rows = np.tile(np.arange(1, siz + 1, dtype=np.int64), nnz_row)
    cols = rng.integers(1, siz + 1, size=siz * nnz_row, dtype=np.int64)
    ii = np.tile(rows, nrep)
    jj = np.tile(cols, nrep)
    p = rng.permutation(ii.shape[0])
    ii = ii[p].astype(np.int32)
    jj = jj[p].astype(np.int32)
    ss = np.ones(ii.shape[0], dtype=np.float64)
    return Triplets(ii, jj, ss, siz, siz, f"ransparse({siz},{nnz_row},{nrep})")


def uniform(L: int, m: int, n: int, seed: int = 0,
            dtype=np.float64) -> Triplets:
    """Independent uniform indices in [1,m] x [1,n], N(0,1) values."""
    rng = np.random.default_rng(seed)
    ii = rng.integers(1, m + 1, size=L, dtype=np.int32)
    jj = rng.integers(1, n + 1, size=L, dtype=np.int32)
    ss = rng.standard_normal(L).astype(dtype)
    return Triplets(ii, jj, ss, m, n, f"uniform(L={L},m={m},n={n})")


# ----------------------------------------------------------------------------
# P1 finite-element meshes
# ----------------------------------------------------------------------------
def fem2d_counts(s: int):
    """(L, nnz) of the 2D mesh with s x s nodes (closed forms)."""
    return 18 * (s - 1) ** 2, s * s + 2 * (s - 1) * (3 * s - 1)


def fem3d_counts(s: int):
    """(L, nnz) of the 3D Kuhn mesh with s^3 nodes (closed forms)."""
    e = 3 * (s - 1) * s * s + 3 * (s - 1) ** 2 * s + (s - 1) ** 3
    return 96 * (s - 1) ** 3, s ** 3 + 2 * e


def _emit(conn: np.ndarray, K: np.ndarray, dtype) -> tuple:
    """Row-major element-matrix emission: (elem, a, b) -> (node_a, node_b)."""
    ne, nv = conn.shape
    ii = np.repeat(conn, nv, axis=1).reshape(-1) + 1
    jj = np.tile(conn, (1, nv)).reshape(-1) + 1
    return (ii.astype(np.int32), jj.astype(np.int32),
            K.reshape(-1).astype(dtype))


def fem2d(s: int, jitter: float = 0.2, seed: int = 0,
          dtype=np.float64) -> Triplets:
    """P1 Laplacian triplets on an s x s node jittered unit-square mesh.

    Each cell (p00,p10,p11,p01) is split along its SW-NE diagonal into the
    triangles (p00,p10,p11) and (p00,p11,p01); 9 triplets per triangle.
    """
    assert s >= 2
    rng = np.random.default_rng(seed)
    h = 1.0 / (s - 1)
    g = np.arange(s, dtype=np.float64) * h
    X = np.empty((s * s, 2))
    X[:, 0] = np.tile(g, s)
    X[:, 1] = np.repeat(g, s)
    X += rng.uniform(-jitter, jitter, size=X.shape) * h

    ci, cj = np.meshgrid(np.arange(s - 1), np.arange(s - 1), indexing="xy")
    ci = ci.reshape(-1).astype(np.int64)
    cj = cj.reshape(-1).astype(np.int64)
    p00 = ci + s * cj
    p10 = p00 + 1
    p01 = p00 + s
    p11 = p01 + 1
    conn = np.empty((2 * p00.shape[0], 3), dtype=np.int64)
    conn[0::2] = np.stack([p00, p10, p11], axis=1)
    conn[1::2] = np.stack([p00, p11, p01], axis=1)

    x = X[conn]                                   # (ne, 3, 2)
    x0, x1, x2 = x[:, 0], x[:, 1], x[:, 2]
    det = ((x1[:, 0] - x0[:, 0]) * (x2[:, 1] - x0[:, 1])
           - (x2[:, 0] - x0[:, 0]) * (x1[:, 1] - x0[:, 1]))
    assert np.all(det > 0), "jitter inverted a triangle"
    area = 0.5 * det
    # gradients of the barycentric coordinates (times 2A), then / 2A
    gx = np.stack([x1[:, 1] - x2[:, 1], x2[:, 1] - x0[:, 1],
                   x0[:, 1] - x1[:, 1]], axis=1) / det[:, None]
    gy = np.stack([x2[:, 0] - x1[:, 0], x0[:, 0] - x2[:, 0],
                   x1[:, 0] - x0[:, 0]], axis=1) / det[:, None]
    K = np.empty((conn.shape[0], 3, 3))
    for a in range(3):
        for b in range(3):
            K[:, a, b] = area * (gx[:, a] * gx[:, b] + gy[:, a] * gy[:, b])
    ii, jj, ss = _emit(conn, K, dtype)
    return Triplets(ii, jj, ss, s * s, s * s, f"fem2d(s={s})", per_elem=9,
                    meta={"s": s, "elements": conn.shape[0],
                          "conn": (conn + 1).astype(np.int32)})


_KUHN = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def fem3d(s: int, jitter: float = 0.15, seed: int = 0,
          dtype=np.float64) -> Triplets:
    """P1 Laplacian triplets on an s^3 node jittered Kuhn tetrahedral mesh.

    Every cube is split into the 6 tetrahedra that walk from its (0,0,0)
    corner to its (1,1,1) corner along the three axes in each order; the
    vertex order is fixed so every tetrahedron is positively oriented.
    16 triplets per tetrahedron.
    """
    assert s >= 2
    rng = np.random.default_rng(seed)
    h = 1.0 / (s - 1)
    g = np.arange(s, dtype=np.float64) * h
    N = s ** 3
    X = np.empty((N, 3))
    X[:, 0] = np.tile(g, s * s)
    X[:, 1] = np.tile(np.repeat(g, s), s)
    X[:, 2] = np.repeat(g, s * s)
    X += rng.uniform(-jitter, jitter, size=X.shape) * h

    c = np.arange((s - 1) ** 3, dtype=np.int64)
    ci = c % (s - 1)
    cj = (c // (s - 1)) % (s - 1)
    ck = c // ((s - 1) ** 2)
    base = ci + s * cj + s * s * ck
    step = np.array([1, s, s * s], dtype=np.int64)
    conn = np.empty((c.shape[0], 6, 4), dtype=np.int64)
    for t, perm in enumerate(_KUHN):
        v1 = base + step[perm[0]]
        v2 = v1 + step[perm[1]]
        v3 = v2 + step[perm[2]]
        # permutation parity decides the orientation of (v0,v1,v2,v3);
        # swap v1/v2 for the odd ones so every element is positive
        odd = t in (1, 2, 5)
        if odd:
            conn[:, t] = np.stack([base, v2, v1, v3], axis=1)
        else:
            conn[:, t] = np.stack([base, v1, v2, v3], axis=1)
    conn = conn.reshape(-1, 4)
    ne = conn.shape[0]

    # process in blocks to bound temporary memory
    K = np.empty((ne, 4, 4))
    blk = 1 << 20
    for lo in range(0, ne, blk):
        hi = min(ne, lo + blk)
        x = X[conn[lo:hi]]                       # (b, 4, 3)
        e1 = x[:, 1] - x[:, 0]
        e2 = x[:, 2] - x[:, 0]
        e3 = x[:, 3] - x[:, 0]
        # cofactors of the edge matrix M (rows e1,e2,e3): inv(M) = adj / det
        c1 = np.cross(e2, e3)
        c2 = np.cross(e3, e1)
        c3 = np.cross(e1, e2)
        det = (e1[:, 0] * c1[:, 0] + e1[:, 1] * c1[:, 1]) + e1[:, 2] * c1[:, 2]
        assert np.all(det > 0), "jitter inverted a tetrahedron"
        vol = det / 6.0
        # grad(l_1..l_3) are the rows c_i / det; grad(l_0) = -sum
        gr = np.empty((hi - lo, 4, 3))
        gr[:, 1] = c1 / det[:, None]
        gr[:, 2] = c2 / det[:, None]
        gr[:, 3] = c3 / det[:, None]
        gr[:, 0] = -((gr[:, 1] + gr[:, 2]) + gr[:, 3])
        for a in range(4):
            for b in range(4):
                K[lo:hi, a, b] = vol * ((gr[:, a, 0] * gr[:, b, 0]
                                         + gr[:, a, 1] * gr[:, b, 1])
                                        + gr[:, a, 2] * gr[:, b, 2])
    ii, jj, ss = _emit(conn, K, dtype)
    return Triplets(ii, jj, ss, N, N, f"fem3d(s={s})", per_elem=16,
                    meta={"s": s, "elements": ne,
                          "conn": (conn + 1).astype(np.int32)})


def element_scale(t: Triplets, step: int, seed: int) -> np.ndarray:
    """New values for a re-assembly step: base values scaled per element.

    One factor U[0.5, 2] per element (``t.per_elem`` consecutive triplets),
    drawn from ``default_rng([seed, step])``.
    """
    rng = np.random.default_rng([seed, step])
    ne = t.L // t.per_elem
    f = rng.uniform(0.5, 2.0, size=ne)
    return (t.ss.reshape(ne, t.per_elem) * f[:, None].astype(t.ss.dtype)
            ).reshape(-1)


# ----------------------------------------------------------------------------
# batched
# ----------------------------------------------------------------------------
@dataclass
class Batch:
    mats: List[Triplets]

    @property
    def nb(self) -> int:
        return len(self.mats)

    @property
    def trip_off(self) -> np.ndarray:
        o = np.zeros(self.nb + 1, dtype=np.int64)
        o[1:] = np.cumsum([t.L for t in self.mats])
        return o

    def concat(self):
        ii = np.concatenate([t.ii for t in self.mats])
        jj = np.concatenate([t.jj for t in self.mats])
        ss = np.concatenate([t.ss for t in self.mats])
        m = np.array([t.m for t in self.mats], dtype=np.int64)
        n = np.array([t.n for t in self.mats], dtype=np.int64)
        return ii, jj, ss, m, n

    @property
    def L(self) -> int:
        return int(sum(t.L for t in self.mats))


def batched_fem2d(nb: int = 64, lo: float = 1e3, hi: float = 1e6,
                  seed: int = 0, jitter: float = 0.2,
                  dtype=np.float64) -> Batch:
    """``nb`` independent 2D meshes, node counts log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    nodes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=nb))
    mats = []
    for b in range(nb):
        s = max(2, int(round(math.sqrt(nodes[b]))))
        mats.append(fem2d(s, jitter, seed=[seed, b], dtype=dtype))
    return Batch(mats)


# ----------------------------------------------------------------------------
# named configurations
# ----------------------------------------------------------------------------
CONFIG_NAMES = {
    "fem2d_100": "2D P1, 100x100 nodes, 19602 triangles x 9 triplets",
    "uniform_1e7": "uniform random, L=1e7, m=n=1e5",
    "fem3d_100": "3D P1 Kuhn, 100^3 nodes, 5821794 tets x 16 triplets",
    "batched_64": "64 x 2D P1 meshes, nodes log-uniform in [1e3,1e6]",
    "fem3d_50": "3D P1 Kuhn, 50^3 nodes, 705894 tets x 16 triplets",
}


def config(name: str, dtype=np.float64):
    """Build a named workload (deterministic seeds)."""
    if name == "fem2d_100":
        return fem2d(100, 0.2, seed=1066, dtype=dtype)
    if name == "uniform_1e7":
        return uniform(10_000_000, 100_000, 100_000, seed=1067, dtype=dtype)
    if name == "fem3d_100":
        return fem3d(100, 0.15, seed=1068, dtype=dtype)
    if name == "batched_64":
        return batched_fem2d(64, 1e3, 1e6, seed=1069, dtype=dtype)
    if name == "fem3d_50":
        return fem3d(50, 0.15, seed=1070, dtype=dtype)
    if name in ("ransparse_d1", "ransparse_d2", "ransparse_d3"):
        siz, nzr, rep = {"ransparse_d1": (10_000, 50, 50),
                         "ransparse_d2": (50_000, 50, 10),
                         "ransparse_d3": (50_000, 10, 50)}[name]
        return ransparse(siz, nzr, rep, seed=1071)
    raise KeyError(name)
