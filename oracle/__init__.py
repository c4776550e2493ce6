"""CPU oracle for sparse assembly -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it and shares no code with it.

``assemble`` wraps the plain-C definition in ``fsparse_oracle.c`` (serial,
one thread); ``brute`` holds an independent pure-Python dense accumulation
used to pin the C oracle on tiny inputs.  ``backward`` and ``reassemble``
are the definitions of the derivative of the assembled values with respect
to the triplet values and of re-assembly with new values; ``postprocess``
is the paper's serial value pass from a known slot map (a fast re-assembly
check at full sizes); ``expand`` writes
out the triplets of an index-expanded input; ``assemble_complex`` sums
complex values (split real and imaginary arrays) on the same pattern;
``assemble_logical`` stores the pairs that have a true triplet.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsparse_oracle.c")
_LIB = os.path.join(_HERE, "libfsparse_oracle.so")

OK, E_INDEX, E_ARG, E_NOMEM = 0, 1, 2, 3


class OracleIndexError(ValueError):
    """An index below 1, or above m / n when those are given."""


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (serial, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                        "-std=c99", "-shared", "-fPIC", _SRC, "-o", tmp],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64 = ctypes.c_int64
        for name, vt in (("oracle_assemble_f64", np.float64),
                         ("oracle_assemble_f32", np.float32)):
            vp = np.ctypeslib.ndpointer(vt, flags="C_CONTIGUOUS")
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [i32p, i32p, vp, i64, i64, i64, i32p, i32p, vp,
                          ctypes.c_void_p, ctypes.POINTER(i64)]
        lib.oracle_dims.restype = ctypes.c_int
        lib.oracle_dims.argtypes = [i32p, i32p, i64, ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
        for name, vt in (("oracle_postprocess_f64", np.float64),
                         ("oracle_postprocess_f32", np.float32)):
            vp = np.ctypeslib.ndpointer(vt, flags="C_CONTIGUOUS")
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [i32p, vp, i64, i64, vp]
        _lib = lib
    return _lib


@dataclass
class Result:
    jcS: np.ndarray      # int32 [n+1]
    irS: np.ndarray      # int32 [nnz]
    prS: np.ndarray      # value dtype [nnz]
    slot: np.ndarray     # int32 [len]
    m: int
    n: int

    @property
    def nnz(self) -> int:
        return int(self.jcS[-1])


def dims(ii, jj):
    """(m, n) = largest row / column index; raises on an index below 1."""
    lib = _load()
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    jj = np.ascontiguousarray(jj, dtype=np.int32)
    m, n = ctypes.c_int64(), ctypes.c_int64()
    st = lib.oracle_dims(ii, jj, ii.shape[0], ctypes.byref(m),
                         ctypes.byref(n))
    if st == E_INDEX:
        raise OracleIndexError("index below 1")
    if st != OK:
        raise RuntimeError("oracle_dims failed: %d" % st)
    return int(m.value), int(n.value)


def assemble(ii, jj, ss, m: Optional[int] = None, n: Optional[int] = None,
             ) -> Result:
    """S = sparse(ii, jj, ss, m, n) by the plain definition (see the C file)."""
    lib = _load()
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    jj = np.ascontiguousarray(jj, dtype=np.int32)
    ss = np.ascontiguousarray(ss)
    if ss.dtype not in (np.float64, np.float32):
        ss = ss.astype(np.float64)
    L = ii.shape[0]
    assert jj.shape[0] == L and ss.shape[0] == L
    if m is None or n is None:
        dm, dn = dims(ii, jj)
        m = dm if m is None else m
        n = dn if n is None else n
    jcS = np.zeros(n + 1, dtype=np.int32)
    irS = np.zeros(max(L, 1), dtype=np.int32)
    prS = np.zeros(max(L, 1), dtype=ss.dtype)
    slot = np.zeros(max(L, 1), dtype=np.int32)
    nnz = ctypes.c_int64()
    f = (lib.oracle_assemble_f64 if ss.dtype == np.float64
         else lib.oracle_assemble_f32)
    st = f(ii, jj, ss, L, m, n, jcS, irS, prS,
           slot.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nnz))
    if st == E_INDEX:
        raise OracleIndexError("index out of range")
    if st != OK:
        raise RuntimeError("oracle assemble failed: %d" % st)
    k = int(nnz.value)
    return Result(jcS, irS[:k].copy(), prS[:k].copy(), slot[:L].copy(),
                  int(m), int(n))


def reassemble(res: Result, ii, jj, ss) -> np.ndarray:
    """Values of a re-assembly with new ``ss`` on the same index pairs.

    By definition this is a fresh assembly of the same triplets; the pattern
    does not depend on the values, so only prS is returned.
    """
    return assemble(ii, jj, ss, res.m, res.n).prS


def postprocess(slot, ss, nnz: int) -> np.ndarray:
    """Values from a known slot map: the serial post-processing of the
    appendix ("Post-processing: finalize CCS format"), prS[slot[k]] += ss[k]
    for k = 0, 1, ... over a prS that starts at +0.0.  With the slot map of
    an assembly this is the value pass alone, i.e. re-assembly of new
    values on the same pattern (written in C, one thread)."""
    lib = _load()
    slot = np.ascontiguousarray(slot, dtype=np.int32)
    ss = np.ascontiguousarray(ss)
    if ss.dtype not in (np.float64, np.float32):
        ss = ss.astype(np.float64)
    assert slot.shape[0] == ss.shape[0]
    prS = np.zeros(max(int(nnz), 1), dtype=ss.dtype)
    f = (lib.oracle_postprocess_f64 if ss.dtype == np.float64
         else lib.oracle_postprocess_f32)
    st = f(slot, ss, ss.shape[0], int(nnz), prS)
    if st != OK:
        raise ValueError("slot map outside [0, nnz)")
    return prS[:int(nnz)].copy()


def backward(slot, grad_prS) -> np.ndarray:
    """d(prS)/d(ss) applied to an upstream gradient.

    prS[t] = sum over k with slot[k] = t of ss[k] (Section 2.2, eq. (2.3)),
    so d prS[t] / d ss[k] = [slot[k] = t] and grad_ss[k] = grad_prS[slot[k]].
    A triplet with slot -1 belongs to a pair that is not stored (a zero sum
    dropped, or a logical pair without a true triplet): no stored value
    depends on it, so its gradient is 0.
    """
    slot = np.asarray(slot)
    g = np.asarray(grad_prS)
    out = np.zeros(slot.shape[0], dtype=g.dtype)
    kept = slot >= 0
    out[kept] = g[slot[kept]]
    return out


def assemble_columns(ii, jj, ss, m: int, n: int, cols: Sequence[int],
                     full_jcS: Optional[np.ndarray] = None):
    """Exact oracle output for a sample of (zero-based) columns only.

    Keeping only the triplets whose column is sampled keeps their relative
    k order, and the sum for a pair only involves that pair's triplets, so
    the per-column row lists and values are exactly those of the full
    assembly.  Returns {col: (rows, values)} and, if ``full_jcS`` is given,
    the global slot of every kept triplet.
    """
    cols = np.asarray(sorted(set(int(c) for c in cols)), dtype=np.int64)
    jj = np.asarray(jj)
    keep = np.isin(jj - 1, cols)
    kidx = np.nonzero(keep)[0]
    sub = assemble(np.asarray(ii)[keep], jj[keep], np.asarray(ss)[keep], m, n)
    out = {}
    for c in cols:
        a, b = sub.jcS[c], sub.jcS[c + 1]
        out[int(c)] = (sub.irS[a:b].copy(), sub.prS[a:b].copy())
    gslot = None
    if full_jcS is not None:
        cj = jj[keep].astype(np.int64) - 1
        gslot = (np.asarray(full_jcS)[cj].astype(np.int64)
                 + (sub.slot.astype(np.int64) - sub.jcS[cj]))
    return out, kidx, gslot


def append(res: Result, ii, jj, ss, m: Optional[int] = None,
           n: Optional[int] = None) -> Result:
    """Delayed assembly (Section 2.1: input not all available at the first
    call), written out: the stored pairs of ``res`` as triplets in storage
    order, then the new triplets, assembled in one call.  m and n default to
    those of ``res`` grown to the largest new index.
    """
    cols = np.repeat(np.arange(res.n, dtype=np.int64),
                     np.diff(res.jcS.astype(np.int64)))
    ii = np.asarray(ii)
    jj = np.asarray(jj)
    if m is None:
        m = max(res.m, int(ii.max()) if ii.size else 0)
    if n is None:
        n = max(res.n, int(jj.max()) if jj.size else 0)
    return assemble(np.concatenate([res.irS.astype(np.int64) + 1, ii]),
                    np.concatenate([cols + 1, jj]),
                    np.concatenate([res.prS, np.asarray(ss, res.prS.dtype)]),
                    m, n)


def drop_zeros(res: Result) -> Result:
    """Matlab's convention on an assembled result: a sparse matrix stores no
    zeros, so the pairs whose sum is +0 or -0 are removed.  The paper keeps
    them (its nnz counts distinct pairs); this is the option that gives
    Matlab's output.  Kept pairs keep their order; jcS counts the kept pairs
    before each column; a triplet of a removed pair gets slot -1.
    """
    keep = res.prS != 0
    before = np.concatenate([[0], np.cumsum(keep)]).astype(np.int64)
    jcS = before[res.jcS.astype(np.int64)].astype(np.int32)
    newpos = (before[:-1]).astype(np.int32)
    slot = np.where(keep[res.slot], newpos[res.slot], -1).astype(np.int32) \
        if res.slot.size else res.slot.copy()
    return Result(jcS, res.irS[keep].copy(), res.prS[keep].copy(), slot,
                  res.m, res.n)


@dataclass
class ComplexResult:
    jcS: np.ndarray      # int32 [n+1]
    irS: np.ndarray      # int32 [nnz]
    prS: np.ndarray      # real parts [nnz]
    piS: np.ndarray      # imaginary parts [nnz]
    slot: np.ndarray     # int32 [len]
    m: int
    n: int

    @property
    def nnz(self) -> int:
        return int(self.jcS[-1])


def assemble_complex(ii, jj, sr, si, m: Optional[int] = None,
                     n: Optional[int] = None) -> ComplexResult:
    """S = sparse(ii, jj, sr + i*si, m, n) for complex values.

    Matlab's compatibility (Section 1) covers complex matrices, which its
    classic external interface stores as two arrays of real and imaginary
    parts beside one pattern (the paper's sr and prS are the real array).
    The pattern and slot do not depend on the values, so they are those of
    the real assembly; every pair's value is its complex triplets summed in
    increasing k from +0 (Section 2.2, eq. (2.3), with complex addition,
    which rounds the real and imaginary sums separately).
    """
    sr = np.ascontiguousarray(sr)
    if sr.dtype not in (np.float64, np.float32):
        sr = sr.astype(np.float64)
    si = np.ascontiguousarray(si, dtype=sr.dtype)
    assert si.shape == sr.shape
    base = assemble(ii, jj, sr, m, n)
    ct = np.complex128 if sr.dtype == np.float64 else np.complex64
    z = np.empty(sr.shape[0], dtype=ct)
    z.real = sr
    z.imag = si
    acc = np.zeros(base.nnz, dtype=ct)
    # unbuffered: repeated slots are added one after another in k order
    np.add.at(acc, base.slot, z)
    return ComplexResult(base.jcS, base.irS, acc.real.copy(), acc.imag.copy(),
                         base.slot, base.m, base.n)


def drop_zeros_complex(res: ComplexResult) -> ComplexResult:
    """Matlab's no-stored-zeros convention for complex values: a pair is
    removed when both its real and its imaginary sum are zero (either
    sign); otherwise as for real values."""
    keep = (res.prS != 0) | (res.piS != 0)
    before = np.concatenate([[0], np.cumsum(keep)]).astype(np.int64)
    jcS = before[res.jcS.astype(np.int64)].astype(np.int32)
    newpos = (before[:-1]).astype(np.int32)
    slot = np.where(keep[res.slot], newpos[res.slot], -1).astype(np.int32) \
        if res.slot.size else res.slot.copy()
    return ComplexResult(jcS, res.irS[keep].copy(), res.prS[keep].copy(),
                         res.piS[keep].copy(), slot, res.m, res.n)


def assemble_logical(ii, jj, sl, m: Optional[int] = None,
                     n: Optional[int] = None) -> Result:
    """S = sparse(ii, jj, sl, m, n) for logical values.

    A Matlab logical matrix holds only true entries, and adding logical
    values gives true when any of them is true.  So a pair is stored when at
    least one of its triplets is true, and its value is true (1, uint8);
    the dimensions come from the indices as for real values.  Written out:
    the real assembly of the 0/1 indicators (exact counts), then the pairs
    with a zero count removed; every triplet of a removed pair gets slot -1.
    """
    sl = np.asarray(sl).astype(bool)
    r = drop_zeros(assemble(ii, jj, sl.astype(np.float64), m, n))
    return Result(r.jcS, r.irS, np.ones(r.irS.size, dtype=np.uint8), r.slot,
                  r.m, r.n)


def indices_from_double(v) -> np.ndarray:
    """Unit-offset indices held in doubles, checked and converted.

    The pre-processing of Section 2.2 (and its appendix listings) rejects a
    value below 1 or one that differs from its ceiling, then converts; NaN
    fails the second test.  Values beyond int32, which the conversion cannot
    hold, are rejected as well (the reading taken for them and for
    infinities).  Raises OracleIndexError.
    """
    v = np.asarray(v, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        bad = (v < 1.0) | (v != np.ceil(v)) | (v > 2147483647.0)
    if bad.any():
        raise OracleIndexError("index %r at %d is not a whole number >= 1"
                               % (float(v[bad][0]), int(np.argmax(bad))))
    return v.astype(np.int32)


def expand(ii, jj, ss):
    """The triplets of an index-expanded input, written out.

    Section 2.1 mentions an extension of the input syntax in which indices
    are used several times as the shapes of the inputs dictate, without
    detail; the reading taken is broadcasting.  ii, jj and ss (at most 3-D)
    broadcast by numpy's rules to one grid of shape (P, C, R), and triplet
    k = r + R*(c + C*p) is the grid element (p, c, r): row-major order, the
    same as Matlab's column-major order of an R x C x P array.  The expanded
    call is, by definition, the assembly of these flat arrays.
    """
    shape = np.broadcast_shapes(np.shape(ii), np.shape(jj), np.shape(ss))
    if len(shape) > 3:
        raise ValueError("operands of at most 3 dimensions")
    return tuple(np.ascontiguousarray(np.broadcast_to(np.asarray(a), shape))
                 .reshape(-1) for a in (ii, jj, ss))


from . import brute  # noqa: E402  (pure Python, no C)
