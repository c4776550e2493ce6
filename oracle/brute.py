"""Dense brute-force assembly for tiny inputs -- TEST INFRASTRUCTURE.

An independent second reading of S = sparse(i,j,s,m,n) (Section 2.1): a dense
m x n table starts at +0.0 everywhere, the triplets are added into it in
increasing k (the order of the paper's serial post-processing), a separate
mask remembers which entries were touched, and the touched entries are read
out column by column, rows increasing.  Pure Python loops, no sorting, no
shared code with the C oracle; only for m*n and len in the hundreds.
"""
from __future__ import annotations

import numpy as np


def assemble(ii, jj, ss, m: int, n: int):
    """Return (jcS, irS, prS, slot) as numpy arrays."""
    f32 = np.asarray(ss).dtype == np.float32
    conv = np.float32 if f32 else float
    D = [[conv(0.0) for _ in range(n)] for _ in range(m)]
    touched = [[False] * n for _ in range(m)]
    for k in range(len(ii)):
        r, c = int(ii[k]) - 1, int(jj[k]) - 1
        if not (0 <= r < m and 0 <= c < n):
            raise IndexError("triplet %d out of range" % k)
        D[r][c] = conv(D[r][c] + conv(ss[k]))
        touched[r][c] = True
    jcS = [0]
    irS, prS = [], []
    where = {}
    for c in range(n):
        for r in range(m):
            if touched[r][c]:
                where[(r, c)] = len(irS)
                irS.append(r)
                prS.append(D[r][c])
        jcS.append(len(irS))
    slot = [where[(int(ii[k]) - 1, int(jj[k]) - 1)] for k in range(len(ii))]
    vt = np.float32 if f32 else np.float64
    return (np.array(jcS, dtype=np.int32), np.array(irS, dtype=np.int32),
            np.array(prS, dtype=vt), np.array(slot, dtype=np.int32))
