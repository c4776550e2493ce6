"""Shared helpers of the GPU parity tests (HIP path against the oracle)."""
import numpy as np
import torch

import oracle


def dev():
    return torch.device("cuda", 0)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def run(fs, ii, jj, ss, m=None, n=None, **kw):
    return fs.sparse(to_dev(ii), to_dev(jj), to_dev(ss), m, n, **kw)


def assert_same(res, ref, slot=True):
    """Pattern bit-exact, values bit-exact, slot bit-exact."""
    jc = res.jcS.cpu().numpy()
    np.testing.assert_array_equal(jc, ref.jcS)
    assert res.nnz == ref.nnz
    np.testing.assert_array_equal(res.irS.cpu().numpy(), ref.irS)
    got = res.prS.cpu().numpy()
    assert got.dtype == ref.prS.dtype
    if got.tobytes() != ref.prS.tobytes():
        bad = np.nonzero(got.view(np.uint8).reshape(-1, got.itemsize).any(1)
                         != ref.prS.view(np.uint8).reshape(
                             -1, got.itemsize).any(1))[0]
        diff = np.nonzero(got != ref.prS)[0]
        raise AssertionError("prS differs at %d positions, first %s: %r vs %r"
                             % (diff.size, diff[:5], got[diff[:5]],
                                ref.prS[diff[:5]]))
    if slot and res.slot is not None:
        np.testing.assert_array_equal(res.slot.cpu().numpy(), ref.slot)


def check(fs, ii, jj, ss, m=None, n=None, **kw):
    ref = oracle.assemble(ii, jj, ss, m, n)
    kw.setdefault("keep_slot", True)
    res = run(fs, ii, jj, ss, m, n, **kw)
    assert (res.m, res.n) == (ref.m, ref.n)
    assert_same(res, ref)
    return res, ref
