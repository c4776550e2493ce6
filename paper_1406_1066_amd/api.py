"""Python binding over the C ABI: torch tensors in, torch tensors out.

Argument marshalling only -- the library does every step of the assembly.
All tensors live on the current HIP device; work is queued on torch's current
stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

__all__ = [
    "FsparseError", "FsparseIndexError", "Assembled", "Batched", "Assembler",
    "SparseAssemble", "sparse", "assemble", "reassemble", "backward",
    "assemble_batched", "dims", "workspace_bytes", "set_tuning", "get_tuning",
    "timing", "stream_copy", "to_torch_csc", "version",
]


class FsparseError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = L.fsparse_status_string(status).decode()
        if status == L.E_HIP:
            msg += " [%s]" % L.fsparse_last_error().decode()
        super().__init__("%s: %s (status %d)" % (what, msg, status))


class FsparseIndexError(FsparseError, IndexError):
    pass


def _check(st: int, what: str):
    if st == L.OK:
        return
    if st == L.E_INDEX:
        raise FsparseIndexError(st, what)
    raise FsparseError(st, what)


def version() -> str:
    return L.fsparse_version().decode()


def _dt(dtype) -> int:
    if dtype == torch.float64:
        return L.F64
    if dtype == torch.float32:
        return L.F32
    raise TypeError("values must be float64 or float32, got %s" % dtype)


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream():
    if _raw_stream is not None:
        return ctypes.c_void_p(_raw_stream(torch.cuda.current_device()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    """Device address of a tensor for the library (None when empty).  A host
    tensor is refused here: its address would reach the kernels."""
    if t is None or t.numel() == 0:
        return None
    if not t.is_cuda:
        raise ValueError("the library takes GPU tensors; got one on %s"
                         % t.device)
    return ctypes.c_void_p(t.data_ptr())


def _as_tensor(x) -> torch.Tensor:
    return x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x))


def _is_float_index(x) -> bool:
    return _as_tensor(x).dtype.is_floating_point


_WIDE = {torch.int64: L.IDX_I64}
for _name, _code in (("uint32", L.IDX_U32), ("uint64", L.IDX_U64)):
    if hasattr(torch, _name):
        _WIDE[getattr(torch, _name)] = _code


def _dev_i32(x, device) -> torch.Tensor:
    """Integer indices as contiguous int32 on the device.  Wider types are
    narrowed by the library (fsparse_indices_i32), which turns a value that
    int32 cannot hold into 0, rejected later as an index below 1 (instead of
    wrapping into range); narrower types convert exactly."""
    if (isinstance(x, torch.Tensor) and x.dtype == torch.int32 and
            x.device == device and x.is_contiguous()):
        return x
    t = _as_tensor(x)
    if t.dtype.is_floating_point or t.dtype.is_complex or t.dtype == torch.bool:
        raise TypeError("integer index arrays expected here, got %s" % t.dtype)
    t = t.to(device).contiguous()
    if t.dtype == torch.int32:
        return t
    code = _WIDE.get(t.dtype)
    if code is None:                      # int8, int16, uint8: exact
        return t.to(torch.int32).contiguous()
    out = torch.empty(t.shape, dtype=torch.int32, device=device)
    _check(L.fsparse_indices_i32(_ptr(t), code, t.numel(), _ptr(out),
                                 _stream()), "fsparse_indices_i32")
    return out


def _need(t: Optional[torch.Tensor], name: str, numel: int, dtype=None,
          device=None):
    """A caller-supplied buffer that a call without capacity arguments will
    write or read: it must be a GPU tensor of the given type, contiguous,
    with at least ``numel`` elements (checked before anything is queued)."""
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d"
                         % (name, t.numel(), numel))


def _dev_f64(x, device) -> torch.Tensor:
    """Floating-point indices as contiguous float64 on the device (exact
    for float32 and float16)."""
    t = _as_tensor(x).to(device)
    if t.dtype != torch.float64:
        t = t.to(torch.float64)
    return t.contiguous()


def _device(*ts):
    for t in ts:
        if isinstance(t, torch.Tensor) and t.is_cuda:
            return t.device
    return torch.device("cuda", torch.cuda.current_device())


def workspace_bytes(L_: int, ncols: int, nb: int = 1,
                    dtype=torch.float64) -> int:
    return int(L.fsparse_workspace_bytes(int(L_), int(ncols), int(nb),
                                         _dt(dtype)))


def append_workspace_bytes(nnzA: int, L_: int, ncols: int,
                           dtype=torch.float64) -> int:
    """Workspace of ``sparse_append``: nnzA stored pairs, L_ new triplets."""
    return int(L.fsparse_append_workspace_bytes(int(nnzA), int(L_),
                                                int(ncols), _dt(dtype)))


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def dims(ii: torch.Tensor, jj: torch.Tensor):
    """Default (m, n): the largest row / column index (Section 2.2).
    Floating-point index arrays are checked as the paper's pre-processing
    does (whole numbers >= 1)."""
    dev = _device(ii, jj)
    fn = L.fsparse_dims
    if _is_float_index(ii) or _is_float_index(jj):
        ii, jj, fn = _dev_f64(ii, dev), _dev_f64(jj, dev), L.fsparse_dims_f64idx
    else:
        ii, jj = _dev_i32(ii, dev), _dev_i32(jj, dev)
    if ii.numel() != jj.numel():
        raise ValueError("ii and jj must have the same length")
    ws = _workspace(256, dev)
    m, n = ctypes.c_int64(), ctypes.c_int64()
    _check(fn(_ptr(ii), _ptr(jj), ii.numel(), ctypes.byref(m),
              ctypes.byref(n), _ptr(ws), ws.numel(), _stream()),
           "fsparse_dims")
    return int(m.value), int(n.value)


@dataclass
class Assembled:
    """CCS result; irS/prS are views of length nnz into capacity buffers."""
    jcS: torch.Tensor
    irS: torch.Tensor
    prS: torch.Tensor
    m: int
    n: int
    nnz: int
    nzmax: int
    slot: Optional[torch.Tensor] = None
    plan: Optional["_Plan"] = None
    ws: Optional[torch.Tensor] = field(default=None, repr=False)
    piS: Optional[torch.Tensor] = None     # imaginary sums (complex values)
    # queued with wait=False: nnz is -1 and irS/prS hold the full capacity
    # until wait() reads the status back
    pending: bool = False

    def wait(self) -> "Assembled":
        """Status and nnz of a call made with wait=False (waits for the
        stream); raises like the waiting call would."""
        if not self.pending:
            return self
        info = L.FsparseInfo()
        _check(L.fsparse_assemble_status(_ptr(self.ws), ctypes.byref(info),
                                         _stream()), "fsparse_assemble_status")
        nnz = int(info.nnz)
        self.nnz = nnz
        self.nzmax = max(self.nzmax, nnz)
        self.irS = self.irS[:nnz]
        self.prS = self.prS[:nnz]
        if self.piS is not None:
            self.piS = self.piS[:nnz]
        if self.plan is not None:
            self.plan.nnz = nnz
        self.pending = False
        return self

    def to_dense(self) -> torch.Tensor:
        return to_torch_csc(self.wait()).to_dense()


class _Plan:
    """Owns a fsparse_plan handle and keeps its device buffers alive."""

    def __init__(self, handle: ctypes.c_void_p, keep: Sequence[torch.Tensor],
                 L_: int, nnz: int, dtype):
        self.handle = handle
        self.keep = list(keep)
        self.len = L_
        self.nnz = nnz
        self.dtype = dtype

    def close(self):
        if self.handle is not None and self.handle.value:
            L.fsparse_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sparse(ii, jj, ss: torch.Tensor, m: Optional[int] = None,
           n: Optional[int] = None, nzmax: Optional[int] = None, *,
           atomic: bool = False, keep_slot: bool = False, plan: bool = False,
           cap: Optional[int] = None,
           ws: Optional[torch.Tensor] = None,
           out: Optional[tuple] = None,
           drop_zeros: bool = False, wait: bool = True) -> Assembled:
    """S = sparse(ii, jj, ss, m, n, nzmax) on the GPU.

    ``ii``/``jj`` unit-offset indices: integer arrays (converted to int32 on
    the device of ``ss``) or floating-point arrays as Matlab passes them
    (read as doubles by the kernels, which reject any index that is not a
    whole number >= 1), ``ss`` float64/float32 on the GPU.
    ``m``/``n`` default to the largest index.  ``cap`` is the capacity of
    irS/prS (default len, always enough).  With ``plan=True`` the result
    carries a re-use plan (see ``reassemble``); ``keep_slot`` returns the
    inverse rank slot[k].  ``out = (jcS, irS, prS[, slot])`` supplies
    preallocated output buffers (irS/prS capacity = their length).
    ``drop_zeros`` removes the pairs whose sum is zero, as Matlab stores no
    zeros (the slot of a dropped pair's triplets is -1; no plan then).
    ``wait=False`` queues the call without waiting (FSPARSE_NO_SYNC; m and n
    must be given): the result's nnz is -1 until ``result.wait()``.
    """
    dev = _device(ss, ii, jj)
    ss = ss.contiguous()
    fn = L.fsparse_assemble
    if _is_float_index(ii) or _is_float_index(jj):
        ii, jj = _dev_f64(ii, dev), _dev_f64(jj, dev)
        fn = L.fsparse_assemble_f64idx
    else:
        ii, jj = _dev_i32(ii, dev), _dev_i32(jj, dev)
    Ln = ss.numel()
    if ii.numel() != Ln or jj.numel() != Ln:
        raise ValueError("ii, jj and ss must have the same length")
    if m is None or n is None:
        dm, dn = dims(ii, jj)
        m = dm if m is None else m
        n = dn if n is None else n

    def call(*a):
        return fn(_ptr(ii), _ptr(jj), _ptr(ss), _dt(ss.dtype), Ln, *a)
    return _fresh(call, Ln, int(m), int(n), ss, dev, nzmax, atomic, keep_slot,
                  plan, cap, ws, out, "fsparse_assemble", drop_zeros,
                  wait=wait)


def _fresh(call, Ln, m, n, ss, dev, nzmax, atomic, keep_slot, plan, cap, ws,
           out, name, drop_zeros=False, ws_need=None, wait=True) -> Assembled:
    """Output buffers and the capacity / workspace retry around one fresh
    assembly call ``call(m, n, nzmax, flags, jcS, jcS_cap, irS, prS, cap,
    slot, ws, ws_bytes, plan_out, info, stream)``."""
    if drop_zeros and plan:
        raise ValueError("drop_zeros: the pattern depends on the values, "
                         "so no re-use plan can be made")
    if not wait and drop_zeros:
        raise ValueError("drop_zeros reads the kept count back: it waits")
    flags = (L.ATOMIC if atomic else L.ORDERED) | (
        L.DROP_ZEROS if drop_zeros else 0) | (0 if wait else L.NO_SYNC)
    if ws_need is None:
        ws_need = lambda: workspace_bytes(Ln, n, 1, ss.dtype)  # noqa: E731
    if ws is None:
        ws = _workspace(ws_need(), dev)
    slot = None
    if ws is not None:
        _need(ws, "ws", 0, torch.uint8, dev)
    if out is not None:
        jcS, irS0, prS0 = out[0], out[1], out[2]
        _need(jcS, "jcS", n + 1, torch.int32, dev)
        _need(irS0, "irS", 0, torch.int32, dev)
        _need(prS0, "prS", 0, ss.dtype, dev)
        if len(out) > 3:
            slot = out[3]
            _need(slot, "slot", Ln, torch.int32, dev)
        cap = min(irS0.numel(), prS0.numel())
    else:
        jcS = torch.empty(n + 1, dtype=torch.int32, device=dev)
        irS0 = prS0 = None
        if cap is None:
            cap = max(Ln, 1)
    if slot is None and (keep_slot or atomic):
        slot = torch.empty(max(Ln, 1), dtype=torch.int32, device=dev)
    while True:
        if irS0 is not None:
            irS, prS = irS0, prS0
        else:
            irS = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            prS = torch.empty(max(cap, 1), dtype=ss.dtype, device=dev)
        info = L.FsparseInfo()
        ph = ctypes.c_void_p()
        st = call(
            m, n, int(nzmax) if nzmax is not None else 0,
            flags, _ptr(jcS), jcS.numel(),
            _ptr(irS), _ptr(prS), cap, _ptr(slot), _ptr(ws), ws.numel(),
            ctypes.byref(ph) if plan else None, ctypes.byref(info), _stream())
        if st == L.E_CAPACITY and info.nnz > cap and irS0 is None:
            cap = int(info.nnz)       # retry with the reported size
            continue
        if st == L.E_CAPACITY:
            need = ws_need()
            if ws.numel() < need:     # a given workspace that is too small
                ws = _workspace(need, dev)
                continue
        _check(st, name)
        break
    nnz = int(info.nnz)
    p = None
    if plan:
        p = _Plan(ph, [ws, slot], Ln, nnz, ss.dtype)
    if not wait:
        return Assembled(jcS, irS, prS, m, n, -1, int(info.nzmax),
                         slot[:Ln] if slot is not None else None, p, ws,
                         pending=True)
    return Assembled(jcS, irS[:nnz], prS[:nnz], m, n, nnz, int(info.nzmax),
                     slot[:Ln] if slot is not None else None, p, ws)


assemble = sparse


def sparse_noalloc(ii, jj, ss: torch.Tensor, m: int, n: int,
                   nzmax: Optional[int] = None, *, atomic: bool = False,
                   out: Optional[tuple] = None) -> Assembled:
    """S = sparse(ii, jj, ss, m, n, nzmax) through fsparse_assemble_noalloc,
    which allocates nothing: its workspace is the library's fixed device
    array (64 MiB per GPU), shared by every call on that GPU, so calls must
    not overlap.  ``m``/``n`` must be given and int32 device indices are
    expected.  ``out = (jcS, irS, prS[, slot])`` are the caller's buffers
    (irS/prS of at least len entries, slot of len); without it they are
    allocated here, before the call.  Waits once, like ``sparse``."""
    dev = _device(ss, ii, jj)
    ss = ss.contiguous()
    ii, jj = _dev_i32(ii, dev), _dev_i32(jj, dev)
    Ln = ss.numel()
    if ii.numel() != Ln or jj.numel() != Ln:
        raise ValueError("ii, jj and ss must have the same length")
    m, n = int(m), int(n)
    if m < 0 or n < 0:
        raise ValueError("m and n must be given")
    slot = None
    if out is not None:
        jcS, irS, prS = out[0], out[1], out[2]
        _need(jcS, "jcS", n + 1, torch.int32, dev)
        _need(irS, "irS", Ln, torch.int32, dev)
        _need(prS, "prS", Ln, ss.dtype, dev)
        if len(out) > 3:
            slot = out[3]
            _need(slot, "slot", Ln, torch.int32, dev)
    else:
        jcS = torch.empty(n + 1, dtype=torch.int32, device=dev)
        irS = torch.empty(max(Ln, 1), dtype=torch.int32, device=dev)
        prS = torch.empty(max(Ln, 1), dtype=ss.dtype, device=dev)
    if atomic and slot is None:
        slot = torch.empty(max(Ln, 1), dtype=torch.int32, device=dev)
    cap = min(irS.numel(), prS.numel())
    info = L.FsparseInfo()
    st = L.fsparse_assemble_noalloc(
        _ptr(ii), _ptr(jj), _ptr(ss), _dt(ss.dtype), Ln, m, n,
        int(nzmax) if nzmax is not None else 0,
        L.ATOMIC if atomic else L.ORDERED, _ptr(jcS), jcS.numel(),
        _ptr(irS), _ptr(prS), cap, _ptr(slot), ctypes.byref(info), _stream())
    _check(st, "fsparse_assemble_noalloc")
    nnz = int(info.nnz)
    return Assembled(jcS, irS[:nnz], prS[:nnz], m, n, nnz, int(info.nzmax),
                     slot[:Ln] if slot is not None else None, None, None)


def sparse_complex(ii, jj, sr: torch.Tensor, si: torch.Tensor,
                   m: Optional[int] = None, n: Optional[int] = None,
                   nzmax: Optional[int] = None, *, atomic: bool = False,
                   keep_slot: bool = False, plan: bool = False,
                   cap: Optional[int] = None,
                   ws: Optional[torch.Tensor] = None,
                   drop_zeros: bool = False) -> Assembled:
    """S = sparse(ii, jj, sr + 1i*si, m, n, nzmax) for complex values.

    Real and imaginary parts come as two float64 (or two float32) arrays,
    the split storage of Matlab's external interface; the result carries
    ``prS`` and ``piS`` on one pattern.  Both parts are summed in increasing
    k from +0.  ``drop_zeros`` removes a pair only when both sums are zero.
    A plan re-assembles one part per ``reassemble`` call.  Integer indices.
    """
    dev = _device(sr, ii, jj)
    sr = sr.contiguous()
    si = si.contiguous()
    if si.dtype != sr.dtype or si.shape != sr.shape or si.device != sr.device:
        raise ValueError("sr and si must match in dtype, shape and device")
    if _is_float_index(ii) or _is_float_index(jj):
        raise TypeError("complex values take integer index arrays")
    ii, jj = _dev_i32(ii, dev), _dev_i32(jj, dev)
    Ln = sr.numel()
    if ii.numel() != Ln or jj.numel() != Ln:
        raise ValueError("ii, jj, sr and si must have the same length")
    if m is None or n is None:
        dm, dn = dims(ii, jj)
        m = dm if m is None else m
        n = dn if n is None else n
    held = {}

    def call(m_, n_, nzmax_, flags, jcS, jcS_cap, irS, prS, cap_, *rest):
        pi = held.get("piS")
        if pi is None or pi.numel() < max(cap_, 1):
            pi = held["piS"] = torch.empty(max(cap_, 1), dtype=sr.dtype,
                                           device=dev)
        return L.fsparse_assemble_complex(
            _ptr(ii), _ptr(jj), _ptr(sr), _ptr(si), _dt(sr.dtype), Ln, m_, n_,
            nzmax_, flags, jcS, jcS_cap, irS, prS, _ptr(pi), cap_, *rest)
    res = _fresh(call, Ln, int(m), int(n), sr, dev, nzmax, atomic, keep_slot,
                 plan, cap, ws, None, "fsparse_assemble_complex", drop_zeros)
    res.piS = held["piS"][:res.nnz]
    return res


def logical_workspace_bytes(L_: int, ncols: int) -> int:
    return int(L.fsparse_logical_workspace_bytes(int(L_), int(ncols)))


def sparse_logical(ii, jj, sl: torch.Tensor, m: Optional[int] = None,
                   n: Optional[int] = None, nzmax: Optional[int] = None, *,
                   keep_slot: bool = False, cap: Optional[int] = None,
                   ws: Optional[torch.Tensor] = None) -> Assembled:
    """S = sparse(ii, jj, sl, m, n, nzmax) for logical values.

    ``sl`` is a bool (or uint8, nonzero = true) tensor on the GPU.  Only
    pairs with at least one true triplet are stored, all with value True
    (``prS`` is a bool tensor); the slot of a triplet whose pair holds no
    true value is -1.  Integer indices; m, n default to the largest index.
    """
    dev = _device(sl, ii, jj)
    if sl.dtype not in (torch.bool, torch.uint8):
        raise TypeError("logical values must be a bool or uint8 tensor")
    sl = sl.contiguous()
    if _is_float_index(ii) or _is_float_index(jj):
        raise TypeError("logical values take integer index arrays")
    ii, jj = _dev_i32(ii, dev), _dev_i32(jj, dev)
    Ln = sl.numel()
    if ii.numel() != Ln or jj.numel() != Ln:
        raise ValueError("ii, jj and sl must have the same length")
    if m is None or n is None:
        dm, dn = dims(ii, jj)
        m = dm if m is None else m
        n = dn if n is None else n
    n = int(n)

    def call(m_, n_, nzmax_, flags, jcS, jcS_cap, irS, prS, cap_, slot, ws_,
             ws_bytes, plan_ref, info, stream):
        return L.fsparse_assemble_logical(
            _ptr(ii), _ptr(jj), _ptr(sl), Ln, m_, n_, nzmax_, jcS, jcS_cap,
            irS, prS, cap_, slot, ws_, ws_bytes, info, stream)
    out_type = torch.empty(0, dtype=torch.bool, device=dev)
    return _fresh(call, Ln, int(m), n, out_type, dev, nzmax, False, keep_slot,
                  False, cap, ws, None, "fsparse_assemble_logical",
                  ws_need=lambda: logical_workspace_bytes(Ln, n))


def sparse_append(A: "Assembled", ii, jj, ss: torch.Tensor,
                  m: Optional[int] = None, n: Optional[int] = None, *,
                  atomic: bool = False, keep_slot: bool = False,
                  plan: bool = False, cap: Optional[int] = None,
                  ws: Optional[torch.Tensor] = None,
                  drop_zeros: bool = False) -> Assembled:
    """Delayed assembly: ``A`` with the triplets (ii, jj, ss) added.

    Bit-identical to one ``sparse`` call on A's triplets followed by the new
    ones (Section 2.1's input that arrives over time).  ``m``/``n`` default to
    A's dimensions grown to the largest new index.  With ``keep_slot`` the
    slot array has A.nnz + len entries: where each of A's pairs went, then
    the new triplets' positions.
    """
    dev = _device(ss, ii, jj)
    ss = ss.contiguous()
    if A.prS.dtype != ss.dtype:
        raise TypeError("values must have the matrix's type %s" % A.prS.dtype)
    ii, jj = _dev_i32(ii, dev), _dev_i32(jj, dev)
    Ln = ss.numel()
    if ii.numel() != Ln or jj.numel() != Ln:
        raise ValueError("ii, jj and ss must have the same length")
    A = A.wait() if getattr(A, "pending", False) else A
    nnzA = int(A.nnz)
    _need(A.jcS, "A.jcS", A.n + 1, torch.int32, dev)
    _need(A.irS, "A.irS", nnzA, torch.int32, dev)
    _need(A.prS, "A.prS", nnzA, ss.dtype, dev)
    if m is None or n is None:
        dm, dn = dims(ii, jj)
        m = max(A.m, dm) if m is None else m
        n = max(A.n, dn) if n is None else n
    jcA = A.jcS.contiguous()
    irA = A.irS.contiguous()
    prA = A.prS.contiguous()

    def call(m_, n_, nzmax_, *rest):
        return L.fsparse_assemble_append(
            _ptr(jcA), _ptr(irA), _ptr(prA), nnzA, A.n, _ptr(ii), _ptr(jj),
            _ptr(ss), Ln, _dt(ss.dtype), m_, n_, *rest)

    def need():
        return append_workspace_bytes(nnzA, Ln, n, ss.dtype)
    return _fresh(call, nnzA + Ln, int(m), int(n), ss, dev, None, atomic,
                  keep_slot, plan, cap, ws, None, "fsparse_assemble_append",
                  drop_zeros, need)


def sparse_stream(chunks, m: Optional[int] = None, n: Optional[int] = None,
                  *, dtype=torch.float64, device=None) -> "Assembled":
    """Delayed assembly of a stream of triplet chunks held in host memory.

    ``chunks`` yields ``(ii, jj, ss)`` triplets (numpy arrays or CPU
    tensors; indices unit-offset).  The stream as a whole may be larger than
    the device memory; the assembled matrix must fit.  Each chunk is copied
    to the device from pinned memory on a side stream while the previous
    one is merged into the matrix, then appended (``sparse_append``).  The
    result is bit-identical to one assembly of the concatenated chunks.
    ``m``/``n`` default to the largest indices seen.
    """
    dev = device or torch.device("cuda", torch.cuda.current_device())
    side = torch.cuda.Stream(device=dev)
    cur = torch.cuda.current_stream(dev)

    def stage(ch):
        ii, jj, ss = (_as_tensor(x) for x in ch)
        ss = ss.to(dtype)
        host = [t.contiguous().pin_memory() for t in (ii, jj, ss)]
        with torch.cuda.stream(side):
            d = [t.to(dev, non_blocking=True) for t in host]
            ev = torch.cuda.Event()
            ev.record(side)
        return d, host, ev

    it = iter(chunks)
    nxt = None
    first = next(it, None)
    if first is None:
        e = torch.empty(0, dtype=torch.int32, device=dev)
        return sparse(e, e, torch.empty(0, dtype=dtype, device=dev),
                      m or 0, n or 0)
    pending = stage(first)
    A = None
    while pending is not None:
        (ii, jj, ss), host, ev = pending
        cur.wait_event(ev)
        for t in (ii, jj, ss):
            t.record_stream(cur)
        nxt = next(it, None)
        pending = stage(nxt) if nxt is not None else None
        if A is None:
            A = sparse(ii, jj, ss, m, n)
        else:
            A = sparse_append(A, ii, jj, ss, m, n)
        del host
    return A


def sparse_expand(ii, jj, ss: torch.Tensor, m: Optional[int] = None,
                  n: Optional[int] = None, nzmax: Optional[int] = None, *,
                  atomic: bool = False, keep_slot: bool = False,
                  plan: bool = False, cap: Optional[int] = None,
                  ws: Optional[torch.Tensor] = None,
                  out: Optional[tuple] = None,
                  drop_zeros: bool = False) -> Assembled:
    """Assembly with index expansion: ``ii``, ``jj``, ``ss`` broadcast.

    The three arrays (at most 3-D) broadcast to one grid of shape
    (P, C, R) by the usual right-aligned rules; the triplets are the grid's
    elements in row-major order (triplet k = r + R*(c + C*p)), each taking
    the broadcast ii, jj and ss there.  No expanded index array is formed.
    For finite elements with connectivity ``conn`` (elements x nv) and
    element matrices ``K`` (elements x nv x nv, K[e, a, b] for row node
    conn[e, a] and column node conn[e, b]):
    ``sparse_expand(conn[:, :, None], conn[:, None, :], K)``.
    Slots, plans and re-assembly count all P*C*R triplets.  Other arguments
    as for ``sparse``.
    """
    dev = _device(ss, ii, jj)
    ss = ss.contiguous()
    ii = _dev_i32(ii, dev)
    jj = _dev_i32(jj, dev)
    if max(ii.dim(), jj.dim(), ss.dim()) > 3:
        raise ValueError("operands of at most 3 dimensions")
    grid = torch.broadcast_shapes(ii.shape, jj.shape, ss.shape)
    grid = (1,) * (3 - len(grid)) + tuple(grid)
    x = L.FsparseExpand()
    for d in range(3):
        x.shape[d] = grid[2 - d]
    for name, t in (("ii_shape", ii), ("jj_shape", jj), ("ss_shape", ss)):
        s = (1,) * (3 - t.dim()) + tuple(t.shape)
        dst = getattr(x, name)
        for d in range(3):
            dst[d] = s[2 - d]
    Ln = grid[0] * grid[1] * grid[2]
    if m is None or n is None:
        if Ln == 0:
            dm = dn = 0
        else:
            # every operand entry is used: its largest index is the default
            dm = dims(ii.reshape(-1), ii.reshape(-1))[0]
            dn = dims(jj.reshape(-1), jj.reshape(-1))[1]
        m = dm if m is None else m
        n = dn if n is None else n

    def call(*a):
        return L.fsparse_assemble_expand(_ptr(ii), _ptr(jj), _ptr(ss),
                                         _dt(ss.dtype), ctypes.byref(x), *a)
    return _fresh(call, Ln, int(m), int(n), ss, dev, nzmax, atomic, keep_slot,
                  plan, cap, ws, out, "fsparse_assemble_expand", drop_zeros)


def reassemble(res: Assembled, ss: torch.Tensor,
               out: Optional[torch.Tensor] = None,
               atomic: bool = False) -> torch.Tensor:
    """Values for new ``ss`` on the pattern of ``res`` (needs plan=True)."""
    if res.plan is None:
        raise ValueError("assembled without plan=True")
    if getattr(res, "pending", False):
        res.wait()
    ss = ss.contiguous()
    if ss.numel() != res.plan.len or ss.dtype != res.plan.dtype:
        raise ValueError("ss does not match the plan")
    _need(ss, "ss", res.plan.len, res.plan.dtype)
    if out is None:
        out = torch.empty(max(res.nnz, 1), dtype=ss.dtype, device=ss.device)
    _need(out, "out", res.nnz, res.plan.dtype, ss.device)
    _check(L.fsparse_assemble_reuse(res.plan.handle, _ptr(ss), _ptr(out),
                                    L.ATOMIC if atomic else L.ORDERED,
                                    _stream()), "fsparse_assemble_reuse")
    return out[:res.nnz]


def backward(slot: torch.Tensor, grad_prS: torch.Tensor,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """grad_ss[k] = grad_prS[slot[k]] (derivative of eq. (2.3)); a triplet
    whose pair is not stored (slot -1) gets 0."""
    grad_prS = grad_prS.contiguous()
    slot = slot.contiguous()
    _dt(grad_prS.dtype)
    _need(slot, "slot", 0, torch.int32)
    _need(grad_prS, "grad_prS", 0, grad_prS.dtype, slot.device)
    if out is None:
        out = torch.empty(slot.numel(), dtype=grad_prS.dtype,
                          device=grad_prS.device)
    _need(out, "out", slot.numel(), grad_prS.dtype, slot.device)
    _check(L.fsparse_backward(_ptr(slot), slot.numel(), _ptr(grad_prS),
                              grad_prS.numel(), _dt(grad_prS.dtype), _ptr(out),
                              _stream()), "fsparse_backward")
    return out


class Assembler:
    """Fresh assembly once, then repeated re-assembly of the values.

    The time-stepping use of Section 2.1: the pattern is computed once and
    later calls only redo the ordered sums (one HIP graph launch each).
    """

    def __init__(self, ii, jj, ss: torch.Tensor, m=None, n=None):
        self.result = sparse(ii, jj, ss, m, n, plan=True, keep_slot=True)

    @property
    def jcS(self):
        return self.result.jcS

    @property
    def irS(self):
        return self.result.irS

    @property
    def slot(self):
        return self.result.slot

    def reassemble(self, ss: torch.Tensor, out: Optional[torch.Tensor] = None,
                   atomic: bool = False) -> torch.Tensor:
        """New values on the pattern: a new tensor per call (so earlier
        results stay as they were), or ``out`` when given."""
        return reassemble(self.result, ss, out, atomic)


class SparseAssemble(torch.autograd.Function):
    """prS = assemble(ii, jj, ss) with d prS / d ss through the slot map."""

    @staticmethod
    def forward(ctx, ss, ii, jj, m=None, n=None):
        res = sparse(ii, jj, ss.detach(), m, n, keep_slot=True)
        ctx.save_for_backward(res.slot)
        ctx.nnz = res.nnz
        ctx.mark_non_differentiable(res.jcS, res.irS)
        return res.prS.clone(), res.jcS, res.irS

    @staticmethod
    def backward(ctx, grad_prS, _gj=None, _gi=None):
        (slot,) = ctx.saved_tensors
        if grad_prS is None:
            return None, None, None, None, None
        return backward(slot, grad_prS), None, None, None, None


@dataclass
class Batched:
    jcS: torch.Tensor          # back-to-back per-matrix column pointers
    irS: torch.Tensor
    prS: torch.Tensor
    nnz_off: List[int]
    col_off: List[int]
    m: List[int]
    n: List[int]
    slot: Optional[torch.Tensor] = None
    plan: Optional[_Plan] = None
    ws: Optional[torch.Tensor] = field(default=None, repr=False)

    @property
    def nb(self) -> int:
        return len(self.m)

    def matrix(self, b: int):
        """(jcS, irS, prS) of matrix b (views)."""
        j0 = self.col_off[b] + b
        jc = self.jcS[j0:j0 + self.n[b] + 1]
        a, e = self.nnz_off[b], self.nnz_off[b + 1]
        return jc, self.irS[a:e], self.prS[a:e]

    @property
    def nnz(self) -> int:
        return self.nnz_off[-1]


def assemble_batched(ii, jj, ss: torch.Tensor, trip_off: Sequence[int],
                     m: Sequence[int], n: Sequence[int], *,
                     atomic: bool = False, keep_slot: bool = False,
                     plan: bool = False, cap: Optional[int] = None,
                     ws: Optional[torch.Tensor] = None,
                     out: Optional[tuple] = None) -> Batched:
    """Assemble nb independent matrices with one set of launches.

    ``out = (jcS, irS, prS[, slot])`` supplies preallocated output buffers
    (jcS at least sum(n) + nb entries; irS/prS capacity = their length; slot
    the total number of triplets), so that repeated calls allocate nothing
    for their results."""
    dev = _device(ss, ii, jj)
    ss = ss.contiguous()
    ii = _dev_i32(ii, dev)
    jj = _dev_i32(jj, dev)
    nb = len(m)
    # the library reads the arrays through trip_off and has no lengths of
    # its own to check them against
    tof = np.ascontiguousarray(np.asarray(trip_off, dtype=np.int64))
    ma = np.ascontiguousarray(np.asarray(m, dtype=np.int64))
    na = np.ascontiguousarray(np.asarray(n, dtype=np.int64))
    if na.size != nb or tof.size != nb + 1:
        raise ValueError("trip_off needs nb+1 entries and m, n nb each")
    if tof[0] != 0 or (nb > 0 and bool((tof[1:] < tof[:-1]).any())):
        raise ValueError("trip_off must start at 0 and not decrease")
    if not (int(tof[-1]) == ii.numel() == jj.numel() == ss.numel()):
        raise ValueError("trip_off[-1] must equal the length of ii, jj, ss")
    _need(ss, "ss", ss.numel(), ss.dtype, dev)
    if ws is not None:
        _need(ws, "ws", 0, torch.uint8, dev)
    to = tof.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    mm = ma.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    nn = na.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    if bool((ma < 0).any()) or bool((na < 0).any()):
        dm = (ctypes.c_int64 * nb)()
        dn = (ctypes.c_int64 * nb)()
        w0 = _workspace(workspace_bytes(0, 0, nb, ss.dtype), dev)
        _check(L.fsparse_dims_batched(nb, to, _ptr(ii), _ptr(jj), dm, dn,
                                      _ptr(w0), w0.numel(), _stream()),
               "fsparse_dims_batched")
        for b in range(nb):
            if ma[b] < 0:
                ma[b] = dm[b]
            if na[b] < 0:
                na[b] = dn[b]
    Ln = int(tof[-1])
    N = int(na.sum())
    need = workspace_bytes(Ln, N, nb, ss.dtype)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    slot = None
    if out is not None:
        jcS, irS, prS = out[0], out[1], out[2]
        _need(jcS, "jcS", N + nb, torch.int32, dev)
        _need(irS, "irS", 0, torch.int32, dev)
        _need(prS, "prS", 0, ss.dtype, dev)
        if len(out) > 3:
            slot = out[3]
            _need(slot, "slot", Ln, torch.int32, dev)
        cap = min(irS.numel(), prS.numel())
    else:
        if cap is None:
            cap = max(Ln, 1)
        jcS = torch.empty(N + nb, dtype=torch.int32, device=dev)
        irS = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        prS = torch.empty(max(cap, 1), dtype=ss.dtype, device=dev)
    if slot is None and (keep_slot or plan or atomic):
        slot = torch.empty(max(Ln, 1), dtype=torch.int32, device=dev)
    off = np.zeros(nb + 1, dtype=np.int64)
    ph = ctypes.c_void_p()
    _check(L.fsparse_assemble_batched(
        nb, to, _ptr(ii), _ptr(jj), _ptr(ss), _dt(ss.dtype), mm, nn,
        L.ATOMIC if atomic else L.ORDERED, _ptr(jcS), jcS.numel(), _ptr(irS),
        _ptr(prS), cap, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        _ptr(slot), _ptr(ws), ws.numel(),
        ctypes.byref(ph) if plan else None, None, _stream()),
        "fsparse_assemble_batched")
    nnz_off = off.tolist()
    col_off = [0] + np.cumsum(na).tolist()
    p = _Plan(ph, [ws, slot], Ln, nnz_off[-1], ss.dtype) if plan else None
    return Batched(jcS, irS[:nnz_off[-1]], prS[:nnz_off[-1]], nnz_off,
                   col_off, ma.tolist(), na.tolist(),
                   slot[:Ln] if slot is not None else None, p, ws)


def to_torch_csc(res: Assembled) -> torch.Tensor:
    """The result as a torch sparse CSC tensor (a conversion for the caller,
    after the assembly); complex results carry prS + i*piS."""
    vals = res.prS if res.piS is None else torch.complex(res.prS, res.piS)
    return torch.sparse_csc_tensor(res.jcS.to(torch.int64),
                                   res.irS.to(torch.int64), vals,
                                   size=(res.m, res.n))


BIN_MODES = {"auto": 0, "dense": 1, "slot": 2, "claim": 3}
SLOT_VALUES = {"binned": 1, "by_k": 2}


def set_tuning(chunk_cap: int = 0, stream_block: int = 0,
               stream_items: int = 0, reuse_block: int = 0,
               chunk_block: int = 0, bin_mode=None, slot_values=None,
               reset: bool = False):
    """Launch-shape tuning (process-wide); zero / None keeps a field.

    ``bin_mode``: "auto", "dense", "slot" or "claim"; ``slot_values``:
    "binned" or "by_k", what the fixed-capacity bins hold for a triplet
    besides its row and k (see fsparse.h)."""
    if reset:
        _check(L.fsparse_set_tuning(None), "fsparse_set_tuning")
        return
    if bin_mode is None:
        bm = get_tuning()["bin_mode"]
    else:
        bm = BIN_MODES[bin_mode] if isinstance(bin_mode, str) else int(bin_mode)
    sv = 0
    if slot_values is not None:
        sv = (SLOT_VALUES[slot_values] if isinstance(slot_values, str)
              else int(slot_values))
    t = L.FsparseTuning(chunk_cap, stream_block, stream_items, reuse_block,
                        chunk_block, bm, sv)
    _check(L.fsparse_set_tuning(ctypes.byref(t)), "fsparse_set_tuning")


def get_tuning() -> dict:
    t = L.FsparseTuning()
    _check(L.fsparse_get_tuning(ctypes.byref(t)), "fsparse_get_tuning")
    return {"chunk_cap": t.chunk_cap, "stream_block": t.stream_block,
            "stream_items": t.stream_items, "reuse_block": t.reuse_block,
            "chunk_block": t.chunk_block, "bin_mode": t.bin_mode,
            "slot_values": t.slot_values}


class timing:
    """Context manager: per-stage HIP-event times of the enclosed calls.

    ``stages`` (names) limits the events to those stages' launches; the
    others then run without events in between.
    """

    NSTAGES = 16

    def __init__(self, stages=None):
        self.mask = 0xFFFFFFFF
        if stages is not None:
            names = [L.fsparse_stage_name(s).decode()
                     for s in range(self.NSTAGES)]
            self.mask = 0
            for nm in stages:
                self.mask |= 1 << names.index(nm)

    def __enter__(self):
        L.fsparse_timing_read(None, None, 0)   # drop stale records
        L.fsparse_timing_select(self.mask)
        L.fsparse_timing_enable(1)
        self.ms = {}
        self.launches = {}
        return self

    def read(self) -> dict:
        ms = (ctypes.c_double * self.NSTAGES)()
        cnt = (ctypes.c_int64 * self.NSTAGES)()
        ns = L.fsparse_timing_read(ms, cnt, self.NSTAGES)
        for s in range(min(ns, self.NSTAGES)):
            name = L.fsparse_stage_name(s).decode()
            if cnt[s]:
                self.ms[name] = self.ms.get(name, 0.0) + ms[s]
                self.launches[name] = self.launches.get(name, 0) + cnt[s]
        return self.ms

    def __exit__(self, *exc):
        self.read()
        L.fsparse_timing_enable(0)
        L.fsparse_timing_select(0xFFFFFFFF)
        return False


def stream_copy(src: torch.Tensor, dst: torch.Tensor):
    nbytes = src.numel() * src.element_size()
    _check(L.fsparse_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream()),
           "fsparse_stream_copy")
