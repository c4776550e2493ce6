"""ctypes view of the C ABI in include/fsparse.h (argument marshalling only).

The shared library is built in-tree by ``paper_1406_1066_amd.build``; if it is
missing this module raises at import time -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

# torch first: it brings its own HIP and HSA runtimes, and the library must
# bind to the ones torch has loaded (loaded the other way round, the
# library's first call reports no device)
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
# FSPARSE_LIBRARY may point at another build of the same ABI
LIB_PATH = os.environ.get("FSPARSE_LIBRARY") or os.path.join(HERE, "libfsparse.so")

F64, F32 = 0, 1
ORDERED, ATOMIC, DROP_ZEROS, NO_SYNC = 0, 1, 2, 4
IDX_I64, IDX_U32, IDX_U64 = 0, 1, 2
OK, E_INDEX, E_ARG, E_CAPACITY, E_PLAN, E_HIP = range(6)


class FsparseInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("nzmax", ctypes.c_int64)]


class FsparseExpand(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int64 * 3), ("ii_shape", ctypes.c_int64 * 3),
                ("jj_shape", ctypes.c_int64 * 3),
                ("ss_shape", ctypes.c_int64 * 3)]


class FsparseTuning(ctypes.Structure):
    _fields_ = [("chunk_cap", ctypes.c_int32), ("stream_block", ctypes.c_int32),
                ("stream_items", ctypes.c_int32),
                ("reuse_block", ctypes.c_int32),
                ("chunk_block", ctypes.c_int32),
                ("bin_mode", ctypes.c_int32),
                ("slot_values", ctypes.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libfsparse.so is not built (expected at %s); run "
        "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)

lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u = ctypes.c_uint
_st = ctypes.c_int


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


fsparse_version = _sig("fsparse_version", ctypes.c_char_p, [])
fsparse_status_string = _sig("fsparse_status_string", ctypes.c_char_p, [_st])
fsparse_workspace_bytes = _sig("fsparse_workspace_bytes", ctypes.c_size_t,
                               [_i64, _i64, _i32, _st])
fsparse_dims = _sig("fsparse_dims", _st,
                    [_vp, _vp, _i64, ctypes.POINTER(_i64),
                     ctypes.POINTER(_i64), _vp, ctypes.c_size_t, _vp])
fsparse_assemble = _sig(
    "fsparse_assemble", _st,
    [_vp, _vp, _vp, _st, _i64, _i64, _i64, _i64, _u, _vp, _i64, _vp, _vp,
     _i64, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp),
     ctypes.POINTER(FsparseInfo), _vp])
fsparse_last_error = _sig("fsparse_last_error", ctypes.c_char_p, [])
fsparse_assemble_noalloc = _sig(
    "fsparse_assemble_noalloc", _st,
    [_vp, _vp, _vp, _st, _i64, _i64, _i64, _i64, _u, _vp, _i64, _vp, _vp,
     _i64, _vp, ctypes.POINTER(FsparseInfo), _vp])
NOALLOC_SCRATCH_BYTES = 64 << 20
fsparse_dims_f64idx = _sig("fsparse_dims_f64idx", _st,
                           [_vp, _vp, _i64, ctypes.POINTER(_i64),
                            ctypes.POINTER(_i64), _vp, ctypes.c_size_t, _vp])
fsparse_assemble_f64idx = _sig(
    "fsparse_assemble_f64idx", _st,
    [_vp, _vp, _vp, _st, _i64, _i64, _i64, _i64, _u, _vp, _i64, _vp, _vp,
     _i64, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp),
     ctypes.POINTER(FsparseInfo), _vp])
fsparse_assemble_complex = _sig(
    "fsparse_assemble_complex", _st,
    [_vp, _vp, _vp, _vp, _st, _i64, _i64, _i64, _i64, _u, _vp, _i64, _vp, _vp,
     _vp, _i64, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp),
     ctypes.POINTER(FsparseInfo), _vp])
fsparse_logical_workspace_bytes = _sig("fsparse_logical_workspace_bytes",
                                       ctypes.c_size_t, [_i64, _i64])
fsparse_assemble_logical = _sig(
    "fsparse_assemble_logical", _st,
    [_vp, _vp, _vp, _i64, _i64, _i64, _i64, _vp, _i64, _vp, _vp, _i64, _vp,
     _vp, ctypes.c_size_t, ctypes.POINTER(FsparseInfo), _vp])
fsparse_append_workspace_bytes = _sig("fsparse_append_workspace_bytes",
                                      ctypes.c_size_t, [_i64, _i64, _i64, _st])
fsparse_assemble_append = _sig(
    "fsparse_assemble_append", _st,
    [_vp, _vp, _vp, _i64, _i64, _vp, _vp, _vp, _i64, _st, _i64, _i64, _u, _vp,
     _i64, _vp, _vp, _i64, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp),
     ctypes.POINTER(FsparseInfo), _vp])
fsparse_assemble_expand = _sig(
    "fsparse_assemble_expand", _st,
    [_vp, _vp, _vp, _st, ctypes.POINTER(FsparseExpand), _i64, _i64, _i64, _u,
     _vp, _i64, _vp, _vp, _i64, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp),
     ctypes.POINTER(FsparseInfo), _vp])
fsparse_assemble_reuse = _sig("fsparse_assemble_reuse", _st,
                              [_vp, _vp, _vp, _u, _vp])
fsparse_backward = _sig("fsparse_backward", _st,
                        [_vp, _i64, _vp, _i64, _st, _vp, _vp])
fsparse_assemble_batched = _sig(
    "fsparse_assemble_batched", _st,
    [_i32, ctypes.POINTER(_i64), _vp, _vp, _vp, _st, ctypes.POINTER(_i64),
     ctypes.POINTER(_i64), _u, _vp, _i64, _vp, _vp, _i64,
     ctypes.POINTER(_i64), _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp),
     ctypes.POINTER(FsparseInfo), _vp])
fsparse_dims_batched = _sig("fsparse_dims_batched", _st,
                            [_i32, ctypes.POINTER(_i64), _vp, _vp,
                             ctypes.POINTER(_i64), ctypes.POINTER(_i64), _vp,
                             ctypes.c_size_t, _vp])
fsparse_plan_destroy = _sig("fsparse_plan_destroy", None, [_vp])
fsparse_plan_query = _sig("fsparse_plan_query", _st,
                          [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                           ctypes.POINTER(_i32)])
fsparse_set_tuning = _sig("fsparse_set_tuning", _st,
                          [ctypes.POINTER(FsparseTuning)])
fsparse_get_tuning = _sig("fsparse_get_tuning", _st,
                          [ctypes.POINTER(FsparseTuning)])
fsparse_timing_enable = _sig("fsparse_timing_enable", _st, [ctypes.c_int])
fsparse_timing_select = _sig("fsparse_timing_select", _st, [ctypes.c_uint32])
fsparse_timing_read = _sig("fsparse_timing_read", ctypes.c_int,
                           [ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(_i64), ctypes.c_int])
fsparse_stage_name = _sig("fsparse_stage_name", ctypes.c_char_p, [ctypes.c_int])
fsparse_stream_copy = _sig("fsparse_stream_copy", _st,
                           [_vp, _vp, ctypes.c_size_t, _vp])
fsparse_assemble_status = _sig("fsparse_assemble_status", _st,
                               [_vp, ctypes.POINTER(FsparseInfo), _vp])
fsparse_indices_i32 = _sig("fsparse_indices_i32", _st,
                           [_vp, _i32, _i64, _vp, _vp])

EXPORTS = [
    "fsparse_version", "fsparse_status_string", "fsparse_last_error",
    "fsparse_workspace_bytes",
    "fsparse_dims", "fsparse_assemble", "fsparse_assemble_noalloc",
    "fsparse_assemble_expand",
    "fsparse_dims_f64idx", "fsparse_assemble_f64idx",
    "fsparse_assemble_complex", "fsparse_logical_workspace_bytes",
    "fsparse_assemble_logical",
    "fsparse_append_workspace_bytes", "fsparse_assemble_append",
    "fsparse_assemble_reuse",
    "fsparse_backward", "fsparse_assemble_batched", "fsparse_dims_batched",
    "fsparse_plan_destroy",
    "fsparse_plan_query", "fsparse_set_tuning", "fsparse_get_tuning",
    "fsparse_timing_enable", "fsparse_timing_read", "fsparse_stage_name",
    "fsparse_timing_select",
    "fsparse_stream_copy", "fsparse_assemble_status", "fsparse_indices_i32",
]
