"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-only entry points (no GPU needed) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsparse.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fsparse_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1406_1066_amd import _lib
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(_lib.lib, name), name
    assert set(_lib.EXPORTS) == set(names)


def test_version_and_status_strings():
    from paper_1406_1066_amd import _lib as L
    assert b"gfx950" in L.fsparse_version()
    assert L.fsparse_status_string(L.OK) == b"ok"
    assert L.fsparse_status_string(L.E_INDEX) == b"index out of range"
    assert L.fsparse_status_string(99) == b"unknown status"


def test_workspace_bytes_host_only():
    from paper_1406_1066_amd import _lib as L
    a = L.fsparse_workspace_bytes(1000, 100, 1, L.F64)
    b = L.fsparse_workspace_bytes(2000, 100, 1, L.F64)
    c = L.fsparse_workspace_bytes(1000, 100, 1, L.F32)
    assert 0 < a < b and c < a
    assert L.fsparse_workspace_bytes(-1, 10, 1, L.F64) == 0
    assert L.fsparse_workspace_bytes(10, 10, 0, L.F64) == 0
    assert L.fsparse_workspace_bytes(10, 10, 1, 7) == 0
    # bucket (16 B/triplet fp64) + long-path scratch + perm/seg/slot
    assert a >= 1000 * (16 + 16 + 4 + 4 + 4)


def test_tuning_validation():
    from paper_1406_1066_amd import _lib as L
    import paper_1406_1066_amd as fs
    fs.set_tuning(reset=True)
    d = fs.get_tuning()
    assert d == {"chunk_cap": 2048, "stream_block": 256, "stream_items": 8,
                 "reuse_block": 512, "chunk_block": 512, "bin_mode": 0,
                 "slot_values": 2}
    fs.set_tuning(chunk_cap=64)
    assert fs.get_tuning()["chunk_cap"] == 64
    fs.set_tuning(slot_values="binned")
    assert fs.get_tuning()["slot_values"] == 1
    fs.set_tuning(chunk_cap=128)          # zero keeps the setting
    assert fs.get_tuning()["slot_values"] == 1
    with pytest.raises(fs.FsparseError):
        fs.set_tuning(chunk_cap=3000)
    with pytest.raises(fs.FsparseError):
        fs.set_tuning(stream_block=100)
    with pytest.raises(fs.FsparseError):
        fs.set_tuning(slot_values=3)
    fs.set_tuning(reset=True)
    assert fs.get_tuning() == d


def test_argument_errors_without_gpu():
    from paper_1406_1066_amd import _lib as L
    info = L.FsparseInfo()
    # NULL jcS / workspace are rejected before any device work
    st = L.fsparse_assemble(None, None, None, L.F64, 0, 3, 3, 0, 0, None, 4,
                            None, None, 0, None, None, 0, None,
                            ctypes.byref(info), None)
    assert st == L.E_ARG
    st = L.fsparse_assemble(None, None, None, 9, 0, 3, 3, 0, 0, None, 4,
                            None, None, 0, None, None, 0, None, None, None)
    assert st == L.E_ARG
    assert L.fsparse_assemble_reuse(None, None, None, 0, None) == L.E_PLAN
    assert L.fsparse_backward(None, -1, None, 0, L.F64, None, None) == L.E_ARG
    assert L.fsparse_plan_query(None, None, None, None) == L.E_PLAN
    L.fsparse_plan_destroy(None)


def test_logical_workspace_bytes_host_only():
    from paper_1406_1066_amd import _lib as L
    for n_, c in ((1000, 100), (12345, 7), (0, 0)):
        w = L.fsparse_logical_workspace_bytes(n_, c)
        base = L.fsparse_workspace_bytes(n_, c, 1, L.F32)
        # the fp32 pipeline's workspace, then indicators and sums
        assert w >= base + 8 * max(n_, 1) and w % 256 == 0
    assert L.fsparse_logical_workspace_bytes(-1, 3) == 0


def test_complex_and_logical_argument_errors_without_gpu():
    from paper_1406_1066_amd import _lib as L
    info = L.FsparseInfo()
    plan = ctypes.c_void_p()
    ws = ctypes.c_void_p(1)          # never dereferenced: rejected before use
    jc = ctypes.c_void_p(1)
    # complex: unknown value type, unknown flag, drop-zeros with a plan,
    # triplets without an imaginary array, NULL jcS
    args = (0, 3, 3, 0)
    assert L.fsparse_assemble_complex(None, None, None, None, 9, *args, 0, jc,
                                      4, None, None, None, 0, None, ws, 1 << 20,
                                      None, ctypes.byref(info), None) == L.E_ARG
    assert L.fsparse_assemble_complex(None, None, None, None, L.F64, *args, 64,
                                      jc, 4, None, None, None, 0, None, ws,
                                      1 << 20, None, None, None) == L.E_ARG
    assert L.fsparse_assemble_complex(None, None, None, None, L.F64, *args,
                                      L.DROP_ZEROS, jc, 4, None, None, None, 0,
                                      None, ws, 1 << 20, ctypes.byref(plan),
                                      None, None) == L.E_ARG
    one = ctypes.c_void_p(1)
    assert L.fsparse_assemble_complex(one, one, one, None, L.F64, 5, 3, 3, 0,
                                      0, jc, 4, None, None, None, 0, None, ws,
                                      1 << 20, None, None, None) == L.E_ARG
    assert L.fsparse_assemble_complex(None, None, None, None, L.F64, *args, 0,
                                      None, 4, None, None, None, 0, None, ws,
                                      1 << 20, None, None, None) == L.E_ARG
    # logical: negative length, triplets without values, NULL workspace
    assert L.fsparse_assemble_logical(None, None, None, -1, 3, 3, 0, jc, 4,
                                      None, None, 0, None, ws, 1 << 20, None,
                                      None) == L.E_ARG
    assert L.fsparse_assemble_logical(one, one, None, 5, 3, 3, 0, jc, 4, None,
                                      None, 0, None, ws, 1 << 20, None,
                                      None) == L.E_ARG
    assert L.fsparse_assemble_logical(None, None, None, 0, 3, 3, 0, jc, 4,
                                      None, None, 0, None, None, 0, None,
                                      None) == L.E_ARG


def test_no_sync_and_narrowing_argument_errors_without_gpu():
    from paper_1406_1066_amd import _lib as L
    jc = ctypes.c_void_p(1)          # never dereferenced: rejected before use
    ws = ctypes.c_void_p(1)
    one = ctypes.c_void_p(1)
    # without a wait the dimensions must be given, and zeros cannot be dropped
    for m, n in ((-1, 3), (3, -1)):
        assert L.fsparse_assemble(one, one, one, L.F64, 5, m, n, 0, L.NO_SYNC,
                                  jc, 4, one, one, 5, None, ws, 1 << 20, None,
                                  None, None) == L.E_ARG
    assert L.fsparse_assemble(one, one, one, L.F64, 5, 3, 3, 0,
                              L.NO_SYNC | L.DROP_ZEROS, jc, 4, one, one, 5,
                              None, ws, 1 << 20, None, None, None) == L.E_ARG
    assert L.fsparse_assemble_f64idx(one, one, one, L.F64, 5, -1, 3, 0,
                                     L.NO_SYNC, jc, 4, one, one, 5, None, ws,
                                     1 << 20, None, None, None) == L.E_ARG
    assert L.fsparse_assemble(one, one, one, L.F64, 5, 3, 3, 0, 8, jc, 4, one,
                              one, 5, None, ws, 1 << 20, None, None,
                              None) == L.E_ARG
    # a batch and an append always wait
    assert L.fsparse_assemble_append(jc, one, one, 1, 3, one, one, one, 1,
                                     L.F64, 3, 3, L.NO_SYNC, jc, 4, one, one,
                                     2, None, ws, 1 << 20, None, None,
                                     None) == L.E_ARG
    to = (ctypes.c_int64 * 2)(0, 1)
    mm = (ctypes.c_int64 * 1)(3)
    assert L.fsparse_assemble_batched(1, to, one, one, one, L.F64, mm, mm,
                                      L.NO_SYNC, jc, 4, one, one, 1, to, None,
                                      ws, 1 << 20, None, None,
                                      None) == L.E_ARG
    assert L.fsparse_assemble_status(None, None, None) == L.E_ARG
    # narrowing: unknown source type, negative length, missing arrays
    assert L.fsparse_indices_i32(one, 7, 4, one, None) == L.E_ARG
    assert L.fsparse_indices_i32(one, L.IDX_I64, -1, one, None) == L.E_ARG
    assert L.fsparse_indices_i32(None, L.IDX_I64, 4, one, None) == L.E_ARG
    assert L.fsparse_indices_i32(None, L.IDX_I64, 0, None, None) == L.OK
    # backward: a negative length is an error, nnz = 0 is not (all zeros)
    assert L.fsparse_backward(one, 0, None, 0, L.F64, one, None) == L.OK


def test_append_workspace_covers_both_paths():
    # the append workspace holds the merge path (the new triplets' own
    # fresh workspace behind B's arrays) and the re-assembly of everything
    from paper_1406_1066_amd import _lib as L
    for nnzA, ln, n in ((0, 0, 0), (10, 0, 5), (0, 1000, 50), (5000, 700, 300),
                        (1 << 20, 1 << 16, 1 << 12)):
        for dt in (L.F64, L.F32):
            a = L.fsparse_append_workspace_bytes(nnzA, ln, n, dt)
            assert a >= L.fsparse_workspace_bytes(nnzA + ln, n, 1, dt)
            assert a >= L.fsparse_workspace_bytes(ln, n, 1, dt) + 4 * (n + 1)
    assert L.fsparse_append_workspace_bytes(-1, 1, 1, L.F64) == 0
    assert L.fsparse_append_workspace_bytes(1, 1, 1, 9) == 0
