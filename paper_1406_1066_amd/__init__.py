"""MI355X-native Matlab-compatible sparse assembly.

``sparse(ii, jj, ss, m, n, nzmax)`` turns unit-offset triplets into the
compressed-column arrays (jcS, irS, prS) of Engblom & Lukarski, Section 2.1,
summing repeated (i,j) pairs in increasing triplet order.  Every step runs in
the HIP library ``libfsparse.so`` (include/fsparse.h); this package only
marshals torch tensors (device memory and the current stream) into it.
"""
from ._lib import LIB_PATH  # noqa: F401  (raises if the library is not built)
from .api import (  # noqa: F401
    Assembled, Assembler, Batched, FsparseError, FsparseIndexError,
    append_workspace_bytes,
    SparseAssemble, assemble, assemble_batched, backward, dims, get_tuning,
    reassemble, set_tuning, sparse, sparse_append, sparse_complex, sparse_expand,
    sparse_logical, sparse_noalloc, sparse_stream, logical_workspace_bytes,
    stream_copy,
    timing,
    to_torch_csc, version, workspace_bytes,
)
