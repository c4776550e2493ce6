"""Build step: compile the HIP library for gfx950 in-tree.

``python -m paper_1406_1066_amd.build`` (or ``__graft_entry__.build()``)
always recompiles.  The library is loaded from this folder at import time.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "fsparse.hip")
OUT = os.path.join(HERE, "libfsparse.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # a ticket taken by one lane is not needed at once: no wave-wide atomic
    # rewrite that waits for its result on the spot
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wno-unused-result", "-Wno-unused-value",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [hipcc] + HIPCC_FLAGS + [SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed (%d)" % r.returncode)
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
