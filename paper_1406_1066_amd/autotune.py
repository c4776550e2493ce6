"""Launch-shape autotuner for the assembly kernels.

For a given input it times every candidate tuning (LDS capacity of the
sort/fold workgroups, their thread count, the streaming block size, the
bin-placement mode and the re-assembly block size) on the device, checks
that every candidate produces byte-identical output, applies the fastest,
and caches the choice per device and per *config class* -- the size of the
problem in powers of two of L (triplets), N (columns) and L/N, plus the
value type -- so later problems of the same class reuse it without timing.

Cache file: ``$FSPARSE_TUNE_CACHE`` or ``~/.cache/fsparse_mi355x/tune.json``.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from typing import Dict, Iterable, List, Optional

import torch

from . import api

DEFAULT_SPACE = {
    "chunk_cap": [2048, 4096],
    "chunk_block": [512, 1024],
    "stream_block": [256, 512],
    "bin_mode": ["auto"],
}
REUSE_BLOCKS = [256, 512, 1024]


def cache_path() -> str:
    p = os.environ.get("FSPARSE_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "fsparse_mi355x",
                        "tune.json")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def config_class(L: int, N: int, dtype, nb: int = 1) -> str:
    # the architecture and compute-unit count (the marketing name is not
    # available in every environment, e.g. under a profiler)
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    dev = "%s/%dcu" % (getattr(p, "gcnArchName", "") or p.name,
                       p.multi_processor_count)
    lg = lambda x: int(math.log2(max(1, x)))
    return "%s|%s|L2^%d|N2^%d|LN2^%d|nb%d" % (
        dev, str(dtype).replace("torch.", ""), lg(L), lg(N),
        lg(max(1, L // max(1, N))), 1 if nb == 1 else 2)


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def _candidates(space: Dict[str, List]) -> Iterable[dict]:
    keys = sorted(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        yield dict(zip(keys, vals))


def _digest(res) -> bytes:
    parts = [res.jcS, res.irS, res.prS]
    if getattr(res, "slot", None) is not None:
        parts.append(res.slot)
    return b"".join(p.cpu().numpy().tobytes() for p in parts)


def tune(ii, jj, ss: torch.Tensor, m: int, n: int, *, trip_off=None,
         space: Optional[Dict[str, List]] = None, reps: int = 3,
         use_cache: bool = True, check: bool = True) -> dict:
    """Pick and apply the fastest tuning for this kind of input.

    With ``trip_off`` (and per-matrix ``m``/``n`` sequences) the batched
    entry point is tuned.  Returns the chosen settings and, when measured,
    the per-candidate times in milliseconds.
    """
    batched = trip_off is not None
    L = int(ss.numel())
    N = int(sum(n)) if batched else int(n)
    key = config_class(L, N, ss.dtype, len(m) if batched else 1)
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["best"]
        api.set_tuning(**best)
        return {"key": key, "best": best, "cached": True}

    space = space or DEFAULT_SPACE

    def fresh(keep=False):
        if batched:
            return api.assemble_batched(ii, jj, ss, trip_off, m, n,
                                        keep_slot=keep)
        return api.sparse(ii, jj, ss, m, n, keep_slot=keep)

    times, ref, best, best_t = {}, None, None, float("inf")
    for cand in _candidates(space):
        api.set_tuning(reset=True)
        api.set_tuning(**cand)
        out = fresh(keep=True)
        if check:
            dig = _digest(out)
            if ref is None:
                ref = dig
            elif dig != ref:
                raise AssertionError("candidate %r changed the result" % cand)
        del out
        t = _time(fresh, reps)  # the plain call, as it is used
        times[json.dumps(cand, sort_keys=True)] = t
        if t < best_t:
            best, best_t = cand, t
    # re-assembly block size, with the best fresh tuning
    api.set_tuning(reset=True)
    api.set_tuning(**best)
    res = (api.assemble_batched(ii, jj, ss, trip_off, m, n, plan=True)
           if batched else api.sparse(ii, jj, ss, m, n, plan=True))
    rbest, rbest_t = None, float("inf")
    for rb in REUSE_BLOCKS:
        api.set_tuning(reuse_block=rb)
        # a plan keeps its launch shape: make a fresh plan per block size
        res = (api.assemble_batched(ii, jj, ss, trip_off, m, n, plan=True)
               if batched else api.sparse(ii, jj, ss, m, n, plan=True))
        out = torch.empty(max(res.nnz, 1), dtype=ss.dtype, device=ss.device)
        t = _time(lambda: api.reassemble(res, ss, out=out), reps)
        times["reuse_block=%d" % rb] = t
        if t < rbest_t:
            rbest, rbest_t = rb, t
    best = dict(best, reuse_block=rbest)
    api.set_tuning(reset=True)
    api.set_tuning(**best)
    if use_cache:
        cache = _load()
        cache[key] = {"best": best, "ms": best_t, "times_ms": times}
        _store(cache)
    return {"key": key, "best": best, "cached": False, "times_ms": times}
