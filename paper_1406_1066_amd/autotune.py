"""Launch-shape autotuner for the assembly kernels.

For a given input it times candidate tunings on the device -- the
bin-placement mode (count matrix, fixed-capacity bins, count then place)
together with the LDS capacity of the bin workgroups and their thread count
(which together set how many bin workgroups share a compute unit), then
whether fixed-capacity bins hold the values or the bin stage reads them by
triplet index, then the streaming block size over the best of those, then
the re-assembly block size --
checks that every candidate produces byte-identical output, applies the
fastest, and caches the choice per device and per *config class* -- the
size of the problem in powers of two of L (triplets), N (columns) and L/N,
the value type, single or batched -- so later problems of the same class
reuse it without timing.

Look-up order: the cache file ``$FSPARSE_TUNE_CACHE`` (default
``~/.cache/fsparse_mi355x/tune.json``), then the table of choices measured
on MI355X that ships beside this module (``tune_table.json``; set
``FSPARSE_TUNE_TABLE=0`` to ignore it), else a measurement.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from typing import Dict, Iterable, List, Optional

import torch

from . import api

# searched in this order, each stage over the best of the stages before.
# The bin capacity and the bin workgroup's thread count are searched
# together: together they set how many bin workgroups share a compute unit
# (LDS and registers), which a search of one with the other fixed misses.
STAGES = [
    {"bin_mode": ["auto", "dense", "slot", "claim"],
     "chunk_cap": [1024, 2048, 4096],
     "chunk_block": [256, 512, 1024]},
    {"slot_values": ["binned", "by_k"]},
    {"stream_block": [256, 512]},
]
START = {"chunk_cap": 2048, "chunk_block": 512, "stream_block": 256,
         "bin_mode": "auto", "slot_values": "by_k"}
REUSE_BLOCKS = [256, 512, 1024]
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                     "tune_table.json")


def cache_path() -> str:
    p = os.environ.get("FSPARSE_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "fsparse_mi355x",
                        "tune.json")


def _load(path: Optional[str] = None) -> dict:
    try:
        with open(path or cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _table() -> dict:
    if os.environ.get("FSPARSE_TUNE_TABLE", "1") == "0":
        return {}
    return _load(TABLE)


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


def _digest(res) -> list:
    """The result's arrays (device copies), compared bit for bit."""
    parts = [res.jcS, res.irS, res.prS]
    if getattr(res, "slot", None) is not None:
        parts.append(res.slot)
    return [p.clone() for p in parts]


def _same(a: list, b: list) -> bool:
    return len(a) == len(b) and all(
        x.shape == y.shape and x.dtype == y.dtype and
        torch.equal(x.view(torch.uint8) if x.dtype.is_floating_point else x,
                    y.view(torch.uint8) if y.dtype.is_floating_point else y)
        for x, y in zip(a, b))


def _effective(c: dict) -> tuple:
    """The launch a candidate gives: the bin workgroup uses at least
    chunk_cap/8 and at most chunk_cap threads (so e.g. 4096/256 runs as
    4096/512)."""
    cap = c["chunk_cap"]
    nt = max(cap // 8, min(c["chunk_block"], cap))
    return (c["bin_mode"], cap, nt, c["stream_block"], c["slot_values"])


def tune(ii, jj, ss: torch.Tensor, m: int, n: int, *, trip_off=None,
         stages: Optional[List[Dict[str, List]]] = None, reps: int = 3,
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
    if use_cache:
        for src, d in (("cache", _load()), ("table", _table())):
            if key in d:
                best = d[key]["best"]
                api.set_tuning(reset=True)
                api.set_tuning(**best)
                return {"key": key, "best": best, "cached": True,
                        "source": src}

    stages = stages or STAGES

    def fresh(keep=False):
        if batched:
            return api.assemble_batched(ii, jj, ss, trip_off, m, n,
                                        keep_slot=keep)
        return api.sparse(ii, jj, ss, m, n, keep_slot=keep)

    times, ref, best_t = {}, None, float("inf")
    best = dict(START)
    seen = {}
    for space in stages:
        base = dict(best)
        for vals in _candidates(space):
            cand = dict(base, **vals)
            eff = _effective(cand)
            if eff in seen:            # the same launch as one already timed
                continue
            api.set_tuning(reset=True)
            api.set_tuning(**cand)
            try:
                out = fresh(keep=True)
            except api.FsparseError as err:
                # a shape the device cannot launch is not a candidate
                seen[eff] = float("inf")
                times[json.dumps(cand, sort_keys=True)] = str(err)
                continue
            if check:
                if ref is None:
                    ref = _digest(out)
                elif not _same(_digest(out), ref):
                    raise AssertionError("candidate %r changed the result"
                                         % cand)
            del out
            t = _time(fresh, reps)  # the plain call, as it is used
            seen[eff] = t
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


def write_table(names: Iterable[str], path: str = TABLE) -> dict:
    """Measure the named workloads (fp64, and fp32 where listed as
    ``name:f32``) and write their choices as the shipped table."""
    import numpy as np
    import workloads as W
    os.environ["FSPARSE_TUNE_TABLE"] = "0"
    dev = torch.device("cuda", torch.cuda.current_device())
    table = {}
    for spec in names:
        # workloads of one config class share an entry: the first listed
        # keeps it
        name, _, dts = spec.partition(":")
        dt = np.float32 if dts == "f32" else np.float64
        t = W.config(name, dtype=dt)
        if isinstance(t, W.Batch):
            ii, jj, ss, m, n = t.concat()
            d = [torch.from_numpy(a).to(dev) for a in (ii, jj, ss)]
            r = tune(*d, list(m), list(n), trip_off=t.trip_off,
                     use_cache=False)
            L, N, nb = t.L, int(n.sum()), t.nb
        else:
            d = [torch.from_numpy(a).to(dev) for a in (t.ii, t.jj, t.ss)]
            r = tune(*d, t.m, t.n, use_cache=False)
            L, N, nb = t.L, t.n, 1
        key = config_class(L, N, d[2].dtype, nb)
        if key in table:
            print(spec, key, "class already measured for",
                  table[key]["workload"], flush=True)
            continue
        best = r["best"]
        table[key] = {"best": best, "workload": spec,
                      "ms": min(v for k, v in r["times_ms"].items()
                                if not k.startswith("reuse_block") and
                                isinstance(v, float)),
                      "times_ms": r["times_ms"]}
        print(spec, key, best, flush=True)
        del t, d
        torch.cuda.empty_cache()
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    return table


if __name__ == "__main__":
    # python -m paper_1406_1066_amd.autotune [out.json] [workload ...]
    import sys
    out = sys.argv[1] if len(sys.argv) > 1 else TABLE
    names = sys.argv[2:] or ["batched_64", "fem3d_100", "uniform_1e7",
                             "fem3d_50", "fem3d_50:f32", "fem2d_100"]
    write_table(names, out)
