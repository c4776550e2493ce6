#!/usr/bin/env python3
"""Throughput of Matlab-compatible sparse assembly on one MI355X.

A step is one fresh assembly S = sparse(ii, jj, ss, m, n) of the workload
(validation, column histogram, look-back scan, bucket scatter, and the chunk
kernel that groups, ranks, orders and folds), inputs resident in HBM.  The
same run also times, on the same workload, pattern re-use (one HIP-graph
replay of the ordered fold), the atomic re-use variant and the backward
gather, and reports them under "modes".

Prints ONE JSON line.  `value` = triplets assembled per second (Gtriplets/s)
over the K timed steps.  The dominant kernel's roofline uses its algorithmic
bytes per launch divided by its average HIP-event duration, measured on the
launch stream inside the timed region.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("Gtriplets/s assembled + % HBM roofline; fresh vs pattern-reuse "
          "vs batched")
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, public spec
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1406_1066_amd", "csrc", "kernels.h")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stage_bytes(stage, L, nnz, n, vb, eb, plan=False, slot=False):
    """Algorithmic bytes of one launch of a stage: every array the stage
    must read or write, touched once.  eb = bytes of one binned triplet
    (row and in-bin column in one word, k, value), vb = bytes of one value.
    (Inputs whose rows and in-bin columns do not share a word add a 4-byte
    column per triplet to the scatter and the bin kernel; none of the
    configured workloads does.)"""
    if stage == "count":
        return 4 * L
    if stage == "scatter":
        return (8 + vb) * L + eb * L
    if stage == "bin":
        b = eb * L + (4 + vb) * nnz + 4 * (n + 1)
        if slot:
            b += 4 * L
        if plan:
            b += 4 * L + 4 * (nnz + 1)
        return b
    if stage == "reuse":
        return 4 * L + 4 * (nnz + 1) + vb * L + vb * nnz
    if stage == "backward":
        return 4 * L + vb * nnz + vb * L
    return None


def path_bytes(L, nnz, n, vb):
    """Bytes the fresh assembly must move: triplets in, CCS out."""
    return (8 + vb) * L + (4 + vb) * nnz + 4 * (n + 1)


def read_traffic(workload, kernel):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel source."""
    path = os.path.join(PROFILE_DIR, "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("bytes_per_launch")


def cpu_baseline(t, seconds):
    import numpy as np  # noqa: F401
    import oracle
    oracle.assemble(t.ii[:1000], t.jj[:1000], t.ss[:1000], t.m, t.n)  # load
    reps, el = 0, 0.0
    while reps == 0 or el < seconds:
        t0 = time.perf_counter()
        oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
        el += time.perf_counter() - t0
        reps += 1
        log("oracle rep %d: %.2f s total" % (reps, el))
    return {"value": t.L * reps / el / 1e9, "unit": "Gtriplets/s", "cores": 1,
            "kind": "oracle",
            "sample": "full %s input (L=%d), %d repetitions, %.1f s, one "
                      "thread" % (t.name, t.L, reps, el)}


def stage_profile(fs, torch, step, steps):
    """Average time per launch of every stage, from an untimed pass with
    events around every launch, and the stage that takes longest."""
    with fs.timing() as tp:
        for _ in range(max(3, min(steps, 10))):
            step()
        torch.cuda.synchronize()
    stages = {k: tp.ms[k] / tp.launches[k] for k in tp.ms}
    return stages, max(stages, key=stages.get)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="uniform_1e7")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the 1 GiB copy kernel (counter calibration)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shapes")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU "
              "path (--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    # tuning choices are cached per device and input class; keep the cache
    # where every process of this machine finds it
    import tempfile
    os.environ.setdefault("FSPARSE_TUNE_CACHE",
                          os.path.join(tempfile.gettempdir(),
                                       "fsparse_mi355x_tune.json"))
    import paper_1406_1066_amd as fs
    import workloads as W

    if args.copy_only:
        gbs = copy_bw(fs, torch)
        print(json.dumps({"copy_bytes_per_launch": 2 * (1 << 30),
                          "copy_gbps": gbs}), flush=True)
        return

    vt = np.float64 if args.dtype == "f64" else np.float32
    vb = 8 if vt == np.float64 else 4
    eb = 16 if vt == np.float64 else 12
    log("building workload", args.config)
    t = W.config(args.config, dtype=vt)
    if isinstance(t, W.Batch):
        return bench_batched(args, t, fs, torch, np, vb, eb)
    dev = torch.device("cuda", 0)
    ii = torch.from_numpy(t.ii).to(dev)
    jj = torch.from_numpy(t.jj).to(dev)
    ss = torch.from_numpy(t.ss).to(dev)
    L, m, n = t.L, t.m, t.n
    tuned = None
    if not args.no_autotune:
        from paper_1406_1066_amd import autotune
        log("autotuning")
        tuned = autotune.tune(ii, jj, ss, m, n)
        log("tuning", tuned["best"], "cached" if tuned["cached"] else "")
    ws = torch.empty(fs.workspace_bytes(L, n, 1, ss.dtype), dtype=torch.uint8,
                     device=dev)
    jcS = torch.empty(n + 1, dtype=torch.int32, device=dev)
    irS = torch.empty(L, dtype=torch.int32, device=dev)
    prS = torch.empty(L, dtype=ss.dtype, device=dev)
    out = (jcS, irS, prS)

    def step():
        return fs.sparse(ii, jj, ss, m, n, ws=ws, out=out)

    log("warmup", args.warmup)
    r = None
    for _ in range(max(1, args.warmup)):
        r = step()
    nnz = r.nnz
    torch.cuda.synchronize()
    stages, dom = stage_profile(fs, torch, step, args.steps)
    log("timed steps", args.steps)
    # events only around the dominant kernel's launches inside the timed
    # region (events around every launch would add their own gaps)
    with fs.timing(stages=[dom]) as tm:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    el = t1 - t0
    dom_ms = tm.ms[dom] / tm.launches[dom]
    ab = stage_bytes(dom, L, nnz, n, vb, eb)
    achieved = ab / (dom_ms * 1e-3) / 1e9
    traffic = read_traffic(args.config, dom)
    line = {
        "metric": METRIC,
        "value": L * args.steps / el / 1e9,
        "unit": "Gtriplets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": args.config, "L": L, "m": m, "n": n,
                   "nnz": nnz, "mode": "fresh"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": ab,
                     "avg_launch_ms": dom_ms},
        "stages_ms": stages,
        "tuning": fs.get_tuning(),
        "path": {"bytes": path_bytes(L, nnz, n, vb),
                 "frac": path_bytes(L, nnz, n, vb) / (el / args.steps)
                 / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_modes:
        line["modes"] = modes(args, fs, torch, ii, jj, ss, m, n, L, vb, eb)
        if "conn" in t.meta:
            line["modes"]["expand"] = expanded(args, fs, torch, t, ss, vb, eb)
        line["modes"]["f64_index"] = double_indices(args, fs, torch, ii, jj,
                                                    ss, m, n)
        line["modes"]["drop_zeros"] = dropped(args, fs, torch, ii, jj, ss, m, n)
        line["modes"]["append"] = appended(args, fs, torch, ii, jj, ss, m, n)
        line["modes"]["complex"] = complexed(args, fs, torch, ii, jj, ss, m, n)
        line["modes"]["logical"] = logical(args, fs, torch, ii, jj, ss, m, n)
        line["copy_gbps"] = copy_bw(fs, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(t, args.cpu_seconds)
        line["cpu_baseline"]["host_cpu"] = host_cpu()
    print(json.dumps(line), flush=True)


def modes(args, fs, torch, ii, jj, ss, m, n, L, vb, eb):
    res = fs.sparse(ii, jj, ss, m, n, plan=True, keep_slot=True)
    nnz = res.nnz
    out = torch.empty(nnz, dtype=ss.dtype, device=ss.device)
    g = torch.randn(nnz, dtype=ss.dtype, device=ss.device)
    gs = torch.empty(L, dtype=ss.dtype, device=ss.device)
    d = {}
    for name, fn, nbytes in (
            ("reuse", lambda: fs.reassemble(res, ss, out=out),
             stage_bytes("reuse", L, nnz, n, vb, eb)),
            ("reuse_atomic",
             lambda: fs.reassemble(res, ss, out=out, atomic=True),
             4 * L + vb * L + vb * nnz),
            ("backward", lambda: fs.backward(res.slot, g, out=gs),
             stage_bytes("backward", L, nnz, n, vb, eb)),
            ("fresh_with_plan",
             lambda: fs.sparse(ii, jj, ss, m, n, plan=True, keep_slot=True,
                               ws=res.ws),
             None),
            ("fresh_plan_no_slot",
             lambda: fs.sparse(ii, jj, ss, m, n, plan=True, ws=res.ws),
             None)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        rec = {"value": L / (ms * 1e-3) / 1e9, "unit": "Gtriplets/s",
               "ms": ms}
        if nbytes:
            rec["gbps"] = nbytes / (ms * 1e-3) / 1e9
            rec["frac"] = rec["gbps"] / HBM_PEAK_GBS
        d[name] = rec
        log(name, "%.4f ms" % ms)
    return d


def expanded(args, fs, torch, t, ss, vb, eb):
    """Fresh assembly from the element connectivity and element matrices
    (index expansion), with the launch shapes of the plain call."""
    conn = torch.from_numpy(t.meta["conn"]).to(ss.device)
    ne, nv = conn.shape
    ci, cj = conn[:, :, None], conn[:, None, :]
    K = ss.view(ne, nv, nv)
    L, n = ss.numel(), t.n
    ws = torch.empty(fs.workspace_bytes(L, n, 1, ss.dtype), dtype=torch.uint8,
                     device=ss.device)
    out = (torch.empty(n + 1, dtype=torch.int32, device=ss.device),
           torch.empty(L, dtype=torch.int32, device=ss.device),
           torch.empty(L, dtype=ss.dtype, device=ss.device))

    def fn():
        return fs.sparse_expand(ci, cj, K, t.m, n, ws=ws, out=out)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    stages, _ = stage_profile(fs, torch, fn, args.steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log("expand", "%.4f ms" % ms)
    # the index bytes of the whole path: the connectivity once
    ib = 4 * ne * nv
    return {"value": L / (ms * 1e-3) / 1e9, "unit": "Gtriplets/s", "ms": ms,
            "index_bytes": ib, "stages_ms": stages}


def double_indices(args, fs, torch, ii, jj, ss, m, n):
    """Fresh assembly from double-valued index arrays (checked and
    converted by the passes that read them), same launch shapes."""
    di, dj = ii.to(torch.float64), jj.to(torch.float64)
    L = ss.numel()
    ws = torch.empty(fs.workspace_bytes(L, n, 1, ss.dtype), dtype=torch.uint8,
                     device=ss.device)
    out = (torch.empty(n + 1, dtype=torch.int32, device=ss.device),
           torch.empty(L, dtype=torch.int32, device=ss.device),
           torch.empty(L, dtype=ss.dtype, device=ss.device))

    def fn():
        return fs.sparse(di, dj, ss, m, n, ws=ws, out=out)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    stages, _ = stage_profile(fs, torch, fn, args.steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log("f64_index", "%.4f ms" % ms)
    del di, dj, ws, out
    return {"value": L / (ms * 1e-3) / 1e9, "unit": "Gtriplets/s", "ms": ms,
            "stages_ms": stages}


def dropped(args, fs, torch, ii, jj, ss, m, n):
    """Fresh assembly with the zero sums removed (Matlab's convention): the
    compaction over the pairs and the second wait, on top of the plain call."""
    L = ss.numel()
    ws = torch.empty(fs.workspace_bytes(L, n, 1, ss.dtype), dtype=torch.uint8,
                     device=ss.device)
    out = (torch.empty(n + 1, dtype=torch.int32, device=ss.device),
           torch.empty(L, dtype=torch.int32, device=ss.device),
           torch.empty(L, dtype=ss.dtype, device=ss.device))

    def fn():
        return fs.sparse(ii, jj, ss, m, n, ws=ws, out=out, drop_zeros=True)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    stages, _ = stage_profile(fs, torch, fn, args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    log("drop_zeros", "%.4f ms" % ms)
    return {"value": L / (ms * 1e-3) / 1e9, "unit": "Gtriplets/s", "ms": ms,
            "nnz_kept": r.nnz, "stages_ms": stages}


def complexed(args, fs, torch, ii, jj, ss, m, n):
    """Complex values, split real and imaginary arrays: the fresh pass on the
    real parts with the sorted order kept, then the ordered fold of the
    imaginary parts along it."""
    L = ss.numel()
    g = torch.Generator(device=ss.device)
    g.manual_seed(1406)
    si = torch.randn(L, dtype=ss.dtype, device=ss.device, generator=g)
    ws = torch.empty(fs.workspace_bytes(L, n, 1, ss.dtype), dtype=torch.uint8,
                     device=ss.device)

    def fn():
        return fs.sparse_complex(ii, jj, ss, si, m, n, ws=ws)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    stages, _ = stage_profile(fs, torch, fn, args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    log("complex", "%.4f ms" % ms)
    return {"value": L / (ms * 1e-3) / 1e9, "unit": "Gtriplets/s (complex)",
            "ms": ms, "nnz": r.nnz, "stages_ms": stages}


def logical(args, fs, torch, ii, jj, ss, m, n):
    """Logical values (true where the workload's value is positive, about
    half the triplets): indicators, the fp32 fold with the pairs that have
    no true triplet removed, and the true values."""
    L = ss.numel()
    sl = ss > 0
    ws = torch.empty(fs.logical_workspace_bytes(L, n), dtype=torch.uint8,
                     device=ss.device)

    def fn():
        return fs.sparse_logical(ii, jj, sl, m, n, ws=ws)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    stages, _ = stage_profile(fs, torch, fn, args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    log("logical", "%.4f ms" % ms)
    return {"value": L / (ms * 1e-3) / 1e9, "unit": "Gtriplets/s (logical)",
            "ms": ms, "nnz": r.nnz, "stages_ms": stages}


def appended(args, fs, torch, ii, jj, ss, m, n):
    """Delayed assembly: the second half of the triplets added to the
    assembled first half (the same matrix as the fresh call)."""
    L = ss.numel()
    h = L // 2
    A = fs.sparse(ii[:h], jj[:h], ss[:h], m, n)
    ws = torch.empty(fs.append_workspace_bytes(A.nnz, L - h, n, ss.dtype),
                     dtype=torch.uint8, device=ss.device)
    i2, j2, s2 = ii[h:].contiguous(), jj[h:].contiguous(), ss[h:].contiguous()

    def fn():
        return fs.sparse_append(A, i2, j2, s2, m, n, ws=ws)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    stages, _ = stage_profile(fs, torch, fn, args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    log("append", "%.4f ms" % ms)
    return {"value": (L - h) / (ms * 1e-3) / 1e9, "unit": "Gtriplets/s (new)",
            "ms": ms, "old_pairs": A.nnz, "new_triplets": L - h,
            "stages_ms": stages}


def copy_bw(fs, torch):
    n = 1 << 27                                   # 1 GiB of doubles
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        fs.stream_copy(a, b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        fs.stream_copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def host_cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return "%s; nproc=%d" % (line.split(":", 1)[1].strip(),
                                         os.cpu_count())
    except OSError:
        pass
    return "nproc=%d" % os.cpu_count()


def bench_batched(args, batch, fs, torch, np, vb, eb):
    dev = torch.device("cuda", 0)
    ii, jj, ss, m, n = batch.concat()
    off = batch.trip_off
    L = batch.L
    iid = torch.from_numpy(ii).to(dev)
    jjd = torch.from_numpy(jj).to(dev)
    ssd = torch.from_numpy(ss).to(dev)
    if not args.no_autotune:
        from paper_1406_1066_amd import autotune
        log("autotuning")
        tuned = autotune.tune(iid, jjd, ssd, list(m), list(n), trip_off=off)
        log("tuning", tuned["best"], "cached" if tuned["cached"] else "")
    ws = torch.empty(fs.workspace_bytes(L, int(n.sum()), batch.nb, ssd.dtype),
                     dtype=torch.uint8, device=dev)

    def step():
        return fs.assemble_batched(iid, jjd, ssd, off, m, n, ws=ws)

    r = None
    for _ in range(max(1, args.warmup)):
        r = step()
    torch.cuda.synchronize()
    stages, dom = stage_profile(fs, torch, step, args.steps)
    with fs.timing(stages=[dom]) as tm:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    dom_ms = tm.ms[dom] / tm.launches[dom]
    nnz, N = r.nnz, int(n.sum())
    ab = stage_bytes(dom, L, nnz, N, vb, eb)
    achieved = ab / (dom_ms * 1e-3) / 1e9
    rp = fs.assemble_batched(iid, jjd, ssd, off, m, n, plan=True)
    outp = torch.empty(nnz, dtype=ssd.dtype, device=dev)
    for _ in range(3):
        fs.reassemble(rp, ssd, out=outp)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        fs.reassemble(rp, ssd, out=outp)
    e1.record()
    torch.cuda.synchronize()
    rms = e0.elapsed_time(e1) / args.steps
    line = {
        "metric": METRIC, "value": L * args.steps / el / 1e9,
        "unit": "Gtriplets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": args.config, "L": L, "nb": batch.nb,
                   "nnz": nnz, "mode": "batched"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": read_traffic(args.config, dom),
                     "algorithmic_bytes": ab, "avg_launch_ms": dom_ms},
        "stages_ms": stages,
        "tuning": fs.get_tuning(),
        "modes": {"reuse": {"value": L / (rms * 1e-3) / 1e9, "ms": rms,
                            "unit": "Gtriplets/s",
                            "frac": stage_bytes("reuse", L, nnz, N, vb, eb)
                            / (rms * 1e-3) / 1e9 / HBM_PEAK_GBS}},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
