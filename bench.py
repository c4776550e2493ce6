#!/usr/bin/env python3
"""Throughput of Matlab-compatible sparse assembly on one MI355X.

A step is one fresh assembly of the workload, inputs resident in HBM: by
default the 64 independent 2D P1 meshes of batched_64 (175M triplets) in one
batched call -- validation, bin counts, look-back scans, the bin scatter and
the bin kernel that groups, ranks, orders and folds.  `value` = triplets
assembled per second (Gtriplets/s) over the K timed steps.

The same run reports, under "modes": the graph-replayed pattern re-use of
the batch; on fem3d_100 (93M triplets) the fresh call, 100 time steps of
re-assembly with new per-element factors (the value update untimed), the
order-free re-use and the backward gather; and on uniform_1e7 the fresh call
and its re-use.  `--config NAME` benchmarks one workload instead, with the
other calls on it (double indices, drop zeros, delayed assembly, complex and
logical values, index expansion).

Roofline: algorithmic bytes are those of the method, triplets in and CCS out
(fresh fp64: 16 L + 12 nnz + 4 (n+1) summed over the matrices; re-use and
backward: 12 L + 8 nnz), divided by the dominant kernel's average HIP-event
duration on its launch stream inside the timed region, against the 8 TB/s
HBM3E peak.  The whole call's fraction and the counter traffic (rocprofv3
FETCH_SIZE + WRITE_SIZE of the committed profiles, when taken on the current
kernel source) stand beside it.

Prints ONE JSON line.
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
# the calls a run can time beside the fresh one (--only)
LEGS = ["reuse", "reuse_atomic", "backward", "fresh_with_plan",
        "fresh_plan_no_slot", "expand", "f64_index", "drop_zeros", "append",
        "complex", "logical", "time_steps"]
# kernel name prefix -> role, the key of a kernel in the traffic summaries
ROLES = [("fsp::k_scatter", "scatter"), ("fsp::k_bin", "bin"),
         ("fsp::k_count", "count"), ("fsp::k_colscan", "colscan"),
         ("fsp::k_reuse_tiles", "reuse_tiles"), ("fsp::k_reuse", "reuse"),
         ("fsp::k_atomic", "atomic"), ("fsp::k_fill", "fill"),
         ("fsp::k_backward", "backward"), ("fsp::k_zero", "init"),
         ("fsp::k_batched_jcs", "batched_jcs"), ("fsp::k_slow", "slow"),
         ("fsp::k_copy16", "copy")]
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, public spec
PROFILE_DIR = os.path.join(ROOT, "profiles")
# the kernels and the host code that chooses their launch shapes
KERNEL_SRC = [os.path.join(ROOT, "paper_1406_1066_amd", "csrc", f)
              for f in ("kernels.h", "fsparse.hip")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def fresh_bytes(L, nnz, ncols, nmat, vb):
    """Bytes fresh assembly must move: triplets in (two int32 indices and a
    value each), CCS out (row and value per pair, n+1 column pointers per
    matrix)."""
    return (8 + vb) * L + (4 + vb) * nnz + 4 * (ncols + nmat)


def reuse_bytes(L, nnz, vb):
    """Re-use and backward: values in and the k -> slot map (4 B) per
    triplet, values out per pair (fp64: 12 L + 8 nnz)."""
    return (4 + vb) * L + vb * nnz


def backward_bytes(L, nnz, vb):
    """Backward: slot and gradient out per triplet, gradient in per pair."""
    return (4 + vb) * L + vb * nnz


def read_traffic(workload, kernel=None):
    """HBM bytes per launch of a kernel role (or, with kernel None, per fresh
    call: all of its kernels) from committed rocprofv3 counter summaries, if
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
    ks = d.get("kernels", {})
    if kernel is None:
        tot = d.get("bytes_per_call")
        return tot if tot else None
    k = ks.get(kernel)
    if not k:
        return None
    return k.get("bytes_per_launch")


def cpu_baseline(mats, seconds, name):
    """The oracle, one host thread, on the full input of the workload (every
    matrix), repeated until `seconds` have passed."""
    import oracle
    t0_ = mats[0]
    oracle.assemble(t0_.ii[:1000], t0_.jj[:1000], t0_.ss[:1000], t0_.m, t0_.n)
    L = sum(t.L for t in mats)
    reps, el = 0, 0.0
    while reps == 0 or el < seconds:
        t0 = time.perf_counter()
        for t in mats:
            oracle.assemble(t.ii, t.jj, t.ss, t.m, t.n)
        el += time.perf_counter() - t0
        reps += 1
        log("oracle rep %d: %.2f s total" % (reps, el))
    return {"value": L * reps / el / 1e9, "unit": "Gtriplets/s", "cores": 1,
            "kind": "oracle",
            "sample": "full %s input (%d matrices, L=%d), %d repetition%s, "
                      "%.1f s, one thread" % (name, len(mats), L, reps,
                                              "" if reps == 1 else "s", el),
            "host_cpu": host_cpu()}


def stage_profile(fs, torch, step, steps):
    """Average time per launch of every stage, from an untimed pass with
    events around every launch, and the stage that takes longest."""
    with fs.timing() as tp:
        for _ in range(max(3, min(steps, 10))):
            step()
        torch.cuda.synchronize()
    stages = {k: tp.ms[k] / tp.launches[k] for k in tp.ms}
    return stages, max(stages, key=stages.get)


def time_fresh(fs, torch, step, steps, warmup):
    """Warm-up, the stage profile, then exactly `steps` timed calls between
    two synchronisations, with events only around the dominant stage's
    launches (on the stream they are launched on).  Returns the last result,
    seconds for the timed calls, the stage times and the dominant stage with
    its average launch time in ms."""
    r = None
    for _ in range(max(1, warmup)):
        r = step()
    torch.cuda.synchronize()
    stages, dom = stage_profile(fs, torch, step, steps)
    with fs.timing(stages=[dom]) as tm:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    return r, el, stages, dom, tm.ms[dom] / tm.launches[dom]


def time_events(torch, fn, steps, warmup=3):
    """ms per call of stream-ordered work (no host waits inside), by events
    on the current stream around `steps` calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def want(args, leg):
    return not args.only or leg in args.only.split(",")


def with_traffic(row, workload, role):
    """The counter bytes per launch of the row's kernel beside its
    algorithmic bytes (null when no summary matches the kernel source)."""
    tr = read_traffic(workload, role)
    row["traffic"] = tr
    row["traffic_ratio"] = tr / row["bytes"] if tr and row.get("bytes") else None
    return row


def rate(L, ms, nbytes=None, unit="Gtriplets/s"):
    r = {"value": L / (ms * 1e-3) / 1e9, "unit": unit, "ms": ms}
    if nbytes:
        r["bytes"] = nbytes
        r["gbps"] = nbytes / (ms * 1e-3) / 1e9
        r["frac"] = r["gbps"] / HBM_PEAK_GBS
    return r


def roofline(nbytes, dom, dom_ms, workload):
    achieved = nbytes / (dom_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": read_traffic(workload, dom),
            "algorithmic_bytes": nbytes, "avg_launch_ms": dom_ms}


def tune(fs, args, *a, **kw):
    if args.no_autotune:
        fs.set_tuning(reset=True)
        return None
    from paper_1406_1066_amd import autotune
    tuned = autotune.tune(*a, **kw)
    log("tuning", tuned["best"], "(cached)" if tuned["cached"] else "")
    return tuned["best"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="batched_64")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true")
    ap.add_argument("--time-steps", type=int, default=100,
                    help="re-assembly steps of the fem3d_100 time-stepping row")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the 1 GiB copy kernel (counter calibration)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shapes")
    ap.add_argument("--only", default="",
                    help="comma list of the calls timed beside the fresh "
                         "one (default all): " + ", ".join(LEGS))
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU "
              "path (--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1406_1066_amd as fs
    import workloads as W

    if args.copy_only:
        gbs = copy_bw(fs, torch)
        print(json.dumps({"copy_bytes_per_launch": 2 * (1 << 30),
                          "copy_gbps": gbs}), flush=True)
        return

    vt = np.float64 if args.dtype == "f64" else np.float32
    vb = 8 if vt == np.float64 else 4
    log("building workload", args.config)
    t = W.config(args.config, dtype=vt)
    if isinstance(t, W.Batch):
        line = bench_batched(args, t, fs, torch, np, vb)
        mats = t.mats
    else:
        line = bench_single(args, t, fs, torch, np, vb)
        mats = [t]
    if not args.no_modes and args.config == "batched_64" and not args.only:
        # the other legs of the metric on the other workloads
        torch.cuda.empty_cache()
        line["modes"]["fem3d_100"] = mesh_steps(args, fs, torch, np, W, vt, vb)
        torch.cuda.empty_cache()
        line["modes"]["uniform_1e7"] = uniform_row(args, fs, torch, W, vt, vb)
    if not args.no_modes and not args.only:
        line["copy_gbps"] = copy_bw(fs, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(mats, args.cpu_seconds,
                                            args.config)
    print(json.dumps(line), flush=True)


def header(args, value, el):
    return {"metric": METRIC, "value": value, "unit": "Gtriplets/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
            "data": "synthetic"}


def bench_batched(args, batch, fs, torch, np, vb):
    """Headline: one batched fresh assembly of all matrices per step, then
    the graph-replayed re-use of the batch."""
    dev = torch.device("cuda", 0)
    ii, jj, ss, m, n = batch.concat()
    off = batch.trip_off
    L, nb, N = batch.L, batch.nb, int(n.sum())
    iid = torch.from_numpy(ii).to(dev)
    jjd = torch.from_numpy(jj).to(dev)
    ssd = torch.from_numpy(ss).to(dev)
    del ii, jj, ss
    tuning = tune(fs, args, iid, jjd, ssd, list(m), list(n), trip_off=off)
    ws = torch.empty(fs.workspace_bytes(L, N, nb, ssd.dtype),
                     dtype=torch.uint8, device=dev)
    # output buffers kept across steps (capacity L: nnz <= L)
    out = (torch.empty(N + nb, dtype=torch.int32, device=dev),
           torch.empty(L, dtype=torch.int32, device=dev),
           torch.empty(L, dtype=ssd.dtype, device=dev))

    def step():
        return fs.assemble_batched(iid, jjd, ssd, off, m, n, ws=ws, out=out)

    log("timed steps", args.steps)
    r, el, stages, dom, dom_ms = time_fresh(fs, torch, step, args.steps,
                                            args.warmup)
    nnz = r.nnz
    fb = fresh_bytes(L, nnz, N, nb, vb)
    line = header(args, L * args.steps / el / 1e9, el)
    line["config"] = {"workload": args.config, "L": L, "nb": nb, "nnz": nnz,
                      "ncols": N, "mode": "batched fresh"}
    line["roofline"] = roofline(fb, dom, dom_ms, args.config)
    tc = read_traffic(args.config)
    line["path"] = {"bytes": fb, "ms": el / args.steps * 1e3,
                    "frac": fb / (el / args.steps) / 1e9 / HBM_PEAK_GBS,
                    "traffic": tc, "traffic_ratio": tc / fb if tc else None}
    line["stages_ms"] = stages
    line["tuning"] = tuning or fs.get_tuning()
    line["modes"] = {}
    if not args.no_modes and want(args, "reuse"):
        rp = fs.assemble_batched(iid, jjd, ssd, off, m, n, plan=True)
        outp = torch.empty(nnz, dtype=ssd.dtype, device=dev)
        ms = time_events(torch, lambda: fs.reassemble(rp, ssd, out=outp),
                         args.steps)
        line["modes"]["batched_reuse"] = with_traffic(
            rate(L, ms, reuse_bytes(L, nnz, vb)), args.config, "reuse")
        log("batched reuse %.4f ms" % ms)
        del rp, outp
    return line


def mesh_steps(args, fs, torch, np, W, vt, vb):
    """fem3d_100: fresh assembly, then the time-stepping shape -- re-use
    with new values scaled per element by U[0.5, 2] every step (the update
    untimed), order-free re-use, the backward gather and the fresh call
    from connectivity and element matrices (index expansion)."""
    dev = torch.device("cuda", 0)
    t = W.config("fem3d_100", dtype=vt)
    ii = torch.from_numpy(t.ii).to(dev)
    jj = torch.from_numpy(t.jj).to(dev)
    ss = torch.from_numpy(t.ss).to(dev)
    L, m, n = t.L, t.m, t.n
    tune(fs, args, ii, jj, ss, m, n)
    ws = torch.empty(fs.workspace_bytes(L, n, 1, ss.dtype), dtype=torch.uint8,
                     device=dev)
    out = (torch.empty(n + 1, dtype=torch.int32, device=dev),
           torch.empty(L, dtype=torch.int32, device=dev),
           torch.empty(L, dtype=ss.dtype, device=dev))

    def step():
        return fs.sparse(ii, jj, ss, m, n, ws=ws, out=out)

    r, el, stages, dom, dom_ms = time_fresh(fs, torch, step, args.steps,
                                            args.warmup)
    nnz = r.nnz
    fb = fresh_bytes(L, nnz, n, 1, vb)
    row = {"L": L, "nnz": nnz}
    row["fresh"] = rate(L, el / args.steps * 1e3, fb)
    row["fresh"]["roofline"] = roofline(fb, dom, dom_ms, "fem3d_100")
    tc = read_traffic("fem3d_100")
    row["fresh"]["traffic"] = tc
    row["fresh"]["traffic_ratio"] = tc / fb if tc else None
    row["fresh"]["stages_ms"] = stages
    log("fem3d_100 fresh %.4f ms" % row["fresh"]["ms"])
    del ws, out, r
    res = fs.sparse(ii, jj, ss, m, n, plan=True, keep_slot=True)
    prS = torch.empty(nnz, dtype=ss.dtype, device=dev)
    # time steps: new per-element factors each step, the update outside the
    # events around each re-use
    ne = L // t.per_elem
    g = torch.Generator(device=dev)
    s_t = torch.empty_like(ss)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    u0 = torch.cuda.Event(enable_timing=True)
    rms, ums = 0.0, 0.0
    for _ in range(3):
        fs.reassemble(res, ss, out=prS)
    for stp in range(args.time_steps):
        g.manual_seed(1068 * 1000 + stp)
        u0.record()
        f = torch.rand(ne, dtype=ss.dtype, device=dev, generator=g) * 1.5 + 0.5
        torch.mul(ss.view(ne, t.per_elem), f[:, None],
                  out=s_t.view(ne, t.per_elem))
        e0.record()
        fs.reassemble(res, s_t, out=prS)
        e1.record()
        torch.cuda.synchronize()
        rms += e0.elapsed_time(e1)
        ums += u0.elapsed_time(e0)
    rb = reuse_bytes(L, nnz, vb)
    row["reuse_steps"] = with_traffic(rate(L, rms / args.time_steps, rb),
                                      "fem3d_100", "reuse")
    row["reuse_steps"]["steps"] = args.time_steps
    row["reuse_steps"]["update_ms"] = ums / args.time_steps
    log("fem3d_100 reuse step %.4f ms" % row["reuse_steps"]["ms"])
    ms = time_events(torch, lambda: fs.reassemble(res, s_t, out=prS,
                                                  atomic=True), args.steps)
    row["reuse_atomic"] = with_traffic(rate(L, ms, rb), "fem3d_100", "atomic")
    gp = torch.randn(nnz, dtype=ss.dtype, device=dev)
    gs = torch.empty(L, dtype=ss.dtype, device=dev)
    ms = time_events(torch, lambda: fs.backward(res.slot, gp, out=gs),
                     args.steps)
    row["backward"] = with_traffic(rate(L, ms, backward_bytes(L, nnz, vb)),
                                   "fem3d_100", "backward")
    log("fem3d_100 atomic %.4f ms, backward %.4f ms"
        % (row["reuse_atomic"]["ms"], ms))
    del res, prS, gp, gs, s_t, ii, jj
    torch.cuda.empty_cache()
    row["expand"] = expanded(args, fs, torch, t, ss)
    return row


def uniform_row(args, fs, torch, W, vt, vb):
    """uniform_1e7 (random triplets): fresh assembly and its re-use."""
    dev = torch.device("cuda", 0)
    t = W.config("uniform_1e7", dtype=vt)
    ii = torch.from_numpy(t.ii).to(dev)
    jj = torch.from_numpy(t.jj).to(dev)
    ss = torch.from_numpy(t.ss).to(dev)
    L, m, n = t.L, t.m, t.n
    tune(fs, args, ii, jj, ss, m, n)
    ws = torch.empty(fs.workspace_bytes(L, n, 1, ss.dtype), dtype=torch.uint8,
                     device=dev)
    out = (torch.empty(n + 1, dtype=torch.int32, device=dev),
           torch.empty(L, dtype=torch.int32, device=dev),
           torch.empty(L, dtype=ss.dtype, device=dev))
    r, el, stages, dom, dom_ms = time_fresh(
        fs, torch, lambda: fs.sparse(ii, jj, ss, m, n, ws=ws, out=out),
        args.steps, args.warmup)
    nnz = r.nnz
    fb = fresh_bytes(L, nnz, n, 1, vb)
    row = {"L": L, "nnz": nnz, "fresh": rate(L, el / args.steps * 1e3, fb)}
    row["fresh"]["roofline"] = roofline(fb, dom, dom_ms, "uniform_1e7")
    tc = read_traffic("uniform_1e7")
    row["fresh"]["traffic"] = tc
    row["fresh"]["traffic_ratio"] = tc / fb if tc else None
    row["fresh"]["stages_ms"] = stages
    res = fs.sparse(ii, jj, ss, m, n, plan=True)
    prS = torch.empty(nnz, dtype=ss.dtype, device=dev)
    ms = time_events(torch, lambda: fs.reassemble(res, ss, out=prS),
                     args.steps)
    row["reuse"] = with_traffic(rate(L, ms, reuse_bytes(L, nnz, vb)),
                                "uniform_1e7", "reuse")
    log("uniform_1e7 fresh %.4f ms, reuse %.4f ms" % (row["fresh"]["ms"], ms))
    return row


def bench_single(args, t, fs, torch, np, vb):
    """One workload: its fresh call as the step; re-use, order-free re-use,
    backward and the other calls on the same input under "modes"."""
    dev = torch.device("cuda", 0)
    ii = torch.from_numpy(t.ii).to(dev)
    jj = torch.from_numpy(t.jj).to(dev)
    ss = torch.from_numpy(t.ss).to(dev)
    L, m, n = t.L, t.m, t.n
    tuning = tune(fs, args, ii, jj, ss, m, n)
    ws = torch.empty(fs.workspace_bytes(L, n, 1, ss.dtype), dtype=torch.uint8,
                     device=dev)
    out = (torch.empty(n + 1, dtype=torch.int32, device=dev),
           torch.empty(L, dtype=torch.int32, device=dev),
           torch.empty(L, dtype=ss.dtype, device=dev))

    def step():
        return fs.sparse(ii, jj, ss, m, n, ws=ws, out=out)

    log("timed steps", args.steps)
    r, el, stages, dom, dom_ms = time_fresh(fs, torch, step, args.steps,
                                            args.warmup)
    nnz = r.nnz
    fb = fresh_bytes(L, nnz, n, 1, vb)
    line = header(args, L * args.steps / el / 1e9, el)
    line["config"] = {"workload": args.config, "L": L, "m": m, "n": n,
                      "nnz": nnz, "mode": "fresh"}
    line["roofline"] = roofline(fb, dom, dom_ms, args.config)
    tc = read_traffic(args.config)
    line["path"] = {"bytes": fb, "ms": el / args.steps * 1e3,
                    "frac": fb / (el / args.steps) / 1e9 / HBM_PEAK_GBS,
                    "traffic": tc, "traffic_ratio": tc / fb if tc else None}
    line["stages_ms"] = stages
    line["tuning"] = tuning or fs.get_tuning()
    line["modes"] = {}
    if args.no_modes:
        return line
    del ws, out, r
    md = line["modes"]
    wl = args.config
    res = fs.sparse(ii, jj, ss, m, n, plan=True, keep_slot=True)
    prS = torch.empty(nnz, dtype=ss.dtype, device=dev)
    rb = reuse_bytes(L, nnz, vb)
    if want(args, "reuse"):
        md["reuse"] = with_traffic(rate(L, time_events(
            torch, lambda: fs.reassemble(res, ss, out=prS), args.steps), rb),
            wl, "reuse")
    if want(args, "reuse_atomic"):
        md["reuse_atomic"] = with_traffic(rate(L, time_events(
            torch, lambda: fs.reassemble(res, ss, out=prS, atomic=True),
            args.steps), rb), wl, "atomic")
    if want(args, "backward"):
        gp = torch.randn(nnz, dtype=ss.dtype, device=dev)
        gs = torch.empty(L, dtype=ss.dtype, device=dev)
        md["backward"] = with_traffic(rate(L, time_events(
            torch, lambda: fs.backward(res.slot, gp, out=gs), args.steps),
            backward_bytes(L, nnz, vb)), wl, "backward")
        del gp, gs
    if want(args, "fresh_with_plan"):
        md["fresh_with_plan"] = rate(L, time_events(
            torch, lambda: fs.sparse(ii, jj, ss, m, n, plan=True,
                                     keep_slot=True, ws=res.ws), args.steps))
    if want(args, "fresh_plan_no_slot"):
        md["fresh_plan_no_slot"] = rate(L, time_events(
            torch, lambda: fs.sparse(ii, jj, ss, m, n, plan=True, ws=res.ws),
            args.steps))
    for k in ("reuse", "reuse_atomic", "backward", "fresh_with_plan",
              "fresh_plan_no_slot"):
        if k in md:
            log(k, "%.4f ms" % md[k]["ms"])
    del res, prS
    if "conn" in t.meta and want(args, "expand"):
        md["expand"] = expanded(args, fs, torch, t, ss)
    if want(args, "f64_index"):
        md["f64_index"] = double_indices(args, fs, torch, ii, jj, ss, m, n)
    if want(args, "drop_zeros"):
        md["drop_zeros"] = dropped(args, fs, torch, ii, jj, ss, m, n)
    if want(args, "append"):
        md["append"] = appended(args, fs, torch, ii, jj, ss, m, n)
    if want(args, "complex"):
        md["complex"] = complexed(args, fs, torch, ii, jj, ss, m, n)
    if want(args, "logical"):
        md["logical"] = logical(args, fs, torch, ii, jj, ss, m, n)
    return line


def expanded(args, fs, torch, t, ss):
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
    """Delayed assembly: the last half (and, beside it, the last tenth) of
    the triplets added to the assembled rest -- the same matrix as the fresh
    call."""
    L = ss.numel()
    out = {}
    for tag, h in (("half", L // 2), ("tenth", L - L // 10)):
        A = fs.sparse(ii[:h], jj[:h], ss[:h], m, n)
        ws = torch.empty(fs.append_workspace_bytes(A.nnz, L - h, n, ss.dtype),
                         dtype=torch.uint8, device=ss.device)
        i2, j2 = ii[h:].contiguous(), jj[h:].contiguous()
        s2 = ss[h:].contiguous()

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
        log("append %s" % tag, "%.4f ms" % ms)
        out[tag] = {"value": (L - h) / (ms * 1e-3) / 1e9,
                    "unit": "Gtriplets/s (new)", "ms": ms, "old_pairs": A.nnz,
                    "new_triplets": L - h, "stages_ms": stages}
        del A, ws, i2, j2, s2
    return out


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


if __name__ == "__main__":
    main()
