#!/usr/bin/env python3
"""Throughput of the GLCM hot path on one MI355X.

Workload: one 4096x4096 uint8 image (smooth: Gaussian noise blurred with
sigma = 8 px, min-max rescaled), N = 32 levels over [0, 255], the four d = 1
offsets of Eq. (2); output [4, 32, 32] uint32.  A step is one glcm_compute
call on a device-resident image (quantize, pair visit, LDS vote, merge).
Timed steps rotate over 32 device copies of the image (512 MiB), the
rotation continuing from the warm-up, and 512 MiB of scratch are written just
before the timed loop: every step reads a copy last touched at least 496 MiB
of traffic earlier, so from HBM rather than from the 256 MiB Infinity Cache.
Every copy's result is checked bit-exact against the CPU oracle.  The plan is
tuned first (untimed) by glcm_plan_autotune on one copy of the same image:
it times the LDS layouts of the strip and slab kernels and, the offsets being
the d = 1 directions, the block-code kernel, and keeps the fastest
(--no-autotune keeps the default layout, --layout fixes one).
`extra.cache_hot_gpairs_s` repeats the timed loop on one image copy, which
then stays in the Infinity Cache: labelled, never the headline value.
`extra.batch` carries the batch workload's ratio of one fused launch over
per-tile calls and its graph-replay time (bench_batch); `extra.tile_stream`
the same tiles as one request each through the request server, which fuses
queued requests of one job into batch launches, against one request at a
time (serve_tile_stream).

Prints one JSON line.  `value` is pairs per second over the timed steps
(wall clock, both kernels of each call).  `roofline` prices the dominant
kernel (the vote kernel) against HBM: algorithmic bytes per launch (image
once + output counts) over that kernel's average duration, from HIP events
that each launch's dispatch stamps with the kernel's start and end (a second,
identically tuned plan with FLAG_TIMING).  `traffic` comes from a committed rocprofv3 counter
summary of the same kernel, used only while the kernel source and layout
still match it.  The CPU-baseline leg times the oracle (plain C, one thread)
on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpairs/s & % HBM roofline (bit-exact); batched vs per-image; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# sources of the vote kernel (the dominant kernel the traffic record describes)
VOTE_SOURCES = [os.path.join(ROOT, "paper_1710_06189_amd", "csrc", f)
                for f in ("glcm_vote.hip", "glcm_device.h", "glcm_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vote_strips_4096x4096_u8_smooth_traffic.json")
# the same for the block-code kernel (the autotuner's pick on smooth images)
BLOCK_SOURCES = [os.path.join(ROOT, "paper_1710_06189_amd", "csrc", f)
                 for f in ("glcm_blocks.hip", "glcm_device.h", "glcm_internal.h")]
BLOCK_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vote_blocks_4096x4096_u8_smooth_traffic.json")
# the same for the histogram kernel
HIST_SOURCES = [os.path.join(ROOT, "paper_1710_06189_amd", "csrc", f)
                for f in ("glcm_hist.hip", "glcm_device.h", "glcm_hist.h", "glcm_internal.h")]
HIST_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "histogram_4096x4096_u8_smooth_traffic.json")
# VALU instruction count of the Haralick kernel (an fp64 ALU-bound kernel)
STATS_SOURCES = [os.path.join(ROOT, "paper_1710_06189_amd", "csrc", f)
                 for f in ("glcm_stats.hip", "glcm_device.h", "glcm_stats.h", "glcm_internal.h")]
HARALICK_VALU_FILE = os.path.join(ROOT, "profiles", "haralick_16384x16x16_glcm_like_valu.json")
# VALU issue peak: 256 CUs x 2.4 GHz x one wave64 instruction per CU-cycle
# (four SIMDs, each finishing a 64-lane instruction every 4 cycles on 16 lanes)
VALU_PEAK_G = 256 * 2.4 * 1.0
TUNING_KEYS = ("path", "replicas", "wg_size", "counter_bits", "merge", "partitions")


def pairs_of(W, H, offsets):
    return sum(max(0, W - abs(dx)) * max(0, H - abs(dy)) for dx, dy in offsets)


def kernel_source_sha256(paths=None):
    h = hashlib.sha256()
    for path in paths or VOTE_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(tuning):
    """HBM bytes per vote-kernel launch from the committed counter summary of
    the kernel the tuning selects, or None when the kernel source or the
    layout differ from what was measured."""
    blocks = tuning.get("path") == 6
    try:
        with open(BLOCK_TRAFFIC_FILE if blocks else TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_sha256(BLOCK_SOURCES if blocks else VOTE_SOURCES):
        return None
    if any(rec.get("tuning", {}).get(k) != tuning.get(k) for k in TUNING_KEYS):
        return None
    return rec.get("hbm_bytes_per_launch")


def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {len(os.sched_getaffinity(0))} cores available"


def recorded_hist_traffic():
    """HBM bytes per histogram-kernel launch (N = 32) from the committed counter
    summary, or None when the kernel's sources differ from what was measured."""
    try:
        with open(HIST_TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_sha256(HIST_SOURCES):
        return None
    return rec.get("hbm_bytes_per_launch")


def recorded_haralick_valu():
    """VALU wave-instructions per Haralick launch on the 16384 x N16 workload
    from the committed counter summary, or None when the sources changed."""
    try:
        with open(HARALICK_VALU_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_sha256(STATS_SOURCES):
        return None
    return rec.get("valu_insts_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kind", default="smooth", choices=["smooth", "uniform", "constant"])
    ap.add_argument("--copies", type=int, default=32)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--others", action="store_true", help="also time the uniform and constant images")
    ap.add_argument("--sweep", action="store_true", help="time the LDS layouts on all three images")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default layout instead of timing the candidates (glcm_plan_autotune)")
    ap.add_argument("--path", default="auto", choices=["auto", "strips", "blocks"],
                    help="auto: the autotuner's pick; strips / blocks: that kernel, untuned (for profiling runs, "
                         "whose per-dispatch overhead would blur the autotuner's timing); multispectral: strips "
                         "moves the stack from the slab kernel onto the strip kernel's reach-4 variant")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch workload's figures in extra")
    ap.add_argument("--layout", default=None,
                    help="fixed layout replicas,counter_bits,wg_size (skips the autotuner)")
    ap.add_argument("--workload", default="square",
                    choices=["square", "multispectral", "batch", "serving", "histogram", "variants", "large_n"],
                    help="square: the 4096^2 device-resident image (the default line); multispectral: "
                         "the 8-band 8192^2 uint16 stack streamed from pinned host memory")
    ap.add_argument("--bands", type=int, default=8)
    ap.add_argument("--tiles", type=int, default=4096)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--requests", type=int, default=1000, help="serving: requests per measurement")
    ap.add_argument("--lanes", type=int, default=4, help="serving: server lanes (streams)")
    ap.add_argument("--budget-gib", type=int, default=32, help="serving: HBM budget of the server")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is a design "
              "note, not a measured configuration", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    import paper_1710_06189_amd as G
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.workload == "multispectral":
        bench_multispectral(args, G, torch, np, oracle, synth, dev)
        return
    if args.workload == "batch":
        bench_batch(args, G, torch, np, oracle, synth, dev)
        return
    if args.workload == "serving":
        bench_serving(args, G, torch, np, oracle, synth, dev)
        return
    if args.workload == "histogram":
        bench_histogram(args, G, torch, np, oracle, synth, dev)
        return
    if args.workload == "variants":
        bench_variants(args, G, torch, np, oracle, synth, dev)
        return
    if args.workload == "large_n":
        bench_large_n(args, G, torch, np, oracle, synth, dev)
        return
    oracle_cache, image_cache = {}, {}
    fixed = None
    if args.layout:
        R, bits, wg = (int(v) for v in args.layout.split(","))
        fixed = {"replicas": R, "counter_bits": bits, "wg_size": wg}

    scratch = torch.empty(512 << 20, dtype=torch.uint8, device=dev)

    def timed_loop(plan, copies, outs, N, lo, hi, offs, steps, warmup):
        stream = torch.cuda.current_stream()
        for i in range(warmup):
            j = i % len(copies)
            G.glcm_compute(copies[j], N, lo, hi, offs, out=outs[j], plan=plan, stream=stream)
        # evict the Infinity Cache (a fill kernel writing 512 MiB)
        scratch.fill_(1)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for i in range(steps):
            j = (warmup + i) % len(copies)
            G.glcm_compute(copies[j], N, lo, hi, offs, out=outs[j], plan=plan, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ev0.elapsed_time(ev1) / max(1, steps)

    def measure(kind, tuning=None, vote_timing=False, ncopies=None):
        ncopies = ncopies or args.copies
        w = image_cache.get(kind)
        if w is None:
            w = image_cache[kind] = synth.square_4096(kind)
        img, N, lo, hi, offs = w["images"][0], w["N"], w["lo"], w["hi"], w["offsets"]
        H, W = img.shape
        K = len(offs)
        want = oracle_cache.get(kind)
        if want is None:
            want = oracle_cache[kind] = oracle.glcm(img, N, lo, hi, offs)
        base = torch.from_numpy(img).to(dev)
        copies = [base.clone() for _ in range(ncopies)]
        outs = [torch.empty((K, N, N), dtype=torch.uint32, device=dev) for _ in range(ncopies)]
        plan = G.glcm_plan_create(np.uint8, N, offs, W, H, G.FLAG_FORCE_BLOCKS if args.path == "blocks" else 0)
        if tuning:
            plan.set_tuning(**tuning)
        elif fixed:
            plan.set_tuning(**fixed)
        elif not args.no_autotune and args.path == "auto":
            plan.autotune(copies[0], lo, hi, repeats=10)
        wall, step_ms = timed_loop(plan, copies, outs, N, lo, hi, offs, args.steps, args.warmup)
        for j in range(min(ncopies, args.steps + args.warmup)):
            got = outs[j].view(torch.int32).cpu().numpy().view(np.uint32)
            if not np.array_equal(got, want):
                raise SystemExit(f"bench: result of copy {j} differs from the oracle ({kind})")
        t = plan.tuning.as_dict()
        vote_ms = None
        if vote_timing:
            blocks = G.PATH_NAMES[t["path"]] == "blocks"
            tp = G.glcm_plan_create(np.uint8, N, offs, W, H, G.FLAG_TIMING | (G.FLAG_FORCE_BLOCKS if blocks else 0))
            if not blocks:
                tp.set_tuning(**{k: t[k] for k in ("replicas", "counter_bits", "wg_size", "merge")})
            assert tp.tuning.as_dict()["path"] == t["path"]
            timed_loop(tp, copies, outs, N, lo, hi, offs, args.warmup, 0)
            tp.kernel_time()  # drop the warm-up launches
            timed_loop(tp, copies, outs, N, lo, hi, offs, args.steps, 0)
            total, n = tp.kernel_time()
            vote_ms = total / n
            tp.close()
        plan.close()
        return dict(name=w["name"], pairs=pairs_of(W, H, offs), bytes=W * H * img.itemsize + K * N * N * 4,
                    wall_s=wall, step_ms=step_ms, vote_ms=vote_ms, tuning=t, img=img, N=N, lo=lo, hi=hi,
                    offs=offs)

    if args.sweep:
        grid = [(R, bits, wg) for R, bits in ((8, 32), (16, 32), (32, 32), (8, 16), (16, 16), (32, 16))
                for wg in (512, 1024)]
        for kind in ("smooth", "uniform", "constant"):
            for R, bits, wg in grid:
                cfg = {"replicas": R, "counter_bits": bits, "wg_size": wg}
                try:
                    r = measure(kind, cfg, vote_timing=True)
                except Exception as e:  # a layout the LDS cannot hold
                    print(json.dumps({"sweep": kind, **cfg, "error": str(e)}), flush=True)
                    continue
                print(json.dumps({"sweep": kind, **cfg, "partitions": r["tuning"]["partitions"],
                                  "us_per_step": round(r["step_ms"] * 1e3, 2),
                                  "vote_us": round(r["vote_ms"] * 1e3, 2) if r["vote_ms"] else None,
                                  "gpairs_s": round(r["pairs"] / (r["step_ms"] * 1e-3) / 1e9, 1)}), flush=True)
        return

    main_res = measure(args.kind, vote_timing=True)
    steps = args.steps
    ms_per_step = main_res["wall_s"] * 1e3 / steps
    value = main_res["pairs"] / (main_res["wall_s"] / steps) / 1e9
    achieved_gbs = main_res["bytes"] / (main_res["vote_ms"] * 1e-3) / 1e9
    traffic = recorded_traffic(main_res["tuning"])

    extra = {"input_sha256": synth.sha256(main_res["img"]),
             "step_ms_events": main_res["step_ms"], "vote_kernel_ms": main_res["vote_ms"],
             "pairs_per_step": main_res["pairs"], "algorithmic_bytes_per_step": main_res["bytes"],
             "tuning": main_res["tuning"], "copies_rotated": args.copies,
             "rotated_bytes": args.copies * 4096 * 4096,
             "lds_vote_rate_tvotes_s": main_res["pairs"] / (main_res["vote_ms"] * 1e-3) / 1e12}
    # per-call latency (events around each call, inputs rotating in HBM) and
    # the features kernel on the same output
    lat = call_latencies(G, torch, np, synth, dev, args)
    extra.update(lat)
    hot = measure(args.kind, ncopies=1)
    extra["cache_hot_gpairs_s"] = hot["pairs"] / (hot["wall_s"] / steps) / 1e9
    if not args.no_batch:
        b = bench_batch(args, G, torch, np, oracle, synth, dev, print_line=False)
        extra["batch"] = {k: b[k] for k in ("workload", "tiles", "pairs", "batched_ms", "batched_device_ms",
                                            "per_image_ms", "per_image_device_ms", "batched_over_per_image",
                                            "graph_replay_ms", "graph_replay_gpairs_s", "autotuned_ms",
                                            "autotuned_layout", "check")}
        # the same tiles as one request each through the request server, which
        # fuses queued requests of one job into batch launches
        extra["tile_stream"] = serve_tile_stream(args, G, torch, np, synth, dev)
    if args.others:
        for kind in ("uniform", "constant", "smooth"):
            if kind == args.kind:
                continue
            r = measure(kind)
            extra[f"{kind}_gpairs_s"] = r["pairs"] / (r["wall_s"] / steps) / 1e9
            extra[f"{kind}_tuning"] = r["tuning"]

    cpu = None
    if not args.no_cpu:
        img, N, lo, hi, offs = (main_res[k] for k in ("img", "N", "lo", "hi", "offs"))
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.glcm(img, N, lo, hi, offs)
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        cpu = {"value": reps * main_res["pairs"] / el / 1e9, "unit": "Gpairs/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full passes over the 4096x4096 {args.kind} image, 4 offsets, single-threaded C "
                         f"oracle, {el:.1f} s; host {host_cpu()}"}
        extra["cpu_all_cores"] = cpu_all_cores(oracle, np, img, N, lo, hi, offs, main_res["pairs"], args.cpu_seconds)

    line = {
        "metric": METRIC, "value": value, "unit": "Gpairs/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": main_res["name"], "image": "4096x4096 uint8", "levels": 32,
                   "offsets": [list(o) for o in main_res["offs"]], "resident": "device"},
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": traffic},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


def cpu_all_cores(oracle, np, img, N, lo, hi, offs, pairs, seconds):
    """The oracle run on row bands by one thread per host core (ctypes releases
    the GIL), each band into its own GLCM, summed: the multi-core CPU figure.
    Checked against the single-threaded oracle."""
    from concurrent.futures import ThreadPoolExecutor
    cores = min(16, len(os.sched_getaffinity(0)))  # the GPU machine's CPU share
    H = img.shape[0]
    bands = [(H * b // cores, H * (b + 1) // cores) for b in range(cores)]

    def once(ex):
        return sum(ex.map(lambda r: oracle.glcm(img, N, lo, hi, offs, rows=r).astype(np.uint64), bands))

    with ThreadPoolExecutor(cores) as ex:
        if not np.array_equal(once(ex), oracle.glcm(img, N, lo, hi, offs)):
            raise SystemExit("bench: the multi-core oracle run differs from the single-threaded one")
        reps, t0 = 0, time.perf_counter()
        while True:
            once(ex)
            reps += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                break
    return {"value": reps * pairs / el / 1e9, "unit": "Gpairs/s", "cores": cores,
            "kind": "oracle on row bands, one thread per core, private GLCMs summed",
            "sample": f"{reps} full passes over the same image, {el:.1f} s"}


def call_latencies(G, torch, np, synth, dev, args, calls=200):
    """p50 / p99 of single glcm_compute calls (and of glcm_features) measured
    with events around each call on the stream, inputs rotating in HBM."""
    w = synth.square_4096(args.kind)
    img, N, lo, hi, offs = w["images"][0], w["N"], w["lo"], w["hi"], w["offsets"]
    base = torch.from_numpy(img).to(dev)
    copies = [base.clone() for _ in range(args.copies)]
    out = torch.empty((len(offs), N, N), dtype=torch.uint32, device=dev)
    plan = G.glcm_plan_create(np.uint8, N, offs, img.shape[1], img.shape[0],
                              G.FLAG_FORCE_BLOCKS if args.path == "blocks" else 0)
    if args.layout:
        R, bits, wg = (int(v) for v in args.layout.split(","))
        plan.set_tuning(replicas=R, counter_bits=bits, wg_size=wg)
    elif not args.no_autotune and args.path == "auto":
        plan.autotune(copies[0], lo, hi, repeats=10)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    fev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    for i in range(20):
        G.glcm_compute(copies[i % len(copies)], N, lo, hi, offs, out=out, plan=plan, stream=stream)
        G.glcm_features(out, stream=stream)
    torch.cuda.synchronize()
    for i in range(calls):
        ev[i][0].record(stream)
        G.glcm_compute(copies[i % len(copies)], N, lo, hi, offs, out=out, plan=plan, stream=stream)
        ev[i][1].record(stream)
        fev[i][0].record(stream)
        G.glcm_features(out, stream=stream)
        fev[i][1].record(stream)
    torch.cuda.synchronize()
    plan.close()
    t = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])
    f = np.array([a.elapsed_time(b) * 1e3 for a, b in fev])
    return {"call_us_p50": float(np.percentile(t, 50)), "call_us_p99": float(np.percentile(t, 99)),
            "features_us_p50": float(np.percentile(f, 50)), "features_us_p99": float(np.percentile(f, 99)),
            "latency_calls": calls}


def bench_batch(args, G, torch, np, oracle, synth, dev, reps=20, print_line=True):
    """4096 uint8 tiles (sides log-uniform in [32, 512], half noise, half
    smooth), N = 16, d = 1 at four angles, counts plus the five statistics:
    one fused launch for the whole batch against one glcm_compute +
    glcm_features pair per tile on one stream.  The two must agree bit for
    bit; 64 tiles are also checked against the oracle."""
    w = synth.batch_tiles(args.tiles)
    imgs, N, offs = w["images"], w["N"], w["offsets"]
    T, K = len(imgs), len(offs)
    print(f"[batch] {T} tiles generated", file=sys.stderr, flush=True)
    tens = [torch.from_numpy(im).to(dev) for im in imgs]
    pairs = sum(pairs_of(im.shape[1], im.shape[0], offs) for im in imgs)
    px = sum(im.size for im in imgs)
    plan = G.glcm_plan_create(np.uint8, N, offs, 512, 512)
    out = torch.empty((T, K, N, N), dtype=torch.uint32, device=dev)
    feats = torch.empty((T, K, 5), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    tiles = G.prepare_tiles(tens, plan)  # the descriptor array a C caller would hold
    aligned = sum(1 for x in tens if (x.data_ptr() % 16 == 0 and x.stride(0) % 16 == 0))
    for _ in range(3):
        G.glcm_batch_compute(tiles, plan, out=out, features=feats, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        G.glcm_batch_compute(tiles, plan, out=out, features=feats, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    batch_wall = (time.perf_counter() - t0) / reps
    batch_dev = e0.elapsed_time(e1) * 1e-3 / reps
    # one launch pair per tile
    out1 = torch.empty_like(out)
    feats1 = torch.empty_like(feats)
    for t in range(min(T, 64)):
        G.glcm_compute(tens[t], N, 0, 255, offs, out=out1[t], plan=plan, stream=stream)
        G.glcm_features(out1[t], out=feats1[t], stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for t in range(T):
        G.glcm_compute(tens[t], N, 0, 255, offs, out=out1[t], plan=plan, stream=stream)
        G.glcm_features(out1[t], out=feats1[t], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    per_wall = time.perf_counter() - t0
    per_dev = e0.elapsed_time(e1) * 1e-3
    # the same batch prepared once and captured in a HIP graph, replayed
    pb = G.PreparedBatch(tiles, plan)
    g_out, g_f = torch.empty_like(out), torch.empty_like(feats)
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        pb.run(out=g_out, features=g_f, stream=side)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        pb.run(out=g_out, features=g_f, stream=side)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    graph_wall = (time.perf_counter() - t0) / reps
    if not (torch.equal(g_out.view(torch.int32), out.view(torch.int32)) and torch.equal(g_f, feats)):
        raise SystemExit("bench: graph-replayed batch differs from glcm_batch_compute")
    del graph
    pb.close()
    # the batch autotuner: every layout timed on this batch, the fastest kept
    default_tuning = plan.batch_tuning.as_dict()
    chosen = plan.batch_autotune(tiles, repeats=3).as_dict()
    a_out, a_f = torch.empty_like(out), torch.empty_like(feats)
    G.glcm_batch_compute(tiles, plan, out=a_out, features=a_f, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        G.glcm_batch_compute(tiles, plan, out=a_out, features=a_f, stream=stream)
    torch.cuda.synchronize()
    tuned_wall = (time.perf_counter() - t0) / reps
    if not (torch.equal(a_out.view(torch.int32), out.view(torch.int32)) and torch.equal(a_f, feats)):
        raise SystemExit("bench: the autotuned batch layout changed the results")
    plan.close()
    a, b = out.view(torch.int32).cpu().numpy(), out1.view(torch.int32).cpu().numpy()
    if not np.array_equal(a, b):
        raise SystemExit("bench: batched counts differ from the per-image calls")
    if not np.array_equal(feats.cpu().numpy(), feats1.cpu().numpy()):
        raise SystemExit("bench: batched statistics differ from the per-image calls")
    got = a.view(np.uint32)
    for t in range(0, T, max(1, T // 64)):
        if not np.array_equal(got[t], oracle.glcm(imgs[t], N, 0, 255, offs)):
            raise SystemExit(f"bench: tile {t} differs from the oracle")
    res = {
        "workload": w["name"], "tiles": T, "pixels": px, "pairs": pairs, "aligned_tiles": aligned,
        "input_sha256": hashlib.sha256("".join(synth.sha256(im) for im in imgs).encode()).hexdigest(),
        "batched_gpairs_s": pairs / batch_wall / 1e9, "batched_ms": batch_wall * 1e3,
        "batched_device_ms": batch_dev * 1e3,
        "per_image_gpairs_s": pairs / per_wall / 1e9, "per_image_ms": per_wall * 1e3,
        "per_image_device_ms": per_dev * 1e3, "batched_over_per_image": per_wall / batch_wall,
        "graph_replay_ms": graph_wall * 1e3, "graph_replay_gpairs_s": pairs / graph_wall / 1e9,
        "default_layout": default_tuning, "autotuned_layout": chosen, "autotuned_ms": tuned_wall * 1e3,
        "autotuned_gpairs_s": pairs / tuned_wall / 1e9,
        "features": True, "check": "batched == per-image calls == graph replay (counts and statistics); "
                                   "64 tiles vs oracle"}
    if print_line:
        print(json.dumps(res), flush=True)
    return res


def time_oracle(fn, seconds):
    reps, t0 = 0, time.perf_counter()
    while True:
        fn()
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return reps, el


def bench_large_n(args, G, torch, np, oracle, synth, dev):
    """GLCMs too large for one workgroup's LDS: 4096x4096 uint8 smooth and
    noise images at N = 256 with all 12 offsets (d = 1, 2, 4) and N = 1024
    with 2, N = 1536 with 1, each with the plan's default path (bin
    partitions over several image passes, or pairs added straight into the
    per-XCD L2 slices).  Every configuration's counts are checked bit-exact
    against the oracle; times are HIP events around `steps` calls."""
    all12 = synth.offsets_for([1, 2, 4])
    cases = [(256, all12), (1024, all12[:2]), (1536, all12[:1])]
    stream = torch.cuda.current_stream()
    rows, pairs_total, ms_total = [], 0, 0.0
    steps = max(1, min(args.steps, 50))
    for kind in ("smooth", "uniform"):
        img = synth.square_4096(kind)["images"][0]
        H, W = img.shape
        t = torch.from_numpy(img).to(dev)
        for N, offs in cases:
            plan = G.glcm_plan_create(np.uint8, N, offs, W, H)
            tun = plan.tuning
            out = torch.empty((len(offs), N, N), dtype=torch.int32, device=dev)
            print(f"[large_n] {kind} N={N} K={len(offs)} path={G.PATH_NAMES[tun.path]}", flush=True)
            for _ in range(min(args.warmup, 5)):
                G.glcm_compute(t, N, 0, 255, offs, out=out, stream=stream, plan=plan)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                G.glcm_compute(t, N, 0, 255, offs, out=out, stream=stream, plan=plan)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            want = oracle.glcm(img, N, 0, 255, offs)
            if not np.array_equal(out.cpu().numpy().view(np.uint32), want):
                raise SystemExit(f"bench: large-N counts differ from the oracle ({kind}, N={N}, K={len(offs)})")
            pairs = int(want.sum(dtype=np.uint64))
            pairs_total += pairs
            ms_total += ms
            passes = tun.partitions if tun.counter_bits == 32 else (tun.partitions + 1) // 2
            rows.append({"image": kind, "N": N, "K": len(offs), "path": G.PATH_NAMES[tun.path],
                         "image_passes": passes if tun.path == 2 else 1, "counter_bits": tun.counter_bits,
                         "ms": ms, "gpairs_s": pairs / (ms * 1e-3) / 1e9})
            plan.close()
    print(json.dumps({
        "metric": "large-N GLCM Gpairs/s (bit-exact)", "value": pairs_total / (ms_total * 1e-3) / 1e9,
        "unit": "Gpairs/s", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 5), "ms_per_step": ms_total,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "4096x4096-u8-smooth+noise-N256K12-N1024K2-N1536K1", "resident": "device"},
        "roofline": None, "cpu_baseline": None,
        "extra": {"cases": rows, "check": "every case bit-exact against the oracle"},
    }), flush=True)


def bench_histogram(args, G, torch, np, oracle, synth, dev):
    """1-D histogram of the 4096x4096 uint8 smooth image (N = 32 levels, also
    N = 256 in `extra`): copies rotated through HBM as for the GLCM line, every
    copy's result checked bit-exact against the oracle.  The roofline prices
    the histogram kernel (image once + N counts) over its kernel-stamped
    average duration; the call also runs the partial reduction."""
    w = synth.square_4096(args.kind)
    img = w["images"][0]
    H, W = img.shape
    base = torch.from_numpy(img).to(dev)
    copies = [base.clone() for _ in range(args.copies)]
    stream = torch.cuda.current_stream()
    res = {}
    for N in (32, 256):
        want = oracle.histogram(img, N, 0, 255)
        outs = [torch.empty(N, dtype=torch.uint32, device=dev) for _ in copies]
        for flags in (0, G.FLAG_TIMING):
            plan = G.glcm_plan_create(np.uint8, N, [(0, 0)], W, H, flags)
            for i in range(args.warmup):
                G.glcm_histogram(copies[i % len(copies)], N, 0, 255, out=outs[i % len(copies)], stream=stream,
                                 plan=plan)
            torch.cuda.synchronize()
            if flags:
                plan.kernel_time()
            t0 = time.perf_counter()
            for i in range(args.steps):
                G.glcm_histogram(copies[i % len(copies)], N, 0, 255, out=outs[i % len(copies)], stream=stream,
                                 plan=plan)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            if flags:
                ms, n = plan.kernel_time()
                res[N]["kernel_ms"] = ms / n
            else:
                res[N] = {"wall_ms": wall * 1e3}
            plan.close()
        for j in range(min(len(copies), args.steps)):
            if not np.array_equal(outs[j].view(torch.int32).cpu().numpy().view(np.uint32), want):
                raise SystemExit(f"bench: histogram of copy {j} differs from the oracle (N={N})")
    px = W * H
    r = res[32]
    nbytes = px + 32 * 4
    achieved = nbytes / (r["kernel_ms"] * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu:
        reps, el = time_oracle(lambda: oracle.histogram(img, 32, 0, 255), args.cpu_seconds)
        cpu = {"value": reps * px / el / 1e9, "unit": "Gpixels/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full passes over the 4096x4096 {args.kind} image, N=32, single-threaded C oracle, "
                         f"{el:.1f} s; host {host_cpu()}"}
    print(json.dumps({
        "metric": "histogram Gpixels/s (bit-exact)", "value": px / (r["wall_ms"] * 1e-3) / 1e9, "unit": "Gpixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["wall_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"histogram-4096x4096-u8-{args.kind}-N32", "resident": "device"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_hist_traffic()},
        "cpu_baseline": cpu,
        "extra": {"input_sha256": synth.sha256(img), "kernel_ms_n32": r["kernel_ms"], "wall_ms_n256": res[256]["wall_ms"],
                  "kernel_ms_n256": res[256]["kernel_ms"],
                  "gpixels_s_n256": px / (res[256]["wall_ms"] * 1e-3) / 1e9, "copies_rotated": len(copies)},
    }), flush=True)


def bench_variants(args, G, torch, np, oracle, synth, dev, reps=50):
    """The post-processing kernels on 16384 GLCM-like matrices of N = 16 (the
    output shape of the 4096-tile batch): symmetric, normalised and
    direction-averaged (m = 4) matrices and the thirteen Haralick statistics.
    Each kernel is timed with events around its own launch; every output is
    checked against the oracle (bit for bit, statistics within 1e-5 rel +
    1e-6 abs)."""
    w = synth.glcm_like_counts()
    P = w["counts"]
    K, N = P.shape[0], P.shape[1]
    t = torch.from_numpy(P.view(np.int32)).to(dev).view(torch.uint32)
    stream = torch.cuda.current_stream()
    sym = torch.empty_like(t)
    nrm = torch.empty((K, N, N), dtype=torch.float32, device=dev)
    avg = torch.empty((K // 4, N, N), dtype=torch.float32, device=dev)
    har = torch.empty((K, 13), dtype=torch.float32, device=dev)
    mcc = torch.empty(K, dtype=torch.float32, device=dev)
    calls = {
        "symmetrize": (lambda: G.glcm_symmetrize(t, out=sym, stream=stream), 2 * K * N * N * 4),
        "normalize": (lambda: G.glcm_normalize(t, out=nrm, stream=stream), 2 * K * N * N * 4),
        "average": (lambda: G.glcm_average(t, 4, out=avg, stream=stream), K * N * N * 4 + K // 4 * N * N * 4),
        "haralick": (lambda: G.glcm_haralick(t, out=har, stream=stream), K * N * N * 4 + K * 13 * 4),
        "haralick_mcc": (lambda: G.glcm_haralick_mcc(t, out=mcc, stream=stream), K * N * N * 4 + K * 4),
    }
    timing = {}
    for name, (fn, nbytes) in calls.items():
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        timing[name] = {"ms": ms, "gb_s": nbytes / (ms * 1e-3) / 1e9, "matrices_per_s": K / (ms * 1e-3)}
    host = lambda x: x.view(torch.int32).cpu().numpy().view(np.uint32) if x.dtype == torch.uint32 else x.cpu().numpy()
    if not np.array_equal(host(sym), oracle.symmetric(P)):
        raise SystemExit("bench: symmetric matrices differ from the oracle")
    if not np.array_equal(host(nrm), oracle.normalize(P).astype(np.float32)):
        raise SystemExit("bench: normalised matrices differ from the oracle")
    if not np.array_equal(host(avg), oracle.average(P, 4).astype(np.float32)):
        raise SystemExit("bench: averaged matrices differ from the oracle")
    want = oracle.haralick(P)
    if (np.abs(host(har).astype(np.float64) - want) > 1e-5 * np.abs(want) + 1e-6).any():
        raise SystemExit("bench: Haralick statistics differ from the oracle")
    wm = oracle.haralick_mcc(P[:1024])  # the maximal correlation coefficient on the first 1024 matrices
    if (np.abs(host(mcc)[:1024].astype(np.float64) - wm) > 1e-5 * np.abs(wm) + 1e-6).any():
        raise SystemExit("bench: maximal correlation coefficients differ from the oracle")
    cpu = None
    if not args.no_cpu:
        sample = P[:2048]
        reps_c, el = time_oracle(lambda: oracle.haralick(sample), args.cpu_seconds)
        cpu = {"value": reps_c * len(sample) / el, "unit": "matrices/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps_c} passes of the C oracle's f1..f13 over the first {len(sample)} matrices, "
                         f"{el:.1f} s; host {host_cpu()}"}
    h = timing["haralick"]
    valu = recorded_haralick_valu()
    if valu:
        achieved = valu / (h["ms"] * 1e-3) / 1e9
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_G, "unit": "G VALU wave-instr/s",
                "frac": achieved / VALU_PEAK_G, "traffic": None,
                "note": f"{valu} VALU wave-instructions per launch (committed counters) over the measured duration; "
                        f"HBM rate {h['gb_s']:.0f} GB/s"}
    else:
        roof = {"bound": "hbm", "achieved": h["gb_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": h["gb_s"] / HBM_PEAK_GBS, "traffic": None}
    print(json.dumps({
        "metric": "Haralick f1..f13 matrices/s (within 1e-5 of the fp64 oracle)", "value": h["matrices_per_s"],
        "unit": "matrices/s", "n_gpus": 1, "steps": reps, "warmup": 5, "ms_per_step": h["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w["name"], "matrices": K, "levels": N, "resident": "device"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": {"input_sha256": synth.sha256(P), "kernels": timing, "check": "symmetric, normalised, averaged bit-exact; statistics within tolerance"},
    }), flush=True)


def bench_multispectral(args, G, torch, np, oracle, synth, dev):
    """8 bands of 8192^2 uint16 (N = 64 over [0, 65535], d in {1, 2, 4} x four
    angles): device-resident counting, the host-to-device copy alone, and the
    whole job from pinned host memory streamed in row tiles (upload of tile
    t+1 overlapping the count of tile t) versus uploaded and counted
    serially.  Band 0 is checked against the oracle bin for bin, every band by
    its per-offset totals."""
    offs = synth.offsets_for([1, 2, 4])
    N, size, bands = 64, args.size, args.bands
    hosts, imgs = [], []
    for b in range(bands):
        img, sigma = synth.multispectral_band(b, size)
        imgs.append(img)
        hosts.append(torch.from_numpy(img.view(np.int16)).pin_memory().view(torch.uint16))
        print(f"[multispectral] band {b} generated (sigma {sigma:.1f})", file=sys.stderr, flush=True)
    pairs_band = pairs_of(size, size, offs)
    pairs = pairs_band * bands
    stream = torch.cuda.current_stream()
    outs = [torch.empty((len(offs), N, N), dtype=torch.uint32, device=dev) for _ in range(bands)]

    def run(plan, srcs):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for b in range(bands):
            G.glcm_compute(srcs[b], N, 0, 65535, offs, out=outs[b], plan=plan, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1) * 1e-3

    def verify(label):
        want_tot = [max(0, size - abs(dx)) * max(0, size - abs(dy)) for dx, dy in offs]
        for b in range(bands):
            got = outs[b].view(torch.int32).cpu().numpy().view(np.uint32)
            if [int(got[k].sum(dtype=np.uint64)) for k in range(len(offs))] != want_tot:
                raise SystemExit(f"bench: multispectral band {b} totals wrong ({label})")
        got0 = outs[0].view(torch.int32).cpu().numpy().view(np.uint32)
        if not np.array_equal(got0, want0):
            raise SystemExit(f"bench: multispectral band 0 differs from the oracle ({label})")

    want0 = oracle.glcm(imgs[0], N, 0, 65535, offs)
    print("[multispectral] oracle for band 0 done", file=sys.stderr, flush=True)
    plan = G.glcm_plan_create(np.uint16, N, offs, size, size)
    plan_serial = G.glcm_plan_create(np.uint16, N, offs, size, size, G.FLAG_SERIAL_UPLOAD)
    if args.path == "blocks":
        raise SystemExit("bench: the block-code kernel takes the d = 1 offsets only")
    if args.path == "strips":
        # the strip kernel's reach-4 variant instead of the slab default
        # (4 dwords per bin in 16-bit pairs, 512 threads unless --layout says)
        R, bits, wg = (int(v) for v in args.layout.split(",")) if args.layout else (4, 16, 512)
        for p in (plan, plan_serial):
            p.set_tuning(path=4, replicas=R, counter_bits=bits, wg_size=wg)
    devs = [h.to(dev) for h in hosts]
    run(plan, devs)  # warm-up (workspace, code objects)
    _, t_dev = run(plan, devs)
    verify("device")
    # the copy alone: every band pinned -> device on the stream
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for b in range(bands):  # byte views: a plain DMA copy whatever the element type
        devs[b].view(torch.uint8).copy_(hosts[b].view(torch.uint8), non_blocking=True)
    c1.record(stream)
    torch.cuda.synchronize()
    t_copy = c0.elapsed_time(c1) * 1e-3
    del devs
    run(plan, hosts)
    wall_stream, _ = run(plan, hosts)
    verify("streamed")
    run(plan_serial, hosts)
    wall_serial, _ = run(plan_serial, hosts)
    verify("serial")
    tiles = plan.tuning.tile_rows
    tuning = plan.tuning.as_dict()
    plan.close()
    plan_serial.close()
    nbytes = bands * size * size * 2
    print(json.dumps({
        "workload": f"{bands}x{size}x{size}-u16-multispectral-N64-K12", "pairs": pairs, "bytes": nbytes,
        "device_resident_gpairs_s": pairs / t_dev / 1e9, "device_resident_ms": t_dev * 1e3,
        "h2d_only_ms": t_copy * 1e3, "h2d_gbs": nbytes / t_copy / 1e9,
        "streamed_ms": wall_stream * 1e3, "streamed_gpairs_s": pairs / wall_stream / 1e9,
        "serial_ms": wall_serial * 1e3, "serial_gpairs_s": pairs / wall_serial / 1e9,
        "streamed_over_serial": wall_serial / wall_stream,
        "h2d_share_of_serial": t_copy / wall_serial, "tile_rows": tiles, "tuning": tuning,
        "resident": "pinned host", "check": "band 0 bit-exact vs oracle; all bands per-offset totals"}), flush=True)


def served_bound(reqs, alone_ms, t_sync, t_closed):
    """How far any server can get above one request at a time on this mix.
    A request of side >= 4096 (16 Mi pixels) keeps every CU busy by itself
    for most of its run (its counting kernels launch hundreds of 512-1024
    thread workgroups per image pass), so such requests cannot together run
    much faster than one after the other: their summed device time alone is
    close to a floor under any schedule's wall time.  For side >= 2048 the
    same sum is only indicative (the measured server beats it: those kernels
    leave CUs idle at their ends, which other requests fill)."""
    out = {"requests_alone_device_ms": sum(alone_ms), "one_at_a_time_ms": t_sync * 1e3, "served_ms": t_closed * 1e3}
    for side in (2048, 4096):
        big = [ms for r, ms in zip(reqs, alone_ms) if r["side"] >= side]
        out[f"side_ge_{side}"] = {"requests": len(big), "device_ms": sum(big),
                                  "one_at_a_time_over_it": t_sync * 1e3 / sum(big) if big else None}
    return out


def bench_serving(args, G, torch, np, oracle, synth, dev):
    """The serving workload: requests are square crops (side uniform in
    [256, 8192]) of a smooth or a noise 8192^2 pool image, N from {8, 16, 32,
    64, 256}, a random non-empty subset of the 12 offsets, statistics with
    probability 1/2.  Measures (a) one request at a time on one stream,
    waiting for each (a plain request loop), (b) all requests queued on one
    stream, (c) the request server with every request submitted at once
    (closed-loop capacity) and (d) Poisson arrivals at 0.5x and 0.9x that
    capacity, with p50/p99 latency from arrival to completion.  Every served
    result must equal the one-at-a-time result bit for bit; 16 small requests
    are also checked against the oracle."""
    all12 = synth.offsets_for([1, 2, 4])
    pool = synth.serving_pool(args.size)
    pool_dev = {k: torch.from_numpy(v).to(dev) for k, v in pool.items()}
    reqs = synth.serving_requests(args.requests, args.size)
    views = [pool_dev[r["kind"]][r["y0"]:r["y0"] + r["side"], r["x0"]:r["x0"] + r["side"]] for r in reqs]
    pairs = [pairs_of(r["side"], r["side"], r["offsets"]) for r in reqs]
    total_pairs = float(sum(pairs))
    print(f"[serving] {len(reqs)} requests, {total_pairs:.3g} pairs", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    outs = [torch.empty((len(r["offsets"]), r["N"], r["N"]), dtype=torch.uint32, device=dev) for r in reqs]
    feats = [torch.empty((len(r["offsets"]), 5), dtype=torch.float32, device=dev) if r["features"] else None
             for r in reqs]
    plans = {N: G.glcm_plan_create(np.uint8, N, all12, args.size, args.size) for N in sorted({r["N"] for r in reqs})}

    def one_stream(sync):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r, v, o, f in zip(reqs, views, outs, feats):
            p = plans[r["N"]]
            G.glcm_plan_rebind(p, r["offsets"])
            G.glcm_compute(v, r["N"], 0, 255, r["offsets"], out=o, plan=p, stream=stream)
            if f is not None:
                G.glcm_features(o, out=f, stream=stream)
            if sync:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def by_n():
        """Device time and counting path of each request alone, summed per N."""
        torch.cuda.synchronize()
        evs = []
        for r, v, o, f in zip(reqs, views, outs, feats):
            p = plans[r["N"]]
            G.glcm_plan_rebind(p, r["offsets"])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            G.glcm_compute(v, r["N"], 0, 255, r["offsets"], out=o, plan=p, stream=stream)
            if f is not None:
                G.glcm_features(o, out=f, stream=stream)
            e1.record(stream)
            aligned = v.data_ptr() % 16 == 0 and v.stride(0) % 16 == 0
            path = G.PATH_NAMES.get(p.tuning.path, "?")
            if not aligned and path in ("strips", "slabs"):
                path = (f"{path} (read in place)" if v.shape[0] * v.shape[1] >= 1 << 16
                        else "generic (misaligned)")
            evs.append((r["N"], path, e0, e1))
        torch.cuda.synchronize()
        agg = {}
        alone.clear()
        for (N, path, e0, e1), pr in zip(evs, pairs):
            a = agg.setdefault(str(N), {"requests": 0, "pairs": 0, "ms": 0.0, "paths": {}})
            a["requests"] += 1
            a["pairs"] += pr
            a["ms"] += e0.elapsed_time(e1)
            a["paths"][path] = a["paths"].get(path, 0) + 1
            alone.append(e0.elapsed_time(e1))
        for a in agg.values():
            a["gpairs_s"] = a["pairs"] / (a["ms"] * 1e-3) / 1e9
        return agg

    alone = []  # device ms of each request alone (counts + statistics)
    one_stream(False)  # warm-up
    per_n = by_n()
    print(f"[serving] per N: {json.dumps(per_n)}", file=sys.stderr, flush=True)
    t_sync = one_stream(True)
    t_stream = one_stream(False)
    print(f"[serving] one at a time {t_sync * 1e3:.1f} ms, one stream {t_stream * 1e3:.1f} ms",
          file=sys.stderr, flush=True)
    # oracle on 16 small requests (bit-exact counts)
    small = sorted(range(len(reqs)), key=lambda i: reqs[i]["side"])[:16]
    for i in small:
        r = reqs[i]
        img = pool[r["kind"]][r["y0"]:r["y0"] + r["side"], r["x0"]:r["x0"] + r["side"]]
        want = oracle.glcm(img, r["N"], 0, 255, r["offsets"])
        if not np.array_equal(outs[i].view(torch.int32).cpu().numpy().view(np.uint32), want):
            raise SystemExit(f"bench: request {i} differs from the oracle")

    srv = G.Server(lanes=args.lanes, hbm_budget=args.budget_gib << 30, result_pool_bytes=min(4 << 30, args.budget_gib << 29))

    def submit_all(arrivals=None):
        tickets, lags = [], []
        t0 = time.perf_counter()
        for i, (r, v) in enumerate(zip(reqs, views)):
            if arrivals is not None:
                due = t0 + arrivals[i]
                while True:
                    now = time.perf_counter()
                    if now >= due:
                        break
                    if due - now > 2e-3:
                        time.sleep(due - now - 1e-3)
                lags.append(max(0.0, time.perf_counter() - due))
            tickets.append(srv.submit(v, r["N"], 0, 255, r["offsets"], features=r["features"]))
        srv.drain()
        wall = time.perf_counter() - t0
        infos = [srv.query(t) for t in tickets]
        return tickets, infos, lags, wall

    def explain(i, P):
        """Which side of a mismatch agrees with the oracle, and by how much the other is off."""
        r = reqs[i]
        img = pool[r["kind"]][r["y0"]:r["y0"] + r["side"], r["x0"]:r["x0"] + r["side"]]
        want = oracle.glcm(img, r["N"], 0, 255, r["offsets"]).astype(np.int64)
        got = {"served": P.view(torch.int32).cpu().numpy().view(np.uint32).astype(np.int64),
               "alone": outs[i].view(torch.int32).cpu().numpy().view(np.uint32).astype(np.int64)}
        parts = []
        for name, g in got.items():
            d = g - want
            per_k = [(tuple(r["offsets"][k]), int(np.count_nonzero(d[k])), int(d[k].sum())) for k in range(len(d))
                     if d[k].any()]
            parts.append(f"{name}: {'== oracle' if not d.any() else f'differs (offset, bins, count delta) {per_k}'}")
        return (f"request {i} N={r['N']} side={r['side']} K={len(r['offsets'])} ptr%16={views[i].data_ptr() % 16}: "
                + "; ".join(parts))

    def check_and_release(tickets, infos):
        bad = []
        for i, (t, info) in enumerate(zip(tickets, infos)):
            if info.status != 0:
                raise SystemExit(f"bench: served request {i} failed with status {info.status}")
            P, F = srv.fetch(t)
            if not torch.equal(P.view(torch.int32), outs[i].view(torch.int32)):
                bad.append(explain(i, P))
                print(f"[serving] MISMATCH {bad[-1]}", file=sys.stderr, flush=True)
            elif F is not None and not torch.equal(F, feats[i]):
                bad.append(f"statistics of request {i}")
            srv.release(t)
        if bad:
            raise SystemExit(f"bench: {len(bad)} served results differ from the same requests alone")

    tk, inf, _, _ = submit_all()  # warm-up: every lane gets its plans
    check_and_release(tk, inf)
    tk, inf, _, t_closed = submit_all()
    check_and_release(tk, inf)
    capacity = len(reqs) / t_closed
    print(f"[serving] closed loop {t_closed * 1e3:.1f} ms, capacity {capacity:.0f} req/s", file=sys.stderr, flush=True)
    open_loop = []
    g = np.random.default_rng(171006189 + 40)
    for load in (0.5, 0.9):
        qps = load * capacity
        arrivals = np.cumsum(g.exponential(1.0 / qps, size=len(reqs)))
        arrivals -= arrivals[0]
        tk, inf, lags, wall = submit_all(arrivals)
        lat_ms = np.array([(i.done_us - i.submit_us) / 1e3 + lag * 1e3 for i, lag in zip(inf, lags)])
        check_and_release(tk, inf)
        open_loop.append({"load": load, "offered_qps": qps, "achieved_qps": len(reqs) / wall,
                          "gpairs_s": total_pairs / wall / 1e9, "p50_ms": float(np.percentile(lat_ms, 50)),
                          "p99_ms": float(np.percentile(lat_ms, 99)), "max_submit_lag_ms": float(max(lags) * 1e3)})
        print(f"[serving] load {load}: p50 {open_loop[-1]['p50_ms']:.3f} ms p99 {open_loop[-1]['p99_ms']:.3f} ms",
              file=sys.stderr, flush=True)
    st = srv.stats()
    srv.close()
    for p in plans.values():
        p.close()
    tile_stream = serve_tile_stream(args, G, torch, np, synth, dev)
    line = {"workload": f"serving-{len(reqs)}-requests-u8-256to{args.size}-N8to256-K1to12",
            "requests": len(reqs), "pairs": total_pairs, "lanes": args.lanes, "hbm_budget_gib": args.budget_gib,
            "one_at_a_time_gpairs_s": total_pairs / t_sync / 1e9, "one_stream_gpairs_s": total_pairs / t_stream / 1e9,
            "served_closed_loop_gpairs_s": total_pairs / t_closed / 1e9, "capacity_req_s": capacity,
            "served_over_one_at_a_time": t_sync / t_closed, "served_over_one_stream": t_stream / t_closed,
            "open_loop": open_loop, "max_inflight": st.max_inflight, "alone_by_N": per_n,
            "served_bound": served_bound(reqs, alone, t_sync, t_closed),
            "max_budgeted_gib": st.max_bytes_in_use / 2 ** 30,
            "fused_launches": st.fused_launches, "fused_requests": st.fused_requests,
            "tile_stream": tile_stream,
            "check": "every served result == the same request alone (counts and statistics, bit for bit); "
                     "16 smallest requests == oracle"}
    print(json.dumps(line), flush=True)


def serve_tile_stream(args, G, torch, np, synth, dev):
    """The batch workload's tiles (sides log-uniform in [32, 512], N = 16, the
    four d = 1 offsets, statistics) as one request each: the request server,
    which fuses queued requests of one job into batch launches, against one
    request at a time (counts, then statistics, then a wait) and against all
    of them queued on one stream.  Every served result must equal the request
    alone, bit for bit."""
    w = synth.batch_tiles(args.tiles)
    N, offs = w["N"], w["offsets"]
    imgs = [torch.from_numpy(im).to(dev) for im in w["images"]]
    K = len(offs)
    outs = [torch.empty((K, N, N), dtype=torch.uint32, device=dev) for _ in imgs]
    feats = [torch.empty((K, 5), dtype=torch.float32, device=dev) for _ in imgs]
    stream = torch.cuda.current_stream()
    plan = G.glcm_plan_create(np.uint8, N, offs, 512, 512)

    def one_by_one(sync):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for im, o, f in zip(imgs, outs, feats):
            G.glcm_compute(im, N, 0, 255, offs, out=o, plan=plan, stream=stream)
            G.glcm_features(o, out=f, stream=stream)
            if sync:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    one_by_one(False)  # warm-up
    t_sync, t_stream = one_by_one(True), one_by_one(False)
    plan.close()
    srv = G.Server(lanes=args.lanes, hbm_budget=8 << 30, result_pool_bytes=1 << 30)

    def served():
        torch.cuda.synchronize()
        # (the collector stays off while the requests are handed over: with
        # the other legs' objects alive its passes would be what is timed)
        gc.disable()
        try:
            t0 = time.perf_counter()
            tickets = [srv.submit(im, N, 0, 255, offs, features=True) for im in imgs]
            t_sub = time.perf_counter() - t0
            srv.drain()
            wall = time.perf_counter() - t0
        finally:
            gc.enable()
        served.submit_s = t_sub
        infos = [srv.query(t) for t in tickets]
        for i, (t, info) in enumerate(zip(tickets, infos)):
            if info.status != 0:
                raise SystemExit(f"bench: tile request {i} failed with status {info.status}")
            P, F = srv.fetch(t)
            if not (torch.equal(P.view(torch.int32), outs[i].view(torch.int32)) and torch.equal(F, feats[i])):
                raise SystemExit(f"bench: served tile {i} differs from the request alone")
            srv.release(t)
        return wall, infos

    served()  # warm-up: the lanes' plans
    before = srv.stats()
    t_served, infos = served()
    st = srv.stats()
    srv.close()
    launches = st.fused_launches - before.fused_launches
    fused = st.fused_requests - before.fused_requests
    res = {"workload": f"{len(imgs)}-tile-requests-u8-32to512-N16-K4-features", "requests": len(imgs),
           "one_at_a_time_ms": t_sync * 1e3, "one_stream_ms": t_stream * 1e3, "served_ms": t_served * 1e3,
           "served_over_one_at_a_time": t_sync / t_served, "served_over_one_stream": t_stream / t_served,
           "submit_ms": served.submit_s * 1e3, "fused_launches": launches, "fused_requests": fused,
           "mean_requests_per_fused_launch": fused / launches if launches else 0.0,
           "largest_fused_launch": max(i.fused for i in infos)}
    print(f"[serving] tile stream: {json.dumps(res)}", file=sys.stderr, flush=True)
    return res


if __name__ == "__main__":
    main()
