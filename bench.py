#!/usr/bin/env python3
"""Benchmark of the LoG feature-extraction pipeline (liblogfx) on one MI355X.

One step = one full pass of the pipeline over one image already resident in
HBM: pass 1 (both LoG responses, zero crossings, per-tile sums, the
crossing-strength pair of every pixel stored), the finalize kernel (global
deviation, thresholds) and pass 2 (3x3 deviation test on the stored
strengths, OR, 5x5 hybrid median, output map).

Workload (default): the 8192 x 8192 11-bit scene -- 20000 rectangles, 500
polylines of width 1-3, Gaussian noise sigma 12, 5 % salt-and-pepper --
with masks 5x5 sigma 0.8 and 9x9 sigma 1.4, threshold 2.0 x the global
deviation and the 5x5 hybrid median.  Three copies of the input are rotated
so the 256 MB last-level cache cannot serve a step from the previous one.
The timed region holds the K steps only; per-kernel times, the spread of
single steps, the FP64 path, the 512^2 latency and the host transfers are
measured after it.

Prints one JSON line (see the keys below).  Progress goes to stderr.

--workload gated: the smoothing gate's workload instead -- four 16384^2
11-bit bands cut into 256 tiles of 2048^2, each tile with its own noise,
run as one batch per step with the gate choosing the median per tile
(SMOOTH_GATE, parameters from paper_1304_3992_amd/gate_weights.bin), next to
the same batch always smoothed and never smoothed; the agreement of each
output with the oracle's best-choice output is computed from the stored
oracle labels (tests/golden/config5_labels.npz).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "Mpixel/s full pipeline, % HBM roofline; gated vs plain at >=99.9% agreement"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one 32-bit VALU lane
# operation per lane per clock.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# The same lane rate as multiply-adds counted as two operations: MI355X's
# published FP64 vector peak (78.6 TFLOP/s); the exact int32 path issues its
# multiply-adds (v_mad_i32_i24, v_dot2_i32_i16 two per lane) at that rate.
ALU_PEAK_TFLOPS = 2 * VALU_PEAK_TOPS
# The pipeline's arithmetic per pixel as the method states it: the two
# direct-form LoG masks of eq. (1), 5x5 and 9x9, 25 + 81 multiply-adds.
LOG_FMA_PER_PX = 106

# Algorithmic ALU operations per output pixel of the recomputing pass 2
# (LOGFX_OPT_STORE_Z = 0: LoG and crossings again, then the deviation), counted
# for the exact orbit-form evaluation the library uses (no halo
# recomputation, no address or loop bookkeeping).  For masks of radius 2 and
# 4 (15 orbits, 6 of them shared by the 5x5 mask):
PASS2_OPS = {
    "pair sums of the 9 taps of a row (4) + row-pair sums (20) + orbit sums (10)": 34,
    "orbit multiply-adds, 6 + 15": 21,
    "zero crossing and strength per mask: 4-neighbour max/min (6), sign tests and "
    "tie rule (6), zero-pixel rule (8), range and threshold (5)": 2 * 25,
    "3x3 deviation per mask: column sums of z and z^2 (5), row sums (4), "
    "9Q - S^2 (2), compare (1)": 2 * 12,
    "OR, output bit, store": 3,
}
PASS2_OPS_PER_PX = sum(PASS2_OPS.values())
# Pass 2 on stored strengths: the deviation (row sums 5, column sums 4,
# 9Q - S^2 2, compare 1 per mask), OR, output.
PASS2Z_OPS_PER_PX = 2 * 12 + 3

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
# (scaled by a plain copy of known size; profiles/pipeline_kernels_8192x8192_u16.md)
# for the kernel sources with this hash and these strip heights.  Reported
# only while both are unchanged.
TRAFFIC_SOURCE_HASH = "c8be2f8aa4a3120f"
TRAFFIC_ROWS = [64, 32]
TRAFFIC_BYTES = {"pass1_kernel": (67492 * 2.0 + 524819 * 1.0) * 1024,
                 "pass2z_kernel": (270230 * 2.0 + 66880 * 1.0) * 1024}
# Algorithmic HBM bytes per pixel of each kernel: pass 1 reads the 16-bit
# image and writes the (Z_1, Z_2) int32 pair; pass 2 reads the pair and
# writes the output byte.
KERNEL_BYTES_PER_PX = {"pass1_kernel": 2 + 8, "pass2z_kernel": 8 + 1}


# The sources the pipeline kernels (pass 1, finalize, pass 2) are compiled
# from; the gate network's files do not take part.
PIPELINE_SOURCES = ("logfx_bits.h", "logfx_dispatch.hip", "logfx_internal.h", "logfx_kernels.h",
                    "logfx_kernels_inst.hip", "logfx_pass2z.hip")


def kernel_source_hash() -> str:
    import hashlib
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1304_3992_amd", "csrc")
    h = hashlib.sha256()
    for f in (os.path.join(here, n) for n in PIPELINE_SOURCES):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cores() -> int:
    """Threads the CPU work may use: the cores this process may run on,
    limited to the job's CPU share when the environment states one
    (OMP_NUM_THREADS; a GPU job of this machine pool gets 16 host threads
    per GPU, whatever the host's core count)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS", "")
    if share.isdigit() and int(share) > 0:
        n = min(n, int(share))
    return max(1, n)


def cpu_info() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"model": model, "nproc": os.cpu_count(), "affinity": affinity,
            "job_share": os.environ.get("OMP_NUM_THREADS")}


# The paper's headline speed-up (Table 7, Sec. 7): its pixel-wise CUDA
# program on a Tesla C2075 against its two-thread pthreads program on an
# 8-core Xeon E5620 (2.4 GHz), AWiFS 2000 x 2000 image: 24500 ms / 1182 ms.
PAPER_SPEEDUP = {"x": round(24500.0 / 1182.0, 1), "gpu": "NVIDIA Tesla C2075",
                 "cpu": "Intel Xeon E5620 (8 cores, 2.4 GHz), 2-thread pthreads program",
                 "image": "AWiFS 2000 x 2000", "source": "Table 7, Sec. 7"}


def cpu_baseline(img, orc_taps, min_seconds: float = 10.0):
    """The oracle, as it stands, on the host cores: whole-scene runs repeated
    until at least min_seconds have passed."""
    import numpy as np
    import oracle
    n = host_cores()
    runs, t0 = 0, time.perf_counter()
    while True:
        oracle.extract(img, orc_taps[0], orc_taps[1], nthreads=n)
        runs += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    res = {"value": runs * img.size / dt / 1e6, "unit": "Mpixel/s", "cores": n, "kind": "oracle",
           "sample": f"whole {img.shape[0]}x{img.shape[1]} scene, {runs} runs, {dt:.1f} s",
           "cpu": cpu_info()}
    # context: one thread on a 2048^2 crop (the paper's CPU program ran one
    # thread per LoG branch, Sec. 6.1)
    crop = np.ascontiguousarray(img[:2048, :2048])
    t0 = time.perf_counter()
    oracle.extract(crop, orc_taps[0], orc_taps[1], nthreads=1)
    res["value_1_thread"] = crop.size / (time.perf_counter() - t0) / 1e6
    res["sample_1_thread"] = f"{crop.shape[0]}x{crop.shape[1]} crop of the scene, 1 run"
    # and two threads, the thread count of the paper's CPU program (the
    # oracle splits rows between them, not LoG branches)
    t0 = time.perf_counter()
    oracle.extract(crop, orc_taps[0], orc_taps[1], nthreads=2)
    res["value_2_threads"] = crop.size / (time.perf_counter() - t0) / 1e6
    return res


def _c5_tile(args):
    import numpy as np
    from paper_1304_3992_amd import scenes
    b, ty, tx = args
    t = scenes.config5_tile(_C5_BASE, b, ty, tx)[0]
    return t, scenes.sha256(t)


_C5_BASE = None


def bench_gated(args):
    """The four-band 16384^2 workload in 2048^2 tiles: gated vs always vs never."""
    import multiprocessing as mp
    import numpy as np
    from paper_1304_3992_amd import scenes
    global _C5_BASE
    root = os.path.dirname(os.path.abspath(__file__))
    t0 = time.time()
    _C5_BASE = scenes.config5_base()
    base_sha = scenes.sha256(_C5_BASE)
    index = scenes.config5_index()
    log(f"base scene {time.time() - t0:.0f} s; generating {len(index)} tiles ...")
    # worker processes are forked before anything touches the GPU
    with mp.get_context("fork").Pool(host_cores()) as pool:
        made = pool.map(_c5_tile, index, chunksize=4)
    _C5_BASE = None
    tiles = [t for t, _ in made]
    tile_shas = [h for _, h in made]
    del made
    log(f"tiles ready ({time.time() - t0:.0f} s)")
    import torch
    from paper_1304_3992_amd import logfx
    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    lib_taps = (logfx.make_log_mask(5, 0.8, 16)[0], logfx.make_log_mask(9, 1.4, 16)[0])
    modes = {"gated": logfx.SMOOTH_GATE, "always": logfx.SMOOTH_ALWAYS, "never": logfx.SMOOTH_NEVER}
    devs = [torch.from_numpy(t.view(np.int16)).cuda() for t in tiles]
    outs = [torch.empty(t.shape, dtype=torch.uint8, device="cuda") for t in tiles]
    px = sum(t.size for t in tiles)
    del tiles
    ctx = logfx.Context(0)
    ctx.gate_load(os.path.join(root, "paper_1304_3992_amd", "gate_weights.bin"))
    stream = torch.cuda.current_stream()
    res = {}
    decisions = None
    for name, mode in modes.items():
        params = logfx.Params(*lib_taps, smooth=mode)
        if not args.no_tune:   # each mode at its own best launch (strip heights, persistence)
            tuned = ctx.tune(devs, params, outs, bits=11, reps=3)
            res[f"tuned_{name}"] = {"rows1": tuned["rows1"], "rows2": tuned["rows2"],
                                    "persistent": tuned["persistent"]}
            log(f"{name} tuned: rows {tuned['rows1']}/{tuned['rows2']}, persistent {tuned['persistent']}")
        _, reps = ctx.extract_batch(devs, params, outs, bits=11, report=True)
        if name == "gated":
            decisions = np.array([r["smoothed"] for r in reps], np.int64)
        for _ in range(args.warmup):
            ctx.extract_batch(devs, params, outs, bits=11)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(args.steps):
            ctx.extract_batch(devs, params, outs, bits=11)
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / args.steps
        res[name] = {"ms_per_step": round(ms, 4), "Mpixel_s": round(px / (ms * 1e-3) / 1e6, 1)}
        log(f"{name}: {ms:.3f} ms/step")
    # the gate alone (features + network + decisions)
    params = logfx.Params(*lib_taps, smooth=logfx.SMOOTH_GATE)
    for _ in range(args.warmup):
        ctx.gate(devs, params, bits=11)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        ctx.gate(devs, params, bits=11)
    stop.record(stream)
    torch.cuda.synchronize()
    res["gate_only_ms"] = round(start.elapsed_time(stop) / args.steps, 4)
    # seamless scene mode: the same tiles stitched back into the four
    # 16384^2 bands, one call per band with one global deviation per mask and
    # the gate deciding per 2048^2 region
    n_side = int(round((len(devs) // 4) ** 0.5))
    T = devs[0].shape[0]
    bands = []
    for b in range(4):
        band = [devs[b * n_side * n_side + ty * n_side:b * n_side * n_side + (ty + 1) * n_side]
                for ty in range(n_side)]
        bands.append(torch.cat([torch.cat(row, dim=1) for row in band], dim=0).contiguous())
    ntiles = len(devs)
    del devs
    bouts = [torch.empty(t.shape, dtype=torch.uint8, device="cuda") for t in bands]
    params = logfx.Params(*lib_taps, smooth=logfx.SMOOTH_GATE, gate_region=T)
    if not args.no_tune:
        tuned = ctx.tune(bands[0], params, [bouts[0]], bits=11, reps=3)
        res["tuned_seamless_gated"] = {"rows1": tuned["rows1"], "rows2": tuned["rows2"]}
        log(f"seamless gated tuned: rows {tuned['rows1']}/{tuned['rows2']}")
    seam_dec = []
    for bt, bo in zip(bands, bouts):
        _, rep = ctx.extract(bt, params, bo, bits=11, report=True)
        seam_dec.append(rep["regions_smoothed"])
    for _ in range(args.warmup):
        for bt, bo in zip(bands, bouts):
            ctx.extract(bt, params, bo, bits=11)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        for bt, bo in zip(bands, bouts):
            ctx.extract(bt, params, bo, bits=11)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    res["seamless_gated"] = {"ms_per_step": round(ms, 4), "Mpixel_s": round(px / (ms * 1e-3) / 1e6, 1),
                             "region": T, "smoothed_regions": int(sum(seam_dec))}
    log(f"seamless gated: {ms:.3f} ms/step")
    # the plain always-smoothed form of the same calls, for the gated vs plain comparison
    p_always = logfx.Params(*lib_taps, smooth=logfx.SMOOTH_ALWAYS)
    if not args.no_tune:
        tuned = ctx.tune(bands[0], p_always, [bouts[0]], bits=11, reps=3)
        res["tuned_seamless_always"] = {"rows1": tuned["rows1"], "rows2": tuned["rows2"]}
        log(f"seamless always tuned: rows {tuned['rows1']}/{tuned['rows2']}")
    for _ in range(args.warmup):
        for bt, bo in zip(bands, bouts):
            ctx.extract(bt, p_always, bo, bits=11)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        for bt, bo in zip(bands, bouts):
            ctx.extract(bt, p_always, bo, bits=11)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_a = start.elapsed_time(stop) / args.steps
    res["seamless_always"] = {"ms_per_step": round(ms_a, 4), "Mpixel_s": round(px / (ms_a * 1e-3) / 1e6, 1)}
    log(f"seamless always: {ms_a:.3f} ms/step")
    # the per-region decisions, in the tiles' order
    seam = np.concatenate([ctx.gate(bt, params, bits=11)[1].cpu().numpy() for bt in bands]).astype(np.int64)
    ctx.close()
    agreement = None
    lab_path = os.path.join(root, "tests", "golden", "config5_labels.npz")
    if os.path.exists(lab_path):
        d = np.load(lab_path)
        lab, diff = d["label"].astype(np.int64), d["diff"].astype(np.float64)
        # the stored labels hold only for the tiles they were computed on
        same_tiles = (str(d["base_sha"]) == base_sha and len(d["sha"]) == len(tile_shas)
                      and all(str(a) == b for a, b in zip(d["sha"], tile_shas)))
        if not same_tiles:
            log("the generated tiles differ from those of the stored labels: no agreement figure")
        if same_tiles and len(lab) == len(decisions):
            def agree(dec):
                return float(1.0 - diff[dec != lab].sum() / px)
            agreement = {"gated": agree(decisions), "always": agree(np.ones_like(lab)),
                         "never": agree(np.zeros_like(lab)),
                         "decision_accuracy": float((decisions == lab).mean()),
                         "smoothed_tiles": int(decisions.sum()), "best_smoothed_tiles": int(lab.sum()),
                         # seamless mode against the tiled labels (each tile's own deviation
                         # and borders): an estimate, since the seamless best choice may differ
                         "seamless_gated_est": agree(seam),
                         "seamless_decision_match": float((seam == lab).mean())}
    ms = res["gated"]["ms_per_step"]
    result = {
        "metric": METRIC, "value": res["gated"]["Mpixel_s"], "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "4 bands x 16384^2 uint16 11-bit (gains 0.9/1.0/1.1/0.7, offsets "
                               "0/40/-40/80), 256 tiles of 2048^2 with per-tile noise sigma~U[0,20], "
                               "salt-and-pepper~U[0,0.2]; gated hybrid median",
                   "pixels": px, "tiles": ntiles, "parallelism": "single GPU"},
        "modes": res, "agreement_with_best_choice": agreement,
    }
    print(json.dumps(result), flush=True)


def bench_batch(args):
    """The 64 uneven tiles (sides log-uniform in [256, 4096]) as one batch
    call: the tuner's choice, each launch form, and the same tiles as single
    calls for comparison."""
    import numpy as np
    import torch
    from paper_1304_3992_amd import logfx, scenes
    tiles = scenes.config3()
    px = sum(t.size for t in tiles)
    devs = [torch.from_numpy(t.view(np.int16)).cuda() for t in tiles]
    outs = [torch.empty(t.shape, dtype=torch.uint8, device="cuda") for t in tiles]
    params = logfx.Params(logfx.make_log_mask(5, 0.8, 16)[0], logfx.make_log_mask(9, 1.4, 16)[0])
    ctx = logfx.Context(0)
    stream = torch.cuda.current_stream()
    if args.rows:
        r1, r2 = (int(v) for v in args.rows.split(","))
        ctx.set_option(logfx.OPT_ROWS1, r1)
        ctx.set_option(logfx.OPT_ROWS2, r2)
    if not args.no_tune:
        ctx.tune(devs, params, outs, bits=8, reps=3)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.steps

    ms = timed(lambda: ctx.extract_batch(devs, params, outs, bits=8))
    chosen = {"persistent": ctx.get_option(logfx.OPT_PERSISTENT), "graph": ctx.get_option(logfx.OPT_GRAPH),
              "rows": [ctx.get_option(logfx.OPT_ROWS1), ctx.get_option(logfx.OPT_ROWS2)]}
    forms = {}
    for pers in (0, 1):
        for graph in (0, 1):
            ctx.set_option(logfx.OPT_PERSISTENT, pers)
            ctx.set_option(logfx.OPT_GRAPH, graph)
            forms[f"persistent{pers}_graph{graph}"] = round(
                timed(lambda: ctx.extract_batch(devs, params, outs, bits=8)), 4)
    ctx.set_option(logfx.OPT_PERSISTENT, chosen["persistent"])
    ctx.set_option(logfx.OPT_GRAPH, chosen["graph"])

    def singles():
        for d, o in zip(devs, outs):
            ctx.extract(d, params, o, bits=8)
    single_ms = timed(singles)
    ctx.close()
    log(f"batch: {ms:.3f} ms, single calls: {single_ms:.3f} ms, forms {forms}")
    result = {
        "metric": METRIC, "value": round(px / (ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "64 uint16 tiles, sides log-uniform in [256, 4096] (seed 3), uint8 values, "
                               "40 rectangles per 512^2, noise sigma 4; LoG 5x5 s0.8 + 9x9 s1.4; "
                               "3x3 deviation > 2.0 global per tile; 5x5 hybrid median; one batch call",
                   "pixels": px, "tiles": len(tiles), "parallelism": "single GPU", "launch": chosen},
        "launch_forms_ms": forms,
        "single_calls": {"ms_per_step": round(single_ms, 4),
                         "Mpixel_s": round(px / (single_ms * 1e-3) / 1e6, 1)},
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=8192, help="scene side (8192 = the workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64-path run of the scene after the timed region")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the 512^2 single-call latency after the timed region")
    ap.add_argument("--no-transfers", action="store_true",
                    help="skip the host transfer timing after the timed region")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (strip heights stay at their defaults, or --rows)")
    ap.add_argument("--rows", default="",
                    help="strip heights of pass 1 and pass 2, e.g. 64,32, set before the run of the "
                         "scene or batch workload (with --no-tune: the launch the tuner picks, "
                         "without the tuner's own launches in a profile)")
    ap.add_argument("--store-z", type=int, default=1, choices=[0, 1],
                    help="1: pass 2 reads the strengths pass 1 stored (default); 0: recomputes them")
    ap.add_argument("--median-cascade", default="",
                    help="further hybrid median windows after the first, e.g. 3,5 (default: none)")
    ap.add_argument("--workload", choices=["scene", "gated", "batch"], default="scene",
                    help="scene: the 8192^2 scene (default); gated: the gate's four-band workload; "
                         "batch: 64 uneven tiles in one call")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run 5 plain device copies of this many MiB (a known-size "
                         "kernel for scaling hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the pipeline is "
                                   "measured on a single MI355X", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "gated":
        return bench_gated(args)
    if args.workload == "batch":
        return bench_batch(args)

    import numpy as np
    import torch
    from paper_1304_3992_amd import logfx, scenes

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    log(f"generating scene {args.size}^2 ...")
    img = scenes.config2(size=args.size)
    H, W = img.shape
    lib_taps = (logfx.make_log_mask(5, 0.8, 16)[0], logfx.make_log_mask(9, 1.4, 16)[0])
    cascade = tuple(int(m) for m in args.median_cascade.split(",") if m)
    params = logfx.Params(*lib_taps, std_k=2.0, smooth=True, median_size=5, median_cascade=cascade)

    dev = torch.device("cuda", 0)
    host = torch.from_numpy(img.view(np.int16))
    bufs = [host.to(dev) for _ in range(3)]
    out = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ctx = logfx.Context(0)
    ctx.set_option(logfx.OPT_STORE_Z, args.store_z)
    stream = torch.cuda.current_stream()

    tuned = None
    if args.rows:
        r1, r2 = (int(v) for v in args.rows.split(","))
        ctx.set_option(logfx.OPT_ROWS1, r1)
        ctx.set_option(logfx.OPT_ROWS2, r2)
    if not args.no_tune:
        # untimed: pick the strip heights of both passes for this workload
        tuned = ctx.tune(bufs[0], params, [out], bits=11, reps=3)
        log(f"tuned rows: pass 1 {tuned['rows1']}, pass 2 {tuned['rows2']}")
    # one reported call to learn the arithmetic path
    _, rep = ctx.extract(bufs[0], params, out, bits=11, report=True)
    log(f"path={'int32' if rep['path'] == logfx.PATH_INT32 else 'fp64'} "
        f"sigma_g={rep['sigma_g']} extracted={rep['extracted']} output={rep['output']}")

    for i in range(args.warmup):
        ctx.extract(bufs[i % 3], params, out, bits=11)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")

    # the timed region: K steps and nothing else
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(args.steps):
        ctx.extract(bufs[i % 3], params, out, bits=11)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_step = total_ms / args.steps
    # after it: per-kernel HIP-event times over the same number of steps, on
    # the stream the kernels run on
    ctx.timing_enable(True)
    for i in range(args.steps):
        ctx.extract(bufs[i % 3], params, out, bits=11)
    kern_ms, calls = ctx.timing_read()
    ctx.timing_enable(False)
    # spread of single steps
    singles = []
    for i in range(min(args.steps, 30)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.extract(bufs[i % 3], params, out, bits=11)
        e1.record(stream)
        singles.append((e0, e1))
    torch.cuda.synchronize()
    step_ms = np.array([a.elapsed_time(b) for a, b in singles])
    # the FP64 path on the same scene: masks on a 23-bit grid (the finest
    # grid an FP32 tap holds), whose sums exceed the int32 bound
    fp64 = None
    if not args.no_fp64:
        p64 = logfx.Params(logfx.make_log_mask(5, 0.8, 23)[0], logfx.make_log_mask(9, 1.4, 23)[0],
                           std_k=2.0, smooth=True, median_size=5, median_cascade=cascade)
        _, rep64 = ctx.extract(bufs[0], p64, out, bits=11, report=True)
        for i in range(args.warmup):
            ctx.extract(bufs[i % 3], p64, out, bits=11)
        torch.cuda.synchronize()
        start.record(stream)
        for i in range(args.steps):
            ctx.extract(bufs[i % 3], p64, out, bits=11)
        stop.record(stream)
        torch.cuda.synchronize()
        ms64 = start.elapsed_time(stop) / args.steps
        fp64 = {"ms_per_step": round(ms64, 4), "Mpixel_s": round(H * W / (ms64 * 1e-3) / 1e6, 1),
                "path": "fp64" if rep64["path"] == logfx.PATH_FP64 else "int32", "mask_grid_bits": 23,
                "rows_per_strip": [ctx.get_option(logfx.OPT_ROWS1), ctx.get_option(logfx.OPT_ROWS2)]}
        log(f"fp64 path: {ms64:.3f} ms/step")
    # latency of one call on the 512^2 uint8 image (40 rectangles, noise
    # sigma 4): it fits in the caches, so launches dominate
    lat = None
    if not args.no_latency:
        small = torch.from_numpy(scenes.config1()).to(dev)
        sout = torch.empty(small.shape, dtype=torch.uint8, device=dev)
        for _ in range(max(args.warmup, 3)):
            ctx.extract(small, params, sout, bits=8)
        torch.cuda.synchronize()
        evs = []
        for _ in range(50):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.extract(small, params, sout, bits=8)
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        lms = np.array([a.elapsed_time(b) for a, b in evs])
        wall = []
        for _ in range(50):
            t0 = time.perf_counter()
            ctx.extract(small, params, sout, bits=8)
            torch.cuda.synchronize()
            wall.append(time.perf_counter() - t0)
        lat = {"workload": "512x512 uint8 image, 40 rectangles, noise sigma 4; same masks, threshold and median",
               "device_ms_p10_p50_p90": [round(float(np.percentile(lms, q)), 4) for q in (10, 50, 90)],
               "host_wall_ms_p50": round(float(np.median(wall)) * 1e3, 4),
               "Mpixel_s_p50": round(small.numel() / (float(np.median(lms)) * 1e-3) / 1e6, 1)}
        del small, sout
        log(f"512^2 latency: {lat['device_ms_p10_p50_p90'][1]:.4f} ms")
    # a plain device copy of 1 GiB: the HBM bandwidth this machine reaches
    csrc = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        cdst.copy_(csrc)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del csrc, cdst
    px = H * W
    # host <-> device transfers (the transfer / kernel split of the paper's
    # Table 6), after the timed region and not part of `value`: the image in
    # from pinned host memory and the output map back to pinned host memory
    transfers = None
    if not args.no_transfers:
        h_img = torch.empty(bufs[0].shape, dtype=bufs[0].dtype, pin_memory=True)
        h_img.copy_(bufs[0].cpu())
        h_out = torch.empty(out.shape, dtype=out.dtype, pin_memory=True)
        d_in = torch.empty_like(bufs[0])
        d_in.copy_(h_img, non_blocking=True)
        h_out.copy_(out, non_blocking=True)
        torch.cuda.synchronize()
        t0, t1, t2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        reps = 5
        t0.record(stream)
        for _ in range(reps):
            d_in.copy_(h_img, non_blocking=True)
        t1.record(stream)
        for _ in range(reps):
            h_out.copy_(out, non_blocking=True)
        t2.record(stream)
        torch.cuda.synchronize()
        h2d, d2h = t0.elapsed_time(t1) / reps, t1.elapsed_time(t2) / reps
        nin, nout = h_img.numel() * h_img.element_size(), h_out.numel()
        transfers = {"h2d_ms": round(h2d, 4), "d2h_ms": round(d2h, 4),
                     "h2d_GBs": round(nin / (h2d * 1e-3) / 1e9, 1), "d2h_GBs": round(nout / (d2h * 1e-3) / 1e9, 1),
                     "pcie_inclusive_Mpixel_s": round(px / ((h2d + ms_step + d2h) * 1e-3) / 1e6, 1),
                     "kernel_share": round(ms_step / (h2d + ms_step + d2h), 4)}
        del h_img, h_out, d_in
        log(f"transfers: in {h2d:.3f} ms, out {d2h:.3f} ms")
    value = px / (ms_step * 1e-3) / 1e6
    avg = [k / max(calls, 1) for k in kern_ms]
    log(f"timed {args.steps} steps: {ms_step:.4f} ms/step, kernels (ms) p1={avg[0]:.4f} "
        f"fin={avg[1]:.4f} p2={avg[2]:.4f}")

    dom = int(np.argmax([avg[0], avg[2]])) * 2  # 0 = pass 1, 2 = pass 2
    stored = ctx.get_option(logfx.OPT_STORE_Z) == 1
    if dom == 2:
        dom_name = "pass2z_kernel" if stored else "pass2_kernel"
        ops_px = PASS2Z_OPS_PER_PX if stored else PASS2_OPS_PER_PX
    else:
        dom_name = "pass1_kernel"
        ops_px = None
    rows = [ctx.get_option(logfx.OPT_ROWS1), ctx.get_option(logfx.OPT_ROWS2)]
    if dom_name == "pass1_kernel":
        # the LoG multiply-adds of the method (two operations each) per second
        # against the ALU peak at that count
        achieved = 2 * LOG_FMA_PER_PX * px / (avg[dom] * 1e-3) / 1e12
        peak, unit, work = ALU_PEAK_TFLOPS, "TFLOP/s", f"{LOG_FMA_PER_PX} LoG multiply-adds per pixel"
    else:
        achieved = ops_px * px / (avg[dom] * 1e-3) / 1e12
        peak, unit, work = VALU_PEAK_TOPS, "Tops/s", f"{ops_px} operations per pixel"
    roofline = {
        "bound": "alu", "kernel": dom_name,
        "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": unit,
        "frac": round(achieved / peak, 4),
        "traffic": (TRAFFIC_BYTES[dom_name] if kernel_source_hash() == TRAFFIC_SOURCE_HASH
                    and dom_name in TRAFFIC_BYTES and H == 8192 and W == 8192
                    and rows == TRAFFIC_ROWS else None),
        "work": work,
        "kernel_hbm": ({"bytes_per_pixel": KERNEL_BYTES_PER_PX[dom_name],
                        "achieved_GBs": round(KERNEL_BYTES_PER_PX[dom_name] * px / (avg[dom] * 1e-3) / 1e9, 1),
                        "frac": round(KERNEL_BYTES_PER_PX[dom_name] * px / (avg[dom] * 1e-3) / 1e9
                                      / HBM_PEAK_GBS, 4)} if dom_name in KERNEL_BYTES_PER_PX else None),
        "measured_copy_GBs": round(copy_gbs, 1),
        "pass2_hbm": ({"kernel": "pass2z_kernel", "bytes_per_pixel": KERNEL_BYTES_PER_PX["pass2z_kernel"],
                       "achieved_GBs": round(KERNEL_BYTES_PER_PX["pass2z_kernel"] * px / (avg[2] * 1e-3) / 1e9, 1),
                       "frac_peak": round(KERNEL_BYTES_PER_PX["pass2z_kernel"] * px / (avg[2] * 1e-3) / 1e9
                                          / HBM_PEAK_GBS, 4),
                       "frac_copy": round(KERNEL_BYTES_PER_PX["pass2z_kernel"] * px / (avg[2] * 1e-3) / 1e9
                                          / copy_gbs, 4)} if stored else None),
        "hbm_view": {"bytes_per_pixel": 3, "achieved_GBs": round(3 * px / (ms_step * 1e-3) / 1e9, 1),
                     "peak_GBs": HBM_PEAK_GBS,
                     "frac": round(3 * px / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    # why the pipeline cannot sit at 70 % of HBM peak: its arithmetic floor
    # (the LoG multiply-adds alone at the ALU peak) against the time its 3
    # bytes per pixel take at that fraction of the 8 TB/s
    roofline["hbm_bar"] = {"target_frac": 0.70,
                           "pipeline_frac": roofline["hbm_view"]["frac"],
                           "alu_floor_ms": round(LOG_FMA_PER_PX * px / (VALU_PEAK_TOPS * 1e12) * 1e3, 4),
                           "hbm_time_at_target_ms": round(3 * px / (0.70 * HBM_PEAK_GBS * 1e9) * 1e3, 4)}
    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32" if rep["path"] == logfx.PATH_INT32 else "f64", "data": "synthetic",
        "config": {"workload": f"{H}x{W} uint16 11-bit scene (20000 rectangles, 500 polylines, "
                               "noise sigma 12, 5% salt-and-pepper); LoG 5x5 s0.8 + 9x9 s1.4; "
                               "3x3 deviation > 2.0 global; 5x5 hybrid median"
                               + "".join(f", then {m}x{m}" for m in cascade),
                   "pixels": px, "parallelism": "single GPU", "store_z": args.store_z,
                   "rows_per_strip": rows},
        "kernels_ms": {"pass1": round(avg[0], 4), "finalize": round(avg[1], 4),
                       "pass2": round(avg[2], 4)},
        "step_ms_p10_p50_p90": [round(float(np.percentile(step_ms, q)), 4) for q in (10, 50, 90)],
        "roofline": roofline,
        "transfers": transfers,
        "fp64_path": fp64,
        "latency_512x512_u8": lat,
        "paper_speedup": PAPER_SPEEDUP,
    }
    ctx.close()
    if args.copy_mib > 0:
        n = args.copy_mib << 20
        src = torch.empty(n, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_mib} MiB x 5")
    if not args.no_cpu_baseline:
        import oracle
        log(f"oracle on {host_cores()} host threads ...")
        orc_taps = (oracle.log_mask(5, 0.8, 16)[0], oracle.log_mask(9, 1.4, 16)[0])
        result["cpu_baseline"] = cpu_baseline(img, orc_taps)
        result["speedup_vs_oracle"] = round(result["value"] / result["cpu_baseline"]["value"], 1)
        log(f"oracle {result['cpu_baseline']['value']:.2f} Mpixel/s")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
