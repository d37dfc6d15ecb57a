#!/usr/bin/env python3
"""Benchmark: exact integral histograms on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (one "step"): the 256-frame uneven batch -- resolutions drawn from
320x240 to 3840x2160 and bin counts from {16, 32, 64, 128}, uniform pixels from
seed 3 (about 3.2e10 entries, 127 GB of uint32 output) -- every frame's
integral histogram computed into its own resident H x W x B tensor by ONE
launch of a batched plan (a hipGraph) whose tile shapes and carry schedules
the autotuner chose per (H, W, B) class.  Inputs are resident in HBM before
the timed region starts.

Prints ONE JSON line: throughput (entries/s) of that step and the roofline of
its dominant kernel, the tile pass (HBM-bound); the same frames through 256
plain per-frame ih_compute calls; the 64-frame 1920x1080 B=64 moving-disc
sequence through a batched plan (with its own roofline), a pipelined plan, a
bin-major plan and the plain loop; the 640x480 B=32 frame and the 8192x8192
B=128 frame through ih_compute with their region queries; one 1920x1080 B=64
frame in each single-frame form; the host-transfer pipeline (frames/s with the
whole integral histogram copied back over PCIe, as the paper measures); device
write references (torch's fill, and the tile pass's own store stream with no
loads); the serving loop's p50/p99 latency and throughput next to the plain
per-frame path at several arrival rates; and the single-threaded CPU oracle
timed on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0

# HBM bytes of the tile pass, from two rocprofv3 --pmc runs per workload
# (FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000, the factors a 1 GiB device copy
# reads on the same counters), summed over the tile-pass dispatches of one
# step.  Valid only for the kernel sources and schedule they were taken with;
# any other combination reports null.
TRAFFIC_RECORDS = {
    "uneven_batch_256": {
        "kernel_sources_sha256": "23c7a9c5a351e4e84255648fdd937497fa1b122128c17abc482c179daabb0cf6",
        "schedule": {
            "1080x1920 B128": "64x120 nt reduce-then-scan",
            "1080x1920 B16": "32x120 reduce-then-scan",
            "1080x1920 B32": "64x120 nt reduce-then-scan",
            "1080x1920 B64": "64x120 nt reduce-then-scan",
            "2160x3840 B128": "64x128 reduce-then-scan",
            "2160x3840 B16": "64x128 reduce-then-scan",
            "2160x3840 B32": "64x240 nt reduce-then-scan",
            "2160x3840 B64": "128x240 reduce-then-scan",
            "240x320 B128": "32x60 nt prefix counts",
            "240x320 B16": "32x16 nt prefix counts",
            "240x320 B32": "32x30 prefix counts",
            "240x320 B64": "32x30 prefix counts",
            "480x640 B128": "32x240 nt prefix counts",
            "480x640 B16": "32x60 prefix counts",
            "480x640 B32": "32x60 prefix counts",
            "480x640 B64": "32x120 nt prefix counts",
            "720x1280 B128": "32x240 reduce-then-scan",
            "720x1280 B16": "32x120 nt prefix counts",
            "720x1280 B32": "32x240 nt prefix counts",
            "720x1280 B64": "64x240 nt prefix counts"
        },
        "fetch_bytes": 2265890098,
        "write_bytes": 126814648608,
        "source": "profiles/uneven_batch_256_tile_pass_hbm_counters.md"
    }
}

KERNEL_SOURCES = ["ih_kernels.hip", "ih_tile.h", "ih_device.h", "ih_internal.h", "ih_tile_regular.hip",
                  "ih_tile_regular_guarded.hip", "ih_tile_nontemporal.hip", "ih_tile_nontemporal_guarded.hip",
                  "ih_tile_table.hip"]


def kernel_digest() -> str | None:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1711_01919_amd", "csrc")
    try:
        for name in KERNEL_SOURCES:
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    return h.hexdigest()


def recorded_traffic(workload: str, schedule) -> float | None:
    r = TRAFFIC_RECORDS.get(workload)
    if r is None or kernel_digest() != r["kernel_sources_sha256"] or schedule != r["schedule"]:
        return None
    return r["fetch_bytes"] + r["write_bytes"]


METRIC = "integral-hist entries/s + % HBM peak; served p50/p99 latency vs plain loop"

# The autotuner's choices for the headline's frame classes, as it wrote them
# (IH_AUTOTUNE_CACHE format) in a run on an MI355X; read unless --retune.
TUNING_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1711_01919_amd", "tuning",
                           "gfx950_autotune.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=64, help="frames of the moving-disc sequence leg")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline workload only (for profiling runs); same as --legs headline")
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs to run (for profiling runs): headline, disc, plain, transfer, "
                         "reference, serving; default all")
    ap.add_argument("--no-transfer", action="store_true", help="skip the host-transfer pipeline leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="time budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the replayed 16-stream arrival trace (0: skip the serving leg)")
    ap.add_argument("--retune", action="store_true",
                    help="autotune the headline's frame classes in this run instead of reading the tuning "
                         "file the autotuner wrote earlier on an MI355X")
    ap.add_argument("--tune-out", default=None,
                    help="with --retune: the file the autotuner writes its choices to")
    ap.add_argument("--copy-reference", action="store_true",
                    help="only run four 1 GiB device-to-device copies (calibrates HBM byte counters)")
    return ap.parse_args()


def copy_reference(torch) -> None:
    """Four copies of 1 GiB between two device buffers: each reads and writes
    exactly 2^30 bytes, which is what FETCH_SIZE / WRITE_SIZE should report
    for one such dispatch."""
    src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": 1 << 30, "dispatches": 4}), flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(frames, bins, budget_s: float) -> dict:
    """The oracle (single-threaded C, as committed) on the workload's frames in
    order, as many as fit in budget_s (at least one); then frame-parallel on up
    to 16 host threads for about the same time."""
    import oracle
    from oracle import _u8p, _u32p
    orc = oracle.get()
    n = len(frames)
    done, t_total, entries = 0, 0.0, 0
    while done < n and (done == 0 or t_total < budget_s):
        f = np.ascontiguousarray(frames[done])
        H, W = f.shape
        B = bins[done]
        out = np.ones((H, W, B), dtype=np.uint32)             # pre-faulted output
        t0 = time.perf_counter()
        rc = orc.lib.ihref_integral_histogram(f.ctypes.data_as(_u8p), H, W, B, out.ctypes.data_as(_u32p))
        t_total += time.perf_counter() - t0
        assert rc == 0
        entries += H * W * B
        done += 1
    res = {"value": entries / t_total, "unit": "entries/s", "cores": 1, "kind": "oracle",
           "sample": f"first {done} of {n} frames of the workload in order ({entries:.3g} entries), "
                     f"{t_total:.1f} s single-threaded, {oracle.compile_flags()}, "
                     f"host: {os.cpu_count()} cpus, {cpu_model()}"}
    # frame-parallel, one oracle call per thread (the call releases the GIL),
    # as the paper's multi-threaded CPU comparison: the same sample split over
    # the threads
    from concurrent.futures import ThreadPoolExecutor
    threads = max(1, min(16, os.cpu_count() or 1))
    sample = list(range(done)) * max(1, threads // max(done, 1))

    def work(k):
        f = np.ascontiguousarray(frames[k])
        H, W = f.shape
        out = np.ones((H, W, bins[k]), dtype=np.uint32)
        t0 = time.perf_counter()
        assert orc.lib.ihref_integral_histogram(f.ctypes.data_as(_u8p), H, W, bins[k],
                                                out.ctypes.data_as(_u32p)) == 0
        return H * W * bins[k], time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        got = list(ex.map(work, sample))
    t_par = time.perf_counter() - t0
    res["parallel"] = {"value": sum(e for e, _ in got) / t_par, "cores": threads,
                       "sample": f"{len(sample)} frames over {threads} threads, {t_par:.1f} s"}
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "cpu model unknown"


def timed(torch, stream, fn, steps):
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


def plain_and_query_legs(torch, ihb, synth, stream) -> dict:
    """The 640x480 B=32 frame through ih_compute (mean over 1000 calls
    rotating 8 outputs) with its 1000 rectangles, and the 8192x8192 B=128
    mixture frame with 1e6 rectangles; queries read rectangles already on the
    device.
    Algorithmic query bytes: 4 corners x B x 4 read + B x 4 written = 20*B
    per rectangle."""
    out = {}
    I, B, rects = synth.plain_frame()
    H, W = I.shape
    f = torch.from_numpy(I).cuda()
    # 8 outputs (315 MB, more than the 256 MB last-level cache) written in turn
    ihs = [torch.empty((H, W, B), dtype=torch.uint32, device="cuda") for _ in range(8)]
    rd = torch.from_numpy(rects).cuda()
    hs = torch.empty((len(rects), B), dtype=torch.uint32, device="cuda")
    for k in range(24):
        ihb.compute(f, B, out=ihs[k % 8], stream=stream)
    reps = 1000
    it = iter(range(1 << 30))
    ms = timed(torch, stream, lambda: ihb.compute(f, B, out=ihs[next(it) % 8], stream=stream), reps) / reps
    it = iter(range(1 << 30))
    qms = timed(torch, stream, lambda: ihb.query_device(ihs[next(it) % 8], rd, out=hs, stream=stream),
                reps) / reps
    out["plain_frame_640x480_B32"] = {"ms_per_frame": ms, "entries_per_s": H * W * B / (ms / 1e3),
                                      "hbm_frac": (H * W + 4 * H * W * B) / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                      "calls": reps, "rotating_outputs": 8, "query_1000_rects_ms": qms}
    del f, ihs, rd, hs
    # the other single-frame forms on one 1920x1080 disc frame, B=64: the
    # bin-major layout and bins from a table (random edges, seed 4)
    frames1, B1 = synth.disc_sequence(n_frames=1)
    f1 = torch.from_numpy(frames1[0]).cuda()
    H1, W1 = frames1.shape[1:]
    o1 = torch.empty((H1, W1, B1), dtype=torch.uint32, device="cuda")
    edges = np.sort(np.random.default_rng(4).integers(0, 257, size=B1 - 1))
    lut = np.searchsorted(edges, np.arange(256), side="right").astype(np.uint8)
    by1 = H1 * W1 + 4 * H1 * W1 * B1
    forms = {}
    for name, fn in (("hwb", lambda: ihb.compute(f1, B1, out=o1, stream=stream)),
                     ("binmajor", lambda: ihb.compute_binmajor(f1, B1, out=o1, stream=stream)),
                     ("table_bins", lambda: ihb.compute_lut(f1, B1, lut, out=o1, stream=stream))):
        fn()
        ms1 = timed(torch, stream, fn, 50) / 50
        forms[name] = {"ms_per_frame": ms1, "hbm_frac": by1 / (ms1 / 1e3) / 1e9 / HBM_PEAK_GBS}
    # region queries on both layouts: 1e5 rectangles (seed 8, drawn as for the
    # 640x480 frame) already on the device
    qr = np.random.default_rng(8)
    nq = 100_000
    xs = np.sort(qr.integers(0, W1, size=(nq, 2)), axis=1)
    ys = np.sort(qr.integers(0, H1, size=(nq, 2)), axis=1)
    rd1 = torch.from_numpy(np.stack([xs[:, 0], ys[:, 0], xs[:, 1], ys[:, 1]], axis=1).astype(np.int32)).cuda()
    h1 = torch.empty((nq, B1), dtype=torch.uint32, device="cuda")
    for name, comp, query, shape in (("hwb", ihb.compute, ihb.query_device, (H1, W1, B1)),
                                     ("binmajor", ihb.compute_binmajor, ihb.query_binmajor_device, (B1, H1, W1))):
        comp(f1, B1, out=o1, stream=stream)
        ihv = o1.view(*shape)
        query(ihv, rd1, out=h1, stream=stream)
        qms = timed(torch, stream, lambda: query(ihv, rd1, out=h1, stream=stream), 20) / 20
        forms[name].update({"query_1e5_rects_ms": qms, "rects_per_s": nq / (qms / 1e3)})
    out["single_frame_1920x1080_B64_forms"] = forms
    del f1, o1, rd1, h1
    I, B, rects = synth.mixture_frame()
    H, W = I.shape
    f = torch.from_numpy(I).cuda()
    ih = torch.empty((H, W, B), dtype=torch.uint32, device="cuda")
    ihb.compute(f, B, out=ih, stream=stream)
    ms = timed(torch, stream, lambda: ihb.compute(f, B, out=ih, stream=stream), 3) / 3
    rd = torch.from_numpy(rects).cuda()
    hs = torch.empty((len(rects), B), dtype=torch.uint32, device="cuda")
    ihb.query_device(ih, rd, out=hs, stream=stream)
    qms = timed(torch, stream, lambda: ihb.query_device(ih, rd, out=hs, stream=stream), 10) / 10
    n = len(rects)
    out["mixture_frame_8192x8192_B128"] = {
        "ms_per_frame": ms, "entries_per_s": H * W * B / (ms / 1e3),
        "hbm_frac": (H * W + 4 * H * W * B) / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        "query_1e6_rects_ms": qms, "rects_per_s": n / (qms / 1e3),
        "query_gbs": 20 * B * n / (qms / 1e3) / 1e9}
    del f, ih, rd, hs
    torch.cuda.empty_cache()
    return out


def device_reference(torch, ihb) -> dict:
    """What plain device writes reach on this GPU: torch's fill of 8 GiB and
    of 32 GiB (write-only streams, one chunk of addresses after another), and
    the tile pass's own store stream with no loads and no arithmetic
    (ih_write_reference) in the moving-disc sequence's geometry: 64 frames of
    1080 x 1920 x 64 stacked into one 69120 x 1920 x 64 tensor (34 GB), tiles
    of 128 x 216, the same work items and store order as that batch's tile
    pass.  Boxes of the same model differ by tens of percent, so the
    integral-histogram figures are best read next to these."""
    res = {}
    stream = torch.cuda.current_stream()
    for gib in (8, 32):
        x = torch.empty(gib << 30, dtype=torch.uint8, device="cuda")
        x.fill_(1)
        ms = timed(torch, stream, lambda: x.fill_(7), 5) / 5
        res[f"fill_{gib}GiB_gbs"] = (gib << 30) / (ms / 1e3) / 1e9
        del x
        torch.cuda.empty_cache()
    H, W, B = 64 * 1080, 1920, 64
    out = torch.empty((H, W, B), dtype=torch.uint32, device="cuda")
    ihb.write_reference(out, (128, 216), stream)
    torch.cuda.synchronize()
    assert int(out[H - 1, W - 1, B - 1]) == H - 1 and int(out[0, 0, 0]) == 0
    ms = timed(torch, stream, lambda: ihb.write_reference(out, (128, 216), stream), 5) / 5
    res["tile_geometry_write_64x1080x1920_B64_128x216_gbs"] = H * W * B * 4 / (ms / 1e3) / 1e9
    del out
    torch.cuda.empty_cache()
    return res


def transfer_leg(torch, ihb) -> dict:
    """The host-transfer pipeline (frames uploaded, whole integral histograms
    downloaded to pinned host memory; one buffer slot, or two so that the
    next frame's upload and kernels overlap this frame's download): frames/s
    including the PCIe copies, the figure the paper reports, next to the
    bound 1 / max(kernel, download) per frame.  Frames: uniform pixels from
    seed 6.  Each case checks one output row against the oracle."""
    import oracle
    orc = oracle.get()
    rng = np.random.default_rng(6)
    res = {}
    for (H, W, B, n) in ((480, 640, 32, 100), (720, 1280, 16, 50), (720, 1280, 128, 12)):
        frames = [torch.from_numpy(rng.integers(0, 256, size=(H, W), dtype=np.uint8)).pin_memory()
                  for _ in range(n)]
        outs = [torch.empty((H, W, B), dtype=torch.uint32).pin_memory() for _ in range(n)]
        case = {}
        for ns in (1, 2):
            ihb.transfer_pipeline(frames, outs, B, n_streams=ns)              # warm-up: every buffer once
        # one and two streams alternate, three runs each, the best of each
        # kept: the host link's rate drifts over seconds on a shared machine
        best = {}
        for rep in range(3):
            for ns in (1, 2):
                st = ihb.transfer_pipeline(frames, outs, B, n_streams=ns)
                if ns not in best or st["wall_ms"] < best[ns]["wall_ms"]:
                    best[ns] = st
        for ns, st in best.items():
            case[f"streams_{ns}"] = {"frames_per_s": st["frames_per_s"], "wall_ms": st["wall_ms"],
                                     "kernel_ms_per_frame": st["kernel_ms"] / n,
                                     "d2h_ms_per_frame": st["d2h_ms"] / n,
                                     "d2h_gbs": H * W * B * 4 * n / (st["d2h_ms"] / 1e3) / 1e9,
                                     "bound_frames_per_s": 1e3 / max(st["kernel_ms"] / n, st["d2h_ms"] / n)}
        k = n - 1
        assert np.array_equal(outs[k][H - 1].numpy(), orc.row_by_definition(frames[k].numpy(), B, H - 1)), \
            f"transfer pipeline parity spot check failed ({H}x{W} B={B})"
        case["dual_buffer_gain"] = case["streams_2"]["frames_per_s"] / case["streams_1"]["frames_per_s"]
        res[f"{W}x{H}_B{B}_{n}_frames"] = case
        del frames, outs
    return res


def schedule_summary(plan, frames, bins):
    """Per (H, W, B) class: the tile, store flavour and carry schedule the plan
    chose (one entry per class; every frame of a class gets the same)."""
    seen = {}
    for k, (f, b) in enumerate(zip(frames, bins)):
        key = f"{f.shape[0]}x{f.shape[1]} B{b}"
        if key not in seen:
            sc = plan.frame_schedule(k)
            cb = sc["carry_bands"]
            sched = " prefix counts" if cb == -2 else (f" fused K={cb}" if cb > 0 else " reduce-then-scan")
            seen[key] = f"{sc['tile'][0]}x{sc['tile'][1]}" + (" nt" if sc["nontemporal"] else "") + sched
    return dict(sorted(seen.items()))


def profiled_steps(torch, stream, plan, ihb, steps):
    """K plan launches with the per-phase event profiler on: HIP events on the
    launch stream bracket each phase's graph (every tile-pass launch of the
    step lies inside the tile phase's pair)."""
    ihb.profile_enable(True)
    ms = timed(torch, stream, lambda: plan.launch(stream), steps)
    ph = ihb.profile_read()
    ihb.profile_enable(False)
    return ms, ph


def uneven_headline(torch, ihb, synth, stream, args) -> dict:
    """The headline: 256 frames of five resolutions and four bin counts (seed
    3) through one autotuned batched plan, one graph launch per step; then
    the same frames through 256 plain ih_compute calls on the same buffers."""
    import oracle
    ub = synth.uneven_batch()
    fr = [torch.from_numpy(f).cuda() for f in ub.frames]
    outs = [torch.empty((f.shape[0], f.shape[1], b), dtype=torch.uint32, device="cuda")
            for f, b in zip(ub.frames, ub.bins)]
    t0 = time.time()
    plan = ihb.BatchPlan(fr, outs, ub.bins, autotune=True, stream=stream)
    tune_s = time.time() - t0
    info = plan.info()
    sched = schedule_summary(plan, ub.frames, ub.bins)
    log(f"[bench] uneven batch plan in {tune_s:.1f}s: {info}")
    for _ in range(args.warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    ms_total = timed(torch, stream, lambda: plan.launch(stream), args.steps)
    ms_prof, ph = profiled_steps(torch, stream, plan, ihb, args.steps)
    ms = ms_total / args.steps
    log(f"[bench] uneven batch: {ms:.3f} ms/step; profiled {ms_prof / args.steps:.3f} ms/step, phases {ph}")
    # parity spot check of the timed outputs: the last row of a few frames
    orc = oracle.get()
    for k in (0, 1, 127, 255):
        H = ub.frames[k].shape[0]
        assert np.array_equal(outs[k][H - 1].cpu().numpy(), orc.row_by_definition(ub.frames[k], ub.bins[k], H - 1)), \
            f"uneven batch parity spot check failed ({k})"

    def plain():
        for k, b in enumerate(ub.bins):
            ihb.compute(fr[k], b, out=outs[k], stream=stream)
    plain()
    ms_plain = timed(torch, stream, plain, 3) / 3
    plan.close()
    del plan, plain, fr, outs
    torch.cuda.empty_cache()
    ent = ub.entries
    alg = 4 * ent + sum(f.size for f in ub.frames)
    tile_ms = ph["tile_ms"] / args.steps                      # tile-pass kernels of one step, back to back
    achieved = alg / (tile_ms / 1e3) / 1e9
    return {"frames": len(ub.frames), "entries": ent, "alg_bytes": alg, "ms_per_step": ms,
            "entries_per_s": ent / (ms / 1e3), "hbm_frac_step": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "profiled_ms_per_step": ms_prof / args.steps,
            "phase_ms_per_step": {k: ph[k] / args.steps for k in ("agg_ms", "scan_ms", "tile_ms")},
            "plain_loop": {"ms_per_step": ms_plain, "entries_per_s": ent / (ms_plain / 1e3),
                           "speedup_batched": ms_plain / ms},
            "autotune_s": tune_s,
            "tuning": ("autotuned in this run" if args.retune or not os.path.exists(TUNING_FILE)
                       else "the autotuner's choices from " + os.path.relpath(TUNING_FILE)),
            "kernel_launches": info["kernel_launches"],
            "tile_launches": info["tile_launches"], "schedules": sched,
            "roofline": {"bound": "hbm", "kernel": "tile_batch_kernel (all variants of the step)",
                         "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": recorded_traffic("uneven_batch_256", sched),
                         "alg_bytes_per_step": alg, "tile_launches_per_step": info["tile_launches"],
                         "tile_ms_per_step": tile_ms}}


def disc_sequence_leg(torch, ihb, synth, stream, args) -> dict:
    """The 64-frame 1920x1080 B=64 moving-disc sequence: one batched plan
    (heuristic tiles, one graph launch), the plain per-frame loop, a
    pipelined plan (4 GiB groups) and a plan writing the bin-major layout."""
    import oracle
    frames, B = synth.disc_sequence(n_frames=args.frames)
    n, H, W = frames.shape
    d_frames = torch.from_numpy(frames).cuda()
    outs = [torch.empty((H, W, B), dtype=torch.uint32, device="cuda") for _ in range(n)]
    plan = ihb.BatchPlan([d_frames[k] for k in range(n)], outs, [B] * n, stream=stream)
    tile = plan.frame_tile(0)
    sched = schedule_summary(plan, list(frames), [B] * n)
    info = plan.info()
    for _ in range(args.warmup):
        plan.launch(stream)
    ms_total = timed(torch, stream, lambda: plan.launch(stream), args.steps)
    ms_prof, ph = profiled_steps(torch, stream, plan, ihb, args.steps)
    ms_step = ms_total / args.steps
    entries_step = n * H * W * B
    alg = n * (H * W + 4 * H * W * B)
    orc = oracle.get()
    for k in (0, n - 1):
        assert np.array_equal(outs[k][H - 1].cpu().numpy(), orc.row_by_definition(frames[k], B, H - 1)), k

    def plain_step():
        for k in range(n):
            ihb.compute(d_frames[k], B, out=outs[k], stream=stream)
    plain_step()
    plain_steps = max(2, min(args.steps, 10))
    ms_plain = timed(torch, stream, plain_step, plain_steps) / plain_steps
    pplan = ihb.BatchPlan([d_frames[k] for k in range(n)], outs, [B] * n, stream=stream, group_bytes=4 << 30)
    pinfo = pplan.info()
    for _ in range(max(1, args.warmup)):
        pplan.launch(stream)
    ms_pipe = timed(torch, stream, lambda: pplan.launch(stream), args.steps) / args.steps
    pplan.close()
    bplan = ihb.BatchPlan([d_frames[k] for k in range(n)], [o.view(B, H, W) for o in outs], [B] * n,
                          stream=stream, binmajor=[True] * n)
    bplan.launch(stream)
    torch.cuda.synchronize()
    got = outs[n - 1].view(B, H, W)[:, H - 1].cpu().numpy().T
    assert np.array_equal(got, orc.row_by_definition(frames[n - 1], B, H - 1)), "bin-major spot check failed"
    ms_bm = timed(torch, stream, lambda: bplan.launch(stream), args.steps) / args.steps
    bm_tile = list(bplan.frame_tile(0)[:2])
    bplan.close()
    plan.close()
    del outs, plan, d_frames
    torch.cuda.empty_cache()
    tile_ms = ph["tile_ms"] / args.steps
    achieved = alg / (tile_ms / 1e3) / 1e9
    return {"workload": f"disc_sequence_{n}x{H}x{W}_B{B}", "ms_per_step": ms_step,
            "entries_per_s": entries_step / (ms_step / 1e3), "hbm_frac_step": alg / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
            "tile": list(tile[:2]), "schedules": sched, "kernel_launches": info["kernel_launches"],
            "profiled_ms_per_step": ms_prof / args.steps,
            "phase_ms_per_step": {k: ph[k] / args.steps for k in ("agg_ms", "scan_ms", "tile_ms")},
            "plain_loop": {"ms_per_step": ms_plain, "entries_per_s": entries_step / (ms_plain / 1e3),
                           "speedup_batched": ms_plain / ms_step},
            "pipelined_4GiB": {"ms_per_step": ms_pipe, "entries_per_s": entries_step / (ms_pipe / 1e3),
                               "groups": pinfo["groups"]},
            "binmajor_batched": {"ms_per_step": ms_bm, "entries_per_s": entries_step / (ms_bm / 1e3),
                                 "hbm_frac": alg / (ms_bm / 1e3) / 1e9 / HBM_PEAK_GBS, "tile": bm_tile},
            "roofline": {"bound": "hbm", "kernel": "tile_batch_kernel", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": recorded_traffic(f"disc_sequence_{n}x{H}x{W}_B{B}", sched),
                         "alg_bytes_per_step": alg, "tile_launches_per_step": info["tile_launches"],
                         "tile_ms_per_step": tile_ms}}


def percentiles(xs):
    a = np.sort(np.asarray(xs, dtype=np.float64))
    return {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean()), "max_ms": float(a.max()), "n": int(a.size)}


def serve_trace(ihb, srv, events, pools, specs, speed: float) -> dict:
    """Replay `events` (arrival seconds, stream, frame index) open-loop at
    `speed` times their rate through the server: a submitting thread follows
    the wall clock, a polling thread collects results as a client would.
    Latency = results in host memory - scheduled arrival, on the monotonic
    clock the library also stamps with; each request's latency splits into
    the submitter's lag behind the schedule, the wait for admission and the
    device part (admission to results in host memory).  Latency from the
    submit call (the server's own part, without the submitting thread's lag)
    is reported beside it."""
    import threading
    n = len(events)
    tickets = [None] * n
    due_ns = [0] * n
    lag = [0.0] * n
    timing = [None] * n
    submitted = threading.Semaphore(0)

    def poller():
        for i in range(n):
            submitted.acquire()
            _, tm = srv.wait(tickets[i], timeout_s=300.0, sleep_s=2e-5)
            timing[i] = tm

    th = threading.Thread(target=poller)
    th.start()
    t0 = time.monotonic_ns()
    for i, (t_arr, sid, k) in enumerate(events):
        due = t0 + int(t_arr / speed * 1e9)
        now = time.monotonic_ns()
        if now < due:
            time.sleep((due - now) / 1e9)
        due_ns[i] = due
        lag[i] = (time.monotonic_ns() - due) / 1e6
        f, r = pools[sid][0][k % len(pools[sid][0])], pools[sid][1][k % len(pools[sid][1])]
        tickets[i] = srv.submit(sid, f, specs[sid].B, r)
        submitted.release()
    th.join()
    wall = (max(tm["t_done_ns"] for tm in timing) - t0) / 1e9
    lat = [(tm["t_done_ns"] - due_ns[i]) / 1e6 for i, tm in enumerate(timing)]
    lat_submit = [(tm["t_done_ns"] - tm["t_submit_ns"]) / 1e6 for tm in timing]
    worst = int(np.argmax(lat))
    tw = timing[worst]
    return {"lat": lat, "lat_submit": lat_submit, "wall_s": wall,
            "submit_lag_p99_ms": float(np.percentile(np.asarray(lag), 99)),
            "worst": {"ms": lat[worst], "submit_lag_ms": lag[worst],
                      "admission_wait_ms": (tw["t_admit_ns"] - tw["t_submit_ns"]) / 1e6,
                      "device_ms": (tw["t_done_ns"] - tw["t_admit_ns"]) / 1e6}}


def plain_trace(torch, ihb, events, pools, specs, speed: float, outs) -> dict:
    """The same arrivals through the plain per-frame path: one host thread,
    FIFO; per frame upload, ih_compute, ih_query, download, synchronize."""
    dev = torch.device("cuda:0")
    lat = []
    t0 = time.monotonic_ns()
    for t_arr, sid, k in events:
        due = t0 + int(t_arr / speed * 1e9)
        now = time.monotonic_ns()
        if now < due:
            time.sleep((due - now) / 1e9)
        sp = specs[sid]
        f = torch.from_numpy(pools[sid][0][k % len(pools[sid][0])]).to(dev)
        ih = ihb.compute(f, sp.B, out=outs[(sp.H, sp.W, sp.B)])
        ihb.query(ih, pools[sid][1][k % len(pools[sid][1])]).cpu()
        lat.append((time.monotonic_ns() - due) / 1e6)
    return {"lat": lat, "wall_s": (time.monotonic_ns() - t0) / 1e9}


def serving_leg(torch, ihb, synth, seconds: float) -> dict:
    """16 synthetic video streams with Poisson arrivals at 30-120 fps, each
    frame followed by 256 rectangle queries: the trace replayed at 1x, 4x and
    16x its arrival rate, through the serving loop (200 GB budget) and through
    the plain per-frame path.  The sweep stops at the first error."""
    sys.setswitchinterval(5e-4)          # the submitting and polling threads share the interpreter
    specs = synth.stream_plan(duration_s=seconds)
    pools = [synth.stream_frame_pool(100 + s, sp, pool=3) for s, sp in enumerate(specs)]
    events = sorted((float(t), s, k) for s, sp in enumerate(specs) for k, t in enumerate(sp.arrivals))
    entries = sum(specs[s].H * specs[s].W * specs[s].B for _, s, _ in events)
    outs = {}
    for sp in specs:
        key = (sp.H, sp.W, sp.B)
        if key not in outs:
            outs[key] = torch.empty(key, dtype=torch.uint32, device="cuda")
    srv = ihb.Server(budget_bytes=200 << 30, max_slots=64, n_hip_streams=4, max_batch=16,
                     pinned_bytes=24 << 30)
    warm = srv.submit(0, pools[0][0][0], specs[0].B, pools[0][1][0])
    srv.wait(warm)
    res = {"workload": f"{len(specs)} streams, {len(events)} frames ({entries:.3g} entries) over {seconds:.0f} s "
                       f"at 1x, 256 queries per frame", "rates": {}}
    try:
        for speed in (1, 4, 16):
            srv_before = srv.stats()
            sv = serve_trace(ihb, srv, events, pools, specs, float(speed))
            st = srv.stats()
            pl = plain_trace(torch, ihb, events, pools, specs, float(speed), outs)
            res["rates"][f"{speed}x"] = {
                "offered_entries_per_s": entries / (seconds / speed),
                "served": {**percentiles(sv["lat"]), "entries_per_s": entries / sv["wall_s"],
                           "from_submit": percentiles(sv["lat_submit"]),
                           "submit_lag_p99_ms": sv["submit_lag_p99_ms"], "worst": sv["worst"],
                           "device_bytes_peak": st["device_bytes_peak"],
                           "budget_blocked": st["budget_blocked"] - srv_before["budget_blocked"]},
                "plain_loop": {**percentiles(pl["lat"]), "entries_per_s": entries / pl["wall_s"]}}
            log(f"[bench] serving at {speed}x: {res['rates'][f'{speed}x']}")
    except Exception as e:                                   # the sweep stops at the first error
        res["error"] = f"{type(e).__name__}: {e}"
    srv.close()
    del outs
    torch.cuda.empty_cache()
    return res


def run_legs(torch, ihb, synth, stream, args, want, legs) -> None:
    if "disc" in want:
        legs["disc_sequence_64x1080x1920_B64"] = disc_sequence_leg(torch, ihb, synth, stream, args)
        log(f"[bench] disc sequence: {legs['disc_sequence_64x1080x1920_B64']}")
    if "plain" in want:
        pl = plain_and_query_legs(torch, ihb, synth, stream)
        legs.update(pl)
        log(f"[bench] plain/query legs: {pl}")
    if "transfer" in want:
        legs["transfer_pipeline"] = transfer_leg(torch, ihb)
        log(f"[bench] transfer pipeline: {legs['transfer_pipeline']}")
    torch.cuda.empty_cache()
    if "reference" in want:
        legs["device_reference"] = device_reference(torch, ihb)
        log(f"[bench] device reference: {legs['device_reference']}")
    if "serving" in want:
        legs["serving"] = serving_leg(torch, ihb, synth, args.serve_seconds)
        log(f"[bench] serving: {legs['serving']}")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    # before the library reads it (at the first autotuned plan)
    if args.retune:
        if args.tune_out:
            os.environ["IH_AUTOTUNE_CACHE"] = args.tune_out
        else:
            os.environ.pop("IH_AUTOTUNE_CACHE", None)
    elif os.path.exists(TUNING_FILE):
        os.environ["IH_AUTOTUNE_CACHE"] = TUNING_FILE
    import torch
    if args.copy_reference:
        copy_reference(torch)
        return
    from paper_1711_01919_amd import binding as ihb
    from paper_1711_01919_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.current_stream()

    names = {"headline", "disc", "plain", "transfer", "reference", "serving"}
    want = names if args.legs == "all" else set(args.legs.split(","))
    if want - names:
        print(f"bench.py: unknown legs {sorted(want - names)}; known: {sorted(names)}", file=sys.stderr)
        sys.exit(2)
    if args.only_headline:
        want = {"headline"}
    if args.no_transfer:
        want.discard("transfer")
    if args.serve_seconds <= 0:
        want.discard("serving")
    legs = {}
    if "headline" not in want:
        # a profiling run of other legs: no JSON line
        run_legs(torch, ihb, synth, stream, args, want, legs)
        return
    head = uneven_headline(torch, ihb, synth, stream, args)
    run_legs(torch, ihb, synth, stream, args, want, legs)

    ms_step = head["ms_per_step"]
    rec = {
        "metric": METRIC, "value": head["entries_per_s"], "unit": "entries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "uneven_batch_256", "frames": head["frames"], "entries": head["entries"],
                   "resolutions": "320x240..3840x2160 (seed 3)", "bins": "16/32/64/128",
                   "form": "batched_graph_autotuned", "parallelism": "single_gpu"},
        "roofline": head.pop("roofline"),
        "uneven_batch_256": head,
    }
    rec.update(legs)
    if not args.no_cpu_baseline:
        ub = synth.uneven_batch()
        rec["cpu_baseline"] = cpu_baseline(ub.frames, ub.bins, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
