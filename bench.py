#!/usr/bin/env python3
"""Benchmark: exact integral histograms on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (one "step"): the 64-frame 1920x1080 moving-disc sequence with B=64
bins (seeded synthetic stand-in for the paper's HD video), every frame's
integral histogram computed into its own resident H x W x B uint32 tensor
(64 x 530.8 MB = 34 GB of output per step) by ONE launch of a batched plan
(a hipGraph holding one launch per phase for all 64 frames).  Inputs are
resident in HBM before the timed region starts.

Prints ONE JSON line: throughput (entries/s) of the batched step; the same
frames through 64 plain per-frame ih_compute calls for comparison; the
roofline of the dominant kernel (the tile pass, HBM-bound); a write-stream
ceiling measured with a plain fill; and the single-threaded CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
METRIC = "integral-hist entries/s + % HBM peak; served p50/p99 latency vs plain loop"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="time budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(frames: np.ndarray, B: int, budget_s: float) -> dict:
    """The oracle (single-threaded C, as committed) on as many frames of the
    workload as fit in budget_s (at least one)."""
    import oracle
    from oracle import _u8p, _u32p
    orc = oracle.get()
    H, W = frames.shape[1:]
    out = np.zeros((H, W, B), dtype=np.uint32)               # pre-faulted output
    done, t_total = 0, 0.0
    while done < frames.shape[0] and (done == 0 or t_total < budget_s):
        f = np.ascontiguousarray(frames[done])
        t0 = time.perf_counter()
        rc = orc.lib.ihref_integral_histogram(f.ctypes.data_as(_u8p), H, W, B, out.ctypes.data_as(_u32p))
        t_total += time.perf_counter() - t0
        assert rc == 0
        done += 1
    entries = done * H * W * B
    return {"value": entries / t_total, "unit": "entries/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {frames.shape[0]} frames ({H}x{W}, B={B}), "
                      f"{t_total:.1f} s single-threaded, {oracle.compile_flags()}, host has {os.cpu_count()} cpus"}


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


def write_ceiling(torch, stream, gib: float = 8.0, reps: int = 5) -> float:
    """GB/s of a plain device fill (torch's own kernel) over a buffer far larger
    than the 256 MB last-level cache: the write-stream ceiling of the chip."""
    n = int(gib * (1 << 30)) // 4
    buf = torch.empty(n, dtype=torch.int32, device="cuda")
    buf.fill_(1)
    ms = timed(torch, stream, lambda: buf.fill_(7), reps)
    del buf
    return n * 4 * reps / (ms / 1e3) / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1711_01919_amd import binding as ihb
    from paper_1711_01919_amd import synth
    import oracle

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    frames, B = synth.disc_sequence(n_frames=args.frames)
    n, H, W = frames.shape
    log(f"[bench] generated {n} frames {H}x{W} B={B} in {time.time() - t0:.1f}s")

    d_frames = torch.from_numpy(frames).to(dev)
    outs = [torch.empty((H, W, B), dtype=torch.uint32, device=dev) for _ in range(n)]
    stream = torch.cuda.current_stream()

    t0 = time.time()
    plan = ihb.BatchPlan([d_frames[k] for k in range(n)], outs, [B] * n,
                         autotune=not args.no_autotune, stream=stream)
    tile = plan.frame_tile(0)
    info = plan.info()
    log(f"[bench] plan ready in {time.time() - t0:.1f}s: tile {tile}, {info}")

    for _ in range(args.warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")

    ihb.profile_enable(True)
    ms_total = timed(torch, stream, lambda: plan.launch(stream), args.steps)
    ph = ihb.profile_read()
    ihb.profile_enable(False)
    log(f"[bench] timed {args.steps} batched steps: {ms_total:.2f} ms; phases {ph}")

    ms_step = ms_total / args.steps
    entries_step = n * H * W * B
    alg_bytes_frame = H * W + 4 * H * W * B                   # frame read + output written
    value = entries_step / (ms_step / 1e3)
    launches = args.steps                                     # one tile launch per step
    tile_ms_launch = ph["tile_ms"] / launches
    alg_bytes_launch = n * alg_bytes_frame
    achieved = alg_bytes_launch / (tile_ms_launch / 1e3) / 1e9
    step_gbs = n * alg_bytes_frame / (ms_step / 1e3) / 1e9

    # parity spot check of the timed outputs: last row of first and last frame
    orc = oracle.get()
    for k in (0, n - 1):
        got = outs[k][H - 1].cpu().numpy()
        assert np.array_equal(got, orc.row_by_definition(frames[k], B, H - 1)), f"parity spot check failed ({k})"

    # the same frames through the plain per-frame loop
    def plain_step():
        for k in range(n):
            ihb.compute(d_frames[k], B, out=outs[k], stream=stream)
    plain_step()
    plain_steps = max(2, min(args.steps, 10))
    ms_plain = timed(torch, stream, plain_step, plain_steps) / plain_steps
    log(f"[bench] plain loop: {ms_plain:.3f} ms/step")

    ceiling = write_ceiling(torch, stream)
    log(f"[bench] write-stream ceiling (fill): {ceiling:.0f} GB/s")

    rec = {
        "metric": METRIC, "value": value, "unit": "entries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"disc_sequence_{n}x{H}x{W}_B{B}", "frames": n, "H": H, "W": W, "B": B,
                   "form": "batched_graph", "tile": list(tile[:2]), "nontemporal": tile[2],
                   "parallelism": "single_gpu"},
        "hbm_frac_step": step_gbs / HBM_PEAK_GBS,
        "plain_loop": {"value": entries_step / (ms_plain / 1e3), "ms_per_step": ms_plain,
                       "speedup_batched": ms_plain / ms_step},
        "phase_ms_per_step": {k: ph[k] / args.steps for k in ("agg_ms", "scan_ms", "tile_ms")},
        "write_ceiling_gbs": ceiling,
        "roofline": {"bound": "hbm", "kernel": "tile_batch_kernel", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_launch": alg_bytes_launch},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(frames, B, args.cpu_seconds)
    plan.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
