#!/usr/bin/env python3
"""Fusion throughput on one MI355X: the 100-frame 640x480 RGB-D room sequence, 4 levels.

A step is one pass of the whole fusion hot path over the sequence: reset the map, then for each of
the 100 frames allocate, integrate (projective update, variance, merging criterion) and finish the
frame.  The depth frames are resident in HBM before the timed region starts.

Prints ONE JSON line: metric / value (M valid points fused per second) plus G voxel updates/s, the
roofline of the dominant kernel (projective update) measured with HIP events on the library's
stream, and the CPU oracle's throughput on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STATE_BYTES = 12  # FP32 D + uint32 W + FP32 S2 per voxel


def algorithmic_bytes_integrate(frames, width, height):
    """Bytes the projective-update kernel must move for the census of one sequence (lower bound):
    read + write of each updated voxel of an existing block, the full zero-initialised write of
    each new block, one read of each depth pixel, the block-table scan (key + info, 12 B per
    allocated block per frame) and the pooled read/write of merged blocks."""
    s = STATE_BYTES
    total = 0
    for f in frames:
        upd_old = f["observations"] - f["fresh_observations"]
        total += 2 * s * upd_old
        total += s * 512 * f["new_blocks"]
        total += 4 * width * height
        total += 12 * f["blocks"]
        m = f["merges"]
        total += s * ((512 + 64) * m[0] + (64 + 8) * m[1] + (8 + 1) * m[2])
    return total


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--cpu-frames", type=int, default=40, help="oracle sample: first N frames")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the fusion of one map runs "
              "on one device; see the sharding notes in the design document)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2511_21459_amd as mrh
    from workloads import configs, room_sequence

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    depths, cam, poses, _ = room_sequence(n_frames=100, frames=range(args.frames))
    H, W = depths.shape[1:]
    dev = torch.from_numpy(depths).cuda()
    frames = [dev[k] for k in range(args.frames)]
    torch.cuda.synchronize()

    fmap = mrh.Map(**configs.ROOM)

    def step():
        fmap.reset()
        for k in range(args.frames):
            fmap.integrate_depth(frames[k], cam.K, poses[k])

    # census: per-frame statistics of one pass (the workload is deterministic)
    fmap.reset()
    census = []
    for k in range(args.frames):
        fmap.integrate_depth(frames[k], cam.K, poses[k])
        last, _ = fmap.sync()
        census.append(last)
    valid_points = sum(f["valid_points"] for f in census)
    updates = sum(f["observations"] for f in census)

    for _ in range(args.warmup):
        step()
    fmap.sync()

    # timed region A: throughput (no profiling events)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    _, tot = fmap.sync()
    ms_per_step = wall * 1e3 / args.steps

    # timed region B: the same steps with every launch bracketed by events on the map's stream
    fmap.profile(True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step()
    prof = fmap.profile_collect()
    fmap.profile(False)
    k_ms, k_launches = prof["integrate_depth"]
    avg_launch_s = k_ms / k_launches / 1e3
    bytes_per_launch = algorithmic_bytes_integrate(census, W, H) / args.frames
    achieved = bytes_per_launch / avg_launch_s / 1e9

    result = {
        "metric": "M points/s fused + G voxel-updates/s; batched/FP16 vs plain FP32 fusion",
        "value": round(valid_points * args.steps / wall / 1e6, 3),
        "unit": "M points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"room RGB-D orbit, {args.frames} frames {W}x{H}, 1/2/4/8 cm levels, tau 3 cm",
                   "frames_per_step": args.frames, "valid_points_per_step": valid_points,
                   "voxel_updates_per_step": updates, "blocks_at_end": census[-1]["blocks"],
                   "merges_per_step": [sum(f["merges"][n] for f in census) for n in range(4)]},
        "g_voxel_updates_per_s": round(updates * args.steps / wall / 1e9, 4),
        "gpu_event_ms_per_step": round(gpu_ms / args.steps, 3),
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in prof.items()},
        "roofline": {"kernel": "k_integrate_depth", "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": int(bytes_per_launch),
                     "avg_launch_us": round(avg_launch_s * 1e6, 3)},
        "cpu_baseline": None,
    }
    if tot["error_flags"]:
        result["errors"] = tot["error_flags"]

    if not args.no_cpu_baseline:
        import oracle

        n = min(args.cpu_frames, args.frames)
        o = oracle.OracleMap(**configs.oracle_kwargs(configs.ROOM))
        t0 = time.perf_counter()
        pts = 0
        for k in range(n):
            pts += o.integrate_depth(depths[k], cam.K, poses[k])["valid_points"]
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(pts / dt / 1e6, 4), "unit": "M points/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"first {n} of the {args.frames} frames, FP64 oracle, one thread "
                                            f"({dt:.1f} s)"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
