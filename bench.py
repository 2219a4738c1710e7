#!/usr/bin/env python3
"""SAFR frames/s at MORFEO scale on one MI355X, with the roofline of the dominant kernel.

Workload: the MORFEO-like geometry with J = 9 guide stars (6 laser stars at
45 arcsec with the cone effect of a 90 km sodium layer, 3 natural tip/tilt
stars at 80 arcsec), L = 9 layers from 0 to 16 km, 69 x 69 pupil grids
zero-extended into 256 x 256 periodic grids, FP32.  One step is one batched
call reconstructing --frames independent frames through the whole
hard-real-time path (Alg. 1); the one-frame-per-call latency (the real-time
loop's mode) is reported beside it.  Inputs are seeded synthetic frames (von
Karman screens, 35-layer synthetic profile, 2% noise, frozen flow) resident in
HBM before timing starts.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SAFR frames/s at MORFEO scale (J=9,L=9,256²) + HBM/MFMA roofline % at rel-L2≤1e-4"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(desc, n, frames=1):
    """Bytes each kernel of one launch must move (inputs + outputs + B read once), per the design notes."""
    M, J, L, G = desc.M, desc.J, desc.L, desc.groups
    Kh = M // 2 + 1
    wf = J * n * n * 4
    R = J * Kh * n * 8
    B = sum(int(desc.B_complex_per_group[g]) for g in range(G)) * 8
    C = G * L * Kh * M * 8
    out = L * M * M * 4
    return {
        "rows": frames * (wf + R),
        "cols": frames * (R + C) + B,
        "out": frames * (C + out),
        "frame": frames * (wf + out) + B,
    }


def cpu_baseline(geo, budget_s: float):
    """The FP64 oracle timed on the host cores on a bounded sample of the same workload."""
    import numpy as np

    import synth
    from oracle import safr as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    plan = O.precompute_geometry(geo)
    frames = synth.frames(geo, 64, first=10_000)
    t0 = time.perf_counter()
    done = 0
    while done < len(frames):
        O.reconstruct(plan, frames[done].astype(np.float64))
        done += 1
        if time.perf_counter() - t0 > budget_s and done >= 2:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} MORFEO-like frames (J=9, L=9, M=256) through the FP64 oracle "
                      f"(dense DFTs, precompute excluded), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--frames", type=int, default=64, help="independent frames per step (one batched call)")
    ap.add_argument("--single-calls", type=int, default=2000, help="one-frame calls timed for the latency figure")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build measures one GPU (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2510_19542_amd import safr as S

    dev = torch.device("cuda:0")
    geo = synth.preset("C2")
    F = args.frames
    print(f"bench: precompute {geo.name} (J={geo.J}, L={geo.L}, M={geo.M}, n={geo.n})", file=sys.stderr, flush=True)
    plan = S.precompute_geometry(geo)             # batched plan
    plan1 = S.precompute_geometry(geo)            # single-frame plan (tuned separately)
    desc = plan.desc
    pool = torch.from_numpy(synth.frames(geo, 2 * F)).to(dev)
    out = torch.empty((F, geo.L, geo.M, geo.M), dtype=torch.float32, device=dev)
    need = S.safr_workspace_size(plan, F)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    stream = torch.cuda.current_stream()
    tuned = tuned1 = None
    if not args.no_autotune:
        tuned = S.safr_autotune(plan, F, pool[:F], out, S.SAFR_FP32, 5, stream)
        tuned1 = S.safr_autotune(plan1, 1, pool[0], out[0], S.SAFR_FP32, 20, stream)
        print(f"bench: autotuned batched {tuned}, single {tuned1}", file=sys.stderr, flush=True)

    # batched throughput: each step reconstructs F frames in one call
    batches = [pool[:F], pool[F:]]
    for i in range(args.warmup):
        S.safr_reconstruct_batched(plan, F, batches[i % 2], out, S.SAFR_FP32, stream)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for i in range(args.steps):
        S.safr_reconstruct_batched(plan, F, batches[i % 2], out, S.SAFR_FP32, stream)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    fps = F * 1000.0 / ms_step

    # single-frame calls (the real-time mode): latency per frame
    for i in range(200):
        S.safr_reconstruct(plan1, pool[i % len(pool)], out[0], stream)
    torch.cuda.synchronize()
    t0.record(stream)
    for i in range(args.single_calls):
        S.safr_reconstruct(plan1, pool[i % len(pool)], out[0], stream)
    t1.record(stream)
    torch.cuda.synchronize()
    us_single = t0.elapsed_time(t1) * 1000.0 / args.single_calls

    # per-kernel durations of the batched call (HIP events on the launch stream, inside the library)
    stage_ms = S.safr_time_stages(plan, F, batches[0], out, S.SAFR_FP32, 20, stream)
    stage1_ms = S.safr_time_stages(plan1, 1, pool[0], out[0], S.SAFR_FP32, 50, stream)
    names = ["rows", "cols", "out"]
    ab = algorithmic_bytes(desc, geo.n, F)
    dom = int(np.argmax(stage_ms))
    achieved = ab[names[dom]] / (stage_ms[dom] * 1e-3) / 1e9
    kernel_names = {"rows": f"safr::rows_kernel<{geo.M}>", "cols": f"safr::cols_fixed<{geo.M}, 9, 6, 3>",
                    "out": f"safr::out_kernel<{geo.M}, rows, true>"}
    result = {
        "metric": METRIC,
        "value": round(fps, 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"MORFEO-like frames: J=9 (6 LGS + 3 NGS, split tomography), L=9, n=69, "
                               f"M=256, FP32; {F} independent frames per step in one batched call",
                   "frames_per_step": F, "J": geo.J, "L": geo.L, "M": geo.M, "n": geo.n,
                   "autotuned": {"batched": tuned, "single": tuned1}},
        "roofline": {"kernel": kernel_names[names[dom]], "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_launch": ab[names[dom]], "kernel_ms": round(stage_ms[dom], 6)},
        "stage_ms": {k: round(v, 6) for k, v in zip(names, stage_ms)},
        "frame_alg_bytes": algorithmic_bytes(desc, geo.n, 1)["frame"],
        "single_frame": {"us_per_frame": round(us_single, 3), "frames_per_s": round(1e6 / us_single, 1),
                         "stage_ms": {k: round(v, 6) for k, v in zip(names, stage1_ms)}},
    }
    if not args.no_cpu_baseline:
        print("bench: CPU baseline (FP64 oracle)", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(geo, args.cpu_budget)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
