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

Prints one JSON line.  ``--gpus`` above 1 is refused: the benchmark runs on one GPU.
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
FP32_PEAK_TFLOPS = 157.3          # MI355X FP32 vector peak (published)

# launch shapes of the MORFEO-like plans, chosen by safr_autotune on an MI355X, the row teams by sweeps (one
# frame: 5 teams cut the 69 pupil rows into 7 chunks, few enough for the passes to add the tip/tilt plane
# shares themselves; 64 frames, inputs rotating over 8 batches as in the timed steps: 12 teams, chunks of 24,
# 24 and 21 rows, 1.5 us per step faster than 16 teams' 32, 32 and 5) (row teams, output rows, column frames
# per block, output frames per block, column frames together)
TUNED_BATCHED = (12, 8, 16, 8, 4)
TUNED_SINGLE = (5, 8, 1, 4, 1)


def apply_shape(S, plan, shape):
    for opt, v in zip((S.SAFR_OPT_ROW_TEAMS, S.SAFR_OPT_OUT_ROWS, S.SAFR_OPT_COL_FRAMES, S.SAFR_OPT_OUT_FRAMES,
                       S.SAFR_OPT_COL_TOGETHER), shape):
        S.safr_set_option(plan, opt, int(v))


def _fft_flops(M):
    """benchFFT convention: 5 M log2 M flops per complex 1-D transform of M points."""
    import math
    return 5.0 * M * math.log2(M)


def algorithmic_flops(desc, n, frames=1):
    """Operations of the hard-real-time step, counted with the cost model of Table 1 (benchFFT
    convention: 5 M log2 M per complex 1-D transform of M points, so a real 2-D transform of M x M
    points costs 2.5 M^2 log2 M^2, half in each direction; 8 flops per complex multiply-add of the
    apply; 2 flops per multiply-add).  Each kernel is credited only with the work it carries out:

    * rows: the forward row transforms of the transformed stars' n pupil rows (two real rows per
      complex M-point transform, ceil(n / 2) per star) and, for split tomography, the tip/tilt
      moments of every star (3 multiply-adds per pupil pixel);
    * cols: for the transformed group (the laser stars of a mixed asterism) the forward column
      transforms of the M / 2 columns below the Nyquist column (B vanishes there), the plane removal
      of split tomography (2 complex-by-real multiply-adds per frequency and star), the apply
      (8 L G flops per frequency) and the inverse column transforms of the L layer spectra;
    * out: the inverse row transforms (M / 2 complex transforms per layer, two real rows each) and,
      for split tomography, the natural-star layers from the basis images (one multiply-add per
      pixel, layer and image).

    ``method`` is the whole step as Table 1 counts it for the geometry (J forward and groups x L
    inverse real 2-D transforms, the apply over the half spectrum): the work of the paper's
    algorithm, which the GPU path does not all perform (pruned rows, natural stars through basis
    images, no Nyquist column)."""
    import math
    M, J, L, G = desc.M, desc.J, desc.L, desc.groups
    Gt = int(desc.group_size[0])                 # stars transformed (laser group when mixed)
    nb = 2 * int(desc.group_size[1]) if G == 2 else 0
    c1 = _fft_flops(M)
    KC = M // 2                                  # columns transformed (below the Nyquist column)
    rows = Gt * ((n + 1) // 2) * c1 + (6.0 * J * n * n if G == 2 else 0.0)
    cols = (Gt + L) * KC * c1 + 8.0 * L * Gt * KC * M + (8.0 * Gt * KC * M if G == 2 else 0.0)
    out = L * KC * c1 + 2.0 * nb * L * M * M
    per = {"rows": rows, "cols": cols, "out": out}
    fft2 = 2.5 * M * M * math.log2(M * M)
    method = J * fft2 + G * L * fft2 + 8.0 * L * J * (M // 2 + 1) * M
    return {"step": frames * (rows + cols + out), "per_kernel": {k: frames * v for k, v in per.items()},
            "method_step": frames * method}


def algorithmic_bytes(desc, n, frames=1):
    """Algorithmic bytes of one launch sequence, with the same split over the kernels as the flops.

    Per kernel, what it must move of the step's inputs, outputs and operators: rows the wavefronts;
    cols the FP32 B of the transformed group for the columns it processes, read once; out the layers
    and, for mixed asterisms, the natural-star basis images, read once.  ``step`` is their sum;
    ``method`` is what the paper's algorithm itself needs (wavefronts in, layers out, both groups' B
    over the half spectrum).  ``with_intermediates`` adds the intermediate spectra each kernel moves
    (R: row spectra of the transformed stars' pupil rows, C: layer half-spectra of the transformed
    group), implementation overhead of the two-pass transforms.
    """
    M, J, L, G = desc.M, desc.J, desc.L, desc.groups
    Kh, KC = M // 2 + 1, M // 2
    Gt = int(desc.group_size[0])
    nb = 2 * int(desc.group_size[1]) if G == 2 else 0
    wf = J * n * n * 4
    R = Gt * KC * n * 8
    B = KC * M * L * Gt * 8
    Bmethod = sum(int(desc.B_complex_per_group[g]) for g in range(G)) * 8
    C = L * KC * M * 8
    out = L * M * M * 4
    basis = L * nb * M * M * 4
    per = {"rows": frames * wf, "cols": B, "out": frames * out + basis}
    return {
        "step": sum(per.values()),
        "per_kernel": per,
        "method_step": frames * (wf + out) + Bmethod,
        "with_intermediates": {"rows": frames * (wf + R), "cols": frames * (R + C) + B,
                               "out": frames * (C + out) + basis},
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_morfeo_step.json")
KERNEL_SOURCES = ["k_rows.hip", "k_cols.hip", "k_out.hip", "fft_device.h", "safr_internal.h"]


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_19542_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# the kernels of each timed stage of the batched MORFEO-like step
KERNEL_NAMES = {"rows": "rows_kernel<256, 69>", "cols": "cols_kernel<256, 4, 6, 9, 1, 1, 69, false>",
                "out": "out_kernel<256, 8, 6, false>"}


def measured_traffic(frames: int, stage: str = None):
    """HBM bytes per step (or per launch of one stage's kernels) from the committed counter summary, if it
    was taken on the current kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_digest") != kernel_source_digest() or int(t.get("frames", -1)) != frames:
        return None
    if stage is None:
        return t.get("bytes_per_step")
    parts = [v["bytes"] for v in t.get("per_kernel", {}).values() if v.get("stage") == stage]
    return sum(parts) if parts else None


def _timed(fn, iters, stream, torch, host=None):
    """GPU milliseconds per call between two events around `iters` back-to-back calls; with a dict `host`,
    also the host's microseconds per call spent issuing them (host["us"])."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(iters):
        fn()
    t1 = time.perf_counter()
    e1.record(stream)
    torch.cuda.synchronize()
    if host is not None:
        host["us"] = (t1 - t0) * 1e6 / iters
    return e0.elapsed_time(e1) / iters


def run_c3(S, torch, stream):
    """1024 consecutive frozen-flow frames of the 8 m geometry in one call, FP32 and BF16x3."""
    import synth
    geo = synth.preset("C3")
    F = 1024
    x = torch.from_numpy(synth.frames(geo, F)).cuda()
    out = torch.empty((F, geo.L, geo.M, geo.M), device="cuda")
    res = {"workload": "C1 geometry (J=4 NGS, L=2, n=33, M=64), 1024 frozen-flow frames per call, replayed "
                       "from a captured HIP graph on a non-default stream (eager launches beside it)"}
    for name, prec in (("fp32", S.SAFR_FP32), ("bf16x3", S.SAFR_BF16X3)):
        plan = S.precompute_geometry(geo)
        _attach_workspace(S, torch, plan, F, prec)
        tuned = S.safr_autotune(plan, F, x, out, prec, 3, stream)
        timing, host = {}, {}
        # eager launches, then the launch sequence captured once in a HIP graph and replayed (the stream is
        # not the legacy default stream, which cannot be captured); the host time spent issuing each call is
        # kept beside the GPU time (a call whose issue takes longer than its kernels leaves the GPU waiting)
        for mode in ("eager", "graph"):
            S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 1 if mode == "graph" else 0)
            # the first replays of a new graph cost the host up to 100 us each, later ones about 20 us
            for _ in range(20):
                S.safr_reconstruct_batched(plan, F, x, out, prec, stream)
            host[mode] = {}
            timing[mode] = _timed(lambda: S.safr_reconstruct_batched(plan, F, x, out, prec, stream), 200, stream,
                                  torch, host[mode])
        S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 0)
        st = S.safr_time_stages(plan, F, x, out, prec, 10, stream)
        ms = timing["graph"]
        res[name] = {"ms_per_call": round(ms, 5), "frames_per_s": round(F * 1000.0 / ms, 1),
                     "ms_per_call_eager": round(timing["eager"], 5),
                     "frames_per_s_eager": round(F * 1000.0 / timing["eager"], 1),
                     "host_us_per_call": {m: round(host[m]["us"], 2) for m in host},
                     "stage_ms": [round(v, 5) for v in st], "autotuned": tuned}
    return res


def run_col_mfma(S, torch, geo, batches, out, stream, steps):
    """The batched MORFEO-like launch with the column pass's per-frequency products on the matrix cores
    (4 x 4 x 1 FP32 products: 4 frames x 4 layers, one star per step) against the vector units, on a plan
    of its own with the stored launch shapes, each after 200 steps of load (switching synchronises)."""
    F = int(batches[0].shape[0])
    plan = S.precompute_geometry(geo)
    apply_shape(S, plan, TUNED_BATCHED)
    _attach_workspace(S, torch, plan, F, S.SAFR_FP32)
    res = {"workload": f"MORFEO-like frames, {F} per call, stored launch shapes"}
    for name, on in (("matrix_cores", 1), ("vector_units", 0)):
        S.safr_set_option(plan, S.SAFR_OPT_COL_MFMA, on)
        for i in range(200):
            S.safr_reconstruct_batched(plan, F, batches[i % len(batches)], out, S.SAFR_FP32, stream)
        ms = _timed(lambda: S.safr_reconstruct_batched(plan, F, batches[0], out, S.SAFR_FP32, stream), steps,
                    stream, torch)
        st = S.safr_time_stages(plan, F, batches[0], out, S.SAFR_FP32, 20, stream)
        res[name] = {"us_per_step": round(ms * 1e3, 2), "cols_us": round(st[1] * 1e3, 2)}
    return res


def run_loop(S, torch, plan, geo, pool, calls):
    """One closed loop of the MORFEO-like geometry: POLC, reconstruction and integrator per time step.

    The measurement and command buffers stay fixed, as in a real-time loop, so the captured graph
    of the step is replayed on every call.
    """
    import numpy as np
    L, M = geo.L, geo.M
    wf = pool[0].clone()
    a = torch.zeros((L, M, M), dtype=torch.float32, device="cuda")
    gain = 0.5
    res = {"workload": "MORFEO-like geometry (J=9, L=9, n=69, M=256), one loop, gain 0.5, "
                       "fixed measurement and command buffers",
           "loop_rate_requirement_hz": [500, 1000]}
    cur = torch.cuda.current_stream()
    for name, graph in (("eager", 0), ("graph", 1)):
        S.safr_set_option(plan, S.SAFR_OPT_GRAPH, graph)
        s = torch.cuda.Stream() if graph else cur
        torch.cuda.synchronize()
        for _ in range(100):
            S.safr_loop_step(plan, 1, wf, a, gain, a, s)
        h = {}
        ms = _timed(lambda: S.safr_loop_step(plan, 1, wf, a, gain, a, s), calls, s, torch, h)
        res[f"us_per_step_{name}"] = round(ms * 1000.0, 3)
        res[f"host_us_per_step_{name}"] = round(h["us"], 3)
    S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 0)
    # per-step latency (events around every eager step): tail against the 1 ms period of a 1 kHz loop
    nstep = 1000
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nstep)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(cur)
        S.safr_loop_step(plan, 1, wf, a, gain, a, cur)
        e1.record(cur)
    torch.cuda.synchronize()
    lat = np.array([e0.elapsed_time(e1) * 1000.0 for e0, e1 in ev])
    res["per_step_latency_us"] = {"steps": nstep, "p50": round(float(np.percentile(lat, 50)), 2),
                                  "p99": round(float(np.percentile(lat, 99)), 2), "max": round(float(lat.max()), 2),
                                  "over_1ms": int((lat > 1000.0).sum())}
    out = torch.empty_like(wf)
    ms = _timed(lambda: S.safr_polc(plan, 1, wf, a, 1.0, out, cur), calls, cur, torch)
    res["us_per_polc_call"] = round(ms * 1000.0, 3)
    # Strehl estimate in a 3 x 3 grid of science directions over the central arcminute
    t = np.linspace(-30.0, 30.0, 3) * np.pi / (180.0 * 3600.0)
    dirs = np.array([(x, y) for x in t for y in t])
    ol = torch.zeros((1, len(dirs), geo.n, geo.n), dtype=torch.float32, device="cuda")
    sr = torch.empty((1, len(dirs)), dtype=torch.float32, device="cuda")
    ms = _timed(lambda: S.safr_strehl(plan, 1, dirs, ol, a, 0.5 / 2.2, sr, None, cur), calls, cur, torch)
    res["us_per_strehl_call_9_directions"] = round(ms * 1000.0, 3)
    best = min(res["us_per_step_eager"], res["us_per_step_graph"])
    res["steps_per_s"] = round(1e6 / best, 1)
    res["fraction_of_1khz_budget"] = round(best / 1000.0, 4)
    return res


def run_loop_strehl(S, torch, plan, geo, steps=60, gain=0.5):
    """Closed loop on a frozen-flow synthetic atmosphere (the 35-layer stand-in), Strehl in K band.

    Step t: the mirror holds a_t; the guide stars measure the residual wavefronts (with noise), the
    science directions see the residual phase; the step's command a_{t+1} = loop_step(residual, a_t)
    is applied at t + 1 (one step of delay).  Long-exposure Strehl: mean of the per-step Marechal
    estimates over the second half of the run.
    """
    import numpy as np
    import synth
    t = np.linspace(-30.0, 30.0, 3) * synth.ARCSEC
    dirs = np.array([(x, y) for x in t for y in t])
    sep = np.round(np.hypot(dirs[:, 0], dirs[:, 1]) / synth.ARCSEC, 1)
    sci = geo.replace(stars=[(float(x), float(y), synth.NGS) for x, y in dirs])
    screens = synth.truth_screens(geo, 0)
    scale = 0.5 / 2.2                                    # screens in rad at 500 nm -> rad at 2.2 um
    a = torch.zeros((1, geo.L, geo.M, geo.M), dtype=torch.float32, device="cuda")
    zero = torch.zeros_like(a)
    res = torch.empty((1, geo.J, geo.n, geo.n), dtype=torch.float32, device="cuda")
    sr = torch.empty((1, len(dirs)), dtype=torch.float32, device="cuda")
    sr0 = torch.empty_like(sr)
    late, open_ = [], []
    for step in range(steps):
        wf = torch.from_numpy(synth.simulate_wavefronts(geo, screens, step, frozen_flow=True)[None]
                              .astype(np.float32)).cuda()
        ol = torch.from_numpy(synth.simulate_wavefronts(sci, screens, step, frozen_flow=True, noise=False)[None]
                              .astype(np.float32)).cuda()
        S.safr_strehl(plan, 1, dirs, ol, a, scale, sr)
        S.safr_strehl(plan, 1, dirs, ol, zero, scale, sr0)
        S.safr_polc(plan, 1, wf, a, -1.0, res)
        S.safr_loop_step(plan, 1, res, a, gain, a)
        if step >= steps // 2:
            late.append(sr.cpu().numpy()[0])
            open_.append(sr0.cpu().numpy()[0])
    late, open_ = np.mean(late, axis=0), np.mean(open_, axis=0)
    out = {"workload": f"MORFEO-like geometry, frozen-flow 35-layer synthetic atmosphere (r0 = {geo.r0} m at "
                       f"500 nm), {steps} steps of 1 ms, gain {gain}, one step of delay, 3 x 3 science directions "
                       "over +-30 arcsec, Strehl at 2.2 um (Marechal), long exposure = mean of the second half",
           "le_strehl_by_separation_arcsec": {}, "uncorrected_strehl_mean": float(f"{open_.mean():.3g}")}
    for s_ in sorted(set(sep.tolist())):
        out["le_strehl_by_separation_arcsec"][str(s_)] = round(float(late[sep == s_].mean()), 4)
    return out


def run_recompute(S, torch, reps=3):
    """Soft-real-time refresh: wall time of the whole precomputation (Alg. 2) when alpha, the layer
    weights or the asterism change, against the loop period."""
    import numpy as np
    import synth
    res = {"what": "safr_precompute wall time (A_n, FP64 Jacobi SVD per frequency, filter, B in FP64/FP32, "
                   "natural-star basis images, BF16 tiles), needed when gamma or the asterism changes; "
                   "safr_update_alpha wall time (filter and B from the kept SVDs) when only the "
                   "regularisation changes", "loop_period_ms_at_1khz": 1.0}
    for name in ("C2", "C1", "C5-Mid"):
        geo = synth.preset(name)
        variants = [geo, geo.replace(alpha=geo.alpha * 2.0), geo.replace(weights=np.roll(geo.weights, 1))]
        ms = []
        for r in range(reps):
            g = variants[r % len(variants)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = S.precompute_geometry(g)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
            plan.close()
        res[name] = {"ms": [round(v, 2) for v in ms], "median_ms": round(float(np.median(ms)), 2),
                     "loop_periods_at_1khz": round(float(np.median(ms)) / 1.0, 1)}
        # refresh of the filter from the kept SVDs (safr_update_alpha): alpha alone, then both alphas
        plan = S.precompute_geometry(geo)
        for what, f_tt in (("alpha_only", 1.0), ("alpha_and_alpha_tt", 2.0)):
            ms = []
            for r in range(reps):
                scale = 1.5 + r
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                S.safr_update_alpha(plan, geo.alpha * scale, geo.alpha_tt * (f_tt ** (r + 1)))
                ms.append((time.perf_counter() - t0) * 1e3)
            res[name]["update_" + what + "_ms"] = round(float(np.median(ms)), 3)
        plan.close()
    return res


_WS = {}


def _attach_workspace(S, torch, plan, frames, prec):
    """Point the plan at one shared workspace (plans here run one after another on one stream)."""
    need = S.safr_workspace_size(plan, frames, prec)
    if _WS.get("bytes", 0) < need:
        _WS["t"] = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        _WS["bytes"] = need
    S.safr_set_workspace(plan, (_WS["t"].data_ptr() + 255) & ~255, need)


def _layer_error(torch, rec, truth):
    """Mean over frames of the relative layer residual after per-layer piston removal."""
    r = rec - rec.mean(dim=(2, 3), keepdim=True)
    t = truth - truth.mean(dim=(2, 3), keepdim=True)
    num = torch.linalg.vector_norm((r - t).flatten(1), dim=1)
    den = torch.linalg.vector_norm(t.flatten(1), dim=1)
    return float((num / den).mean())


def run_c4(S, torch, stream, frames):
    """Learned filter on the 8 m geometry (periodic-exact data on the whole grid)."""
    import numpy as np

    import synth
    from paper_2510_19542_amd import learn as Lrn
    base = synth.preset("C1")
    geo = base.replace(n=base.M)
    t0 = time.perf_counter()
    params, _ = Lrn.train(geo, frames=frames, epochs=3, batch=16, lr=2e-3, seed=1)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    etas = (0.005, 0.01, 0.02, 0.05)
    truth, wfs = synth.periodic_frames(geo, range(20000, 21000), etas)
    tt = torch.from_numpy(truth.astype(np.float32)).cuda()
    alphas = [geo.alpha] + [float(a) for a in np.logspace(-6, 0, 25)]
    tik = [S.precompute_geometry(geo, pupil=None, alpha=a) for a in alphas]
    F = len(truth)
    for p in tik:
        _attach_workspace(S, torch, p, F, S.SAFR_FP32)
    out = torch.empty((F, geo.L, geo.M, geo.M), device="cuda")
    # truncated SVD over the same alpha grid: one plan, B rebuilt from its kept SVDs for each alpha
    tsvd = S.precompute_geometry(geo, pupil=None, filter=S.SAFR_FILTER_TSVD)
    _attach_workspace(S, torch, tsvd, F, S.SAFR_FP32)
    # Tikhonov with a per-frequency alpha_n = alpha (1 + |n|^2 / 64)^(1/3): the exponent is the gap between the
    # von Karman spectral slope (11/6) and the Sobolev beta = 1.5 the operator already carries
    nidx = np.where(np.arange(geo.M) <= (geo.M - 1) // 2, np.arange(geo.M), np.arange(geo.M) - geo.M)
    wmap = (1.0 + (nidx[:, None] ** 2 + nidx[None, :] ** 2) / 64.0) ** (1.0 / 3.0)
    wtik = S.precompute_geometry(geo, pupil=None)
    _attach_workspace(S, torch, wtik, F, S.SAFR_FP32)
    # the Sobolev smoothness beta of the layer prior (Sec. 3.1): one plan per beta, alpha swept on each
    betas = (0.0, 0.5, 1.0, 1.5, 2.0, 2.5)
    bplans = [S.precompute_geometry(geo.replace(beta=bt), pupil=None) for bt in betas]
    for p in bplans:
        _attach_workspace(S, torch, p, F, S.SAFR_FP32)
    balphas = [float(a) for a in np.logspace(-8, 0, 17)]
    res = {"workload": f"C1 geometry with data on the whole 64x64 grid; trained on {frames} frames "
                       f"(eta ~ U[0.5%, 5%]), evaluated on 1000 held-out seeds",
           "train_s": round(train_s, 2), "heldout": {}}
    speed = {}
    for eta, wf in zip(etas, wfs):
        x = torch.from_numpy(wf).cuda()
        lrn = S.precompute_geometry(geo, pupil=None, filter=S.SAFR_FILTER_MLP, mlp=params, noise=eta)
        _attach_workspace(S, torch, lrn, F, S.SAFR_FP32)
        S.safr_reconstruct_batched(lrn, F, x, out, S.SAFR_FP32, stream)
        e_l = _layer_error(torch, out, tt)
        errs = []
        for p in tik:
            S.safr_reconstruct_batched(p, F, x, out, S.SAFR_FP32, stream)
            errs.append(_layer_error(torch, out, tt))
        b = int(np.argmin(errs[1:])) + 1
        terrs = []
        for a in alphas[1:]:
            S.safr_update_alpha(tsvd, a, a, S.SAFR_FILTER_TSVD)
            S.safr_reconstruct_batched(tsvd, F, x, out, S.SAFR_FP32, stream)
            terrs.append(_layer_error(torch, out, tt))
        tb = int(np.argmin(terrs))
        werrs = []
        for a in alphas[1:]:
            S.safr_update_alpha(wtik, a, a, S.SAFR_FILTER_TIKHONOV, wmap)
            S.safr_reconstruct_batched(wtik, F, x, out, S.SAFR_FP32, stream)
            werrs.append(_layer_error(torch, out, tt))
        wb = int(np.argmin(werrs))
        bsweep = {}
        for bt, p in zip(betas, bplans):
            berrs = []
            for a in balphas:
                S.safr_update_alpha(p, a, a)
                S.safr_reconstruct_batched(p, F, x, out, S.SAFR_FP32, stream)
                berrs.append(_layer_error(torch, out, tt))
            bb = int(np.argmin(berrs))
            bsweep[str(bt)] = {"best": round(berrs[bb], 5), "best_alpha": float(f"{balphas[bb]:.3g}")}
        res["heldout"][str(eta)] = {"learned": round(e_l, 5), f"tikhonov_alpha_{geo.alpha:g}": round(errs[0], 5),
                                    "tikhonov_best": round(errs[b], 5), "best_alpha": float(f"{alphas[b]:.3g}"),
                                    "tsvd_best": round(terrs[tb], 5), "tsvd_best_alpha": float(f"{alphas[1 + tb]:.3g}"),
                                    "weighted_tikhonov_best": round(werrs[wb], 5),
                                    "weighted_best_alpha": float(f"{alphas[1 + wb]:.3g}"),
                                    "tikhonov_best_by_beta": bsweep}
        if not speed:
            for name, p in (("learned", lrn), ("tikhonov", tik[0])):
                speed[name] = round(F * 1000.0 / _timed(
                    lambda: S.safr_reconstruct_batched(p, F, x, out, S.SAFR_FP32, stream), 20, stream, torch), 1)
    res["frames_per_s"] = speed
    res["training_objective"] = c4_objective_bound(torch, geo, params, etas, alphas[1:])
    res["heldout_metapupil"] = c4_metapupil(S, torch, stream, base, params, etas, alphas[1:])
    return res, params


def metapupil_masks(geo):
    """(L, M, M) bool: the pixels of each output layer's grid that some guide star's line of sight through
    the aperture crosses (the union over stars of the aperture footprint at that height; layer l's grid has
    spacing c_l pitch, centred at index M / 2)."""
    import numpy as np
    M, p = geo.M, geo.pitch
    has_lgs = any(int(s[2]) == 1 for s in geo.stars)
    idx = (np.arange(M) - M / 2.0) * p
    out = np.zeros((len(geo.heights), M, M), dtype=bool)
    r_out, r_in = geo.diameter / 2.0, geo.obstruction * geo.diameter / 2.0
    for l, h in enumerate(geo.heights):
        c_l = (1.0 - h / geo.h_lgs) if has_lgs else 1.0
        X, Y = np.meshgrid(c_l * idx, c_l * idx, indexing="ij")
        for ax, ay, kind in geo.stars:
            c_g = (1.0 - h / geo.h_lgs) if int(kind) == 1 else 1.0
            # the pupil point r maps to c_g r + theta h on the layer
            rx, ry = (X - ax * h) / c_g, (Y - ay * h) / c_g
            rr = np.hypot(rx, ry)
            out[l] |= (rr <= r_out) & (rr >= r_in)
    return out


def c4_metapupil(S, torch, stream, geo, params, etas, alphas, count=250):
    """The learned filter (trained on periodic whole-grid data) and best-tuned Tikhonov on pupil-masked frames of
    the 8 m geometry: bilinear line-of-sight wavefronts of frozen von Karman screens with white noise, held-out
    frames 20000.., the relative layer residual over each layer's metapupil after per-layer piston removal
    (mean over frames)."""
    import numpy as np
    import synth
    masks = torch.from_numpy(metapupil_masks(geo)).cuda()
    ids = range(20000, 20000 + count)
    screens = [synth.truth_screens(geo, f) for f in ids]
    truth = torch.from_numpy(np.stack([synth.truth_layers(geo, sc, f) for sc, f in zip(screens, ids)])
                             .astype(np.float32)).cuda()
    F = count
    out = torch.empty((F, geo.L, geo.M, geo.M), device="cuda")
    m = masks[None].float()
    cnt = m.sum(dim=(2, 3), keepdim=True)

    def err():
        r = (out - truth) * m
        r = (r - r.sum(dim=(2, 3), keepdim=True) / cnt) * m
        t = truth * m
        t = (t - t.sum(dim=(2, 3), keepdim=True) / cnt) * m
        num = torch.linalg.vector_norm(r.flatten(1), dim=1)
        den = torch.linalg.vector_norm(t.flatten(1), dim=1)
        return float((num / den).mean())

    tik = S.precompute_geometry(geo)
    _attach_workspace(S, torch, tik, F, S.SAFR_FP32)
    res = {"workload": f"C1 geometry with its pupil (n=33, M=64), {count} held-out frames: bilinear line-of-sight "
                       "wavefronts of von Karman screens with white noise; layer residual over each layer's "
                       "metapupil after per-layer piston removal; the network trained on periodic whole-grid data"}
    for eta in etas:
        x = torch.from_numpy(np.stack([synth.simulate_wavefronts(geo, sc, f, eta=eta) for sc, f in zip(screens, ids)])
                             .astype(np.float32)).cuda()
        lrn = S.precompute_geometry(geo, filter=S.SAFR_FILTER_MLP, mlp=params, noise=eta)
        _attach_workspace(S, torch, lrn, F, S.SAFR_FP32)
        S.safr_reconstruct_batched(lrn, F, x, out, S.SAFR_FP32, stream)
        e_l = err()
        errs = []
        for a in alphas:
            S.safr_update_alpha(tik, a, a)
            S.safr_reconstruct_batched(tik, F, x, out, S.SAFR_FP32, stream)
            errs.append(err())
        b = int(np.argmin(errs))
        res[str(eta)] = {"learned": round(e_l, 5), "tikhonov_best": round(errs[b], 5), "best_alpha": float(f"{alphas[b]:.3g}"),
                         "tikhonov_alpha_0.001": round(errs[int(np.argmin(np.abs(np.log(np.asarray(alphas) / 1e-3))))], 5)}
    return res


def c4_objective_bound(torch, geo, params, etas, alphas, count=1000):
    """The learned filter's training objective (frame-averaged full-grid layer residual, normalised by the
    expected layer energy) on held-out method-generated frames at each noise level, beside best-tuned
    Tikhonov over the alpha grid and the closed-form optimal filter factors for those frames, which bound
    every filter's objective from below (Sec. 3.1 filter functions)."""
    import numpy as np

    import synth
    from paper_2510_19542_amd import learn as Lrn
    out = {"frames": count, "first_seed": 20000}
    for eta in etas:
        tr = Lrn.Trainer(geo, synth.vk_amplitude(geo).reshape(geo.L, -1), count)
        Lrn.add_seeded_frames(tr, 20000, count, eta_range=(eta, eta))
        idx = np.arange(count)
        net = tr.network_loss(params, idx)
        tik = [tr.tikhonov_loss(idx, a) for a in alphas]
        b = int(np.argmin(tik))
        opt = tr.optimal_filter(idx)
        tr.close()
        out[str(eta)] = {"learned": float(f"{net:.6g}"), "tikhonov_best": float(f"{tik[b]:.6g}"),
                         "tikhonov_best_alpha": float(f"{alphas[b]:.3g}"), "optimal_bound": float(f"{opt:.6g}"),
                         "learned_gain_over_tikhonov_pct": round(100.0 * (tik[b] - net) / tik[b], 3),
                         "learned_gap_to_bound_pct": round(100.0 * (net - opt) / opt, 3),
                         "share_of_tikhonov_gap_closed": round((tik[b] - net) / (tik[b] - opt), 3)}
    return out


def run_c5(S, torch, stream, params):
    """64 instances of three sizes (16 frames each) with the learned filter, one graph launch per step."""
    import collections

    import synth
    count = collections.Counter(synth.c5_instances(64))
    names = [n for n in synth.C5_SIZES if count[n]]
    geos = [synth.preset(n) for n in names]
    frames = [16 * count[n] for n in names]
    plans = [S.precompute_geometry(g, filter=S.SAFR_FILTER_MLP, mlp=params, noise=0.02) for g in geos]
    wf_host = [synth.random_wavefronts(g, f, seed=50 + i) for i, (g, f) in enumerate(zip(geos, frames))]
    wf = [torch.from_numpy(w).cuda() for w in wf_host]
    outs = [torch.empty((f, g.L, g.M, g.M), device="cuda") for g, f in zip(geos, frames)]
    m = S.Multi(plans, frames)
    m.autotune(wf, outs, iters=3, stream=stream)
    for _ in range(3):
        m.execute(wf, outs, stream=stream)
    ms = _timed(lambda: m.execute(wf, outs, stream=stream), 20, stream, torch)
    total = sum(frames)
    torch.cuda.synchronize()
    # one frame of every size (its first and last), for the oracle check of the CPU leg
    samples = {n: (g, w[[0, -1]], o[[0, -1]].cpu().numpy()) for n, g, w, o in zip(names, geos, wf_host, outs)}
    m.close()
    return {"workload": "64 instances drawn from {8 m/4 NGS/M=64/L=3, 20 m/6 LGS/M=128/L=5, "
                        "39 m MORFEO-like/M=256/L=9}, 16 frames each, learned filter (eta 2%), one graph launch "
                        "per step on a non-default stream (the sizes as parallel branches)",
            "instances": {n: count[n] for n in names}, "frames_per_step": total,
            "ms_per_step": round(ms, 5), "frames_per_s": round(total * 1000.0 / ms, 1)}, samples


def cpu_baseline(geo, budget_s: float, frames_in=None, gpu_out=None):
    """The FP64 oracle timed on the host cores on a bounded sample of the same workload.

    frames_in / gpu_out: the timed launch's first input batch and the GPU layers it produced; the
    frames the oracle reconstructs are taken from that batch and compared with the GPU layers
    (relative L2 per frame, the FP32 tolerance is 1e-5)."""
    import numpy as np

    import synth
    from oracle import safr as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    tp = time.perf_counter()
    plan = O.precompute_geometry(geo)
    precompute_s = time.perf_counter() - tp
    frames = frames_in if frames_in is not None else synth.frames(geo, 64, first=10_000)
    t0 = time.perf_counter()
    done = 0
    errs = []
    while done < len(frames):
        want = O.reconstruct(plan, frames[done].astype(np.float64))
        if gpu_out is not None:
            errs.append(float(np.linalg.norm(gpu_out[done].astype(np.float64) - want) / np.linalg.norm(want)))
        done += 1
        if time.perf_counter() - t0 > budget_s and done >= 2:
            break
    dt = time.perf_counter() - t0
    # the same oracle on one thread (BLAS pool limited), a shorter bounded sample
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            k = 0
            while k < len(frames):
                O.reconstruct(plan, frames[k].astype(np.float64))
                k += 1
                if time.perf_counter() - t1 > budget_s / 2:
                    break
            one = round(k / (time.perf_counter() - t1), 4)
    except Exception:
        pass
    res = {"value": done / dt, "unit": "frames/s", "cores": cores, "kind": "oracle", "value_1_thread": one,
           "sample": f"frames 0..{done - 1} of the timed launch's first input batch (MORFEO-like, J=9, L=9, "
                     f"M=256) through the FP64 oracle (dense DFTs, precompute excluded), {dt:.1f} s",
           "precompute_s": round(precompute_s, 2)}
    if errs:
        res["gpu_vs_oracle_rel_l2"] = {"frames": done, "max": float(f"{max(errs):.3e}"),
                                       "tolerance": 1e-5, "pass": bool(max(errs) <= 1e-5)}
    return res


def c5_oracle_check(samples, params, eta=0.02):
    """Part of the CPU leg: the first and last frame of every size of the mixed-size step against the FP64
    oracle with the same network (its BF16 evaluation emulated), relative L2 per frame (tolerance 1e-4, the
    learned filter's inference precision)."""
    import numpy as np
    from oracle import safr as O
    out = {}
    for name, (g, wf, got) in samples.items():
        ref = O.precompute_geometry(g, mlp_params=np.asarray(params, np.float64), eta=np.float32(eta), mlp_bf16=True)
        errs = [float(np.linalg.norm(got[k].astype(np.float64) - want) / np.linalg.norm(want))
                for k in range(len(wf)) for want in [O.reconstruct(ref, wf[k].astype(np.float64))]]
        out[name] = float(f"{max(errs):.3e}")
    return {"frames_per_size": 2, "max_rel_l2": out, "tolerance": 1e-4,
            "pass": bool(max(out.values()) <= 1e-4) if out else None}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--frames", type=int, default=64, help="independent frames per step (one batched call)")
    ap.add_argument("--batches", type=int, default=8,
                    help="distinct input batches cycled through (each is re-read only every this many steps)")
    ap.add_argument("--single-calls", type=int, default=2000, help="one-frame calls timed for the latency figure")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="re-tune the launch shapes instead of the stored ones")
    ap.add_argument("--only-batched", action="store_true",
                    help="time the batched step only (no single-frame, extra or CPU legs): for counter runs")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="after timing, copy 256 MiB device to device three times (counter calibration)")
    ap.add_argument("--no-extras", action="store_true", help="skip the 1024-frame, learned-filter and mixed-size runs")
    ap.add_argument("--col-mfma", action="store_true",
                    help="the column pass's per-frequency products on the matrix cores (SAFR_OPT_COL_MFMA) in the "
                         "timed batched step: for counter runs of that variant")
    ap.add_argument("--c4-frames", type=int, default=20000, help="training frames of the learned filter")
    ap.add_argument("--only-c3", action="store_true",
                    help="only the 1024-frame FP32 and BF16x3 (matrix-core) runs, printed as one JSON line")
    ap.add_argument("--only-c4", action="store_true",
                    help="only the learned-filter run and the classical filter sweeps, printed as one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the benchmark measures one GPU (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2510_19542_amd import safr as S

    if args.only_c3:
        print(json.dumps({"c3_batched_1024": run_c3(S, torch, torch.cuda.Stream())}), flush=True)
        return
    if args.only_c4:
        print(json.dumps({"c4_learned_filter": run_c4(S, torch, torch.cuda.current_stream(), args.c4_frames)[0]}),
              flush=True)
        return

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
    if args.autotune:
        tuned = S.safr_autotune(plan, F, pool[:F], out, S.SAFR_FP32, 5, stream)
        tuned1 = S.safr_autotune(plan1, 1, pool[0], out[0], S.SAFR_FP32, 20, stream)
        print(f"bench: autotuned batched {tuned}, single {tuned1}", file=sys.stderr, flush=True)
    else:
        tuned, tuned1 = TUNED_BATCHED, TUNED_SINGLE
        apply_shape(S, plan, tuned)
        apply_shape(S, plan1, tuned1)
    if args.col_mfma:
        S.safr_set_option(plan, S.SAFR_OPT_COL_MFMA, 1)
    # distinct input buffers (the two synthetic batches, then sign-flipped copies in their own memory), so
    # that a step's inputs were last read several steps earlier
    batches = [pool[:F], pool[F:]]
    while len(batches) < args.batches:
        batches.append(-batches[len(batches) % 2])
    # the timed launch on its first input batch, kept for the oracle check of the CPU-baseline leg
    S.safr_reconstruct_batched(plan, F, batches[0], out, S.SAFR_FP32, stream)
    torch.cuda.synchronize()
    ref_out = out.cpu().numpy()

    result = {}
    c5_samples, params = None, None
    # Order of the legs: the one-frame latency, the closed loop, the refreshes and the other workloads
    # run first and the headline batched step right after the GPU-heavy batched workloads (1024-frame
    # batches, mixed sizes), with no host-side pause in between; the CPU-only oracle leg comes last.
    # After any idle gap (0.1 s is enough) the batched step starts about 10% slow and needs some 25 ms of
    # continuous load to settle, so a 20-step window right after the precomputation or after a
    # host-bound leg measures the settling, not the kernels.
    if not args.only_batched:
        for i in range(200):
            S.safr_reconstruct(plan1, pool[i % len(pool)], out[0], stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(args.single_calls):
            S.safr_reconstruct(plan1, pool[i % len(pool)], out[0], stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us_single = e0.elapsed_time(e1) * 1000.0 / args.single_calls
        stage1_ms = S.safr_time_stages(plan1, 1, pool[0], out[0], S.SAFR_FP32, 50, stream)
        result["single_frame"] = {"us_per_frame": round(us_single, 3), "frames_per_s": round(1e6 / us_single, 1),
                                  "stage_ms": {k: round(v, 6) for k, v in zip(("rows", "cols", "out"), stage1_ms)}}
        print("bench: closed-loop step (Alg. 3)", file=sys.stderr, flush=True)
        result["closed_loop"] = run_loop(S, torch, plan1, geo, pool, args.single_calls)
        print("bench: precompute refresh", file=sys.stderr, flush=True)
        result["recompute"] = run_recompute(S, torch)
        if not args.no_extras:
            gstream = torch.cuda.Stream()
            print("bench: closed loop on a frozen-flow atmosphere (Strehl)", file=sys.stderr, flush=True)
            result["closed_loop_strehl"] = run_loop_strehl(S, torch, plan1, geo)
            print("bench: learned filter (train 20k frames, held-out evaluation)", file=sys.stderr, flush=True)
            result["c4_learned_filter"], params = run_c4(S, torch, stream, args.c4_frames)
            print("bench: 1024-frame batches (C1 geometry)", file=sys.stderr, flush=True)
            result["c3_batched_1024"] = run_c3(S, torch, gstream)
            print("bench: mixed-size bundle", file=sys.stderr, flush=True)
            result["c5_mixed_sizes"], c5_samples = run_c5(S, torch, gstream, params)
        if not args.col_mfma:
            print("bench: column apply on the matrix cores", file=sys.stderr, flush=True)
            result["column_apply_on_matrix_cores"] = run_col_mfma(S, torch, geo, batches, out, stream, args.steps)

    # headline: each step reconstructs F frames in one batched call
    print(f"bench: batched step, {F} frames per call, {args.warmup} warm-up + {args.steps} timed steps",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        S.safr_reconstruct_batched(plan, F, batches[i % len(batches)], out, S.SAFR_FP32, stream)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for i in range(args.steps):
        S.safr_reconstruct_batched(plan, F, batches[i % len(batches)], out, S.SAFR_FP32, stream)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    fps = F * 1000.0 / ms_step
    # five more timed runs of the same length, for the spread (not part of the reported value)
    reruns = []
    if not args.only_batched:
        for _ in range(5):
            torch.cuda.synchronize()
            t0.record(stream)
            for i in range(args.steps):
                S.safr_reconstruct_batched(plan, F, batches[i % len(batches)], out, S.SAFR_FP32, stream)
            t1.record(stream)
            torch.cuda.synchronize()
            reruns.append(round(F * 1000.0 / (t0.elapsed_time(t1) / args.steps), 1))
    # per-kernel durations of the batched call (HIP events on the launch stream, inside the library, around 20
    # back-to-back launches of each stage's kernel)
    stage_ms = S.safr_time_stages(plan, F, batches[0], out, S.SAFR_FP32, 20, stream)
    # the launch is deterministic: the first batch again gives the layers the oracle leg checks
    S.safr_reconstruct_batched(plan, F, batches[0], out, S.SAFR_FP32, stream)
    torch.cuda.synchronize()
    same = bool(np.array_equal(out.cpu().numpy(), ref_out))
    names = ["rows", "cols", "out"]
    if args.calibration_copy:
        a = torch.empty(64 * 1024 * 1024, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ab = algorithmic_bytes(desc, geo.n, F)
    af = algorithmic_flops(desc, geo.n, F)
    step_kernel_ms = float(sum(stage_ms))
    t_hbm = ab["step"] / (HBM_PEAK_GBS * 1e9)
    t_alu = af["step"] / (FP32_PEAK_TFLOPS * 1e12)
    gbs = ab["step"] / (step_kernel_ms * 1e-3) / 1e9
    tfl = af["step"] / (step_kernel_ms * 1e-3) / 1e12
    traffic = measured_traffic(F)
    # whole step (rows, cols, out): the larger of its algorithmic HBM and ALU times
    if t_alu >= t_hbm:
        step_roof = {"bound": "alu", "achieved": round(tfl, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tfl / FP32_PEAK_TFLOPS, 4), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        step_roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "alu_frac": round(tfl / FP32_PEAK_TFLOPS, 4)}
    step_roof.update({"kernel_ms": round(step_kernel_ms, 6), "alg_bytes": ab["step"], "alg_flops": af["step"],
                      "method_alg_bytes": ab["method_step"], "method_alg_flops": af["method_step"],
                      "traffic": traffic})
    # the dominant (longest) kernel against its own binding resource: algorithmic bytes or flops of one
    # launch over its duration (HIP events on the launch stream)
    dom = int(np.argmax(stage_ms))
    dk = names[dom]
    dsec = stage_ms[dom] * 1e-3
    dom_tfl = af["per_kernel"][dk] / dsec / 1e12
    dom_gbs = ab["per_kernel"][dk] / dsec / 1e9
    dom_hbm_bound = ab["per_kernel"][dk] / (HBM_PEAK_GBS * 1e9) >= af["per_kernel"][dk] / (FP32_PEAK_TFLOPS * 1e12)
    if dom_hbm_bound:
        roof = {"bound": "hbm", "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom_gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(dom_tfl, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(dom_tfl / FP32_PEAK_TFLOPS, 4)}
    roof.update({"traffic": measured_traffic(F, dk), "kernel": KERNEL_NAMES[dk], "kernel_ms": round(stage_ms[dom], 6),
                 "duration_source": "HIP events on the launch stream around 20 back-to-back launches of the "
                                    "stage's kernel (after one full call), mean per launch",
                 "alg_bytes_per_launch": ab["per_kernel"][dk], "alg_flops_per_launch": af["per_kernel"][dk],
                 "hbm_frac": round(dom_gbs / HBM_PEAK_GBS, 4), "alu_frac": round(dom_tfl / FP32_PEAK_TFLOPS, 4),
                 "GBs_with_intermediates": round(ab["with_intermediates"][dk] / dsec / 1e9, 1),
                 "step": step_roof,
                 "per_kernel_alg_flops": af["per_kernel"], "per_kernel_alg_bytes": ab["per_kernel"],
                 "per_kernel_GBs_with_intermediates": {
                     k: round(ab["with_intermediates"][k] / (v * 1e-3) / 1e9, 1) for k, v in zip(names, stage_ms)}})
    head = {
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
                   "frames_per_step": F, "input_batches_cycled": len(batches), "J": geo.J, "L": geo.L, "M": geo.M,
                   "n": geo.n,
                   "launch_shapes": {"batched": list(tuned), "single": list(tuned1), "autotuned_now": args.autotune},
                   "leg_order": "single-frame, closed loop, refresh, Strehl loop, C4, C3, C5, matrix-core apply, "
                                "then the headline (warm-up, timed steps, reruns, stage timing, determinism "
                                "check), then the CPU oracle"},
        "roofline": roof,
        "stage_ms": {k: round(v, 6) for k, v in zip(names, stage_ms)},
        "reruns_frames_per_s": {"runs": reruns, "median": float(np.median(reruns)) if reruns else None},
        "timed_launch_deterministic": same,
        "frame_alg_bytes": algorithmic_bytes(desc, geo.n, 1)["step"],
        "frame_alg_flops": algorithmic_flops(desc, geo.n, 1)["step"],
        "frame_method_flops": algorithmic_flops(desc, geo.n, 1)["method_step"],
    }
    head.update(result)
    result = head
    if not args.only_batched and not args.no_cpu_baseline:
        print("bench: CPU baseline (FP64 oracle) on the timed launch's first batch", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(geo, args.cpu_budget, batches[0].cpu().numpy(), ref_out)
        if c5_samples:
            result["c5_mixed_sizes"]["oracle_check"] = c5_oracle_check(c5_samples, params)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
