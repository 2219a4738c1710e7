"""Parity of the benchmark's own launch with the FP64 oracle.

The throughput benchmark reconstructs 64 MORFEO-like frames per call with the stored
launch shapes (12 row teams, 8 output rows, 16 column frames per block, 8 output frames
per block, 4 frames transformed together in the column pass), i.e. the column kernel
that applies B to four frames at once and walks four runs of 16 frames per column.
These tests run exactly that launch and hold its output to the FP32 tolerance of the
reconstruction (relative L2 <= 1e-5 against the oracle, per frame), on frames that land
in every slot of the four-frame groups (f mod 4) and in every frame run (f // 16), the
first and last frame included.  Alg. 1 and Sec. 3.3 define what is computed.
"""
import numpy as np
import pytest

import bench
import synth
from oracle import safr as O

pytestmark = pytest.mark.gpu

# f % 4 covers 0..3 and f // 16 covers 0..3; frames 0 and 63 included
BENCH_FRAMES = [0, 5, 10, 15, 17, 22, 27, 35, 40, 45, 50, 63]


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _lib():
    from paper_2510_19542_amd import safr as S
    S.lib()
    return S


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


_CACHE = {}


def _oracle_plan(geo):
    if geo.name not in _CACHE:
        _CACHE[geo.name] = O.precompute_geometry(geo)
    return _CACHE[geo.name]


def _batched(S, torch, plan, x, stream):
    F = int(x.shape[0])
    geo_L, M = plan.desc.L, plan.desc.M
    need = S.safr_workspace_size(plan, F)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    out = torch.full((F, geo_L, M, M), float("nan"), dtype=torch.float32, device="cuda")
    S.safr_reconstruct_batched(plan, F, x, out, S.SAFR_FP32, stream)
    stream.synchronize()
    res = out.cpu().numpy()
    S.safr_set_workspace(plan, 0, 0)
    return res


@pytest.fixture(scope="module")
def c2_bench_run():
    """The timed launch: C2, 64 frozen-flow frames (the benchmark's first input batch), stored shapes."""
    torch = _torch()
    S = _lib()
    geo = synth.preset("C2")
    F = 64
    wf = synth.frames(geo, F)
    x = torch.from_numpy(wf).cuda()
    plan = S.precompute_geometry(geo)
    bench.apply_shape(S, plan, bench.TUNED_BATCHED)
    stream = torch.cuda.Stream()
    got = _batched(S, torch, plan, x, stream)
    return geo, wf, plan, x, got


def test_bench_shapes_select_the_four_frame_column_kernel():
    # the stored shape asks for 4 frames transformed together and 16 frames per column block
    assert bench.TUNED_BATCHED[4] == 4 and bench.TUNED_BATCHED[2] == 16
    assert 64 % bench.TUNED_BATCHED[2] == 0 and bench.TUNED_BATCHED[2] % bench.TUNED_BATCHED[4] == 0


@pytest.mark.parametrize("f", BENCH_FRAMES)
def test_bench_launch_matches_oracle(c2_bench_run, f):
    geo, wf, _, _, got = c2_bench_run
    assert np.isfinite(got[f]).all(), f
    want = O.reconstruct(_oracle_plan(geo), wf[f].astype(np.float64))
    err = rel_l2(got[f], want)
    print(f"C2 bench launch, frame {f} (slot {f % 4}, run {f // 16}): rel-L2 {err:.3e}")
    assert err <= 1e-5, (f, err)


def test_bench_launch_four_frames_together_equals_one(c2_bench_run):
    """The four-frame column kernel and the one-frame kernel compute every frame alike (<= 1e-6)."""
    torch = _torch()
    S = _lib()
    geo, _, plan, x, got = c2_bench_run
    S.safr_set_option(plan, S.SAFR_OPT_COL_TOGETHER, 1)
    try:
        one = _batched(S, torch, plan, x, torch.cuda.Stream())
    finally:
        S.safr_set_option(plan, S.SAFR_OPT_COL_TOGETHER, bench.TUNED_BATCHED[4])
    worst = max(rel_l2(got[f], one[f].astype(np.float64)) for f in range(len(got)))
    print(f"C2, 64 frames: four frames together vs one at a time, worst rel-L2 {worst:.3e}")
    assert worst <= 1e-6


def test_bench_launch_replayed_from_a_graph(c2_bench_run):
    """The same launch captured in a HIP graph on a non-default stream and replayed three times, the
    program's own work and synchronisations in between, equals the eager launch bit for bit."""
    torch = _torch()
    S = _lib()
    geo, _, plan, x, got = c2_bench_run
    F = int(x.shape[0])
    need = S.safr_workspace_size(plan, F)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    out = torch.empty((F, geo.L, geo.M, geo.M), dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 1)
    try:
        for rep in range(3):
            out.fill_(float(rep + 1))
            torch.cuda.synchronize()
            S.safr_reconstruct_batched(plan, F, x, out, S.SAFR_FP32, stream)
            stream.synchronize()
            assert np.array_equal(out.cpu().numpy(), got), rep
    finally:
        S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 0)
        S.safr_set_workspace(plan, 0, 0)


def test_c5_big_tikhonov_32_frames_matches_oracle():
    """The MORFEO-scale entry of the mixed-size workload with the Tikhonov filter, 32 frames in one call
    (default launch shapes: the four-frame column kernel), sampled frames against the oracle."""
    torch = _torch()
    S = _lib()
    geo = synth.preset("C5-Big")
    F = 32
    wf = synth.frames(geo, F)
    plan = S.precompute_geometry(geo)
    got = _batched(S, torch, plan, torch.from_numpy(wf).cuda(), torch.cuda.Stream())
    ref = _oracle_plan(geo)
    for f in (0, 9, 18, 31):
        err = rel_l2(got[f], O.reconstruct(ref, wf[f].astype(np.float64)))
        print(f"C5-Big Tikhonov, 32 frames, frame {f}: rel-L2 {err:.3e}")
        assert err <= 1e-5, (f, err)


def test_stage_timing_leaves_the_batched_result(c2_bench_run):
    """safr_time_stages runs one batched call and then each stage's kernels back to back on the inputs that
    call left in the workspace: every stage time is positive and the layers are the batched call's, bit
    for bit."""
    torch = _torch()
    S = _lib()
    geo, _, plan, x, got = c2_bench_run
    F = int(x.shape[0])
    need = S.safr_workspace_size(plan, F)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    out = torch.full((F, geo.L, geo.M, geo.M), float("nan"), dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    try:
        ms = S.safr_time_stages(plan, F, x, out, S.SAFR_FP32, 5, stream)
        stream.synchronize()
        print("stage ms:", ms)
        assert len(ms) == 3 and all(0.0 < t < 10.0 for t in ms)
        assert np.array_equal(out.cpu().numpy(), got)
    finally:
        S.safr_set_workspace(plan, 0, 0)


def test_odd_frame_count_matches_oracle():
    """65 frames with the stored shapes (a partial last group of the four-frame column kernel and of the
    output pass's frame runs; Alg. 1 per frame): frames at both ends against the oracle."""
    torch = _torch()
    S = _lib()
    geo = synth.preset("C2")
    F = 65
    wf = synth.random_wavefronts(geo, F, seed=17)
    plan = S.precompute_geometry(geo)
    bench.apply_shape(S, plan, bench.TUNED_BATCHED)
    got = _batched(S, torch, plan, torch.from_numpy(wf).cuda(), torch.cuda.Stream())
    ref = _oracle_plan(geo)
    for f in (0, 1, 33, 63, 64):
        err = rel_l2(got[f], O.reconstruct(ref, wf[f].astype(np.float64)))
        print(f"C2, 65 frames, frame {f}: rel-L2 {err:.3e}")
        assert err <= 1e-5, (f, err)
