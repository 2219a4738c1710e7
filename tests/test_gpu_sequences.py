"""Calls with more frames than one launch sequence takes (SAFR_OPT_SEQ_FRAMES): the library runs the row,
column and output passes for groups of frames one after the other.  Frames are independent, so every
grouping gives the same layers bit for bit; checked against one sequence for the FP32 and BF16x3 paths,
eager and replayed from a graph, for the closed-loop step (integrator read per group), and at MORFEO scale,
where the automatic grouping splits 70 frames in two, against the oracle on the first and last frame of
each group (relative L2 1e-5)."""
import numpy as np
import pytest

import synth
from oracle import safr as O

pytestmark = pytest.mark.gpu

ONE_SEQUENCE = 65535


def _mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2510_19542_amd import safr as S
    S.lib()                      # fails loudly if the library is missing
    return torch, S


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _run(S, torch, plan, x, seq, precision=0, stream=None, graph=False, reps=1):
    F = int(x.shape[0])
    d = plan.desc
    S.safr_set_option(plan, S.SAFR_OPT_SEQ_FRAMES, seq)
    S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 1 if graph else 0)
    need = S.safr_workspace_size(plan, F, precision)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    out = torch.empty((F, d.L, d.M, d.M), dtype=torch.float32, device="cuda")
    res = []
    for _ in range(reps):
        out.fill_(float("nan"))
        S.safr_reconstruct_batched(plan, F, x, out, precision, stream)
        torch.cuda.synchronize()
        res.append(out.cpu().numpy())
    S.safr_set_workspace(plan, 0, 0)
    S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 0)
    return res


@pytest.mark.parametrize("name,F,seq", [("C1", 20, 7), ("C1", 20, 1), ("C5-Mid", 9, 4), ("C2", 5, 2)])
def test_groups_equal_one_sequence(name, F, seq):
    torch, S = _mods()
    geo = synth.preset(name)
    plan = S.precompute_geometry(geo)
    x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=31 + F)).cuda()
    ref = _run(S, torch, plan, x, ONE_SEQUENCE)[0]
    got = _run(S, torch, plan, x, seq)[0]
    assert np.isfinite(got).all()
    assert np.array_equal(got, ref), (name, F, seq)


def test_groups_equal_one_sequence_bf16x3_and_graph():
    torch, S = _mods()
    geo = synth.preset("C1")
    F = 20
    plan = S.precompute_geometry(geo)
    x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=5)).cuda()
    ref = _run(S, torch, plan, x, ONE_SEQUENCE, precision=S.SAFR_BF16X3)[0]
    got = _run(S, torch, plan, x, 6, precision=S.SAFR_BF16X3)[0]
    assert np.array_equal(got, ref)
    # the groups captured in one graph and replayed on a non-default stream, three times
    ref32 = _run(S, torch, plan, x, ONE_SEQUENCE)[0]
    stream = torch.cuda.Stream()
    for rep, res in enumerate(_run(S, torch, plan, x, 6, stream=stream, graph=True, reps=3)):
        assert np.array_equal(res, ref32), rep


def test_loop_step_groups():
    torch, S = _mods()
    geo = synth.preset("C1")
    F = 5
    plan = S.precompute_geometry(geo)
    d = plan.desc
    wf = torch.from_numpy(synth.random_wavefronts(geo, F, seed=8)).cuda()
    a0 = torch.from_numpy(np.random.default_rng(3).standard_normal((F, d.L, d.M, d.M)).astype(np.float32)).cuda()
    outs = []
    for seq in (ONE_SEQUENCE, 2):
        S.safr_set_option(plan, S.SAFR_OPT_SEQ_FRAMES, seq)
        need = S.safr_workspace_size(plan, F)
        ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
        a = a0.clone()
        S.safr_loop_step(plan, F, wf, a, 0.5, a)            # in place: each group reads its own commands
        torch.cuda.synchronize()
        outs.append(a.cpu().numpy())
        S.safr_set_workspace(plan, 0, 0)
    assert np.array_equal(outs[1], outs[0])
    assert not np.array_equal(outs[0], a0.cpu().numpy())


def test_automatic_groups_at_morfeo_scale():
    torch, S = _mods()
    geo = synth.preset("C2")
    F = 70                                   # more than the 69 frames of one automatic group: 35 + 35
    wf = synth.random_wavefronts(geo, F, seed=13)
    plan = S.precompute_geometry(geo)
    x = torch.from_numpy(wf).cuda()
    auto = _run(S, torch, plan, x, 0)[0]
    one = _run(S, torch, plan, x, ONE_SEQUENCE)[0]
    assert np.array_equal(auto, one)
    ref = O.precompute_geometry(geo)
    for f in (0, 34, 35, 69):
        err = rel_l2(auto[f], O.reconstruct(ref, wf[f].astype(np.float64)))
        print(f"C2, {F} frames in two groups, frame {f}: rel-L2 to the oracle {err:.3e}")
        assert err <= 1e-5, (f, err)


def test_sequence_option_rejects_bad_values():
    torch, S = _mods()
    plan = S.precompute_geometry(synth.preset("C1"))
    for bad in (-1, 65536):
        with pytest.raises(S.SafrError):
            S.safr_set_option(plan, S.SAFR_OPT_SEQ_FRAMES, bad)


def test_workspace_holds_one_sequence():
    """The workspace holds the spectra of one launch sequence (each sequence reuses it) plus the closed-loop
    wavefronts of every frame: it grows with the frame count only by the latter beyond one sequence."""
    torch, S = _mods()
    geo = synth.preset("C2")
    plan = S.precompute_geometry(geo)
    J, n = len(geo.stars), geo.n
    one = S.safr_workspace_size(plan, 69)
    big = S.safr_workspace_size(plan, 2000)
    polc = lambda F: F * J * n * n * 4
    assert big - one <= polc(2000) - polc(69) + 256
    assert big - one >= polc(2000) - polc(69) - 256
    # 150 frames (three sequences of 50) in exactly that workspace, against one sequence
    F = 150
    x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=2)).cuda()
    got = _run(S, torch, plan, x, 0)[0]
    ref = _run(S, torch, plan, x, ONE_SEQUENCE)[0]
    assert np.array_equal(got, ref)


def test_stage_timing_and_autotune_over_groups():
    """safr_time_stages and safr_autotune on a call of several launch sequences: the stage timing covers every
    group, the autotuner times the first, and the tuned call still equals one sequence bit for bit."""
    torch, S = _mods()
    geo = synth.preset("C1")
    F = 20
    plan = S.precompute_geometry(geo)
    S.safr_set_option(plan, S.SAFR_OPT_FUSED, 0)     # the three passes (the one-kernel step has one stage)
    d = plan.desc
    x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=17)).cuda()
    out = torch.empty((F, d.L, d.M, d.M), dtype=torch.float32, device="cuda")
    S.safr_set_option(plan, S.SAFR_OPT_SEQ_FRAMES, 7)
    need = S.safr_workspace_size(plan, F)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    stream = torch.cuda.current_stream()
    ms = S.safr_time_stages(plan, F, x, out, S.SAFR_FP32, 5, stream)
    assert all(v > 0.0 for v in ms), ms
    choice = S.safr_autotune(plan, F, x, out, S.SAFR_FP32, 3, stream)
    assert len(choice) == 5 and all(v >= 1 for v in choice), choice
    S.safr_set_workspace(plan, 0, 0)
    got = _run(S, torch, plan, x, 7)[0]
    ref = _run(S, torch, plan, x, ONE_SEQUENCE)[0]
    assert np.array_equal(got, ref)
