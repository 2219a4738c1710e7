"""The one-kernel step of the small configured shape (SAFR_OPT_FUSED: M = 64, n = 33, 4 stars of one kind,
L = 2 or 3): every frame's spectra stay in one block's LDS.  It runs the same transform routines, apply and
packing formulas in the same order as the row, column and output passes, so the layers must be the same
bit for bit; and within 1e-5 (relative L2) of the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import safr as O

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2510_19542_amd import safr as S
    S.lib()                      # fails loudly if the library is missing
    return torch, S


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _run(S, torch, plan, x, fused, stream=None, graph=False):
    F = int(x.shape[0])
    d = plan.desc
    S.safr_set_option(plan, S.SAFR_OPT_FUSED, 1 if fused else 0)
    S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 1 if graph else 0)
    need = S.safr_workspace_size(plan, F)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    out = torch.full((F, d.L, d.M, d.M), float("nan"), dtype=torch.float32, device="cuda")
    S.safr_reconstruct_batched(plan, F, x, out, S.SAFR_FP32, stream)
    torch.cuda.synchronize()
    S.safr_set_workspace(plan, 0, 0)
    S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 0)
    return out.cpu().numpy()


@pytest.mark.parametrize("name,F", [("C1", 1), ("C1", 7), ("C3", 1024), ("C5-S", 5)])
def test_one_kernel_step_equals_three_passes(name, F):
    torch, S = _mods()
    geo = synth.preset(name)
    plan = S.precompute_geometry(geo)
    x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=40 + F)).cuda()
    fused = _run(S, torch, plan, x, True)
    three = _run(S, torch, plan, x, False)
    assert np.isfinite(fused).all()
    assert np.array_equal(fused, three), (name, F, float(np.abs(fused - three).max()))


@pytest.mark.parametrize("name", ["C1", "C5-S"])
def test_one_kernel_step_matches_oracle(name):
    torch, S = _mods()
    geo = synth.preset(name)
    F = 3
    wf = synth.random_wavefronts(geo, F, seed=7)
    plan = S.precompute_geometry(geo)
    got = _run(S, torch, plan, torch.from_numpy(wf).cuda(), True)
    ref = O.precompute_geometry(geo)
    for f in range(F):
        err = rel_l2(got[f], O.reconstruct(ref, wf[f].astype(np.float64)))
        print(f"{name}, frame {f}: one-kernel step vs oracle rel-L2 {err:.3e}")
        assert err <= 1e-5, (name, f, err)


def test_one_kernel_step_from_a_graph():
    torch, S = _mods()
    geo = synth.preset("C1")
    F = 64
    plan = S.precompute_geometry(geo)
    x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=3)).cuda()
    eager = _run(S, torch, plan, x, True)
    stream = torch.cuda.Stream()
    for rep in range(3):
        assert np.array_equal(_run(S, torch, plan, x, True, stream=stream, graph=True), eager), rep


def test_one_kernel_step_stage_timing():
    """safr_time_stages reports the one-kernel step as the row stage and (about) nothing for the other two."""
    torch, S = _mods()
    geo = synth.preset("C1")
    F = 256
    plan = S.precompute_geometry(geo)
    d = plan.desc
    x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=1)).cuda()
    out = torch.empty((F, d.L, d.M, d.M), dtype=torch.float32, device="cuda")
    need = S.safr_workspace_size(plan, F)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    ms = S.safr_time_stages(plan, F, x, out, S.SAFR_FP32, 5)
    S.safr_set_workspace(plan, 0, 0)
    assert ms[0] > 0.0 and ms[1] < 0.2 * ms[0] and ms[2] < 0.2 * ms[0], ms


def test_one_kernel_loop_step_equals_three_passes():
    """The closed-loop step (POLC, reconstruction, integrator in place) with the one-kernel step gives the
    commands of the three passes bit for bit, at gain 0.5 and at gain 0 (the commands unchanged)."""
    torch, S = _mods()
    geo = synth.preset("C1")
    F = 6
    plan = S.precompute_geometry(geo)
    d = plan.desc
    wf = torch.from_numpy(synth.random_wavefronts(geo, F, seed=12)).cuda()
    a0 = torch.from_numpy(np.random.default_rng(9).standard_normal((F, d.L, d.M, d.M)).astype(np.float32)).cuda()
    need = S.safr_workspace_size(plan, F)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    for gain in (0.5, 0.0):
        res = []
        for fused in (1, 0):
            S.safr_set_option(plan, S.SAFR_OPT_FUSED, fused)
            a = a0.clone()
            S.safr_loop_step(plan, F, wf, a, gain, a)
            torch.cuda.synchronize()
            res.append(a.cpu().numpy())
        assert np.array_equal(res[0], res[1]), gain
        if gain == 0.0:
            assert np.array_equal(res[0], a0.cpu().numpy())
    S.safr_set_workspace(plan, 0, 0)
