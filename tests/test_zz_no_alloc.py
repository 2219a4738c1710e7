"""The allocation-free variant of the batched reconstruction (safr_reconstruct_batched_static): the same
launch sequence with the workspace in the library's static device array.  Checked through the C ABI against
safr_reconstruct_batched with a caller-bound workspace, bit for bit, on two calls in a row, the second with
fewer frames (the array keeps the first call's contents: nothing in the path may depend on it)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    from paper_2510_19542_amd import safr as S
    assert torch.cuda.is_available()
    L = S.lib()                                  # the C ABI: safr_reconstruct_batched_static is called directly
    return torch, S, L


def _reference(S, torch, plan, x, prec):
    F = int(x.shape[0])
    d = plan.desc
    need = S.safr_workspace_size(plan, F, prec)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    out = torch.empty((F, d.L, d.M, d.M), device="cuda")
    S.safr_reconstruct_batched(plan, F, x, out, prec)
    torch.cuda.synchronize()
    S.safr_set_workspace(plan, 0, 0)
    return out


@pytest.mark.parametrize("name,prec,frames", [("C2", 0, (12, 5)), ("C1", 0, (40, 7)), ("C1", 1, (40, 7)),
                                              ("C5-Mid", 0, (16, 3))])
def test_static_workspace_equals_bound_workspace(name, prec, frames):
    torch, S, L = _mods()
    geo = synth.preset(name)
    plan = S.precompute_geometry(geo)
    d = plan.desc
    stream = torch.cuda.current_stream()
    for i, F in enumerate(frames):
        x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=20 + i)).cuda()
        want = _reference(S, torch, plan, x, prec)
        got = torch.full((F, d.L, d.M, d.M), float("nan"), device="cuda")
        st = L.safr_reconstruct_batched_static(plan.handle, F, x.data_ptr(), got.data_ptr(), prec,
                                               stream.cuda_stream)
        assert st == 0, S.safr_last_error()
        torch.cuda.synchronize()
        assert torch.equal(got, want), (name, prec, F)


def test_static_workspace_rejects_frames_beyond_its_size():
    torch, S, L = _mods()
    geo = synth.preset("C2")
    plan = S.precompute_geometry(geo)
    cap = int(L.safr_static_workspace_bytes())
    per = S.safr_workspace_size(plan, 1)
    F = cap // per + 1
    while S.safr_workspace_size(plan, F) <= cap:
        F += 1
    x = torch.zeros((1,), device="cuda")
    st = L.safr_reconstruct_batched_static(plan.handle, F, x.data_ptr(), x.data_ptr(), 0,
                                           torch.cuda.current_stream().cuda_stream)
    assert st == S.SAFR_ERR_ARG and "static workspace" in S.safr_last_error()
