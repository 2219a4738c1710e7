"""The FP32 column pass with its per-frequency products on the matrix cores (SAFR_OPT_COL_MFMA).

When the column pass transforms four frames together, b_l(n) = sum_g B_n[l][g] d_g(n) (Alg. 1, the apply)
for those frames runs as 4 x 4 x 1 FP32 matrix products: the four frames are the rows, four layers the
columns, one star per step, real and imaginary parts as four real products.  The arithmetic type is the
vector path's (FP32 products, FP32 sums); only the summation order differs.  These tests hold it

* to the vector-unit apply of the same launch, frame by frame (relative L2 <= 1e-6), at every shape with a
  compile-time column kernel (M = 64 with L = 2 and 3, M = 128, M = 256 with the split-tomography group),
  with ragged frame counts whose last group of four is partly empty;
* to the FP64 oracle (relative L2 <= 1e-5, the FP32 bound of the reconstruction);
* after B changes: a refreshed regularisation (safr_update_alpha) and an imported B (safr_import_B) both
  reach the matrix-core layout of B.
"""
import numpy as np
import pytest

import synth
from oracle import safr as O

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    from paper_2510_19542_amd import safr as S
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    S.lib()
    return torch, S


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(S, torch, plan, x, mfma):
    F = int(x.shape[0])
    d = plan.desc
    S.safr_set_option(plan, S.SAFR_OPT_COL_MFMA, 1 if mfma else 0)
    need = S.safr_workspace_size(plan, F)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    out = torch.full((F, d.L, d.M, d.M), float("nan"), dtype=torch.float32, device="cuda")
    S.safr_reconstruct_batched(plan, F, x, out, S.SAFR_FP32)
    torch.cuda.synchronize()
    S.safr_set_workspace(plan, 0, 0)
    return out.cpu().numpy()


def _four_frame_plan(S, geo, **kw):
    plan = S.precompute_geometry(geo, **kw)
    S.safr_set_option(plan, S.SAFR_OPT_COL_TOGETHER, 4)
    return plan


@pytest.mark.parametrize("name,F", [("C1", 7), ("C5-S", 5), ("C5-Mid", 13), ("C2", 4), ("C2", 10)])
def test_matrix_core_apply_equals_vector_apply(name, F):
    torch, S = _mods()
    geo = synth.preset(name)
    plan = _four_frame_plan(S, geo)
    x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=11 + F)).cuda()
    mf = _run(S, torch, plan, x, True)
    va = _run(S, torch, plan, x, False)
    assert np.isfinite(mf).all()
    worst = max(rel_l2(mf[f], va[f]) for f in range(F))
    print(f"{name}, {F} frames: matrix-core vs vector apply, worst rel-L2 {worst:.3e}")
    assert worst <= 1e-6, (name, F, worst)


@pytest.mark.parametrize("name", ["C1", "C5-Mid", "C2"])
def test_matrix_core_apply_matches_oracle(name):
    torch, S = _mods()
    geo = synth.preset(name)
    F = 6                                               # groups of 4 and 2 frames
    wf = synth.random_wavefronts(geo, F, seed=5)
    plan = _four_frame_plan(S, geo)
    got = _run(S, torch, plan, torch.from_numpy(wf).cuda(), True)
    ref = O.precompute_geometry(geo)
    for f in (0, 3, 4, 5):
        err = rel_l2(got[f], O.reconstruct(ref, wf[f].astype(np.float64)))
        print(f"{name}, frame {f} of {F}: rel-L2 to the oracle {err:.3e}")
        assert err <= 1e-5, (name, f, err)


def test_matrix_core_layout_follows_refresh_and_import():
    torch, S = _mods()
    geo = synth.preset("C5-Mid")
    F = 8
    x = torch.from_numpy(synth.random_wavefronts(geo, F, seed=21)).cuda()
    plan = _four_frame_plan(S, geo)
    base = _run(S, torch, plan, x, True)
    # a refresh with another alpha: the matrix-core result follows the new B
    S.safr_update_alpha(plan, geo.alpha * 10.0, geo.alpha_tt * 10.0)
    mf = _run(S, torch, plan, x, True)
    va = _run(S, torch, plan, x, False)
    assert rel_l2(mf, base) > 1e-3                      # B did change
    assert max(rel_l2(mf[f], va[f]) for f in range(F)) <= 1e-6
    # an import of the first plan's B: back to the first result
    src = S.precompute_geometry(geo)
    S.safr_import_B(plan, 0, S.safr_export_B(src, 0))
    again = _run(S, torch, plan, x, True)
    assert np.array_equal(again, base)
