"""BF16 matrix-core apply with the split correction (batched path) against the FP64 oracle.

Bound: relative L2 <= 1e-4 per frame (the BF16 tolerance of the batched path).  The
split hi/lo products leave ~2^-16 relative error per product; the FP32 path on
the same frames is also checked, and the two GPU paths must differ by no more
than the BF16 bound.
"""
import numpy as np
import pytest

import synth
from oracle import safr as O

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    from paper_2510_19542_amd import safr as S
    assert torch.cuda.is_available()
    S.lib()
    return torch, S


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _small_mixed():
    rng = np.random.default_rng(5)
    h = np.array([0.0, 3000.0, 8000.0])
    stars = [(float(x), float(y), k) for (x, y), k in zip(rng.uniform(-1.5e-4, 1.5e-4, (5, 2)), [1, 1, 1, 0, 0])]
    return synth.Geometry(name="mixed32", n=19, M=32, pitch=0.5, diameter=9.0, obstruction=0.1, stars=stars,
                          h_lgs=90e3, heights=h, weights=np.array([0.5, 0.3, 0.2]), alpha=5e-3, alpha_tt=1e-3,
                          beta=1.5, truth_heights=h, truth_fracs=np.ones(3) / 3, r0=0.15, L0=25.0, eta=0.01,
                          config_id=77)


@pytest.mark.parametrize("name,frames", [("C1", 40), ("C1", 1), ("C5-S", 20), ("C5-Mid", 9), ("mixed32", 17)])
def test_bf16x3_matches_oracle(name, frames):
    torch, S = _setup()
    geo = _small_mixed() if name == "mixed32" else synth.preset(name)
    plan = S.precompute_geometry(geo)
    wf = synth.frames(geo, frames)
    x = torch.from_numpy(wf).cuda()
    got = S.reconstruct(plan, x, precision=S.SAFR_BF16X3).cpu().numpy()
    fp32 = S.reconstruct(plan, x, precision=S.SAFR_FP32).cpu().numpy()
    ref = O.precompute_geometry(geo)
    worst = 0.0
    for f in range(frames):
        want = O.reconstruct(ref, wf[f].astype(np.float64))
        e = _rel(got[f], want)
        worst = max(worst, e)
        assert e <= 1e-4, (name, f, e)
        assert _rel(fp32[f], want) <= 1e-5
    print(f"{name}: worst BF16x3 rel-L2 {worst:.2e} over {frames} frames")


def test_bf16x3_unsupported_for_large_grids():
    torch, S = _setup()
    geo = synth.preset("C2")
    plan = S.precompute_geometry(geo)
    x = torch.zeros((2, geo.J, geo.n, geo.n), device="cuda")
    with pytest.raises(S.SafrError) as e:
        S.reconstruct(plan, x, precision=S.SAFR_BF16X3)
    assert e.value.status == S.SAFR_ERR_UNSUPPORTED


@pytest.mark.parametrize("nf", [4, 8, 16])
def test_bf16x3_frames_per_block_options_agree(nf):
    torch, S = _setup()
    geo = synth.preset("C1")
    plan = S.precompute_geometry(geo)
    x = torch.from_numpy(synth.random_wavefronts(geo, 23)).cuda()
    S.safr_set_option(plan, S.SAFR_OPT_MFMA_FRAMES, 16)
    ref = S.reconstruct(plan, x, precision=S.SAFR_BF16X3)
    S.safr_set_option(plan, S.SAFR_OPT_MFMA_FRAMES, nf)
    got = S.reconstruct(plan, x, precision=S.SAFR_BF16X3)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)          # frames are independent columns of the matrix product


def test_batched_1024_frozen_flow_frames():
    """1024 consecutive frozen-flow frames of the 8 m geometry in one batched call, both precisions,
    every frame against the oracle (BF16x3 <= 1e-4, FP32 <= 1e-5)."""
    torch, S = _setup()
    geo = synth.preset("C3")
    wf = synth.frames(geo, 1024)
    plan = S.precompute_geometry(geo)
    x = torch.from_numpy(wf).cuda()
    got = S.reconstruct(plan, x, precision=S.SAFR_BF16X3).cpu().numpy()
    fp32 = S.reconstruct(plan, x, precision=S.SAFR_FP32).cpu().numpy()
    ref = O.precompute_geometry(geo)
    eb, ef = [], []
    for f in range(1024):
        want = O.reconstruct(ref, wf[f].astype(np.float64))
        eb.append(_rel(got[f], want))
        ef.append(_rel(fp32[f], want))
    print(f"1024 frames: BF16x3 worst {max(eb):.2e} mean {np.mean(eb):.2e}; FP32 worst {max(ef):.2e}")
    assert max(eb) <= 1e-4
    assert max(ef) <= 1e-5
