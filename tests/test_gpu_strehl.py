"""Marechal Strehl estimate (safr_strehl) through the C ABI, against the oracle, and a closed loop.

Parity: residual variances within 1e-4 relative of the oracle's (FP32 sample
positions and FP32 accumulation over a few thousand pupil pixels; the residual is
a difference of two fields of similar size), Strehl ratios within 1e-4 (1 + var)
relative.  The closed-loop run is a property check: on a frozen-flow atmosphere
the loop's Strehl in the science directions must rise far above the uncorrected one.
"""
import numpy as np
import pytest

import synth
from oracle import safr as O

pytestmark = pytest.mark.gpu

ARCSEC = np.pi / (180.0 * 3600.0)
K_BAND = 0.5 / 2.2               # phase in rad at 500 nm -> rad at 2.2 um


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _lib():
    from paper_2510_19542_amd import safr as S
    S.lib()
    return S


def _grid(half_arcsec, k=3):
    t = np.linspace(-half_arcsec, half_arcsec, k) * ARCSEC
    return np.array([(x, y) for x in t for y in t])


def _open_loop(geo, dirs, frame):
    """Noise-free open-loop phase along the science directions (synthetic atmosphere of frame)."""
    sci = geo.replace(stars=[(float(x), float(y), synth.NGS) for x, y in dirs])
    screens = synth.truth_screens(geo, frame)
    return synth.simulate_wavefronts(sci, screens, frame, noise=False).astype(np.float32)


CASES = {
    "C1": (lambda: synth.preset("C1"), 20.0),
    "C2": (lambda: synth.preset("C2"), 30.0),
    "C5-Mid": (lambda: synth.preset("C5-Mid"), 30.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_strehl_matches_oracle(case):
    torch = _torch()
    S = _lib()
    mk, half = CASES[case]
    geo = mk()
    plan = S.precompute_geometry(geo)
    ref = O.precompute_geometry(geo)
    dirs = _grid(half)
    F = 2
    ol = np.stack([_open_loop(geo, dirs, f) for f in range(F)])
    layers = np.stack([(0.9 * synth.frame(geo, f)[1]).astype(np.float32) for f in range(F)])
    x = torch.from_numpy(ol).cuda()
    la = torch.from_numpy(layers).cuda()
    sr = torch.full((F, len(dirs)), np.nan, device="cuda")
    var = torch.full((F, len(dirs)), np.nan, device="cuda")
    S.safr_strehl(plan, F, dirs, x, la, K_BAND, sr, var)
    torch.cuda.synchronize()
    sr, var = sr.cpu().numpy(), var.cpu().numpy()
    for f in range(F):
        want_sr, want_var = O.strehl(ref, ol[f], layers[f], dirs, K_BAND)
        assert np.all(np.abs(var[f] - want_var) <= 1e-4 * want_var), (case, f, var[f], want_var)
        assert np.all(np.abs(sr[f] - want_sr) <= 1e-4 * (1 + want_var) * want_sr), (case, f)
    sr2 = torch.empty((F, len(dirs)), device="cuda")                 # without the variance output
    S.safr_strehl(plan, F, dirs, x, la, K_BAND, sr2, None)
    torch.cuda.synchronize()
    assert np.array_equal(sr2.cpu().numpy(), sr)


def test_strehl_errors():
    torch = _torch()
    S = _lib()
    geo = synth.preset("C1")
    plan = S.precompute_geometry(geo)
    x = torch.zeros((1, 33, geo.n, geo.n), device="cuda")
    la = torch.zeros((1, geo.L, geo.M, geo.M), device="cuda")
    sr = torch.zeros((1, 33), device="cuda")
    for dirs, scale in ((np.zeros((33, 2)), 1.0), (np.zeros((0, 2)), 1.0), (np.zeros((1, 2)), float("inf")),
                        (np.array([[np.nan, 0.0]]), 1.0)):
        with pytest.raises(S.SafrError) as e:
            S.safr_strehl(plan, 1, dirs, x, la, scale, sr)
        assert e.value.status == S.SAFR_ERR_ARG


def test_closed_loop_raises_the_strehl():
    # frozen flow, 1 ms steps; the command computed from the measurement of step t (taken with the
    # mirror a_t) is applied at step t + 1.  After 30 steps the K-band Strehl in the science
    # directions is compared with the uncorrected one.
    torch = _torch()
    S = _lib()
    geo = synth.preset("C1")
    plan = S.precompute_geometry(geo)
    dirs = _grid(20.0)
    sci = geo.replace(stars=[(float(x), float(y), synth.NGS) for x, y in dirs])
    screens = synth.truth_screens(geo, 0)
    a = torch.zeros((1, geo.L, geo.M, geo.M), device="cuda")
    zero = torch.zeros_like(a)
    res = torch.empty((1, geo.J, geo.n, geo.n), device="cuda")
    sr = torch.empty((1, len(dirs)), device="cuda")
    sr0 = torch.empty_like(sr)
    late, open_ = [], []
    for t in range(30):
        wf = synth.simulate_wavefronts(geo, screens, t, frozen_flow=True).astype(np.float32)
        ol = synth.simulate_wavefronts(sci, screens, t, frozen_flow=True, noise=False).astype(np.float32)
        xs = torch.from_numpy(ol[None]).cuda()
        S.safr_strehl(plan, 1, dirs, xs, a, K_BAND, sr)              # mirror a_t during step t
        S.safr_strehl(plan, 1, dirs, xs, zero, K_BAND, sr0)
        S.safr_polc(plan, 1, torch.from_numpy(wf[None]).cuda(), a, -1.0, res)   # measured residual
        S.safr_loop_step(plan, 1, res, a, 0.5, a)                    # a_{t+1}
        torch.cuda.synchronize()
        if t >= 20:
            late.append(sr.cpu().numpy()[0])
            open_.append(sr0.cpu().numpy()[0])
    late, open_ = np.mean(late, axis=0), np.mean(open_, axis=0)
    assert np.all(np.isfinite(late))
    assert late.mean() > 0.3 and late.mean() > 10.0 * open_.mean(), (late, open_)
