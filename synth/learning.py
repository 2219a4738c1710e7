"""Seeded random draws and the von Karman amplitude model for learned-filter training data.

Periodic-exact mode: a layer's spectrum on its own M x M periodic grid (spacing
c_l * pitch) is F_l(n) = amp_l(n) z(n) with z complex normal (E|z|^2 = 1) and
amp_l(n)^2 = M^4 df^2 PSD_l(|f_n|), df = 1 / (M c_l pitch), the von Karman phase
spectrum PSD(f) = 0.023 r0_l^(-5/3) (f^2 + L0^-2)^(-11/6), r0_l = r0 w_l^(-3/5),
DC removed.  Noise draws are complex normal per star and frequency; the noise
level eta of a frame is drawn uniformly in [eta_min, eta_max].  Nothing here
applies the tomography operator; the draws are inputs to it.
"""
from __future__ import annotations

import numpy as np

from .atmosphere import rng_for
from .configs import Geometry, LGS

STREAM_LEARN = 4


def _cone(geo: Geometry) -> np.ndarray:
    has_lgs = any(int(s[2]) == LGS for s in geo.stars)
    h = np.asarray(geo.heights, dtype=np.float64)
    return 1.0 - h / geo.h_lgs if has_lgs else np.ones_like(h)


def vk_amplitude(geo: Geometry) -> np.ndarray:
    """amp[l][k][j] on the half spectrum (k = 0..M/2, j = 0..M-1) of each reconstruction layer's grid."""
    M = geo.M
    w = np.asarray(geo.weights, dtype=np.float64)
    w = w / w.sum()
    idx = np.arange(M)
    n = np.where(idx <= (M - 1) // 2, idx, idx - M)
    K, J = np.meshgrid(np.arange(M // 2 + 1), np.arange(M), indexing="ij")
    out = np.zeros((len(w), M // 2 + 1, M))
    for l, (wl, cl) in enumerate(zip(w, _cone(geo))):
        d = cl * geo.pitch
        df = 1.0 / (M * d)
        f = np.hypot(n[J], n[K]) * df
        r0 = geo.r0 * wl ** (-3.0 / 5.0)
        psd = 0.023 * r0 ** (-5.0 / 3.0) * (f ** 2 + 1.0 / geo.L0 ** 2) ** (-11.0 / 6.0)
        a = M * M * df * np.sqrt(psd)
        a[0, 0] = 0.0
        out[l] = a
    return out


MLP_SHAPES = [(64, 4), (64,), (64, 64), (64,), (64, 64), (64,), (64,), (1,)]


def mlp_init(seed: int = 0) -> np.ndarray:
    """Seeded initial network parameters (FP32, packed in the order of MLP_SHAPES):
    weight matrices N(0, 1 / fan_in), output weights N(0, 1/64), biases zero."""
    rng = np.random.default_rng([19542, 4, seed, 7])
    parts = []
    for i, shp in enumerate(MLP_SHAPES):
        if len(shp) == 2:
            parts.append(rng.standard_normal(shp) / np.sqrt(shp[1]))
        elif i == 6:
            parts.append(rng.standard_normal(shp) / 8.0)
        else:
            parts.append(np.zeros(shp))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def learn_draws(geo: Geometry, first: int, count: int, eta_range=(0.005, 0.05), config_id: int = 4):
    """Frames first .. first+count-1: zl (F, L, K, J), zn (F, J_stars, K, J) complex128 and eta (F,)."""
    M, K = geo.M, geo.M // 2 + 1
    zl = np.empty((count, geo.L, K, M), dtype=np.complex128)
    zn = np.empty((count, geo.J, K, M), dtype=np.complex128)
    eta = np.empty(count)
    for i in range(count):
        rng = rng_for(config_id, first + i, STREAM_LEARN)
        a = rng.standard_normal((2, geo.L + geo.J, K, M)) / np.sqrt(2.0)
        z = a[0] + 1j * a[1]
        zl[i], zn[i] = z[: geo.L], z[geo.L:]
        eta[i] = rng.uniform(*eta_range)
    return zl, zn, eta


def periodic_layers(geo: Geometry, seed: int, config_id: int = 4) -> np.ndarray:
    """Real periodic von Karman layers (L, M, M) on the layer grids with E|F|^2 = amp^2, DC and Nyquist removed."""
    M = geo.M
    rng = rng_for(config_id, seed, 3)
    amp_h = vk_amplitude(geo)                                   # [l][k][j]
    idx = np.arange(M)
    n = np.where(idx <= (M - 1) // 2, idx, idx - M)
    amp = np.zeros((geo.L, M, M))                               # [l][j][k] full spectrum
    for k in range(M):
        kk = k if k <= M // 2 else M - k
        amp[:, :, k] = amp_h[:, kk, :] if k <= M // 2 else amp_h[:, kk, (-idx) % M]
    z = (rng.standard_normal((geo.L, M, M)) + 1j * rng.standard_normal((geo.L, M, M))) / np.sqrt(2.0)
    Z = amp * z
    neg = (-idx) % M
    F = (Z + np.conj(Z[:, neg][:, :, neg])) / np.sqrt(2.0)
    if M % 2 == 0:
        F[:, M // 2, :] = 0.0
        F[:, :, M // 2] = 0.0
    F[:, 0, 0] = 0.0
    return np.fft.ifft2(F).real


def periodic_wavefronts(geo: Geometry, layers: np.ndarray) -> np.ndarray:
    """Noise-free data of periodic layers (L, M, M) on the full M x M grid (periodic-exact mode).

    Star g sees layer l shifted by alpha_g h_l / (c_l pitch) layer pixels: an exact
    Fourier shift of the layer's trigonometric interpolant (Nyquist dropped for even M).
    Returns (J, M, M).
    """
    M = geo.M
    idx = np.arange(M)
    n = np.where(idx <= (M - 1) // 2, idx, idx - M).astype(np.float64)
    keep = np.ones(M, dtype=bool)
    if M % 2 == 0:
        keep[M // 2] = False
    K = keep[:, None] & keep[None, :]
    Fl = np.fft.fft2(layers) * K
    h = np.asarray(geo.heights, dtype=np.float64)
    out = np.empty((geo.J, M, M))
    for g, (ax, ay, kind) in enumerate(np.asarray(geo.stars, dtype=np.float64).reshape(-1, 3)):
        c = 1.0 - h / geo.h_lgs if int(kind) == LGS else np.ones_like(h)
        sx = ax * h / (c * geo.pitch)
        sy = ay * h / (c * geo.pitch)
        ph = np.exp(2j * np.pi * (n[None, :, None] * sx[:, None, None] + n[None, None, :] * sy[:, None, None]) / M)
        out[g] = np.fft.ifft2(np.sum(ph * Fl, axis=0)).real
    return out


def periodic_frames(geo: Geometry, seeds, etas, config_id: int = 4):
    """Held-out periodic-exact frames: truth (F, L, M, M) from periodic_layers and, for each noise
    level in etas, data (F, J, M, M) float32 with white noise of std eta x the RMS of each star's
    noise-free data (one noise draw per seed, scaled by eta).  Returns (truth, [data per eta])."""
    seeds = list(seeds)
    etas = list(np.atleast_1d(etas))
    truth = np.empty((len(seeds), geo.L, geo.M, geo.M))
    wfs = [np.empty((len(seeds), geo.J, geo.M, geo.M), dtype=np.float32) for _ in etas]
    for i, s in enumerate(seeds):
        truth[i] = periodic_layers(geo, s, config_id)
        d = periodic_wavefronts(geo, truth[i])
        rms = np.sqrt(np.mean(d ** 2, axis=(1, 2)))
        z = rng_for(config_id, s, 9).standard_normal(d.shape)
        for wf, eta in zip(wfs, etas):
            wf[i] = d + eta * rms[:, None, None] * z
    return truth, wfs
