"""Seeded synthetic data: von Karman phase screens, simulated wavefronts, noise.

This is the data *simulator*, not the reconstruction: truth screens are drawn
by FFT filtering of seeded Gaussian noise (the standard method of Johansson &
Gavel, 1994, with the von Karman phase spectrum 0.023 r0^(-5/3) (f^2 +
L0^(-2))^(-11/6)), and each guide-star wavefront is the sum over truth layers of
the screen sampled, by bilinear interpolation, at the point where the line of
sight crosses the layer (the layered model of the paper's Sec. 2, with the cone
effect for laser guide stars).  Noise is white Gaussian with a standard
deviation of eta times the RMS of the clean wavefront over the pupil pixels.

Random streams use ``numpy.random.default_rng([19542, config_id, frame_id,
stream_id])`` with stream 0 = screens, 1 = noise, 2 = instance draws.
"""
from __future__ import annotations

import numpy as np

from .configs import Geometry, LGS

STREAM_SCREENS, STREAM_NOISE, STREAM_DRAWS = 0, 1, 2


def rng_for(config_id: int, frame_id: int, stream_id: int) -> np.random.Generator:
    return np.random.default_rng([19542, int(config_id), int(frame_id), int(stream_id)])


def truth_grid_size(M: int) -> int:
    return 4 * M if M <= 128 else 2 * M


def vk_screen(N: int, dx: float, r0: float, L0: float, rng: np.random.Generator) -> np.ndarray:
    """One periodic N x N von Karman phase screen [rad at 500 nm], spacing dx, zero mean."""
    f = np.fft.fftfreq(N, d=dx)
    f2 = f[:, None] ** 2 + f[None, :] ** 2
    psd = 0.023 * r0 ** (-5.0 / 3.0) * (f2 + 1.0 / L0 ** 2) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    df = 1.0 / (N * dx)
    c = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    return (np.fft.ifft2(c * np.sqrt(psd) * df) * (N * N)).real


def truth_screens(geo: Geometry, frame_id: int = 0) -> np.ndarray:
    """Truth screens, one per truth layer, on a periodic grid of spacing ``pitch``."""
    rng = rng_for(geo.config_id, frame_id, STREAM_SCREENS)
    N = truth_grid_size(geo.M)
    fr = np.asarray(geo.truth_fracs, dtype=np.float64)
    fr = fr / fr.sum()
    out = np.empty((len(fr), N, N))
    for i, w in enumerate(fr):
        r0_i = geo.r0 * w ** (-3.0 / 5.0)
        out[i] = vk_screen(N, geo.pitch, r0_i, geo.L0, rng)
    return out


def _sample_periodic(screen: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Bilinear sample of a periodic screen at fractional indices (u, v)."""
    N0, N1 = screen.shape
    i0 = np.floor(u).astype(np.int64)
    j0 = np.floor(v).astype(np.int64)
    fu = u - i0
    fv = v - j0
    i0 %= N0
    j0 %= N1
    i1 = (i0 + 1) % N0
    j1 = (j0 + 1) % N1
    return ((1 - fu) * (1 - fv) * screen[i0, j0] + fu * (1 - fv) * screen[i1, j0]
            + (1 - fu) * fv * screen[i0, j1] + fu * fv * screen[i1, j1])


def cone(kind: int, h: float, h_lgs: float) -> float:
    return 1.0 - h / h_lgs if kind == LGS else 1.0


def wind_offset(layer: int, frame_id: int, speed: float = 10.0, dt: float = 1e-3) -> np.ndarray:
    """Frozen-flow displacement [m] of truth layer ``layer`` after ``frame_id`` steps."""
    ang = layer * np.pi / 2.0
    d = speed * dt * frame_id
    return np.array([d * np.cos(ang), d * np.sin(ang)])


def simulate_wavefronts(geo: Geometry, screens: np.ndarray, frame_id: int = 0,
                        eta: float | None = None, frozen_flow: bool = False,
                        noise: bool = True) -> np.ndarray:
    """Noisy pupil wavefronts (J, n, n) float64: bilinear line-of-sight sums + white noise."""
    n, p = geo.n, geo.pitch
    N = screens.shape[-1]
    x = (np.arange(n) - (n - 1) / 2.0) * p
    X, Y = np.meshgrid(x, x, indexing="ij")
    mask = geo.pupil().astype(bool)
    out = np.zeros((geo.J, n, n))
    for g, (ax, ay, kind) in enumerate(geo.stars):
        acc = np.zeros((n, n))
        for i, h in enumerate(geo.truth_heights):
            c = cone(int(kind), float(h), geo.h_lgs)
            off = wind_offset(i, frame_id) if frozen_flow else np.zeros(2)
            u = (c * X + ax * h - off[0]) / p + N / 2.0
            v = (c * Y + ay * h - off[1]) / p + N / 2.0
            acc += _sample_periodic(screens[i], u, v)
        out[g] = np.where(mask, acc, 0.0)
    if noise:
        e = geo.eta if eta is None else eta
        rng = rng_for(geo.config_id, frame_id, STREAM_NOISE)
        for g in range(geo.J):
            rms = np.sqrt(np.mean(out[g][mask] ** 2))
            out[g][mask] += e * rms * rng.standard_normal(int(mask.sum()))
    return out


def truth_layers(geo: Geometry, screens: np.ndarray, frame_id: int = 0,
                 frozen_flow: bool = False) -> np.ndarray:
    """Truth binned to the reconstruction heights, sampled on each output layer's own grid.

    Output layer l has spacing c_l * pitch (c_l of the laser-star group when the
    asterism has laser stars, else 1), centred on x = 0 at index M / 2.
    """
    M, p = geo.M, geo.pitch
    N = screens.shape[-1]
    has_lgs = any(int(s[2]) == LGS for s in geo.stars)
    rec_h = np.asarray(geo.heights)
    out = np.zeros((len(rec_h), M, M))
    idx = (np.arange(M) - M / 2.0)
    for i, h in enumerate(geo.truth_heights):
        l = int(np.argmin(np.abs(rec_h - h)))
        c_l = (1.0 - rec_h[l] / geo.h_lgs) if has_lgs else 1.0
        off = wind_offset(i, frame_id) if frozen_flow else np.zeros(2)
        X, Y = np.meshgrid(c_l * idx * p, c_l * idx * p, indexing="ij")
        u = (X - off[0]) / p + N / 2.0
        v = (Y - off[1]) / p + N / 2.0
        out[l] += _sample_periodic(screens[i], u, v)
    return out


def frame(geo: Geometry, frame_id: int = 0, eta: float | None = None,
          frozen_flow: bool = False, screens: np.ndarray | None = None):
    """(wavefronts float32 (J,n,n), truth layers float64 (L,M,M)) for one frame."""
    if screens is None:
        screens = truth_screens(geo, 0 if frozen_flow else frame_id)
    wf = simulate_wavefronts(geo, screens, frame_id, eta=eta, frozen_flow=frozen_flow)
    tl = truth_layers(geo, screens, frame_id, frozen_flow=frozen_flow)
    return wf.astype(np.float32), tl


def frames(geo: Geometry, count: int, first: int = 0, eta: float | None = None,
           frozen_flow: bool = True) -> np.ndarray:
    """(count, J, n, n) float32 wavefronts of consecutive frames (frozen flow by default)."""
    screens = truth_screens(geo, 0)
    out = np.empty((count, geo.J, geo.n, geo.n), dtype=np.float32)
    for f in range(count):
        out[f] = simulate_wavefronts(geo, screens, first + f, eta=eta,
                                     frozen_flow=frozen_flow).astype(np.float32)
    return out


def random_wavefronts(geo: Geometry, count: int, seed: int = 0) -> np.ndarray:
    """(count, J, n, n) float32 white-noise wavefronts on the pupil (cheap bench inputs)."""
    rng = rng_for(geo.config_id, seed, STREAM_DRAWS)
    mask = geo.pupil().astype(np.float32)
    w = rng.standard_normal((count, geo.J, geo.n, geo.n)).astype(np.float32)
    return w * mask
