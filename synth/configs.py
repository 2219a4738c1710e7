"""Workload presets: the synthetic stand-ins for the paper's experiments.

Every preset is plain data (sizes, angles, heights, weights, seeds).  Nothing in
this module computes any part of the reconstruction method; it only describes
the problem instances that the oracle, the GPU library, the tests and the
benchmark all consume.

Conventions shared with the rest of the project:

* angles are in radians; 1 arcsec = pi / (180 * 3600) rad;
* ``kind`` 0 is a natural guide star (NGS, no cone effect), 1 a laser guide
  star (LGS, cone effect with the sodium height ``h_lgs``) (paper, Sec. 2);
* the pupil grid is n x n with spacing ``pitch`` [m]; the periodic grid is
  M x M with the same spacing, so T = M * pitch / 2 (paper, Sec. 3.2 grids);
* heights in metres, ascending; weights are relative turbulence strengths
  (normalised to sum 1 by the consumers, paper Sec. 2).

The MORFEO-like values (6 LGS on a 45 arcsec radius, 3 NGS, sodium at 90 km,
0-16 km reconstruction layers, Table 5 regularisation parameters) follow the
paper's Sec. 4.1 setup and Table 5; the ESO 35-layer profile is not available,
so a synthetic 35-layer profile stands in for it (see ``synthetic_35_layers``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

ARCSEC = math.pi / (180.0 * 3600.0)
NGS, LGS = 0, 1


@dataclasses.dataclass
class Geometry:
    """One reconstruction geometry plus the truth atmosphere used to make data."""

    name: str
    n: int                      # pupil grid n x n
    M: int                      # periodic FFT grid M x M
    pitch: float                # grid spacing [m]
    diameter: float             # aperture diameter [m]
    obstruction: float          # central obstruction, fraction of the diameter
    stars: List[Tuple[float, float, int]]   # (alpha_x, alpha_y [rad], kind)
    h_lgs: float                # sodium layer height [m]
    heights: np.ndarray         # reconstruction layer heights [m], ascending
    weights: np.ndarray         # reconstruction layer weights gamma (unnormalised)
    alpha: float                # Tikhonov parameter (LGS group, or the only group)
    alpha_tt: float             # Tikhonov parameter of the NGS group in mixed asterisms
    beta: float                 # Sobolev smoothness
    # truth atmosphere for synthetic data
    truth_heights: np.ndarray
    truth_fracs: np.ndarray
    r0: float                   # Fried parameter at 500 nm [m]
    L0: float                   # outer scale [m]
    eta: float                  # relative measurement noise
    config_id: int

    @property
    def J(self) -> int:
        return len(self.stars)

    @property
    def L(self) -> int:
        return len(self.heights)

    @property
    def T(self) -> float:
        return self.M * self.pitch / 2.0

    def pupil(self) -> np.ndarray:
        return circular_pupil(self.n, self.pitch, self.diameter, self.obstruction)

    def star_array(self) -> np.ndarray:
        return np.array(self.stars, dtype=np.float64).reshape(-1, 3)

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)


def circular_pupil(n: int, pitch: float, diameter: float, obstruction: float = 0.0) -> np.ndarray:
    """Circular aperture of the given diameter inscribed in the n x n grid (uint8 mask)."""
    c = (n - 1) / 2.0
    i = (np.arange(n) - c) * pitch
    r = np.hypot(i[:, None], i[None, :])
    R = diameter / 2.0
    tol = 1e-9 * max(R, 1.0)
    mask = r <= R + tol
    if obstruction > 0.0:
        mask &= r >= obstruction * R - tol
    return mask.astype(np.uint8)


def ring(count: int, radius_arcsec: float, angles_deg, kind: int):
    out = []
    for a in angles_deg[:count]:
        t = math.radians(a)
        out.append((radius_arcsec * ARCSEC * math.cos(t), radius_arcsec * ARCSEC * math.sin(t), kind))
    return out


def synthetic_35_layers() -> Tuple[np.ndarray, np.ndarray]:
    """Stand-in for a measured 35-layer profile: h_i = 0.5 km * i, fractions ~ exp(-h/3 km)."""
    h = 500.0 * np.arange(35, dtype=np.float64)
    f = np.exp(-h / 3000.0)
    return h, f / f.sum()


def bin_weights(truth_h: np.ndarray, truth_f: np.ndarray, rec_h: np.ndarray) -> np.ndarray:
    """Reconstruction weights: truth fractions binned onto the nearest reconstruction height."""
    w = np.zeros(len(rec_h))
    for h, f in zip(truth_h, truth_f):
        w[int(np.argmin(np.abs(rec_h - h)))] += f
    return w / w.sum()


def c1() -> Geometry:
    """8 m aperture, 4 NGS at 30 arcsec on a square, 33^2 pupil grid in 64^2, L = 2."""
    stars = ring(4, 30.0, [45.0, 135.0, 225.0, 315.0], NGS)
    h = np.array([0.0, 6000.0])
    w = np.array([0.7, 0.3])
    return Geometry(name="C1", n=33, M=64, pitch=0.25, diameter=8.0, obstruction=0.0,
                    stars=stars, h_lgs=90e3, heights=h, weights=w, alpha=1e-3, alpha_tt=1e-3,
                    beta=1.5, truth_heights=h.copy(), truth_fracs=w.copy(), r0=0.16, L0=25.0,
                    eta=0.01, config_id=1)


def c2() -> Geometry:
    """MORFEO-like: 39 m, 6 LGS at 45 arcsec + 3 NGS at 80 arcsec, 69^2 in 256^2, L = 9."""
    lgs = ring(6, 45.0, [0.0, 60.0, 120.0, 180.0, 240.0, 300.0], LGS)
    ngs = ring(3, 80.0, [60.0, 180.0, 300.0], NGS)
    th, tf = synthetic_35_layers()
    h = 2000.0 * np.arange(9, dtype=np.float64)
    return Geometry(name="C2", n=69, M=256, pitch=0.574, diameter=39.0, obstruction=0.11,
                    stars=lgs + ngs, h_lgs=90e3, heights=h, weights=bin_weights(th, tf, h),
                    alpha=0.005, alpha_tt=0.001, beta=1.5, truth_heights=th, truth_fracs=tf,
                    r0=0.157, L0=25.0, eta=0.02, config_id=2)


def c5_small() -> Geometry:
    g = c1()
    h = np.array([0.0, 4000.0, 12700.0])
    w = np.array([0.75, 0.15, 0.10])
    return g.replace(name="C5-S", heights=h, weights=w, truth_heights=h.copy(),
                     truth_fracs=w.copy(), eta=0.02, config_id=5)


def c5_mid() -> Geometry:
    """20 m, 6 LGS at 45 arcsec, 41^2 in 128^2 (pitch 0.5 m), L = 5 at 0..16 km."""
    lgs = ring(6, 45.0, [0.0, 60.0, 120.0, 180.0, 240.0, 300.0], LGS)
    th, tf = synthetic_35_layers()
    h = 4000.0 * np.arange(5, dtype=np.float64)
    return Geometry(name="C5-Mid", n=41, M=128, pitch=0.5, diameter=20.0, obstruction=0.0,
                    stars=lgs, h_lgs=90e3, heights=h, weights=bin_weights(th, tf, h),
                    alpha=0.005, alpha_tt=0.001, beta=1.5, truth_heights=th, truth_fracs=tf,
                    r0=0.157, L0=25.0, eta=0.02, config_id=5)


def c5_big() -> Geometry:
    return c2().replace(name="C5-Big", config_id=5)


def c3() -> Geometry:
    """The C1 geometry with its own seeds, for batches of consecutive frozen-flow frames."""
    return c1().replace(name="C3", config_id=3)


PRESETS = {"C1": c1, "C2": c2, "C3": c3, "C5-S": c5_small, "C5-Mid": c5_mid, "C5-Big": c5_big}
C5_SIZES = ("C5-S", "C5-Mid", "C5-Big")


def c5_instances(count: int = 64) -> list:
    """Sizes of the mixed-size workload's instances, drawn uniformly (config 5, stream 2)."""
    rng = np.random.default_rng([19542, 5, 0, 2])
    return [C5_SIZES[i] for i in rng.integers(0, len(C5_SIZES), count)]


def preset(name: str) -> Geometry:
    return PRESETS[name]()
