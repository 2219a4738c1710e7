"""Pins of the oracle's Strehl estimate (Marechal approximation of Sec. 4), CPU only."""
import numpy as np
import pytest

from oracle import safr as O

RNG = np.random.default_rng(4471)


def _plan(M=16, n=12, kinds=(O.NGS, O.NGS, O.LGS), pupil=None):
    stars = [(1e-4 * (i + 1), -5e-5 * i, k) for i, k in enumerate(kinds)]
    plan = O.precompute(n=n, M=M, pitch=0.5, stars=stars, h_lgs=20e3, heights=np.array([0.0, 3000.0]),
                        weights=np.array([0.6, 0.4]), alpha=1e-3, alpha_tt=1e-3, beta=1.5, pupil=pupil)
    return plan


def test_piston_only_residual_has_unit_strehl():
    plan = _plan()
    n = plan.n
    D = 3
    ol = np.full((D, n, n), 2.5) + np.arange(D)[:, None, None]
    sr, var = O.strehl(plan, ol, np.zeros((2, plan.M, plan.M)), RNG.uniform(-1e-4, 1e-4, (D, 2)))
    assert np.all(var <= 1e-28) and np.all(sr == 1.0)


def test_sinusoid_over_whole_periods_gives_the_closed_form():
    # over a full square pupil holding whole periods, A cos(2 pi k i / n + c) has variance A^2 / 2
    n = 12
    plan = _plan(n=n)
    i = np.arange(n)
    amp = np.array([0.3, 0.7])
    ol = np.stack([a * np.cos(2 * np.pi * 3 * i / n + 0.4)[:, None] * np.ones((1, n)) for a in amp])
    for scale in (1.0, 2.5):
        sr, var = O.strehl(plan, ol, np.zeros((2, plan.M, plan.M)), np.zeros((2, 2)), scale=scale)
        assert np.allclose(var, scale ** 2 * amp ** 2 / 2, rtol=1e-13, atol=0)
        assert np.allclose(sr, np.exp(-scale ** 2 * amp ** 2 / 2), rtol=1e-13, atol=0)


def test_variance_matches_brute_force_on_an_annular_pupil():
    n = 9
    x = np.arange(n) - 4.0
    r = np.hypot(x[:, None], x[None, :])
    pupil = ((r <= 4.2) & (r >= 1.5)).astype(np.uint8)
    plan = _plan(n=n, pupil=pupil)
    ph = RNG.standard_normal((2, n, n))
    var = O.pupil_variance(ph, plan.pupil)
    for d in range(2):
        vals = [ph[d, a, b] for a in range(n) for b in range(n) if pupil[a, b]]
        mu = sum(vals) / len(vals)
        ref = sum((v - mu) ** 2 for v in vals) / len(vals)
        assert abs(var[d] - ref) <= 1e-14 * ref


def test_correction_along_a_guide_star_direction_uses_the_natural_star_line_of_sight():
    # a science direction equal to a natural guide star's sees exactly that star's A a, also when the
    # output grids are the laser stars' (mixed asterism: cone 1 on grids of spacing c_l pitch)
    for kinds in ((O.NGS, O.NGS), (O.NGS, O.NGS, O.LGS)):
        plan = _plan(kinds=kinds)
        layers = RNG.standard_normal((2, plan.M, plan.M))
        fwd = O.forward_layers(plan, layers)[:2]
        dirs = np.asarray(plan.stars)[:2, :2]
        res = O.residual_phase(plan, fwd, layers, dirs)
        assert np.max(np.abs(res)) <= 1e-13
