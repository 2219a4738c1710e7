"""Pins of the oracle's closed-loop pieces (Alg. 3 without wavefront reconstruction), CPU only.

The line-of-sight operator used by POLC is pinned by exact cases of its sampling
(integer shifts, where it is a periodic roll of the layers; affine layers, which
bilinear interpolation reproduces exactly, so the result must equal the layer
functions evaluated at the physical crossing points of Sec. 2).  The loop step is
pinned by the closed form of the integrator recursion under a static atmosphere.
"""
import numpy as np
import pytest

from oracle import safr as O

RNG = np.random.default_rng(3519)


def _plan(M, n, stars, heights, h_lgs=20e3, pitch=1.0, alpha=1e-3):
    w = np.linspace(1.0, 0.5, len(heights))
    return O.precompute(n=n, M=M, pitch=pitch, stars=stars, h_lgs=h_lgs, heights=heights,
                        weights=w, alpha=alpha, alpha_tt=alpha, beta=1.5)


def test_line_of_sight_integer_shift_is_periodic_roll():
    # natural stars, pitch 1 m: a direction of k mrad at 1 km height is a shift of k pixels
    M, n = 16, 7
    heights = np.array([0.0, 1000.0, 2000.0])
    stars = [(3e-3, -2e-3, O.NGS), (-1e-3, 4e-3, O.NGS)]
    plan = _plan(M, n, stars, heights)
    layers = RNG.standard_normal((3, M, M))
    got = O.forward_layers(plan, layers)
    p0 = (M - n + 1) // 2
    for g, (ax, ay, _) in enumerate(stars):
        ref = np.zeros((n, n))
        for l, h in enumerate(heights):
            sx, sy = int(round(ax * h)), int(round(ay * h))
            rolled = np.roll(layers[l], (-sx, -sy), axis=(0, 1))      # rolled[p] = layers[p + s]
            ref += rolled[p0:p0 + n, p0:p0 + n]
        assert np.max(np.abs(got[g] - ref)) <= 1e-12


def test_line_of_sight_affine_layers_mixed_asterism():
    # laser stars see layer l scaled by 1 - h_l / h_LGS, natural stars unscaled; the output grids are
    # those of the laser stars.  Affine layers are interpolated exactly away from the periodic seam.
    M, n, pitch, h_lgs = 32, 9, 0.5, 20e3
    heights = np.array([0.0, 2500.0, 5000.0])
    stars = [(4e-4, 0.0, O.LGS), (-2e-4, 3e-4, O.LGS), (1e-4, -5e-4, O.NGS), (-4e-4, -1e-4, O.NGS)]
    plan = _plan(M, n, stars, heights, h_lgs=h_lgs, pitch=pitch)
    coef = RNG.standard_normal((3, 3))                 # f_l(x, y) = c0 + c1 x + c2 y, x, y in metres
    c_grid = 1.0 - heights / h_lgs
    layers = np.empty((3, M, M))
    xg = (np.arange(M) - M / 2.0) * pitch
    for l in range(3):
        X, Y = np.meshgrid(c_grid[l] * xg, c_grid[l] * xg, indexing="ij")
        layers[l] = coef[l, 0] + coef[l, 1] * X + coef[l, 2] * Y
    u, v = O.line_of_sight_points(plan)
    assert u.min() > 0.0 and u.max() < M - 1 and v.min() > 0.0 and v.max() < M - 1
    got = O.forward_layers(plan, layers)
    p0 = (M - n + 1) // 2
    r = (p0 + np.arange(n) - M / 2.0) * pitch           # pupil pixel positions on the grid
    RX, RY = np.meshgrid(r, r, indexing="ij")
    for g, (ax, ay, kind) in enumerate(stars):
        ref = np.zeros((n, n))
        for l, h in enumerate(heights):
            cs = 1.0 - h / h_lgs if kind == O.LGS else 1.0
            x, y = cs * RX + ax * h, cs * RY + ay * h
            ref += coef[l, 0] + coef[l, 1] * x + coef[l, 2] * y
        assert np.max(np.abs(got[g] - ref)) <= 1e-11


def test_polc_masks_and_is_linear_in_the_commands():
    M, n = 16, 9
    stars = [(2e-4, 1e-4, O.NGS), (-1e-4, 2e-4, O.NGS), (1e-4, -2e-4, O.NGS)]
    plan = _plan(M, n, stars, np.array([0.0, 4000.0]), pitch=0.5)
    pup = RNG.integers(0, 2, (n, n)).astype(bool)
    pup[n // 2, n // 2] = True
    plan.pupil = pup
    wf = RNG.standard_normal((3, n, n))
    a1, a2 = RNG.standard_normal((2, 2, M, M))
    assert np.array_equal(O.polc(plan, wf, np.zeros((2, M, M))), np.where(pup, wf, 0.0))
    lin = O.polc(plan, wf, 2.0 * a1 - a2, -0.5)
    ref = np.where(pup, wf, 0.0) - 1.0 * O.forward_layers(plan, a1) + 0.5 * O.forward_layers(plan, a2)
    assert np.max(np.abs(lin - ref)) <= 1e-12
    assert np.all(lin[:, ~pup] == 0.0)


@pytest.mark.parametrize("mixed", [False, True])
def test_loop_static_atmosphere_closed_form(mixed):
    # residuals measured with the current commands: Psi_i = Psi_atm - A a_i.  POLC restores Psi_atm, so
    # a_{i+1} = (1 - g) a_i + g R(Psi_atm) and a_K = (1 - g)^K a_0 + (1 - (1 - g)^K) R(Psi_atm).
    M, n, pitch = 16, 9, 0.5
    if mixed:
        stars = [(3e-4, 0.0, O.LGS), (-3e-4, 1e-4, O.LGS), (0.0, -3e-4, O.LGS), (2e-4, 2e-4, O.NGS)]
    else:
        stars = [(3e-4, 0.0, O.NGS), (-3e-4, 1e-4, O.NGS), (0.0, -3e-4, O.NGS)]
    plan = _plan(M, n, stars, np.array([0.0, 3000.0]), pitch=pitch)
    psi = RNG.standard_normal((len(stars), n, n))
    a = RNG.standard_normal((2, M, M))
    a0 = a.copy()
    g, K = 0.3, 4
    for _ in range(K):
        a = O.loop_step(plan, O.polc(plan, psi, a, -1.0), a, g)
    phi = O.reconstruct(plan, psi)
    ref = (1 - g) ** K * a0 + (1 - (1 - g) ** K) * phi
    assert np.max(np.abs(a - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_loop_gain_limits():
    M, n = 16, 9
    stars = [(3e-4, 0.0, O.NGS), (-3e-4, 1e-4, O.NGS)]
    plan = _plan(M, n, stars, np.array([0.0, 3000.0]), pitch=0.5)
    psi = RNG.standard_normal((2, n, n))
    a = RNG.standard_normal((2, M, M))
    assert np.array_equal(O.loop_step(plan, psi, a, 0.0), a)
    full = O.loop_step(plan, psi, a, 1.0)
    assert np.max(np.abs(full - O.reconstruct(plan, O.polc(plan, psi, a)))) <= 1e-13 * np.max(np.abs(full))


def test_oracle_closed_loop_raises_the_strehl():
    # frozen-flow synthetic atmosphere, natural stars; the command computed from the measurement of step t
    # (taken with the mirror a_t) is applied at step t + 1.  A property of the whole loop, not a pin.
    import synth
    geo = synth.preset("C1")
    plan = O.precompute_geometry(geo)
    t = np.linspace(-20.0, 20.0, 3) * synth.ARCSEC
    dirs = np.array([(x, y) for x in t for y in t])
    sci = geo.replace(stars=[(float(x), float(y), synth.NGS) for x, y in dirs])
    screens = synth.truth_screens(geo, 0)
    a = np.zeros((geo.L, geo.M, geo.M))
    late, open_ = [], []
    for step in range(25):
        wf = synth.simulate_wavefronts(geo, screens, step, frozen_flow=True)
        ol = synth.simulate_wavefronts(sci, screens, step, frozen_flow=True, noise=False)
        sr, _ = O.strehl(plan, ol, a, dirs, 0.5 / 2.2)
        sr0, _ = O.strehl(plan, ol, np.zeros_like(a), dirs, 0.5 / 2.2)
        a = O.loop_step(plan, O.polc(plan, wf, a, -1.0), a, 0.5)
        if step >= 15:
            late.append(sr)
            open_.append(sr0)
    assert np.mean(late) > 0.3 and np.mean(late) > 10.0 * np.mean(open_)
