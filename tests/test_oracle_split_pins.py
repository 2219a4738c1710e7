"""Pins of the split-tomography sum (Sec. 3.3: the layers reconstructed from the laser stars with their
tip/tilt removed, plus those reconstructed from the tip/tilt stars, resampled onto the laser layer grids),
against values fixed independently of the oracle's code (CPU only).

* A closed form: one layer at the ground (both groups' cone coefficient 1, so the resampling is the
  identity), beta = 0 and alpha = alpha_TT = 0.  Then A_n = 1 (one column of ones) at every frequency, the
  pseudo-inverse gives b = the mean over a group's stars, and the mixed reconstruction must be the mean
  laser-star data with its tip/tilt removed plus the mean tip/tilt of the natural stars, zero-extended, with
  the Nyquist row and column dropped.  The inputs are built so that these are known without a fit: laser
  data even in x and y on a centred symmetric pupil (no tip/tilt), natural data = a known plane + an even
  field + a piston (tip/tilt = the plane).  Swapped tip/tilt modes, an average instead of a sum, a lost
  normalisation or a sign all fail it.
* The resampling onto the cone-scaled grids against scipy's periodic linear interpolation
  (scipy.ndimage.map_coordinates, order 1, grid-wrap) at the grid points c_l (p - M/2) + M/2.
"""
import numpy as np

from oracle import safr as O

RNG = np.random.default_rng(2510)


def _even(n, rng):
    """A random field even in both axes about the pupil centre."""
    r = rng.standard_normal((n, n))
    return (r + r[::-1, :] + r[:, ::-1] + r[::-1, ::-1]) / 4.0


def _symmetric_pupil(n):
    x = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(x, x, indexing="ij")
    R = np.hypot(X, Y)
    m = (R <= (n - 1) / 2.0 + 1e-9) & (R >= 1.2)               # annulus: symmetric under x -> -x, y -> -y
    assert np.array_equal(m, m[::-1, :]) and np.array_equal(m, m[:, ::-1])
    return m.astype(np.uint8), X, Y


def _expected(field, M):
    """Zero extension at p0 = (M - n + 1) // 2, without the Nyquist row and column (numpy FFT)."""
    n = field.shape[0]
    z = np.zeros((M, M))
    p0 = (M - n + 1) // 2
    z[p0:p0 + n, p0:p0 + n] = field
    X = np.fft.fft2(z)
    X[M // 2, :] = 0.0
    X[:, M // 2] = 0.0
    return np.fft.ifft2(X).real


def test_ground_layer_split_tomography_closed_form():
    M, n = 16, 11
    pupil, X, Y = _symmetric_pupil(n)
    m = pupil.astype(bool)
    lgs = [(RNG.uniform(-1, 1) * 1e-4, RNG.uniform(-1, 1) * 1e-4, O.LGS) for _ in range(3)]
    ngs = [(RNG.uniform(-1, 1) * 1e-4, RNG.uniform(-1, 1) * 1e-4, O.NGS) for _ in range(2)]
    plan = O.precompute(n=n, M=M, pitch=1.0, stars=lgs + ngs, h_lgs=90e3, heights=[0.0], weights=[1.0],
                        alpha=0.0, alpha_tt=0.0, beta=0.0, pupil=pupil)
    assert plan.mixed
    laser = [_even(n, RNG) for _ in lgs]                         # no tip/tilt on a symmetric pupil
    tilts = [(RNG.uniform(-1, 1), RNG.uniform(-1, 1)) for _ in ngs]
    natural = [b * X + c * Y + _even(n, RNG) + RNG.uniform(-3, 3) for b, c in tilts]
    wf = np.stack(laser + natural)
    got = O.reconstruct(plan, wf)[0]
    want = _expected(np.where(m, np.mean(laser, axis=0) + np.mean([b * X + c * Y for b, c in tilts], axis=0), 0.0),
                     M)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    # each group alone: the laser part carries no tilt of the natural stars, and vice versa
    only_l = O.reconstruct(plan, np.stack(laser + [np.zeros((n, n))] * 2))[0]
    assert np.max(np.abs(only_l - _expected(np.where(m, np.mean(laser, axis=0), 0.0), M))) <= 1e-12 * np.max(np.abs(want))


def test_resample_matches_scipy_periodic_linear_interpolation():
    from scipy.ndimage import map_coordinates
    M = 32
    X = RNG.standard_normal((3, M, M))
    c = np.array([1.0, 0.83, 0.61])
    got = O.resample_onto_cone_grid(X, c)
    p = np.arange(M)
    for l in range(3):
        u = c[l] * (p - M / 2.0) + M / 2.0
        U, V = np.meshgrid(u, u, indexing="ij")
        want = map_coordinates(X[l], [U, V], order=1, mode="grid-wrap")
        assert np.max(np.abs(got[l] - want)) <= 1e-12 * np.max(np.abs(X[l]))
