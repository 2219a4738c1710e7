"""Property tests of the oracle over random tiny geometries (hypothesis; CPU only).

Each property holds for every admissible geometry, so a plausible mistake (a
dropped conjugate, a transposed index, a sign in a shift) fails on some draw:
B is Hermitian in frequency, the reconstruction is linear and invariant under a
permutation of the stars, the Tikhonov inverse equals its normal-equations form at
every frequency, and the closed-loop and Strehl pieces respect their identities.
"""
import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

from oracle import safr as O  # noqa: E402

SETTINGS = settings(max_examples=15, deadline=None, derandomize=True)


@st.composite
def geometries(draw):
    M = draw(st.sampled_from([8, 9, 16]))
    n = draw(st.integers(min_value=3, max_value=M))
    L = draw(st.integers(min_value=1, max_value=3))
    J = draw(st.integers(min_value=1, max_value=4))
    kinds = draw(st.lists(st.sampled_from([O.NGS, O.LGS]), min_size=J, max_size=J))
    if len(set(kinds)) > 1:
        kinds = [O.NGS] * J                     # mixed asterisms have their own tests; keep one kind here
    pitch = draw(st.sampled_from([0.25, 0.5, 1.0]))
    h = np.cumsum(draw(st.lists(st.floats(min_value=200.0, max_value=4000.0), min_size=L, max_size=L)))
    h = h - h[0]
    amax = 0.3 * M * pitch / max(h[-1], 1.0) / 2.0
    ang = draw(st.lists(st.tuples(st.floats(-amax, amax), st.floats(-amax, amax)), min_size=J, max_size=J))
    stars = [(float(a), float(b), int(k)) for (a, b), k in zip(ang, kinds)]
    w = draw(st.lists(st.floats(min_value=0.1, max_value=1.0), min_size=L, max_size=L))
    alpha = draw(st.sampled_from([1e-3, 1e-2, 0.3]))
    beta = draw(st.sampled_from([0.0, 1.5]))
    seed = draw(st.integers(min_value=0, max_value=2 ** 16))
    return dict(n=n, M=M, pitch=pitch, stars=stars, h_lgs=90e3, heights=h, weights=np.asarray(w),
                alpha=alpha, alpha_tt=alpha, beta=beta), seed


def _plan(g, **kw):
    return O.precompute(**g, **kw)


@SETTINGS
@given(geometries())
def test_B_is_hermitian_in_frequency(gs):
    g, _ = gs
    B = _plan(g).groups[0].B
    M = g["M"]
    neg = (-np.arange(M)) % M
    assert np.max(np.abs(B - np.conj(B[neg][:, neg]))) <= 1e-12 * max(np.max(np.abs(B)), 1e-300)


@SETTINGS
@given(geometries())
def test_tikhonov_B_equals_normal_equations_at_every_frequency(gs):
    g, _ = gs
    plan = _plan(g, keep_svd=True)
    grp = plan.groups[0]
    M, L = g["M"], len(g["heights"])
    nidx, keep = O.shifted_index(M)
    NX, NY = np.meshgrid(nidx, nidx, indexing="ij")
    st_ = np.asarray(g["stars"], dtype=np.float64)
    gamma = O.normalise_weights(g["weights"])
    T = M * g["pitch"] / 2.0
    c = O.cone_coefficients(g["heights"], int(st_[0, 2]), g["h_lgs"])
    A = O.tomography_matrix(NX, NY, st_[:, :2], g["heights"], c, gamma, T, g["beta"])
    scale = O.layer_scale(NX, NY, c, gamma, T, g["beta"])
    AH = np.conj(np.swapaxes(A, -1, -2))
    R = AH @ np.linalg.inv(A @ AH + g["alpha"] * np.eye(A.shape[-2]))
    ref = np.where((keep[:, None] & keep[None, :])[..., None, None], scale[..., :, None] * R, 0.0)
    assert np.max(np.abs(grp.B - ref)) <= 1e-9 * max(np.max(np.abs(ref)), 1e-300)
    assert L == grp.B.shape[2]


@SETTINGS
@given(geometries())
def test_reconstruction_is_linear_and_star_permutation_invariant(gs):
    g, seed = gs
    rng = np.random.default_rng(seed)
    plan = _plan(g)
    J, n = len(g["stars"]), g["n"]
    x, y = rng.standard_normal((2, J, n, n))
    a, b = rng.standard_normal(2)
    lhs = O.reconstruct(plan, a * x + b * y)
    rhs = a * O.reconstruct(plan, x) + b * O.reconstruct(plan, y)
    assert np.max(np.abs(lhs - rhs)) <= 1e-10 * max(np.max(np.abs(rhs)), 1.0)
    perm = rng.permutation(J)
    gp = dict(g, stars=[g["stars"][i] for i in perm])
    got = O.reconstruct(_plan(gp), x[perm])
    assert np.max(np.abs(got - O.reconstruct(plan, x))) <= 1e-9 * max(np.max(np.abs(got)), 1.0)


@SETTINGS
@given(geometries())
def test_loop_step_and_strehl_identities(gs):
    g, seed = gs
    rng = np.random.default_rng(seed)
    plan = _plan(g)
    J, n, M, L = len(g["stars"]), g["n"], g["M"], len(g["heights"])
    psi = rng.standard_normal((J, n, n))
    a = rng.standard_normal((L, M, M))
    # POLC with the residual formed by the same operator restores the open-loop data
    back = O.polc(plan, O.polc(plan, psi, a, -1.0), a, 1.0)
    assert np.max(np.abs(back - np.where(plan.pupil[None], psi, 0.0))) <= 1e-12 * max(np.max(np.abs(psi)), 1.0)
    # integrator: gain g gives (1 - g) a + g R(POLC)
    g_ = float(rng.uniform(0.1, 0.9))
    step = O.loop_step(plan, psi, a, g_)
    phi = O.reconstruct(plan, O.polc(plan, psi, a))
    assert np.max(np.abs(step - ((1 - g_) * a + g_ * phi))) <= 1e-12 * max(np.max(np.abs(step)), 1.0)
    # Strehl in (0, 1], 1 for a residual that is a pure piston
    dirs = rng.uniform(-1e-4, 1e-4, (3, 2))
    sr, var = O.strehl(plan, rng.standard_normal((3, n, n)), a, dirs, 0.3)
    assert np.all((sr > 0.0) & (sr <= 1.0)) and np.all(var >= 0.0)
    piston = O.forward_layers(plan, a, dirs, np.ones((3, L))) + 2.0
    sr1, _ = O.strehl(plan, piston, a, dirs)
    assert np.allclose(sr1, 1.0, rtol=0, atol=1e-12)
