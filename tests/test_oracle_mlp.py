"""Pins of the oracle's learned-filter network and of the learned-filter path of Alg. 2 (CPU only)."""
import math

import numpy as np
import pytest

from oracle import mlp as N
from oracle import safr as O

RNG = np.random.default_rng(7)


def _params(scale=0.3):
    return RNG.standard_normal(N.N_PARAMS) * scale


def test_parameter_count():
    assert N.N_PARAMS == 8705
    p = _params()
    assert np.array_equal(N.pack(N.unpack(p)), p)


def test_gelu_special_values():
    # x Phi(x): 0 at 0, Phi(1) = 0.8413447460685429 at 1, and gelu(x) - gelu(-x) = x
    assert N.gelu(np.array(0.0)) == 0.0
    assert abs(N.gelu(np.array(1.0)) - 0.8413447460685429) <= 1e-15
    x = RNG.standard_normal(50) * 3
    assert np.max(np.abs(N.gelu(x) - N.gelu(-x) - x)) <= 1e-14
    # large |x|: identity / zero
    assert abs(N.gelu(np.array(12.0)) - 12.0) <= 1e-14 and abs(N.gelu(np.array(-12.0))) <= 1e-14


def test_gelu_grad_central_difference():
    x = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (N.gelu(x + h) - N.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - N.gelu_grad(x))) <= 1e-8


def test_backward_matches_central_differences():
    p = _params()
    X = RNG.standard_normal((9, 4))
    dphi = RNG.standard_normal(9)
    phi, cache = N.forward(p, X, cache=True)
    g = N.backward(p, cache, dphi)
    h = 1e-6
    idx = RNG.choice(N.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [0, 255, 256, 8703, 8704]])       # first/last of each end
    for i in idx:
        e = np.zeros(N.N_PARAMS)
        e[i] = h
        fd = (np.dot(dphi, N.forward(p + e, X)) - np.dot(dphi, N.forward(p - e, X))) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_quadratic_loss_gradient():
    r = 2
    phi = RNG.uniform(0, 1, (5, r))
    A = RNG.standard_normal((5, r, r))
    Q = A @ np.swapaxes(A, 1, 2)
    c = RNG.standard_normal((5, r))
    w = RNG.uniform(0.5, 2, 5)
    g = N.quadratic_loss_grad(phi, Q, c, w)
    h = 1e-6
    for n in range(5):
        for i in range(r):
            e = np.zeros_like(phi)
            e[n, i] = h
            fd = (N.quadratic_loss(phi + e, Q, c, w) - N.quadratic_loss(phi - e, Q, c, w)) / (2 * h)
            assert abs(fd - g[n, i]) <= 1e-7


def test_adam_first_step_is_signed_lr():
    """At t = 1 the bias-corrected ratio is g / |g| (up to eps): each parameter moves by -lr sign(g)."""
    p = _params()
    g = RNG.standard_normal(N.N_PARAMS)
    new, m, v = N.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-3)
    assert np.max(np.abs((new - p) + 1e-3 * np.sign(g))) <= 1e-3 * 1e-8 / np.min(np.abs(g)) + 1e-15
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_round_known_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, 3.14159265, -2.5e-3])
    r = N.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie -> even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6            # tie -> even (upwards)
    assert abs(r[4] - 3.140625) == 0.0
    assert abs(r[5] / -2.5e-3 - 1) <= 2 ** -8


def test_learned_path_with_tikhonov_phi_reproduces_tikhonov_B():
    """phi = s^2 / (s^2 + alpha) through the learned-filter branch gives the Tikhonov B (A21 reading)."""
    import synth
    geo = synth.preset("C1")
    alpha = geo.alpha
    ref = O.precompute_geometry(geo)

    def phi_fn(F):
        s2 = 10.0 ** (2.0 * F[:, 1])
        return s2 / (s2 + alpha)

    got = O.precompute_geometry(geo, phi_fn=phi_fn)
    B0, B1 = ref.groups[0].B, got.groups[0].B
    assert np.max(np.abs(B0 - B1)) <= 1e-13 * np.max(np.abs(B0))


def test_features_are_basis_invariant_layer_weights():
    """sum_l gamma_l |V_li|^2 lies in [min gamma, max gamma] and sums (over i, L <= G) to 1."""
    import synth
    geo = synth.preset("C1")
    plan = O.precompute_geometry(geo, keep_svd=True)
    g = plan.groups[0]
    nidx, _ = O.shifted_index(geo.M)
    NX, NY = np.meshgrid(nidx, nidx, indexing="ij")
    F = O.mlp_features(NX, NY, geo.M * geo.pitch / 2, g.sigma, g.V, plan.gamma, 0.01)
    w = F[..., 3]
    assert np.all(w >= plan.gamma.min() - 1e-12) and np.all(w <= plan.gamma.max() + 1e-12)
    assert np.max(np.abs(w.sum(-1) - 1.0)) <= 1e-12          # L = 2 <= G = 4: V is square unitary
    assert abs(F[0, 1, 0, 0] - 1.0 / (2 * 8.0)) <= 1e-15      # |n| = 1 -> 1 / (2T) cycles per metre
    assert np.all(F[..., 2] == math.log10(0.01))


@pytest.mark.parametrize("bf16", [False, True])
def test_forward_range(bf16):
    p = _params()
    phi = N.forward(p, RNG.standard_normal((100, 4)), bf16=bf16)
    assert np.all((phi > 0) & (phi < 1))


def test_learned_branch_with_unit_phi_is_library_pinv_with_half_precision_cutoff():
    """phi = 1 turns g = phi / sigma into the pseudo-inverse with relative cutoff sqrt(eps): on the
    8 m / 4-star / 3-layer geometry (rank 2 along the frequency axes) B_n = diag(s_l) pinv(A_n)
    with numpy's pinv at rcond = sqrt(eps), frequencies with rounding-level singular values included."""
    import synth
    geo = synth.preset("C5-S")
    got = O.precompute_geometry(geo, phi_fn=lambda F: np.ones(len(F)))
    M, T = geo.M, geo.T
    gamma = O.normalise_weights(geo.weights)
    c = O.cone_coefficients(geo.heights, 0, geo.h_lgs)
    nidx, keep = O.shifted_index(M)
    stars = np.asarray(geo.stars, dtype=np.float64)[:, :2]
    rank_deficient = 0
    # includes (29, 0), (0, 35), (39, 0): rank 2 with a smallest singular value at rounding level
    # that happens to exceed max(G, L) eps sigma_1
    for j, k in [(j, k) for j in (0, 1, 5, 31, 33, 40) for k in (0, 3, 17, 60)] + [(29, 0), (0, 35), (39, 0)]:
        if not (keep[j] and keep[k]):
            continue
        A = O.tomography_matrix(np.array([[nidx[j]]]), np.array([[nidx[k]]]), stars, geo.heights, c, gamma, T,
                                geo.beta)[0, 0]
        sv = np.linalg.svd(A, compute_uv=False)
        rank_deficient += int(sv[-1] < 1e-12 * sv[0])
        s = O.layer_scale(np.array([[nidx[j]]]), np.array([[nidx[k]]]), c, gamma, T, geo.beta)[0, 0]
        want = s[:, None] * np.linalg.pinv(A, rcond=np.sqrt(np.finfo(float).eps))
        B = got.groups[0].B[j, k]
        assert np.max(np.abs(B - want)) <= 1e-10 * np.max(np.abs(want)), (j, k)
    assert rank_deficient >= 3
