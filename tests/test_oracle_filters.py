"""Pins of the oracle's other filters of Sec. 3.1: truncated SVD and a per-frequency alpha (CPU only).

Truncation is pinned against numpy's pseudo-inverse with a relative cutoff (a
LAPACK SVD, not the oracle's Jacobi); the per-frequency Tikhonov parameter
against the normal-equations form of each frequency's regularised inverse.
"""
import numpy as np
import pytest

from oracle import safr as O

RNG = np.random.default_rng(7319)


def _geometry(M=16, G=4, L=3, seed=0):
    rng = np.random.default_rng(seed)
    stars = [(float(x), float(y), O.NGS) for x, y in rng.uniform(-2e-4, 2e-4, (G, 2))]
    heights = np.linspace(0.0, 9000.0, L)
    weights = rng.uniform(0.3, 1.0, L)
    return dict(n=M, M=M, pitch=0.5, stars=stars, h_lgs=90e3, heights=heights, weights=weights,
                alpha_tt=0.0, beta=1.5)


def _A_and_scale(geo):
    M = geo["M"]
    nidx, keep = O.shifted_index(M)
    NX, NY = np.meshgrid(nidx, nidx, indexing="ij")
    st = np.asarray(geo["stars"], dtype=np.float64)
    c = np.ones(len(geo["heights"]))
    gamma = O.normalise_weights(geo["weights"])
    T = M * geo["pitch"] / 2.0
    A = O.tomography_matrix(NX, NY, st[:, :2], geo["heights"], c, gamma, T, geo["beta"])
    scale = O.layer_scale(NX, NY, c, gamma, T, geo["beta"])
    return A, scale, keep[:, None] & keep[None, :]


def _symmetric_weights(M, rng):
    """Point-symmetric w[j, k] = w[-j, -k] (so B stays Hermitian), not symmetric under transposition."""
    w = rng.uniform(0.1, 10.0, (M, M))
    w = 0.5 * (w + np.roll(w[::-1, ::-1], (1, 1), axis=(0, 1)))
    assert not np.allclose(w, w.T)
    return w


def test_tsvd_matches_library_pinv_with_relative_cutoff():
    geo = _geometry()
    A, scale, K = _A_and_scale(geo)
    sig = np.linalg.svd(A, compute_uv=False)                 # (M, M, min(G, L)), LAPACK
    alpha = float(np.median(sig ** 2))
    while np.min(np.abs(sig ** 2 - alpha)) <= 1e-8 * alpha:  # keep every decision clear of rounding
        alpha *= 1.01
    kept = np.sum(sig ** 2 > alpha, axis=-1)
    assert np.any((kept > 0) & (kept < sig.shape[-1]))      # the truncation is partial somewhere
    plan = O.precompute(alpha=alpha, filter="tsvd", **geo)
    ref = scale[..., :, None] * np.linalg.pinv(A, rcond=np.sqrt(alpha) / sig[..., 0])
    ref = np.where(K[..., None, None], ref, 0.0)
    B = plan.groups[0].B
    assert np.max(np.abs(B - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_tsvd_with_zero_alpha_is_the_pseudo_inverse():
    geo = _geometry(seed=1)
    a = O.precompute(alpha=0.0, filter="tsvd", **geo).groups[0].B
    b = O.precompute(alpha=0.0, **geo).groups[0].B
    assert np.array_equal(a, b)


@pytest.mark.parametrize("G,L", [(4, 3), (2, 3)])
def test_per_frequency_alpha_equals_normal_equations(G, L):
    geo = _geometry(G=G, L=L, seed=2)
    M = geo["M"]
    A, scale, K = _A_and_scale(geo)
    w = _symmetric_weights(M, RNG)
    alpha = 2e-3
    plan = O.precompute(alpha=alpha, alpha_weight=w, **geo)
    AH = np.conj(np.swapaxes(A, -1, -2))
    an = (alpha * w)[..., None, None]
    if L <= G:
        R = np.linalg.solve(AH @ A + an * np.eye(L), AH)
    else:
        R = AH @ np.linalg.inv(A @ AH + an * np.eye(G))
    ref = np.where(K[..., None, None], scale[..., :, None] * R, 0.0)
    B = plan.groups[0].B
    assert np.max(np.abs(B - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_per_frequency_alpha_scales_both_groups_of_a_mixed_asterism():
    geo = _geometry(seed=3)
    geo["stars"] = geo["stars"][:3] + [(1e-4, -1e-4, O.LGS), (-1e-4, 1e-4, O.LGS)]
    geo["alpha_tt"] = 4e-3
    M = geo["M"]
    w = np.full((M, M), 3.0)
    a = O.precompute(alpha=1e-3, alpha_weight=w, **geo)
    b = O.precompute(alpha=3e-3, **dict(geo, alpha_tt=1.2e-2))
    for ga, gb in zip(a.groups, b.groups):
        assert np.max(np.abs(ga.B - gb.B)) <= 1e-14 * np.max(np.abs(gb.B))


def test_tsvd_reconstruction_is_exact_on_the_kept_subspace():
    # data in the span of the kept right singular vectors is reconstructed exactly per frequency
    geo = _geometry(G=4, L=2, seed=4)
    A, scale, K = _A_and_scale(geo)
    sig = np.linalg.svd(A, compute_uv=False)
    alpha = float(np.percentile(sig ** 2, 30))
    plan = O.precompute(alpha=alpha, filter="tsvd", keep_svd=True, **geo)
    grp = plan.groups[0]
    j, k = 3, 5
    keep = grp.sigma[j, k] ** 2 > alpha
    assert keep.any()
    x = grp.V[j, k][:, keep] @ (RNG.standard_normal(keep.sum()) + 1j * RNG.standard_normal(keep.sum()))
    d = A[j, k] @ x                                          # A x for layer coefficients x (scaled basis)
    rec = grp.B[j, k] @ d                                    # scale_l * (A^+ d)_l
    assert np.max(np.abs(rec - scale[j, k] * x)) <= 1e-11 * np.max(np.abs(scale[j, k] * x))
