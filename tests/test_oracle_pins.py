"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test ties one part of the oracle to something other than itself: a
library routine of a different algorithm, a closed form, an invariant, a
brute-force construction, or a value the paper prints.
"""
import json
import os

import numpy as np
import pytest

from oracle import safr as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(20251019)


def _stars(G, scale=1e-4, kind=O.NGS, rng=RNG):
    a = rng.uniform(-1.0, 1.0, (G, 2)) * scale
    return [(float(x), float(y), kind) for x, y in a]


def _plan(M, stars, heights, weights, alpha=0.0, beta=1.5, h_lgs=90e3, pitch=1.0, n=None, **kw):
    return O.precompute(n=M if n is None else n, M=M, pitch=pitch, stars=stars, h_lgs=h_lgs,
                        heights=heights, weights=weights, alpha=alpha, alpha_tt=alpha,
                        beta=beta, **kw)


def _bandlimited(L, M, rng=RNG, piston=False):
    """Random real layers with no Nyquist content (and no piston unless asked)."""
    F = O.dft2(rng.standard_normal((L, M, M)))
    _, keep = O.shifted_index(M)
    K = keep[:, None] & keep[None, :]
    if not piston:
        K = K.copy()
        K[0, 0] = False
    return O.idft2(F * K).real


# ----------------------------------------------------------------------------------------
# Sec. 3.2: DFT2 / IDFT2
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("M", [8, 9, 16, 64])
def test_dft2_matches_library_fft(M):
    X = RNG.standard_normal((3, M, M)) + 1j * RNG.standard_normal((3, M, M))
    ref = np.fft.fft2(X)
    assert np.max(np.abs(O.dft2(X) - ref)) <= 1e-12 * np.max(np.abs(ref))
    refi = np.fft.ifft2(X)
    assert np.max(np.abs(O.idft2(X) - refi)) <= 1e-12 * np.max(np.abs(refi))


@pytest.mark.parametrize("M", [7, 8, 16])
def test_dft2_closed_forms(M):
    # a unit impulse at (p, q) transforms to exp(-2 pi i (j p + k q) / M)
    p, q = 2, M - 3
    X = np.zeros((M, M))
    X[p, q] = 1.0
    j = np.arange(M)
    expect = np.exp(-2j * np.pi * (j[:, None] * p + j[None, :] * q) / M)
    assert np.max(np.abs(O.dft2(X) - expect)) <= 1e-13
    # a constant transforms to M^2 at the origin and 0 elsewhere
    C = O.dft2(np.ones((M, M)))
    e = np.zeros((M, M))
    e[0, 0] = M * M
    assert np.max(np.abs(C - e)) <= 1e-11


@pytest.mark.parametrize("M", [8, 9, 32])
def test_parseval_and_inverse(M):
    X = RNG.standard_normal((M, M))
    Y = O.dft2(X)
    assert abs(np.sum(X ** 2) - np.sum(np.abs(Y) ** 2) / M ** 2) <= 1e-13 * np.sum(X ** 2)
    assert np.max(np.abs(O.idft2(Y) - X)) <= 1e-13


# ----------------------------------------------------------------------------------------
# SVD and the Tikhonov filter (Sec. 3.1)
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("G,L", [(4, 2), (6, 9), (3, 9), (5, 5), (1, 3), (3, 1)])
def test_jacobi_svd(G, L):
    A = RNG.standard_normal((7, G, L)) + 1j * RNG.standard_normal((7, G, L))
    U, s, V = O.jacobi_svd(A)
    r = min(G, L)
    assert U.shape == (7, G, r) and V.shape == (7, L, r) and s.shape == (7, r)
    rec = np.einsum("bgr,br,blr->bgl", U, s, np.conj(V))
    assert np.max(np.abs(rec - A)) <= 1e-13 * np.max(np.abs(A))
    I = np.eye(r)
    assert np.max(np.abs(np.einsum("bgr,bgs->brs", np.conj(U), U) - I)) <= 1e-13
    assert np.max(np.abs(np.einsum("blr,bls->brs", np.conj(V), V) - I)) <= 1e-13
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - ref)) <= 1e-13 * np.max(ref)
    assert np.all(np.diff(s, axis=-1) <= 0)


def test_jacobi_svd_rank_deficient():
    # rank one: every row equal (the structure of A at the zero frequency)
    v = RNG.standard_normal(5) + 1j * RNG.standard_normal(5)
    A = np.tile(v, (4, 1))[None]
    U, s, V = O.jacobi_svd(A)
    assert abs(s[0, 0] - 2.0 * np.linalg.norm(v)) <= 1e-13 * s[0, 0]
    assert np.all(s[0, 1:] <= 1e-13 * s[0, 0])


@pytest.mark.parametrize("G,L,alpha", [(4, 2, 1e-3), (6, 9, 5e-3), (3, 9, 1e-3), (2, 2, 0.3)])
def test_tikhonov_equals_closed_form(G, L, alpha):
    """R_alpha = V g(Sigma^T) U^H with g(s) = s/(s^2+alpha) equals (A^H A + alpha I)^-1 A^H."""
    A = RNG.standard_normal((5, G, L)) + 1j * RNG.standard_normal((5, G, L))
    U, s, V = O.jacobi_svd(A)
    R = O.regularised_inverse(U, s, V, O.tikhonov_filter(s, alpha, G, L))
    AH = np.conj(np.swapaxes(A, -1, -2))
    if L <= G:
        ref = np.linalg.solve(AH @ A + alpha * np.eye(L), AH)
    else:   # the same matrix by the push-through identity, better conditioned when G < L
        ref = AH @ np.linalg.inv(A @ AH + alpha * np.eye(G))
    assert np.max(np.abs(R - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_pinv_filter_matches_library_pinv():
    A = RNG.standard_normal((6, 4, 3)) + 1j * RNG.standard_normal((6, 4, 3))
    U, s, V = O.jacobi_svd(A)
    R = O.regularised_inverse(U, s, V, O.tikhonov_filter(s, 0.0, 4, 3))
    assert np.max(np.abs(R - np.linalg.pinv(A))) <= 1e-12


# ----------------------------------------------------------------------------------------
# B: structure (Eq. sparseM, Alg. 2)
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("M,kind", [(8, O.NGS), (9, O.LGS), (16, O.LGS)])
def test_B_hermitian_and_nyquist(M, kind):
    st = _stars(4, kind=kind)
    plan = _plan(M, st, [0.0, 3000.0, 9000.0], [0.5, 0.3, 0.2], alpha=1e-3, h_lgs=20e3)
    B = plan.groups[0].B
    neg = (-np.arange(M)) % M
    Bm = B[neg][:, neg]
    _, keep = O.shifted_index(M)
    K = keep[:, None] & keep[None, :]
    assert np.max(np.abs(Bm[K] - np.conj(B[K]))) <= 1e-14 * np.max(np.abs(B))
    assert np.all(B[~K] == 0)


def test_B_nonzero_count_matches_paper():
    """B has L G M^2 nonzeros, i.e. 2 L G N floats of storage (Eq. sparseM, Table 1)."""
    spec = json.load(open(os.path.join(GOLDEN, "paper_cost_table.json")))
    for case in spec["cases"]:
        L, G, M = case["L"], case["G"], case["M"]
        assert M % 2 == 1          # the paper's odd-M setting: no Nyquist to drop
        st = _stars(G)
        plan = _plan(M, st, list(1000.0 * np.arange(L)), list(np.ones(L)), alpha=1e-3)
        B = plan.groups[0].B
        nnz = int(np.count_nonzero(B))
        assert nnz == L * G * M * M
        assert 2 * nnz == 2 * L * G * M * M      # floats, N = M^2


def test_paper_parameters_fixture_matches_morfeo_preset():
    import synth
    p = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    g = synth.preset("C2")
    assert g.alpha == p["safr_alpha"] and g.alpha_tt == p["safr_alpha_tt_low_flux"]
    assert g.beta == p["safr_beta"] and g.h_lgs == p["sodium_height_m"]
    assert sum(1 for s in g.stars if s[2] == synth.LGS) == p["n_lgs"]
    r = np.hypot(g.stars[0][0], g.stars[0][1]) / synth.ARCSEC
    assert abs(2 * r - p["lgs_ring_diameter_arcsec"]) < 1e-9


@pytest.mark.parametrize("M", [8, 9])
def test_dense_mvm_form(M):
    """Phi = IDFT2_L . B . DFT2_G . Psi with explicit dense matrices and the index maps u, v."""
    st = _stars(3)
    plan = _plan(M, st, [0.0, 5000.0], [0.6, 0.4], alpha=1e-2)
    B = plan.groups[0].B
    IL, Bs, DG = O.dense_operators(B)
    Psi = RNG.standard_normal((3, M, M))
    dense = (IL @ (Bs @ (DG @ Psi.reshape(-1)))).reshape(2, M, M)
    assert np.max(np.abs(dense.imag)) <= 1e-12
    assert np.max(np.abs(dense.real - O.reconstruct(plan, Psi))) <= 1e-12 * np.max(np.abs(dense))


# ----------------------------------------------------------------------------------------
# Eq. (defAperonly): the forward operator
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("M", [9, 16])
def test_forward_fourier_equals_space_domain(M):
    layers = RNG.standard_normal((2, M, M))
    if M % 2 == 0:
        layers = _bandlimited(2, M, piston=True)
    shifts = RNG.uniform(-2.5, 2.5, (3, 2, 2))
    a = O.forward_fourier(layers, shifts)
    b = O.forward_dirichlet(layers, shifts)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_forward_integer_shift_is_roll():
    M = 12
    layers = _bandlimited(2, M, piston=True)
    shifts = np.array([[[2.0, -1.0], [0.0, 3.0]]])
    expect = np.roll(layers[0], (-2, 1), axis=(0, 1)) + np.roll(layers[1], (0, -3), axis=(0, 1))
    assert np.max(np.abs(O.forward_fourier(layers, shifts)[0] - expect)) <= 1e-12
    assert np.max(np.abs(O.forward_bilinear(layers, shifts)[0] - expect)) <= 1e-14


def test_shift_geometry_of_cone():
    """On layer l's grid the line of sight of star g is displaced by alpha_g h_l / (c_l pitch) pixels."""
    st = [(1e-4, -2e-4, O.LGS)]
    c = O.cone_coefficients([4000.0], O.LGS, 90e3)
    s = O.layer_shifts(st, [4000.0], c, 0.5)
    assert abs(s[0, 0, 0] - 1e-4 * 4000.0 / (c[0] * 0.5)) <= 1e-15
    assert abs(s[0, 0, 1] + 2e-4 * 4000.0 / (c[0] * 0.5)) <= 1e-15
    assert abs(c[0] - (1.0 - 4000.0 / 90e3)) <= 1e-16


# ----------------------------------------------------------------------------------------
# Whole-method pins (Sec. 3.1 least squares, Alg. 1 + Alg. 2)
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("M,kind", [(8, O.NGS), (9, O.NGS), (16, O.NGS), (9, O.LGS), (16, O.LGS)])
def test_exact_recovery(M, kind):
    """Noise-free periodic data from the exact operator, alpha -> 0, J >= L: the layers come back."""
    st = [(1.3e-4, 0.2e-4, kind), (-0.5e-4, 1.1e-4, kind), (0.3e-4, -1.2e-4, kind),
          (-1.0e-4, -0.6e-4, kind)]
    h = [0.0, 4000.0, 8000.0]
    plan = _plan(M, st, h, [0.5, 0.3, 0.2], alpha=0.0, h_lgs=20e3, keep_svd=True)
    sig = plan.groups[0].sigma
    _, keep = O.shifted_index(M)
    K = keep[:, None] & keep[None, :]
    K[0, 0] = False
    assert np.min(sig[K][:, -1] / sig[K][:, 0]) > 1e-4       # full column rank away from DC
    truth = _bandlimited(3, M)
    c = O.cone_coefficients(h, kind, 20e3)
    wf = O.forward_fourier(truth, O.layer_shifts(st, h, c, 1.0))
    rec = O.reconstruct(plan, wf)
    assert np.max(np.abs(rec - truth)) <= 1e-10 * np.max(np.abs(truth))


@pytest.mark.parametrize("M,shift", [(9, (3, -2)), (16, (-5, 4))])
def test_single_star_integer_shift(M, shift):
    """J = L = 1, NGS, beta = 0, alpha = 0: the layer is the wavefront rolled by the shift."""
    h = 1000.0
    st = [(shift[0] / h, shift[1] / h, O.NGS)]
    plan = _plan(M, st, [h], [1.0], alpha=0.0, beta=0.0)
    psi = _bandlimited(1, M, piston=True)
    rec = O.reconstruct(plan, psi)[0]
    assert np.max(np.abs(rec - np.roll(psi[0], shift, axis=(0, 1)))) <= 1e-12
    assert np.max(np.abs(rec - np.roll(psi[0], (-shift[0], -shift[1]), axis=(0, 1)))) > 0.5


def test_single_star_tikhonov_closed_form():
    """J = L = 1: B_n = sigma_n^2 / (sigma_n^2 + alpha) exp(-i theta_n), theta_n = pi h (n . alpha_g) / T."""
    M, h, alpha, beta = 9, 3000.0, 0.05, 1.5
    st = [(0.7e-4, -0.4e-4, O.NGS)]
    plan = _plan(M, st, [h], [1.0], alpha=alpha, beta=beta, pitch=0.5)
    T = M * 0.5 / 2.0
    nidx, _ = O.shifted_index(M)
    NX, NY = np.meshgrid(nidx, nidx, indexing="ij")
    s = (1.0 + np.pi ** 2 / T ** 2 * (NX ** 2 + NY ** 2)) ** (-beta / 2.0)
    theta = np.pi * h * (NX * st[0][0] + NY * st[0][1]) / T
    expect = s ** 2 / (s ** 2 + alpha) * np.exp(-1j * theta)
    assert np.max(np.abs(plan.groups[0].B[..., 0, 0] - expect)) <= 1e-14


@pytest.mark.parametrize("M", [8, 9])
def test_identity(M):
    plan = _plan(M, [(2e-4, 1e-4, O.NGS)], [0.0], [1.0], alpha=0.0, beta=0.0)
    psi = _bandlimited(1, M, piston=True)
    assert np.max(np.abs(O.reconstruct(plan, psi) - psi)) <= 1e-13


@pytest.mark.parametrize("kind", [O.NGS, O.LGS])
def test_dc_closed_form(kind):
    """A_0 = 1_G s^T is rank one; Sherman-Morrison: B_0[l, g] = (gamma_l / c_l^2) / (G sum gamma/c^2 + alpha)."""
    M, alpha = 8, 0.02
    h = [0.0, 5000.0, 11000.0]
    w = np.array([0.5, 0.3, 0.2])
    st = _stars(4, kind=kind)
    plan = _plan(M, st, h, w, alpha=alpha, h_lgs=30e3)
    c = O.cone_coefficients(h, kind, 30e3)
    gam = w / w.sum()
    e = (gam / c ** 2) / (4 * np.sum(gam / c ** 2) + alpha)
    B0 = plan.groups[0].B[0, 0]
    assert np.max(np.abs(B0 - e[:, None])) <= 1e-13


def test_metamorphic_linearity_translation_permutation_transpose():
    M = 16
    st = _stars(4)
    h = [0.0, 6000.0]
    plan = _plan(M, st, h, [0.7, 0.3], alpha=1e-3)
    a = RNG.standard_normal((4, M, M))
    b = RNG.standard_normal((4, M, M))
    ra, rb = O.reconstruct(plan, a), O.reconstruct(plan, b)
    assert np.max(np.abs(O.reconstruct(plan, 2.0 * a - 3.0 * b) - (2.0 * ra - 3.0 * rb))) <= 1e-12
    # translation covariance: rolling every wavefront rolls every layer by the same amount
    rs = O.reconstruct(plan, np.roll(a, (3, -5), axis=(1, 2)))
    assert np.max(np.abs(rs - np.roll(ra, (3, -5), axis=(1, 2)))) <= 1e-12
    # star permutation invariance
    perm = [2, 0, 3, 1]
    plan_p = _plan(M, [st[i] for i in perm], h, [0.7, 0.3], alpha=1e-3)
    assert np.max(np.abs(O.reconstruct(plan_p, a[perm]) - ra)) <= 1e-12
    # transpose symmetry: swap axes of the data and alpha^x <-> alpha^y
    plan_t = _plan(M, [(y, x, k) for x, y, k in st], h, [0.7, 0.3], alpha=1e-3)
    rt = O.reconstruct(plan_t, np.swapaxes(a, 1, 2))
    assert np.max(np.abs(rt - np.swapaxes(ra, 1, 2))) <= 1e-12


def test_lgs_tends_to_ngs():
    """As h_LGS -> infinity the cone coefficients tend to 1 and the laser plan to the natural one,
    with a difference of first order in h / h_LGS."""
    M = 9
    st = _stars(3)
    h = [0.0, 4000.0, 9000.0]
    ngs = _plan(M, st, h, [0.5, 0.3, 0.2], alpha=1e-3).groups[0].B
    scale = np.max(np.abs(ngs))

    def diff(hl):
        lgs = _plan(M, [(x, y, O.LGS) for x, y, _ in st], h, [0.5, 0.3, 0.2], alpha=1e-3, h_lgs=hl)
        return np.max(np.abs(lgs.groups[0].B - ngs)) / scale

    assert diff(1e15) <= 1e-9
    r = diff(1e8) / diff(1e9)
    assert 5.0 < r < 20.0


# ----------------------------------------------------------------------------------------
# Sec. 3.3: tip/tilt handling and the split-tomography sum
# ----------------------------------------------------------------------------------------

def test_tip_tilt_remove_and_keep():
    import synth
    n = 21
    pup = synth.circular_pupil(n, 1.0, 20.0, 0.2)
    x = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(x, x, indexing="ij")
    plane = 0.7 + 0.3 * X - 1.1 * Y
    m = pup.astype(bool)
    assert np.max(np.abs(O.prepare(plane, pup, 1) - np.where(m, 0.7, 0.0))) <= 1e-12
    assert np.max(np.abs(O.prepare(plane, pup, 2) - np.where(m, 0.3 * X - 1.1 * Y, 0.0))) <= 1e-12
    psi = RNG.standard_normal((n, n))
    both = O.prepare(psi, pup, 1) + O.prepare(psi, pup, 2)
    assert np.max(np.abs(both - np.where(m, psi, 0.0))) <= 1e-12
    # the removed residual carries no tilt: it is orthogonal to x and y after its mean is taken out
    r = O.prepare(psi, pup, 1)[m]
    r = r - r.mean()
    assert abs(np.dot(r, X[m] - X[m].mean())) <= 1e-10 and abs(np.dot(r, Y[m] - Y[m].mean())) <= 1e-10


def test_resample_reproduces_linear_functions_and_identity():
    M = 32
    p = np.arange(M) - M / 2.0
    P, Q = np.meshgrid(p, p, indexing="ij")
    lin = np.stack([0.2 + 0.05 * P - 0.03 * Q])
    c = np.array([0.8])
    out = O.resample_onto_cone_grid(lin, c)
    # interior points (no periodic wrap between the two samples) are reproduced exactly
    expect = 0.2 + 0.05 * c[0] * P - 0.03 * c[0] * Q
    assert np.max(np.abs(out[0] - expect)) <= 1e-13
    X = RNG.standard_normal((2, M, M))
    assert np.max(np.abs(O.resample_onto_cone_grid(X, np.ones(2)) - X)) == 0.0


def test_mixed_asterism_is_sum_of_groups():
    """A mixed plan returns the laser-group layers plus the resampled natural-group layers."""
    M, n = 16, 9
    lgs = _stars(3, kind=O.LGS)
    ngs = _stars(2, kind=O.NGS)
    h = [0.0, 5000.0]
    mixed = O.precompute(n=n, M=M, pitch=1.0, stars=lgs + ngs, h_lgs=20e3, heights=h,
                         weights=[0.6, 0.4], alpha=5e-3, alpha_tt=1e-3, beta=1.5)
    only_l = O.precompute(n=n, M=M, pitch=1.0, stars=lgs, h_lgs=20e3, heights=h,
                          weights=[0.6, 0.4], alpha=5e-3, alpha_tt=5e-3, beta=1.5)
    only_n = O.precompute(n=n, M=M, pitch=1.0, stars=ngs, h_lgs=20e3, heights=h,
                          weights=[0.6, 0.4], alpha=1e-3, alpha_tt=1e-3, beta=1.5)
    assert mixed.mixed and [g.kind for g in mixed.groups] == [O.LGS, O.NGS]
    wf = RNG.standard_normal((5, n, n))
    pup = np.ones((n, n), dtype=np.uint8)
    lw = np.stack([O.prepare(w, pup, 1) for w in wf[:3]])
    nw = np.stack([O.prepare(w, pup, 2) for w in wf[3:]])
    expect = O.reconstruct(only_l, lw) + O.resample_onto_cone_grid(O.reconstruct(only_n, nw),
                                                                    mixed.groups[0].c)
    assert np.max(np.abs(O.reconstruct(mixed, wf) - expect)) <= 1e-12


def test_natural_star_layers_are_linear_in_the_plane_coefficients():
    """Sec. 3.3 with keepTT: the natural stars see only b_g x + c_g y over the pupil, and Alg. 1 and the
    resampling are linear, so the natural-star part of a mixed reconstruction equals
    sum_g b_g P[2g] + c_g P[2g+1] with P the (resampled) reconstructions of the unit planes x * mask,
    y * mask of one star at a time (the identity the GPU path's precomputed basis images rest on)."""
    M, n = 16, 9
    lgs = _stars(3, kind=O.LGS)
    ngs = _stars(2, kind=O.NGS)
    plan = O.precompute(n=n, M=M, pitch=1.0, stars=lgs + ngs, h_lgs=20e3, heights=[0.0, 4000.0, 9000.0],
                        weights=[0.5, 0.3, 0.2], alpha=5e-3, alpha_tt=1e-3, beta=1.5)
    pup = np.ones((n, n), dtype=np.uint8)
    pup[0, 0] = pup[-1, -1] = 0
    plan.pupil = pup.astype(bool)
    lg, ng = plan.groups
    wf = RNG.standard_normal((5, n, n))
    laser = O.reconstruct_group(lg.B, O.zero_extend(np.stack([O.prepare(w, pup, 1) for w in wf[:3]]), M))
    natural = O.reconstruct(plan, wf) - laser
    x = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(x, x, indexing="ij")
    m = pup.astype(bool)
    basis = np.stack([X[m], Y[m], np.ones(m.sum())], axis=1)
    expect = np.zeros_like(natural)
    for g in range(2):
        coef, *_ = np.linalg.lstsq(basis, wf[3 + g][m], rcond=None)
        for a, img in ((coef[0], X), (coef[1], Y)):
            unit = np.zeros((2, n, n))
            unit[g] = np.where(m, img, 0.0)
            P = O.resample_onto_cone_grid(O.reconstruct_group(ng.B, O.zero_extend(unit, M)), lg.c)
            expect += a * P
    assert np.max(np.abs(natural - expect)) <= 1e-12 * np.max(np.abs(natural))


def test_zero_extension_centres_pupil():
    M, n = 16, 5
    psi = np.arange(n * n, dtype=float).reshape(n, n)
    Z = O.zero_extend(psi, M)
    assert Z[M // 2, M // 2] == psi[(n - 1) // 2, (n - 1) // 2]
    assert Z.sum() == psi.sum()
