"""Pins of the oracle's learned-filter training objective (CPU only)."""
import numpy as np

import synth
from oracle import learn as LR
from oracle import mlp as N
from oracle import safr as O

RNG = np.random.default_rng(11)


def _fs(M=16):
    st = [(1.3e-4, 0.2e-4, 0), (-0.5e-4, 1.1e-4, 0), (0.3e-4, -1.2e-4, 0), (-1.0e-4, -0.6e-4, 0)]
    return LR.frequency_svd(M=M, pitch=1.0, stars=st, h_lgs=90e3, heights=[0.0, 6000.0], weights=[0.7, 0.3],
                            beta=1.5), st


def _draws(F, L, G, M):
    K = M // 2 + 1
    zl = (RNG.standard_normal((F, L, K, M)) + 1j * RNG.standard_normal((F, L, K, M))) / np.sqrt(2)
    zn = (RNG.standard_normal((F, G, K, M)) + 1j * RNG.standard_normal((F, G, K, M))) / np.sqrt(2)
    return zl, zn


def test_multiplicity_is_parseval_for_real_fields():
    M = 16
    X = RNG.standard_normal((M, M))
    Fh = O.dft2(X)
    _, keep = O.shifted_index(M)
    Kf = keep[:, None] & keep[None, :]
    full = np.sum(np.abs(Fh[Kf]) ** 2)
    half = np.transpose(Fh[:, : M // 2 + 1])                  # [k][j]
    assert abs(np.sum(LR.multiplicity(M) * np.abs(half) ** 2) - full) <= 1e-10 * full


def test_wavefront_spectra_match_the_space_domain_forward_operator():
    """Noise-free d from the statistics' forward model = DFT2 of the oracle's Fourier-form forward operator."""
    M = 16
    fs, st = _fs(M)
    _, keep = O.shifted_index(M)
    Kf = keep[:, None] & keep[None, :]
    layers = O.idft2(O.dft2(RNG.standard_normal((2, M, M))) * Kf).real
    F = np.transpose(O.dft2(layers)[:, :, : M // 2 + 1], (0, 2, 1))    # (L, K, J)
    amp = np.ones_like(F.real)
    Fl, D = LR.wavefront_spectra(fs, amp, F[None], np.zeros((1, 4) + F.shape[1:]), np.zeros(1), M)
    wf = O.forward_fourier(layers, fs["shifts"])
    Dw = np.transpose(O.dft2(wf)[:, :, : M // 2 + 1], (0, 2, 1))
    w = LR.multiplicity(M) > 0
    assert np.max(np.abs(D[0][:, w] - Dw[:, w])) <= 1e-10 * np.max(np.abs(Dw))


def test_quadratic_form_equals_direct_residual():
    """phi^T Q phi - 2 c^T phi + |F|^2 equals |b - F|^2 with b = diag(s) V diag(phi / sigma) U^H d, per frequency."""
    M = 16
    fs, st = _fs(M)
    amp = RNG.uniform(0.5, 2.0, (2, M // 2 + 1, M))
    zl, zn = _draws(3, 2, 4, M)
    eta = np.array([0.01, 0.03, 0.1])
    Q, c, F2 = LR.statistics(fs, amp, zl, zn, eta, M)
    Fl, D = LR.wavefront_spectra(fs, amp, zl, zn, eta, M)
    phi = RNG.uniform(0, 1, Q.shape[:-1])
    sig = fs["sigma"]
    ok = sig > O.learned_cutoff(sig)
    g = np.where(ok, phi / np.where(ok, sig, 1.0), 0.0)               # (F, K, J, r)
    R = np.einsum("kjlr,fkjr,kjgr->fkjlg", fs["V"], g, np.conj(fs["U"]))
    b = fs["s"][None, :, :, :, None] * R
    b = np.einsum("fkjlg,fgkj->fklj", b, D)                           # (F, K, L, J)
    resid = np.sum(np.abs(b - np.transpose(Fl, (0, 2, 1, 3))) ** 2, axis=2)   # (F, K, J)
    quad = np.einsum("fkjr,fkjrq,fkjq->fkj", phi, Q, phi) - 2 * np.einsum("fkjr,fkjr->fkj", c, phi) + F2
    assert np.max(np.abs(quad - resid)) <= 1e-9 * np.max(resid)


def test_batch_gradient_central_differences():
    M = 8
    fs, st = _fs(M)
    amp = RNG.uniform(0.5, 2.0, (2, M // 2 + 1, M))
    zl, zn = _draws(2, 2, 4, M)
    eta = np.array([0.02, 0.05])
    p = RNG.standard_normal(N.N_PARAMS) * 0.3
    loss, grad = LR.batch_loss_and_grad(p, fs, amp, zl, zn, eta, M)
    h = 1e-6
    for i in list(RNG.choice(N.N_PARAMS, 25, replace=False)) + [8704, 8640]:
        e = np.zeros(N.N_PARAMS)
        e[i] = h
        lp, _ = LR.batch_loss_and_grad(p + e, fs, amp, zl, zn, eta, M)
        lm, _ = LR.batch_loss_and_grad(p - e, fs, amp, zl, zn, eta, M)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])), i


def test_vk_amplitude_matches_screen_variance():
    """The synthetic amplitude model: E sum_n w |F|^2 / M^4 equals the screen's variance (Parseval)."""
    geo = synth.preset("C1")
    amp = synth.vk_amplitude(geo)
    var_model = np.sum(LR.multiplicity(geo.M) * np.sum(amp ** 2, axis=0)) / geo.M ** 4
    screens = [synth.periodic_layers(geo, s) for s in range(40)]
    var_emp = np.mean([np.mean(np.sum(x, axis=0) ** 2) - np.mean(np.sum(x, axis=0)) ** 2 for x in screens])
    assert 0.5 < var_emp / var_model < 1.5


def _stats(F=5, M=16, eta=0.02):
    fs, st = _fs(M)
    amp = np.abs(RNG.standard_normal((2, M // 2 + 1, M))) + 0.1
    zl, zn = _draws(F, 2, 4, M)
    Q, c, F2 = LR.statistics(fs, amp, zl, zn, np.full(F, eta), M)
    w = LR.multiplicity(M)
    Z = float(np.sum(w * np.sum(amp ** 2, axis=0)))
    keep = fs["sigma"] > O.learned_cutoff(fs["sigma"])
    return fs, Q, c, F2, w, Z, keep


def test_optimal_filter_is_a_stationary_minimum():
    """The objective's gradient in phi vanishes at phi* on every kept component, and random perturbations
    of phi* (kept components) only increase it: the quadratic is convex (Qbar is a Gram matrix)."""
    fs, Q, c, F2, w, Z, keep = _stats()
    phi, best = LR.optimal_filter(Q, c, F2, w, Z, keep)
    grad = 2.0 * (np.einsum("fkjrq,kjq->kjr", Q, phi) - c.sum(axis=0))
    assert np.max(np.abs(np.where(keep, grad, 0.0))) <= 1e-9 * np.max(np.abs(c.sum(axis=0)))
    for _ in range(20):
        d = np.where(keep, RNG.standard_normal(phi.shape) * 1e-2, 0.0)
        assert LR.objective(phi + d, Q, c, F2, w, Z) > best
    # below the objective of every Tikhonov filter on the same frames
    for alpha in (1e-6, 1e-3, 1e-1, 10.0):
        tik = LR.tikhonov_factors(fs["sigma"], alpha, keep)
        assert LR.objective(tik, Q, c, F2, w, Z) >= best


def test_optimal_filter_one_component_closed_form_and_brute_force():
    """With one kept component the optimum is sum_f c_f / sum_f Q_f; with two, a direct numerical
    minimisation of the objective at one frequency (scipy, no use of the normal equations) finds phi*."""
    from scipy.optimize import minimize
    fs, Q, c, F2, w, Z, keep = _stats(F=3)
    k, j = 3, 5
    assert keep[k, j].all()
    one = keep.copy()
    one[k, j, 1] = False
    phi1, _ = LR.optimal_filter(Q, c, F2, w, Z, one)
    assert abs(phi1[k, j, 0] - c[:, k, j, 0].sum() / Q[:, k, j, 0, 0].sum()) <= 1e-12 * abs(phi1[k, j, 0])
    assert phi1[k, j, 1] == 0.0
    phi, _ = LR.optimal_filter(Q, c, F2, w, Z, keep)
    f = lambda x: float(np.sum(x @ Q[:, k, j] @ x) - 2.0 * np.sum(c[:, k, j] @ x))
    res = minimize(f, np.zeros(2), method="Nelder-Mead", options={"xatol": 1e-12, "fatol": 1e-18, "maxiter": 4000})
    assert np.max(np.abs(res.x - phi[k, j])) <= 1e-6 * np.max(np.abs(phi[k, j]))


def test_tikhonov_factors_reproduce_the_tikhonov_filter():
    """g = phi / sigma with phi = s^2 / (s^2 + alpha) is Tikhonov's g(s) = s / (s^2 + alpha) (Sec. 3.1)."""
    s = np.array([[[3.0, 0.5, 1e-3]]])
    keep = np.ones_like(s, dtype=bool)
    phi = LR.tikhonov_factors(s, 0.25, keep)
    assert np.allclose(phi / s, s / (s ** 2 + 0.25), rtol=1e-15)
