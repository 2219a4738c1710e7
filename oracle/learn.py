"""FP64 reference of the learned spectral filter's training objective (test infrastructure only).

The learned filter replaces Tikhonov's g(s) = s / (s^2 + alpha) by g_r = phi_r / s_r
with phi = MLP(features) (Sec. 3.1 allows any regularising filter).  Training
pairs are generated in periodic-exact mode: truth layer spectra F_l(n) drawn
with a von Karman amplitude, wavefront spectra from the exact Fourier form of
the tomography operator (Eq. defAperonly on the periodic grids:
d_g(n) = sum_l exp(2 pi i n . s_gl / M) F_l(n), s_gl = alpha_g h_l / (c_l pitch)),
plus white measurement noise.

With b_l = s_l sum_r V[l, r] (phi_r / sigma_r) (U_r^H d) (Alg. 2 with the learned
filter), the full-grid layer residual sum_n sum_l |b_l - F_l|^2 (Parseval) is
quadratic in phi at every frequency:
    |b - F|^2 = phi^T Q phi - 2 c^T phi + |F|^2,
    y_r  = U_r^H d,
    Q_rq = Re(conj(y_r) y_q sum_l s_l^2 conj(V_lr) V_lq) / (sigma_r sigma_q),
    c_r  = Re(y_r sum_l conj(F_l) s_l V_lr) / sigma_r.
Singular values at or below the learned filter's cutoff sqrt(eps) sigma_1 get no filter.
The frame loss is sum_n w_n (...) / Z with w_n the half-spectrum multiplicity
(2 for 0 < k < M/2, 1 for k = 0, 0 on the Nyquist row/column) and
Z = sum_n w_n sum_l amp_l(n)^2 (the expected |F|^2).
"""
from __future__ import annotations

import numpy as np

from . import mlp as _mlp
from . import safr as O


def half_spectrum_indices(M: int):
    """(j, k) array indices of the half spectrum in the layout [k][j], k = 0..M/2."""
    K, J = np.meshgrid(np.arange(M // 2 + 1), np.arange(M), indexing="ij")
    return J, K


def multiplicity(M: int) -> np.ndarray:
    """w[k][j]: 2 for 0 < k < M/2, 1 for k = 0, 0 on the Nyquist row or column (even M)."""
    J, K = half_spectrum_indices(M)
    w = np.where(K == 0, 1.0, 2.0)
    if M % 2 == 0:
        w = np.where((J == M // 2) | (K == M // 2), 0.0, w)
    return w


def frequency_svd(*, M, pitch, stars, h_lgs, heights, weights, beta):
    """SVD of A_n (Sec. 3.1) on the half spectrum [k][j]; also the layer scale s_l(n) and the shifts."""
    stars = np.asarray(stars, dtype=np.float64).reshape(-1, 3)
    kinds = stars[:, 2].astype(int)
    assert np.all(kinds == kinds[0]), "one kind of guide star"
    T = M * pitch / 2.0
    gamma = O.normalise_weights(weights)
    c = O.cone_coefficients(heights, int(kinds[0]), h_lgs)
    nidx, _ = O.shifted_index(M)
    J, K = half_spectrum_indices(M)
    NX, NY = nidx[J], nidx[K]
    A = O.tomography_matrix(NX, NY, stars[:, :2], heights, c, gamma, T, beta)
    U, sig, V = O.jacobi_svd(A)
    s = O.layer_scale(NX, NY, c, gamma, T, beta)
    shifts = O.layer_shifts(stars, heights, c, pitch)
    return dict(U=U, sigma=sig, V=V, s=s, NX=NX, NY=NY, T=T, gamma=gamma, shifts=shifts,
                G=len(stars), L=len(heights))


def noise_std(amp: np.ndarray, M: int) -> float:
    """Expected RMS of a wavefront over the grid per unit eta: sqrt(sum_n w |d|^2) / M^2 with E|d|^2 = sum_l amp^2."""
    return float(np.sqrt(np.sum(multiplicity(M) * np.sum(amp ** 2, axis=0))) / M ** 2)


def wavefront_spectra(fs, amp, zl, zn, eta, M):
    """Layer spectra F = amp zl and wavefront spectra d = sum_l exp(2 pi i n . s_gl / M) F_l + eta sigma M zn."""
    NX, NY = fs["NX"], fs["NY"]
    sn = noise_std(amp, M)
    Fl = amp[None] * zl                                              # (F, L, K, J)
    ph = np.exp(2j * np.pi * (NX[None, None] * fs["shifts"][:, :, 0, None, None]
                              + NY[None, None] * fs["shifts"][:, :, 1, None, None]) / M)   # (G, L, K, J)
    D = np.einsum("glkj,flkj->fgkj", ph, Fl) + (np.asarray(eta)[:, None, None, None] * sn * M) * zn
    return Fl, D


def statistics(fs, amp, zl, zn, eta, M):
    """Per frame and frequency: Q (F, K, J, r, r), c (F, K, J, r) and |F|^2 (F, K, J).

    amp (L, K, J); zl (F, L, K, J) and zn (F, G, K, J) complex draws with E|z|^2 = 1; eta (F,).
    """
    U, sig, V, s = fs["U"], fs["sigma"], fs["V"], fs["s"]
    G, L = fs["G"], fs["L"]
    Fl, D = wavefront_spectra(fs, amp, zl, zn, eta, M)
    y = np.einsum("kjgr,fgkj->fkjr", np.conj(U), D)                  # U_r^H d
    ok = sig > O.learned_cutoff(sig)
    inv = np.where(ok, 1.0 / np.where(ok, sig, 1.0), 0.0)            # (K, J, r)
    W = np.einsum("kjl,kjlr,kjlq->kjrq", s ** 2, np.conj(V), V)
    Q = np.real(np.conj(y)[..., :, None] * y[..., None, :] * W[None]) * inv[None, ..., :, None] * inv[None, ..., None, :]
    c = np.real(y * np.einsum("flkj,kjl,kjlr->fkjr", np.conj(Fl), s, V)) * inv[None]
    F2 = np.sum(np.abs(Fl) ** 2, axis=1)
    return Q, c, F2


def features(fs, eta):
    """Network inputs per (frame, k, j, r): (|n|/(2T), log10 sigma, log10 eta, sum_l gamma_l |V_lr|^2)."""
    f = O.mlp_features(fs["NX"], fs["NY"], fs["T"], fs["sigma"], fs["V"], fs["gamma"], 1.0)   # (K, J, r, 4)
    out = np.broadcast_to(f, (len(eta),) + f.shape).copy()
    out[..., 2] = np.log10(np.asarray(eta))[:, None, None, None]
    return out


def batch_loss_and_grad(params, fs, amp, zl, zn, eta, M):
    """Mean over the frames of sum_n w (phi^T Q phi - 2 c^T phi + |F|^2) / Z, and its parameter gradient."""
    Q, c, F2 = statistics(fs, amp, zl, zn, eta, M)
    w = multiplicity(M)
    Z = np.sum(w * np.sum(amp ** 2, axis=0))
    X = features(fs, eta)
    nb = len(eta)
    r = X.shape[-2]
    phi, cache = _mlp.forward(params, X.reshape(-1, 4), cache=True)
    phi = phi.reshape(X.shape[:-1])
    ww = (np.broadcast_to(w, phi.shape[:-1]) / (Z * nb)).reshape(-1)
    Qf, cf, pf = Q.reshape(-1, r, r), c.reshape(-1, r), phi.reshape(-1, r)
    loss = _mlp.quadratic_loss(pf, Qf, cf, ww) + float(np.sum(w[None] * F2) / (Z * nb))
    dphi = _mlp.quadratic_loss_grad(pf, Qf, cf, ww)
    grad = _mlp.backward(params, cache, dphi.reshape(-1))
    return loss, grad


def objective(phi, Q, c, F2, w, Z):
    """The training objective for given filter factors phi (F-independent, (K, J, r)) on the frames of the
    statistics: sum over frames and frequencies of w (phi^T Q phi - 2 c^T phi + |F|^2), divided by Z and
    the number of frames."""
    nb = Q.shape[0]
    quad = np.einsum("kjr,fkjrq,kjq->fkj", phi, Q, phi) - 2.0 * np.einsum("fkjr,kjr->fkj", c, phi) + F2
    return float(np.sum(w[None] * quad) / (Z * nb))


def optimal_filter(Q, c, F2, w, Z, keep):
    """The filter factors minimising the training objective over the frames of the statistics: at each
    frequency the objective is the quadratic phi^T Qbar phi - 2 cbar^T phi + const (Qbar, cbar summed over
    the frames), minimised by phi* = Qbar^-1 cbar over the components kept (keep: (K, J, r) bool, the
    singular values above the learned filter's cutoff; the others have phi = 0).  Returns (phi*, the
    objective at phi*)."""
    Qb = Q.sum(axis=0)
    cb = c.sum(axis=0)
    K, Jn, r = cb.shape
    phi = np.zeros((K, Jn, r))
    for k in range(K):
        for j in range(Jn):
            idx = np.flatnonzero(keep[k, j])
            if idx.size:
                phi[k, j, idx] = np.linalg.solve(Qb[k, j][np.ix_(idx, idx)], cb[k, j, idx])
    return phi, objective(phi, Q, c, F2, w, Z)


def tikhonov_factors(sigma, alpha, keep):
    """Tikhonov's filter factors phi = sigma^2 / (sigma^2 + alpha) (Sec. 3.1), 0 where not kept."""
    return np.where(keep, sigma ** 2 / (sigma ** 2 + alpha), 0.0)
