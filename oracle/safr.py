"""FP64 CPU oracle of SAFR (arXiv 2510.19542): slow, plain, test infrastructure only.

This module is the correctness reference for the GPU library.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
library never calls it and shares no code with it.

It follows the paper step by step:

* Sec. 2: layered model, cone coefficients c_l, weights gamma_l normalised to 1;
* Sec. 3.1: the per-frequency matrix A_jk built from the bases w_jk and
  w^(beta)_{jk,l}, its SVD and the filtered inverse R_alpha = V g(Sigma^T) U^H
  with the Tikhonov filter g(s) = s / (s^2 + alpha);
* Sec. 3.2: grids, DFT2 / IDFT2 (unnormalised forward, 1/M^2 on the inverse),
  the shifted index n(j), the coefficients b_{jk,lg}, Alg. 2 (soft real time,
  builds B) and Alg. 1 (hard real time: fft2 -> multiply by B -> ifft2);
* Sec. 3.3: split tomography for mixed asterisms (laser stars with tip/tilt
  removed, natural stars reconstructing only tip/tilt, layers added).

Every floating-point step is FP64.  Transforms are direct (dense DFT matrices),
the SVD is a one-sided (Hestenes) complex Jacobi iteration.

Readings taken where the paper is silent or assumes odd M (all documented in
the design notes):

* even M: symmetric truncation with m = M/2 - 1; frequencies on the Nyquist row
  or column (j = M/2 or k = M/2) get B = 0, which keeps B Hermitian;
* the (-1)^(j+k) factors of Appendix A appear in analysis and synthesis alike and
  cancel, so Alg. 1 is used without them;
* Alg. 2's sum is read with V[l, r] (R = V g(Sigma^T) U^H of Sec. 3.1);
* alpha = 0 means the pseudo-inverse, singular values below
  max(G, L) * eps * sigma_1 being dropped;
* pupil data sits centred in the M x M grid: pupil sample i -> p = (M - n + 1) // 2 + i;
* split tomography: laser-star data has its least-squares tip/tilt plane (fit of
  1, x, y over the pupil pixels) subtracted; natural-star data is reduced to that
  plane; the natural-star layers (spacing = pitch) are resampled bilinearly
  (periodically) at the points of the laser-star layer grids (spacing c_l * pitch)
  and added;
* Alg. 3 (closed loop): the mirror commands are the reconstructed layers on their
  output grids; POLC adds A(a) with A evaluated by periodic bilinear interpolation
  along each star's line of sight, at the pupil pixels only.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import mlp as _mlp

NGS, LGS = 0, 1
EPS = np.finfo(np.float64).eps


# --------------------------------------------------------------------------------------
# Sec. 2: geometry
# --------------------------------------------------------------------------------------

def normalise_weights(weights) -> np.ndarray:
    """gamma_l normalised so that sum_l gamma_l = 1 (Sec. 2, Sobolev weights)."""
    w = np.asarray(weights, dtype=np.float64)
    return w / w.sum()


def cone_coefficients(heights, kind: int, h_lgs: float) -> np.ndarray:
    """c_l = 1 for natural stars, 1 - h_l / h_LGS for laser stars (Sec. 2)."""
    h = np.asarray(heights, dtype=np.float64)
    if kind == LGS:
        return 1.0 - h / h_lgs
    return np.ones_like(h)


def pupil_offset(M: int, n: int) -> int:
    """Index in the M-grid of pupil sample 0, so that the pupil centre sits at x = 0."""
    return (M - n + 1) // 2


# --------------------------------------------------------------------------------------
# Sec. 3.2: the shifted frequency index n(j)
# --------------------------------------------------------------------------------------

def shifted_index(M: int):
    """n(j) for j = 0..M-1, and the mask of kept frequencies.

    Odd M = 2m + 1: n(j) = j for j <= m, j - M otherwise (Sec. 3.2).
    Even M: m = M/2 - 1 and the Nyquist index j = M/2 is dropped (kept = False).
    """
    j = np.arange(M)
    m = (M - 1) // 2
    n = np.where(j <= m, j, j - M)
    keep = np.ones(M, dtype=bool)
    if M % 2 == 0:
        keep[M // 2] = False
    return n, keep


# --------------------------------------------------------------------------------------
# Sec. 3.1: the per-frequency tomography matrix A_jk
# --------------------------------------------------------------------------------------

def layer_scale(nx, ny, c, gamma, T: float, beta: float) -> np.ndarray:
    """gamma_l^(1/2) / c_l * (1 + tau_l |(j,k)|^2)^(-beta/2), tau_l = pi^2 (c_l T)^(-2).

    This is the factor in front of w_jk in w^(beta)_{jk,l} (Sec. 3.1) and in
    b_{jk,lg} (Sec. 3.2).  Shape: broadcast(nx, ny) + (L,).
    """
    nx = np.asarray(nx, dtype=np.float64)[..., None]
    ny = np.asarray(ny, dtype=np.float64)[..., None]
    c = np.asarray(c, dtype=np.float64)
    tau = np.pi ** 2 / (c * T) ** 2
    return np.sqrt(gamma) / c * (1.0 + tau * (nx ** 2 + ny ** 2)) ** (-beta / 2.0)


def tomography_matrix(nx, ny, angles, heights, c, gamma, T: float, beta: float) -> np.ndarray:
    """A_jk[g, l] = (2T) w^(beta)_{jk,l}(alpha_g^x h_l, alpha_g^y h_l) (Sec. 3.1).

    With w_jk(x, y) = exp(i omega (j x + k y)) / (2T), omega = pi / T, and the layer
    basis evaluated at (x, y) / c_l, the 2T cancels:
    A[g, l] = scale_l * exp(i pi (j alpha_g^x + k alpha_g^y) h_l / (c_l T)).
    Shape: broadcast(nx, ny) + (G, L).
    """
    s = layer_scale(nx, ny, c, gamma, T, beta)                 # (..., L)
    nx = np.asarray(nx, dtype=np.float64)[..., None, None]
    ny = np.asarray(ny, dtype=np.float64)[..., None, None]
    ax = np.asarray(angles)[:, 0][:, None]                     # (G, 1)
    ay = np.asarray(angles)[:, 1][:, None]
    h = np.asarray(heights, dtype=np.float64)[None, :]          # (1, L)
    cc = np.asarray(c, dtype=np.float64)[None, :]
    phase = np.pi * (nx * ax + ny * ay) * h / (cc * T)
    return s[..., None, :] * np.exp(1j * phase)


# --------------------------------------------------------------------------------------
# SVD: one-sided (Hestenes) complex Jacobi, batched over leading axes
# --------------------------------------------------------------------------------------

def _jacobi_columns(X: np.ndarray, tol: float = 1e-15, max_sweeps: int = 100):
    """Orthogonalise the columns of X (..., m, n) by plane rotations; returns (X V, V).

    A pair is rotated while its inner product exceeds tol * |x_p| |x_q| and is not
    negligible against the whole matrix (1e-30 |X|_F^2), so that columns of a
    rank-deficient X that are zero up to rounding are left alone.
    """
    X = np.array(X, dtype=np.complex128, copy=True)
    n = X.shape[-1]
    floor = 1e-30 * np.sum(np.abs(X) ** 2, axis=(-2, -1))
    V = np.broadcast_to(np.eye(n, dtype=np.complex128), X.shape[:-2] + (n, n)).copy()
    for _ in range(max_sweeps):
        rotated = False
        for p in range(n - 1):
            for q in range(p + 1, n):
                xp = X[..., :, p]
                xq = X[..., :, q]
                a = np.sum(np.abs(xp) ** 2, axis=-1)
                b = np.sum(np.abs(xq) ** 2, axis=-1)
                cpq = np.sum(np.conj(xp) * xq, axis=-1)
                mag = np.abs(cpq)
                act = (mag > tol * np.sqrt(a * b)) & (mag > floor)
                if not np.any(act):
                    continue
                rotated = True
                safe = np.where(act, mag, 1.0)
                e = np.where(act, np.conj(cpq) / safe, 1.0)          # exp(-i theta)
                zeta = (b - a) / (2.0 * safe)
                t = np.where(zeta >= 0, 1.0, -1.0) / (np.abs(zeta) + np.hypot(1.0, zeta))
                cs = 1.0 / np.sqrt(1.0 + t ** 2)
                sn = t * cs
                cs = np.where(act, cs, 1.0)
                sn = np.where(act, sn, 0.0)
                for Y in (X, V):
                    yp = Y[..., :, p].copy()
                    yq = Y[..., :, q].copy()
                    Y[..., :, p] = cs[..., None] * yp - (sn * e)[..., None] * yq
                    Y[..., :, q] = sn[..., None] * yp + (cs * e)[..., None] * yq
        if not rotated:
            break
    return X, V


def jacobi_svd(A: np.ndarray):
    """A = U diag(sigma) V^H for A (..., G, L); U (..., G, r), sigma (..., r) descending, V (..., L, r).

    r = min(G, L).  The columns of the thinner side are orthogonalised: A itself
    when L <= G, else A^H (then the roles of U and V swap).
    """
    A = np.asarray(A, dtype=np.complex128)
    G, L = A.shape[-2:]
    flip = L > G
    X = np.conj(np.swapaxes(A, -1, -2)) if flip else A
    W, Q = _jacobi_columns(X)
    sig = np.sqrt(np.sum(np.abs(W) ** 2, axis=-2))             # (..., r)
    order = np.argsort(-sig, axis=-1)
    sig = np.take_along_axis(sig, order, axis=-1)
    W = np.take_along_axis(W, order[..., None, :], axis=-1)
    Q = np.take_along_axis(Q, order[..., None, :], axis=-1)
    safe = np.where(sig > 0, sig, 1.0)
    Wn = np.where(sig[..., None, :] > 0, W / safe[..., None, :], 0.0)
    if flip:
        # A^H = Wn diag(sig) Q^H  =>  A = Q diag(sig) Wn^H
        return Q, sig, Wn
    return Wn, sig, Q


# --------------------------------------------------------------------------------------
# Sec. 3.1: filters and the regularised inverse
# --------------------------------------------------------------------------------------

def rank_tolerance(sigma: np.ndarray, G: int, L: int) -> np.ndarray:
    """max(G, L) * eps * sigma_1: singular values at or below it count as zero."""
    return max(G, L) * EPS * sigma[..., :1]


def learned_cutoff(sigma: np.ndarray) -> np.ndarray:
    """sqrt(eps) * sigma_1: below it the learned filter treats a singular value as zero.

    A filter factor phi in (0, 1) does not vanish as sigma -> 0, so phi / sigma would
    turn singular values at rounding level (exactly rank-deficient frequencies) into
    gains of order 1 / eps; singular directions below sqrt(eps) sigma_1 are not
    resolved to half the working precision and are dropped instead.
    """
    return np.sqrt(EPS) * sigma[..., :1]


def tikhonov_filter(sigma: np.ndarray, alpha, G: int, L: int) -> np.ndarray:
    """g(s) = s / (s^2 + alpha) (Sec. 3.1); alpha = 0 gives 1/s above the rank tolerance.

    alpha is a scalar or an array broadcastable against sigma (one value per frequency,
    Sec. 3.1 allows a different parameter for each A_jk).
    """
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), sigma.shape)
    tol = rank_tolerance(sigma, G, L)
    keep = sigma > tol
    pinv = np.where(keep, 1.0 / np.where(keep, sigma, 1.0), 0.0)
    tik = sigma / (sigma ** 2 + np.where(alpha > 0.0, alpha, 1.0))
    return np.where(alpha > 0.0, tik, pinv)


def tsvd_filter(sigma: np.ndarray, alpha, G: int, L: int) -> np.ndarray:
    """Truncated SVD (Sec. 3.1 admits truncation): g(s) = 1/s for s^2 > alpha, else 0.

    The cut sits where Tikhonov's filter factor s^2 / (s^2 + alpha) equals 1/2, so
    alpha plays the same role in both filters; alpha = 0 is the pseudo-inverse.
    """
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), sigma.shape)
    keep = (sigma > rank_tolerance(sigma, G, L)) & (sigma ** 2 > alpha)
    return np.where(keep, 1.0 / np.where(keep, sigma, 1.0), 0.0)


def regularised_inverse(U, sigma, V, gvals) -> np.ndarray:
    """R = V g(Sigma^T) U^H, shape (..., L, G) (Sec. 3.1)."""
    return np.einsum("...lr,...r,...gr->...lg", V, gvals, np.conj(U))


def mlp_features(nx, ny, T: float, sigma, V, gamma, eta: float) -> np.ndarray:
    """Per singular value: (|n| / (2T) [cycles/m], log10 sigma_i, log10 eta, sum_l gamma_l |V_li|^2)."""
    r = sigma.shape[-1]
    f0 = np.broadcast_to((np.hypot(nx, ny) / (2.0 * T))[..., None], sigma.shape)
    f1 = np.log10(np.maximum(sigma, 1e-30))
    f2 = np.full(sigma.shape, np.log10(eta))
    f3 = np.einsum("l,...lr->...r", np.asarray(gamma), np.abs(V) ** 2)
    assert f3.shape[-1] == r
    return np.stack([f0, f1, f2, f3], axis=-1)


# --------------------------------------------------------------------------------------
# Alg. 2: soft-real-time precomputation of B
# --------------------------------------------------------------------------------------

@dataclasses.dataclass
class Group:
    """One SAFR instance of the split tomography (Sec. 3.3)."""
    stars: np.ndarray        # indices into the star list
    kind: int                # NGS or LGS
    alpha: float
    c: np.ndarray            # (L,) cone coefficients
    B: np.ndarray            # (M, M, L, G) complex128, indexed by array indices (j, k)
    tt_mode: int             # 0 none, 1 remove tip/tilt (laser stars), 2 keep tip/tilt (natural)
    sigma: Optional[np.ndarray] = None
    U: Optional[np.ndarray] = None
    V: Optional[np.ndarray] = None


@dataclasses.dataclass
class Plan:
    n: int
    M: int
    pitch: float
    T: float
    L: int
    gamma: np.ndarray
    pupil: np.ndarray
    groups: List[Group]
    mixed: bool
    stars: Optional[np.ndarray] = None      # (J, 3): alpha_x, alpha_y [rad], kind
    heights: Optional[np.ndarray] = None    # (L,) layer heights [m]
    h_lgs: float = 0.0

    @property
    def c_out(self) -> np.ndarray:
        """Cone coefficients of the output layer grids: those of the first group (laser stars when mixed)."""
        return self.groups[0].c


def split_groups(kinds, alpha: float, alpha_tt: float):
    """Single-kind asterisms: one group with alpha.  Mixed: laser group with alpha, natural with alpha_TT."""
    kinds = np.asarray(kinds, dtype=int)
    if np.all(kinds == kinds[0]):
        return [(np.arange(len(kinds)), int(kinds[0]), alpha, 0)], False
    lgs = np.nonzero(kinds == LGS)[0]
    ngs = np.nonzero(kinds == NGS)[0]
    return [(lgs, LGS, alpha, 1), (ngs, NGS, alpha_tt, 2)], True


def precompute(*, n: int, M: int, pitch: float, stars, h_lgs: float, heights, weights,
               alpha: float, alpha_tt: float, beta: float, pupil=None, mlp_params=None,
               eta: float = 0.01, mlp_bf16: bool = False, phi_fn=None,
               keep_svd: bool = False, filter: str = "tikhonov", alpha_weight=None) -> Plan:
    """Alg. 2 for every frequency of the M x M grid and every group.

    For each array index pair (j, k): n = (n(j), n(k)); A_n per Sec. 3.1; SVD;
    filter; b_{n,lg} = scale_l(n) * sum_r g(sigma_r) conj(U[g, r]) V[l, r].
    With ``mlp_params`` the filter is g_r = phi_r / sigma_r, phi = MLP(features);
    ``phi_fn`` (features (N, 4) -> phi (N,)) replaces the network by any other map.
    ``filter`` = "tikhonov" or "tsvd"; ``alpha_weight`` (M, M), indexed by the array
    indices (j, k) like B, scales the group's alpha per frequency.
    """
    if filter not in ("tikhonov", "tsvd"):
        raise ValueError(f"unknown filter {filter}")
    if mlp_params is not None and phi_fn is None:
        def phi_fn(F):
            return _mlp.forward(mlp_params, F, bf16=mlp_bf16)
    stars = np.asarray(stars, dtype=np.float64).reshape(-1, 3)
    T = M * pitch / 2.0
    gamma = normalise_weights(weights)
    heights = np.asarray(heights, dtype=np.float64)
    L = len(heights)
    nidx, keep = shifted_index(M)
    NX, NY = np.meshgrid(nidx, nidx, indexing="ij")
    KEEP = keep[:, None] & keep[None, :]
    groups = []
    spec, mixed = split_groups(stars[:, 2], alpha, alpha_tt)
    for idx, kind, a, tt in spec:
        c = cone_coefficients(heights, kind, h_lgs)
        A = tomography_matrix(NX, NY, stars[idx, :2], heights, c, gamma, T, beta)  # (M,M,G,L)
        U, sig, V = jacobi_svd(A)
        G = len(idx)
        a_n = a if alpha_weight is None else a * np.asarray(alpha_weight, dtype=np.float64)[..., None]
        if phi_fn is None:
            g = (tikhonov_filter if filter == "tikhonov" else tsvd_filter)(sig, a_n, G, L)
        else:
            feats = mlp_features(NX, NY, T, sig, V, gamma, eta)
            phi = np.asarray(phi_fn(feats.reshape(-1, 4))).reshape(sig.shape)
            ok = sig > learned_cutoff(sig)
            g = np.where(ok, phi / np.where(ok, sig, 1.0), 0.0)
        R = regularised_inverse(U, sig, V, g)                                     # (M,M,L,G)
        scale = layer_scale(NX, NY, c, gamma, T, beta)                            # (M,M,L)
        B = scale[..., :, None] * R
        B = np.where(KEEP[..., None, None], B, 0.0)
        grp = Group(stars=idx, kind=kind, alpha=a, c=c, B=B, tt_mode=tt)
        if keep_svd:
            grp.sigma, grp.U, grp.V = sig, U, V
        groups.append(grp)
    if pupil is None:
        pupil = np.ones((n, n), dtype=np.uint8)
    return Plan(n=n, M=M, pitch=pitch, T=T, L=L, gamma=gamma,
                pupil=np.asarray(pupil).astype(bool), groups=groups, mixed=mixed,
                stars=stars, heights=heights, h_lgs=float(h_lgs))


def precompute_geometry(geo, **kw) -> Plan:
    """Alg. 2 for an object with the fields of a workload preset."""
    return precompute(n=geo.n, M=geo.M, pitch=geo.pitch, stars=geo.stars, h_lgs=geo.h_lgs,
                      heights=geo.heights, weights=geo.weights, alpha=kw.pop("alpha", geo.alpha),
                      alpha_tt=kw.pop("alpha_tt", geo.alpha_tt), beta=kw.pop("beta", geo.beta),
                      pupil=geo.pupil(), **kw)


# --------------------------------------------------------------------------------------
# Sec. 3.2: DFT2 / IDFT2 (direct, dense)
# --------------------------------------------------------------------------------------

def dft_matrix(M: int, sign: int) -> np.ndarray:
    """F[j, p] = exp(sign * 2 pi i (j p mod M) / M), the product reduced in integers first."""
    j = np.arange(M)
    r = np.outer(j, j) % M
    ang = 2.0 * np.pi * r / M
    return np.cos(ang) + 1j * sign * np.sin(ang)


def dft2(X: np.ndarray) -> np.ndarray:
    """DFT2(X)[j, k] = sum_{p,q} exp(-2 pi i (j p + k q) / M) X[p, q] over the last two axes."""
    M = X.shape[-1]
    F = dft_matrix(M, -1)
    return F @ X @ F.T


def idft2(Y: np.ndarray) -> np.ndarray:
    """IDFT2(Y)[p, q] = M^-2 sum_{j,k} exp(+2 pi i (j p + k q) / M) Y[j, k]."""
    M = Y.shape[-1]
    F = dft_matrix(M, +1)
    return (F @ Y @ F.T) / (M * M)


# --------------------------------------------------------------------------------------
# Sec. 2 / 3.3: pupil data, zero extension and tip/tilt handling
# --------------------------------------------------------------------------------------

def tt_plane(psi: np.ndarray, pupil: np.ndarray) -> np.ndarray:
    """Least-squares fit a + b x + c y of psi over the pupil pixels; returns b x + c y on the grid.

    x, y are pixel coordinates measured from the pupil centre.
    """
    n = psi.shape[-1]
    x = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(x, x, indexing="ij")
    m = pupil.astype(bool)
    basis = np.stack([np.ones(m.sum()), X[m], Y[m]], axis=1)
    coef, *_ = np.linalg.lstsq(basis, psi[m], rcond=None)
    return coef[1] * X + coef[2] * Y


def prepare(psi: np.ndarray, pupil: np.ndarray, tt_mode: int) -> np.ndarray:
    """Pupil-masked data with removeTT (mode 1) or keepTT (mode 2) applied (Sec. 3.3)."""
    m = pupil.astype(bool)
    psi = np.where(m, np.asarray(psi, dtype=np.float64), 0.0)
    if tt_mode == 0:
        return psi
    plane = np.where(m, tt_plane(psi, m), 0.0)
    return psi - plane if tt_mode == 1 else plane


def zero_extend(psi: np.ndarray, M: int) -> np.ndarray:
    """Extension by zero of the n x n pupil data to the periodic M x M grid (Sec. 2), centred."""
    n = psi.shape[-1]
    p0 = pupil_offset(M, n)
    out = np.zeros(psi.shape[:-2] + (M, M))
    out[..., p0:p0 + n, p0:p0 + n] = psi
    return out


# --------------------------------------------------------------------------------------
# Alg. 1: hard-real-time reconstruction
# --------------------------------------------------------------------------------------

def apply_B(B: np.ndarray, D: np.ndarray) -> np.ndarray:
    """b_l(j, k) = sum_g B[j, k, l, g] d_g(j, k); D (G, M, M) -> (L, M, M)."""
    return np.einsum("jklg,gjk->ljk", B, D)


def reconstruct_group(B: np.ndarray, Psi: np.ndarray) -> np.ndarray:
    """Alg. 1 for one group: d_g = DFT2(Psi_g), b_l = sum_g B d_g, Phi_l = IDFT2(b_l) (real part)."""
    D = dft2(Psi)
    b = apply_B(B, D)
    Phi = idft2(b)
    scale = max(np.max(np.abs(Phi.real)), 1e-300)
    assert np.max(np.abs(Phi.imag)) <= 1e-9 * scale, "B is not Hermitian"
    return Phi.real


def resample_onto_cone_grid(Phi: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Natural-star layers (spacing pitch) sampled bilinearly, periodically, on the grids of spacing c_l pitch.

    Layer l, output index p corresponds to x = c_l (p - M/2) pitch, i.e. the
    fractional input index u = c_l (p - M/2) + M/2.
    """
    L, M, _ = Phi.shape
    out = np.empty_like(Phi)
    idx = np.arange(M) - M / 2.0
    for l in range(L):
        u = c[l] * idx + M / 2.0
        i0 = np.floor(u).astype(int)
        f = u - i0
        a0 = i0 % M
        a1 = (i0 + 1) % M
        rows = (1.0 - f)[:, None] * Phi[l][a0, :] + f[:, None] * Phi[l][a1, :]
        out[l] = (1.0 - f)[None, :] * rows[:, a0] + f[None, :] * rows[:, a1]
    return out


def reconstruct(plan: Plan, wavefronts: np.ndarray) -> np.ndarray:
    """One frame: wavefronts (J, n, n) -> layers (L, M, M) on the output layer grids (Alg. 1, Sec. 3.3)."""
    wf = np.asarray(wavefronts, dtype=np.float64)
    parts = []
    for grp in plan.groups:
        psi = np.stack([prepare(wf[g], plan.pupil, grp.tt_mode) for g in grp.stars])
        parts.append(reconstruct_group(grp.B, zero_extend(psi, plan.M)))
    if not plan.mixed:
        return parts[0]
    lgs = 0 if plan.groups[0].kind == LGS else 1
    return parts[lgs] + resample_onto_cone_grid(parts[1 - lgs], plan.groups[lgs].c)


def reconstruct_batch(plan: Plan, wavefronts: np.ndarray) -> np.ndarray:
    """(F, J, n, n) -> (F, L, M, M), frame by frame."""
    return np.stack([reconstruct(plan, w) for w in wavefronts])


# --------------------------------------------------------------------------------------
# Sec. 3.2: the matrix representation Phi = IDFT2_L . B . DFT2_G . Psi
# --------------------------------------------------------------------------------------

def dense_operators(B: np.ndarray):
    """(IDFT2_L, B_sparse, DFT2_G) as dense matrices with the index maps u, v of Eq. (sparseM).

    u(j, k, l) = l M^2 + j M + k and v(j, k, g) = g M^2 + j M + k (0-based).
    Tiny M only (the matrices are M^2 L x M^2 G).
    """
    M, _, L, G = B.shape
    F = dft_matrix(M, -1)
    Fi = dft_matrix(M, +1) / M
    D2 = np.kron(F, F)                  # acts on X flattened row-major
    I2 = np.kron(Fi, Fi)
    Bs = np.zeros((L * M * M, G * M * M), dtype=np.complex128)
    for l in range(L):
        for g in range(G):
            for j in range(M):
                for k in range(M):
                    Bs[l * M * M + j * M + k, g * M * M + j * M + k] = B[j, k, l, g]
    DG = np.kron(np.eye(G), D2)
    IL = np.kron(np.eye(L), I2)
    return IL, Bs, DG


# --------------------------------------------------------------------------------------
# Eq. (defAperonly): the tomography operator, on the discrete periodic grids
# --------------------------------------------------------------------------------------

def layer_shifts(stars, heights, c, pitch: float) -> np.ndarray:
    """Shift alpha_g h_l / (c_l pitch) in layer pixels of the line of sight of star g at layer l.

    (A_g phi)(r) = sum_l phi_l(c_l r + alpha_g h_l); on layer l's own grid (spacing
    c_l pitch) this is the point r / pitch + alpha_g h_l / (c_l pitch).
    Returns (G, L, 2).
    """
    s = np.asarray(stars, dtype=np.float64).reshape(-1, 3)[:, :2]
    h = np.asarray(heights, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    return s[:, None, :] * (h / (c * pitch))[None, :, None]


def forward_fourier(layers: np.ndarray, shifts: np.ndarray) -> np.ndarray:
    """Psi_g = sum_l phi_l(p + s_gl) with phi_l the symmetric trigonometric interpolant of layer l.

    In frequency: d_g(j, k) = sum_l exp(2 pi i (n(j) s^x + n(k) s^y) / M) DFT2(Phi_l)(j, k),
    Nyquist dropped for even M.  layers (L, M, M), shifts (G, L, 2) -> (G, M, M).
    """
    L, M, _ = layers.shape
    nidx, keep = shifted_index(M)
    K = keep[:, None] & keep[None, :]
    Fl = dft2(layers) * K
    out = []
    for g in range(shifts.shape[0]):
        acc = np.zeros((M, M), dtype=np.complex128)
        for l in range(L):
            sx, sy = shifts[g, l]
            acc += np.exp(2j * np.pi * (nidx[:, None] * sx + nidx[None, :] * sy) / M) * Fl[l]
        out.append(idft2(acc).real)
    return np.stack(out)


def dirichlet_kernel(t: np.ndarray, M: int) -> np.ndarray:
    """(1/M) sum_{|n| <= m} exp(2 pi i n t / M) = sin(pi (2m+1) t / M) / (M sin(pi t / M)), m as in n(j)."""
    m = (M - 1) // 2
    K = 2 * m + 1
    t = np.asarray(t, dtype=np.float64)
    den = M * np.sin(np.pi * t / M)
    near = np.abs(den) < 1e-12
    num = np.sin(np.pi * K * t / M)
    # at t = 0 mod M the limit is K / M times the sign pattern of the ratio
    lim = K / M * np.cos(np.pi * K * t / M) / np.cos(np.pi * t / M)
    return np.where(near, lim, num / np.where(near, 1.0, den))


def forward_dirichlet(layers: np.ndarray, shifts: np.ndarray) -> np.ndarray:
    """Space-domain shift-and-sum with the periodic Dirichlet (trigonometric) interpolation kernel.

    Psi_g[p, q] = sum_l sum_{p',q'} Phi_l[p', q'] D(p + s^x - p') D(q + s^y - q').
    Independent of the DFT code; brute force, tiny grids only.
    """
    L, M, _ = layers.shape
    p = np.arange(M)
    out = np.zeros((shifts.shape[0], M, M))
    for g in range(shifts.shape[0]):
        for l in range(L):
            sx, sy = shifts[g, l]
            Kx = dirichlet_kernel(p[:, None] + sx - p[None, :], M)
            Ky = dirichlet_kernel(p[:, None] + sy - p[None, :], M)
            out[g] += Kx @ layers[l] @ Ky.T
    return out


def forward_bilinear(layers: np.ndarray, shifts: np.ndarray) -> np.ndarray:
    """Space-domain shift-and-sum with periodic bilinear interpolation (the paper's POLC operator)."""
    L, M, _ = layers.shape
    p = np.arange(M, dtype=np.float64)
    out = np.zeros((shifts.shape[0], M, M))
    for g in range(shifts.shape[0]):
        for l in range(L):
            sx, sy = shifts[g, l]
            u = p + sx
            v = p + sy
            i0 = np.floor(u).astype(int)
            j0 = np.floor(v).astype(int)
            fu = u - i0
            fv = v - j0
            a0, a1 = i0 % M, (i0 + 1) % M
            b0, b1 = j0 % M, (j0 + 1) % M
            X = layers[l]
            rows = (1 - fu)[:, None] * X[a0, :] + fu[:, None] * X[a1, :]
            out[g] += (1 - fv)[None, :] * rows[:, b0] + fv[None, :] * rows[:, b1]
    return out


# --------------------------------------------------------------------------------------
# Alg. 3: three-step closed loop (the wavefront-reconstruction step excluded)
# --------------------------------------------------------------------------------------

def bilinear_periodic(X: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """X sampled at fractional indices (u, v) by bilinear interpolation on the periodic grid."""
    M0, M1 = X.shape
    i0 = np.floor(u).astype(np.int64)
    j0 = np.floor(v).astype(np.int64)
    fu = u - i0
    fv = v - j0
    a0, a1 = i0 % M0, (i0 + 1) % M0
    b0, b1 = j0 % M1, (j0 + 1) % M1
    return ((1 - fu) * (1 - fv) * X[a0, b0] + fu * (1 - fv) * X[a1, b0]
            + (1 - fu) * fv * X[a0, b1] + fu * fv * X[a1, b1])


def line_of_sight_points(plan: Plan, directions=None, cones=None):
    """Fractional indices (u, v) on each output layer grid seen from every pupil pixel.

    Pupil pixel (i, j) sits at grid point p = p0 + i, q = p0 + j, i.e. at
    r = ((p - M/2) pitch, (q - M/2) pitch).  A source in direction theta with cone
    coefficient c^s_l (Sec. 2: 1 for a natural star, 1 - h_l / h_LGS for a laser star)
    crosses layer l at c^s_l r + theta h_l, which on the layer's output grid (spacing
    c_l pitch, centred at index M/2) is the index (c^s_l r + theta h_l) / (c_l pitch) + M/2.
    ``directions`` (D, 2) and ``cones`` (D, L) default to the plan's guide stars.
    Returns u, v of shape (D, L, n, n).
    """
    M, n, pitch = plan.M, plan.n, plan.pitch
    if directions is None:
        st = np.asarray(plan.stars, dtype=np.float64).reshape(-1, 3)
        directions = st[:, :2]
        cones = np.stack([cone_coefficients(plan.heights, int(k), plan.h_lgs) for k in st[:, 2]])
    directions = np.asarray(directions, dtype=np.float64).reshape(-1, 2)
    cones = np.asarray(cones, dtype=np.float64).reshape(len(directions), -1)
    p0 = pupil_offset(M, n)
    r = (p0 + np.arange(n) - M / 2.0) * pitch
    X, Y = np.meshgrid(r, r, indexing="ij")
    h = np.asarray(plan.heights, dtype=np.float64)
    co = plan.c_out
    D, L = len(directions), len(h)
    u = np.empty((D, L, n, n))
    v = np.empty((D, L, n, n))
    for d in range(D):
        for l in range(L):
            u[d, l] = (cones[d, l] * X + directions[d, 0] * h[l]) / (co[l] * pitch) + M / 2.0
            v[d, l] = (cones[d, l] * Y + directions[d, 1] * h[l]) / (co[l] * pitch) + M / 2.0
    return u, v


def forward_layers(plan: Plan, layers: np.ndarray, directions=None, cones=None) -> np.ndarray:
    """(A a)_g on the pupil: sum over layers of a_l at the line-of-sight points, zero outside the pupil.

    layers (L, M, M) on the output grids -> (D, n, n); D = J guide stars by default.
    """
    u, v = line_of_sight_points(plan, directions, cones)
    out = np.zeros(u.shape[:1] + u.shape[2:])
    for d in range(u.shape[0]):
        for l in range(u.shape[1]):
            out[d] += bilinear_periodic(np.asarray(layers[l], dtype=np.float64), u[d, l], v[d, l])
    return np.where(plan.pupil[None], out, 0.0)


def polc(plan: Plan, wavefronts: np.ndarray, layers: np.ndarray, weight: float = 1.0) -> np.ndarray:
    """Pseudo-open-loop data Psi + weight * A(a) on the pupil pixels, zero outside (Alg. 3, POLC step)."""
    wf = np.where(plan.pupil[None], np.asarray(wavefronts, dtype=np.float64), 0.0)
    return wf + weight * forward_layers(plan, layers)


def loop_step(plan: Plan, wavefronts: np.ndarray, a: np.ndarray, gain: float) -> np.ndarray:
    """One time step of Alg. 3 from given closed-loop wavefronts.

    POLC, tip/tilt removal of the laser stars and the two SAFR reconstructions
    (both inside ``reconstruct``), then the integrator
    a_next = (1 - gain) a + gain Phi.
    """
    phi = reconstruct(plan, polc(plan, wavefronts, a))
    return (1.0 - gain) * np.asarray(a, dtype=np.float64) + gain * phi


# --------------------------------------------------------------------------------------
# Sec. 4: Strehl ratio by the Marechal approximation
# --------------------------------------------------------------------------------------

def residual_phase(plan: Plan, open_loop: np.ndarray, layers: np.ndarray, directions) -> np.ndarray:
    """Phase left in science directions after the correction: open_loop - A_theta(a), on the pupil.

    Science objects are at infinity (cone coefficient 1 on every layer).  open_loop (D, n, n).
    """
    directions = np.asarray(directions, dtype=np.float64).reshape(-1, 2)
    cones = np.ones((len(directions), plan.L))
    corr = forward_layers(plan, layers, directions, cones)
    return np.where(plan.pupil[None], np.asarray(open_loop, dtype=np.float64), 0.0) - corr


def pupil_variance(phase: np.ndarray, pupil: np.ndarray) -> np.ndarray:
    """Variance over the pupil pixels (piston removed) of each (n, n) map in ``phase``."""
    m = pupil.astype(bool)
    vals = phase[..., m]
    return np.mean((vals - vals.mean(axis=-1, keepdims=True)) ** 2, axis=-1)


def marechal_strehl(variance_rad2) -> np.ndarray:
    """Strehl ratio exp(-sigma^2) from the residual phase variance in rad^2 (Marechal)."""
    return np.exp(-np.asarray(variance_rad2, dtype=np.float64))


def strehl(plan: Plan, open_loop: np.ndarray, layers: np.ndarray, directions, scale: float = 1.0):
    """(Strehl ratios, variances in rad^2) of the residual in each direction; ``scale`` converts the
    data's phase unit to radians at the science wavelength."""
    var = scale ** 2 * pupil_variance(residual_phase(plan, open_loop, layers, directions), plan.pupil)
    return marechal_strehl(var), var
