"""FP64 reference of the learned spectral filter network (test infrastructure only).

Network: 4 -> 64 -> 64 -> 64 -> 1 with the exact GELU x * Phi(x) =
x/2 (1 + erf(x / sqrt 2)) (Hendrycks & Gimpel, 2016) after each hidden layer and
a logistic output phi = 1 / (1 + exp(-z)) in (0, 1).  The filter factor that
replaces Tikhonov's is g = phi / sigma (Tikhonov is the member phi = s^2 / (s^2 + alpha)).

Flat parameter packing, 8,705 values:
W1 (64 x 4, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (64 x 64), b3 (64),
w4 (64), b4 (1).  Layer k computes z = W x + b with W[out, in].

Adam follows Kingma & Ba (2015): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

HIDDEN = 64
N_IN = 4
SHAPES = [(HIDDEN, N_IN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,),
          (HIDDEN,), (1,)]
N_PARAMS = int(sum(np.prod(s) for s in SHAPES))          # 8705


def unpack(params):
    p = np.asarray(params, dtype=np.float64).ravel()
    assert p.size == N_PARAMS
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(p[o:o + k].reshape(s))
        o += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in parts])


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64. Finite inputs only."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((a + 0x7FFF + ((a >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, X, bf16: bool = False, cache: bool = False):
    """phi for feature rows X (N, 4).  ``bf16`` rounds every layer input and weight to bfloat16
    (the arithmetic of reduced-precision inference), accumulating in FP64."""
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    r = bf16_round if bf16 else (lambda t: t)
    z1 = r(X) @ r(W1).T + b1
    a1 = gelu(z1)
    z2 = r(a1) @ r(W2).T + b2
    a2 = gelu(z2)
    z3 = r(a2) @ r(W3).T + b3
    a3 = gelu(z3)
    z4 = r(a3) @ r(w4) + b4[0]
    phi = sigmoid(z4)
    if cache:
        return phi, (X, z1, a1, z2, a2, z3, a3, z4, phi)
    return phi


def backward(params, cache, dphi) -> np.ndarray:
    """Gradient of sum_rows dphi * phi with respect to the flat parameters (FP64, hand-derived)."""
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(params)
    X, z1, a1, z2, a2, z3, a3, z4, phi = cache
    dz4 = np.asarray(dphi, dtype=np.float64) * phi * (1.0 - phi)        # (N,)
    gw4 = a3.T @ dz4
    gb4 = np.array([dz4.sum()])
    dz3 = np.outer(dz4, w4) * gelu_grad(z3)                               # (N, 64)
    gW3 = dz3.T @ a2
    gb3 = dz3.sum(0)
    dz2 = (dz3 @ W3) * gelu_grad(z2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3, gw4, gb4])


def adam_step(params, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015) at step t >= 1; returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def quadratic_loss(phi, Q, c, w):
    """sum_rows w * (phi^T Q phi - 2 c^T phi) for rows of r filter values; phi (N, r), Q (N, r, r)."""
    quad = np.einsum("ni,nij,nj->n", phi, Q, phi)
    lin = np.einsum("ni,ni->n", c, phi)
    return float(np.sum(w * (quad - 2.0 * lin)))


def quadratic_loss_grad(phi, Q, c, w):
    """d/dphi of ``quadratic_loss`` (Q symmetric): 2 w (Q phi - c)."""
    return 2.0 * w[:, None] * (np.einsum("nij,nj->ni", Q, phi) - c)
