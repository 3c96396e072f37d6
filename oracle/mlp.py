"""FP64 reference of the learned surrogate's arithmetic (test infrastructure only).

The surrogate embeds a feature vector with a three-layer perceptron
f(x) = ((gelu(gelu(x W1 + b1) W2 + b2)) W3 + b3) and predicts a kernel entry
(the kernel of §2, Eq. 3) from the embeddings, with one of two heads:

* log domain (the default):   ln K_hat(x, y) = -c (1 - exp(-s d^2)) with
  d^2 = ||x - y||^2 + ||f(x) - f(y)||^2, the squared distance between the
  embeddings [x, f(x)] (the input itself and the MLP output), trained by the
  mean squared error of ln K_hat against the exact ln K, scaled by a fixed
  constant; ln K_hat(x, x) = 0, and large distances saturate at -c, the
  level to which kernels of unrelated points concentrate at many qubits;
* sigmoid:   K_hat(x, y) = sigmoid(alpha <f(x), f(y)> + beta), trained by
  squared error or soft-target cross-entropy against K.

Weights are updated with AdamW.  This module writes those definitions out in
float64 NumPy so the GPU kernels (BF16 operands, FP32 accumulation) can be
compared with them.  GELU is the exact form x Phi(x).  Nothing here is shared
with the GPU path; only tests, the build's smoke check and the benchmark's CPU
baseline use it.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT_HALF = math.sqrt(0.5)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x * SQRT_HALF))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x * SQRT_HALF)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, X):
    """params = (W1, b1, W2, b2, W3, b3); returns dict of H1, A1, H2, A2, E."""
    W1, b1, W2, b2, W3, b3 = params
    H1 = X @ W1 + b1
    A1 = gelu(H1)
    H2 = A1 @ W2 + b2
    A2 = gelu(H2)
    E = A2 @ W3 + b3
    return {"H1": H1, "A1": A1, "H2": H2, "A2": A2, "E": E}


def softplus(z):
    return np.logaddexp(0.0, z)


def pair_loss(E, target, alpha, beta, kind="mse"):
    """Rows p and P + p of E are the two points of pair p.

    Returns (loss, dE, dalpha, dbeta) for loss = mean_p l_p with
    l_p = (K_hat_p - t_p)^2 ("mse") or the soft-target cross-entropy
    -t_p log K_hat_p - (1 - t_p) log(1 - K_hat_p) ("bce").
    """
    P = target.shape[0]
    ei, ej = E[:P], E[P:]
    dot = np.sum(ei * ej, axis=1)
    z = alpha * dot + beta
    kh = sigmoid(z)
    if kind == "bce":
        loss = float(np.mean(target * softplus(-z) + (1.0 - target) * softplus(z)))
        ds = (kh - target) / P
    else:
        err = kh - target
        loss = float(np.mean(err * err))
        ds = (2.0 * err / P) * kh * (1.0 - kh)
    dE = np.concatenate([(ds * alpha)[:, None] * ej, (ds * alpha)[:, None] * ei])
    return loss, dE, float(np.sum(ds * dot)), float(np.sum(ds))


def backward(params, X, acts, dE):
    """Gradients (dW1, db1, dW2, db2, dW3, db3) of a loss with dloss/dE = dE."""
    W1, b1, W2, b2, W3, b3 = params
    dW3 = acts["A2"].T @ dE
    db3 = dE.sum(axis=0)
    dH2 = (dE @ W3.T) * gelu_grad(acts["H2"])
    dW2 = acts["A1"].T @ dH2
    db2 = dH2.sum(axis=0)
    dH1 = (dH2 @ W2.T) * gelu_grad(acts["H1"])
    dW1 = X.T @ dH1
    db1 = dH1.sum(axis=0)
    return dW1, db1, dW2, db2, dW3, db3


def adamw_step(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One AdamW update (decoupled weight decay, bias-corrected moments)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1**step)
    vhat = v / (1.0 - beta2**step)
    w = w * (1.0 - lr * weight_decay) - lr * mhat / (np.sqrt(vhat) + eps)
    return w, m, v


def surrogate_gram(E, alpha, beta):
    """K_hat = sigmoid(alpha E E^T + beta) with the diagonal set to 1."""
    K = sigmoid(alpha * (E @ E.T) + beta)
    np.fill_diagonal(K, 1.0)
    return K


def bf16_round(a):
    """Round float64/float32 values to the nearest bfloat16 (ties to even)."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def sat_log_head(d2, log_c, log_s):
    """ln K_hat as a function of the squared embedding distance d2:
    -c (1 - exp(-s d2)) with c = exp(log_c), s = exp(log_s).  It is 0 at
    d2 = 0 (K_hat(x, x) = 1), -c s d2 for small d2, and saturates at -c."""
    c, s = math.exp(log_c), math.exp(log_s)
    return -c * (1.0 - np.exp(-s * d2))


def sat_log_pair_loss(Xr, E, target, log_c, log_s, scale):
    """Log-domain pair head on the embedding [x, f(x)].

    Rows p and P + p of Xr (the input features) and E (the MLP output) are
    the two points of pair p; d2_p = ||x_p - x_{P+p}||^2 + ||e_p - e_{P+p}||^2,
    ln K_hat_p = sat_log_head(d2_p), loss = mean_p ((ln K_hat_p - t_p) / scale)^2
    with t_p the exact ln K.  The input part carries no parameters, so only E
    receives a gradient.  Returns (loss, dE, dlog_c, dlog_s, ln_k_hat, d2).
    """
    P = target.shape[0]
    dx = Xr[:P] - Xr[P:]
    de = E[:P] - E[P:]
    d2 = np.sum(dx * dx, axis=1) + np.sum(de * de, axis=1)
    c, s = math.exp(log_c), math.exp(log_s)
    ex = np.exp(-s * d2)
    lh = -c * (1.0 - ex)
    r = (lh - target) / scale
    loss = float(np.mean(r * r))
    dl = 2.0 * r / (scale * P)             # d loss / d ln K_hat_p
    g = dl * (-c * s * ex)                 # d loss / d d2_p
    gi = (2.0 * g)[:, None] * de
    dE = np.concatenate([gi, -gi])
    dlog_c = float(np.sum(dl * lh))        # d ln K_hat / d log_c = ln K_hat
    dlog_s = float(np.sum(dl * (-c * s * d2 * ex)))
    return loss, dE, dlog_c, dlog_s, lh, d2


def sat_log_gram(Xr, E, log_c, log_s):
    """ln K_hat for all pairs of the rows of [Xr, E], with the diagonal rule
    ln K_hat[i][i] = 0.  Returns (ln_k_hat, k_hat)."""
    Z = np.concatenate([np.asarray(Xr, dtype=np.float64), np.asarray(E, dtype=np.float64)], axis=1)
    D2 = np.sum((Z[:, None, :] - Z[None, :, :]) ** 2, axis=2)
    L = sat_log_head(D2, log_c, log_s)
    np.fill_diagonal(L, 0.0)
    with np.errstate(under="ignore"):
        K = np.exp(L)
    return L, K


def tile_max_offdiag(M, tile=64):
    """Largest off-diagonal entry of every tile x tile block of the square M
    (row-major over tiles, -inf for a block with none)."""
    N = M.shape[0]
    T = -(-N // tile)
    out = np.full((T, T), -np.inf)
    off = ~np.eye(N, dtype=bool)
    for a in range(T):
        for b in range(T):
            blk = M[a * tile:(a + 1) * tile, b * tile:(b + 1) * tile]
            msk = off[a * tile:(a + 1) * tile, b * tile:(b + 1) * tile]
            if msk.any():
                out[a, b] = blk[msk].max()
    return out
