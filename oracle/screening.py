"""FP64 reference of the learned pair screen (not part of the paper's method).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The screen predicts ||t_ij||_F, the Frobenius norm of the first-order doubles of
a core pair (Eq. A7), before the pair is computed, and drops pairs whose
predicted norm is below a threshold.

Pair quantities (unordered core pairs i <= j, row-major):
  q_iQ  = ||B^Q_i.||_2 = (sum_a (B^Q_ia)^2)^(1/2)           column norms of the slab B_i
  U_ij  = sum_Q q_iQ q_jQ                                    ||V_ij||_F <= U_ij (triangle inequality
                                                             over the rank-one terms of V_ij)
  W_ij  = (sum_Q q_iQ^2 q_jQ^2)^(1/2)                        ||V_ij||_F when the rank-one terms
                                                             are mutually orthogonal
  g_ij  = max |1 - exp(-s D^2)| / |D| over D in [e_i + e_j - 2 e_vmax, e_i + e_j - 2 e_vmin]
  so that ||t_ij||_F <= g_ij ||V_ij||_F <= g_ij U_ij  (a rigorous screen).
Features (FP32 in the kernels):
  x = (e_i, e_j, log(U_ij / W_ij), 0.1 (log W_ij - (log W_ii + log W_jj)/2), 0.1 log(g_ij W_ij))
Target: y = log ||t_ij||_F - log(g_ij W_ij); the predicted norm is exp(log(g_ij W_ij) + mlp(x)).
Network: x -> tanh(W1 x + b1) (64) -> tanh(W2 h1 + b2) (64) -> w3 . h2 + b3, mean squared
error, Adam (Kingma & Ba, 2015).  Parameters are packed as
  [W1 (64x5 row-major), b1 (64), W2 (64x64), b2 (64), w3 (64), b3 (1)] = 4609 values.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

H = 64
N_IN = 5
N_PARAMS = H * N_IN + H + H * H + H + H + 1
U_STAR_EQ = "2 u^2 exp(-u^2) = 1 - exp(-u^2)"


def unpack(w: np.ndarray):
    o = 0
    W1 = w[o:o + H * N_IN].reshape(H, N_IN); o += H * N_IN
    b1 = w[o:o + H]; o += H
    W2 = w[o:o + H * H].reshape(H, H); o += H * H
    b2 = w[o:o + H]; o += H
    w3 = w[o:o + H]; o += H
    b3 = w[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]]).astype(np.float64)


def regularizer_max(s: float, d_lo: float, d_hi: float) -> float:
    """max of |1 - e^{-s D^2}| / |D| for D in [d_lo, d_hi] (both < 0 or both > 0).

    With u = sqrt(s)|D| the function is sqrt(s) (1 - e^{-u^2}) / u, increasing up to
    the root u* of 2 u^2 e^{-u^2} = 1 - e^{-u^2} and decreasing after it."""
    a, b = sorted((abs(d_lo), abs(d_hi)))
    rs = math.sqrt(s)

    def f(x):
        return -math.expm1(-s * x * x) / x if x > 0 else 0.0

    # bisection on the stationarity condition
    lo, hi = 0.5, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if 2 * mid * mid * math.exp(-mid * mid) > -math.expm1(-mid * mid):
            lo = mid
        else:
            hi = mid
    x_star = 0.5 * (lo + hi) / rs
    if a <= x_star <= b:
        return f(x_star)
    return max(f(a), f(b))


def pair_quantities(inp, s: float) -> Dict[str, np.ndarray]:
    """Features, scales and targets-to-be for the unordered core pairs of one input set."""
    nc = inp.n_core
    q = np.sqrt(np.einsum("iaQ,iaQ->iQ", inp.B[:nc], inp.B[:nc]))      # [nc, n_aux]
    U = q @ q.T
    W = np.sqrt((q * q) @ (q * q).T)
    ev = inp.eps_vir
    e = inp.eps_core
    pairs = [(i, j) for i in range(nc) for j in range(i, nc)]
    n = len(pairs)
    feats = np.zeros((n, N_IN))
    log_gw = np.zeros(n)
    log_gu = np.zeros(n)
    for p, (i, j) in enumerate(pairs):
        g = regularizer_max(s, e[i] + e[j] - 2 * ev.max(), e[i] + e[j] - 2 * ev.min())
        feats[p] = (e[i], e[j], math.log(U[i, j] / W[i, j]),
                    0.1 * (math.log(W[i, j]) - 0.5 * (math.log(W[i, i]) + math.log(W[j, j]))),
                    0.1 * math.log(g * W[i, j]))
        log_gw[p] = math.log(g * W[i, j])
        log_gu[p] = math.log(g * U[i, j])
    return dict(pairs=np.array(pairs), feats=feats, log_gw=log_gw, log_gu=log_gu, U=U, W=W)


def targets(pair_tnorm: np.ndarray, pairs: np.ndarray, log_gw: np.ndarray) -> np.ndarray:
    return np.log(pair_tnorm[pairs[:, 0], pairs[:, 1]]) - log_gw


# ----------------------------------------------------------------------------- MLP


def mlp_forward(w: np.ndarray, X: np.ndarray) -> Tuple[np.ndarray, Dict]:
    W1, b1, W2, b2, w3, b3 = unpack(w)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    out = h2 @ w3 + b3
    return out, dict(X=X, h1=h1, h2=h2)


def mlp_backward(w: np.ndarray, cache: Dict, dout: np.ndarray) -> np.ndarray:
    """Gradient of sum_n dout_n * out_n with respect to the packed parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    X, h1, h2 = cache["X"], cache["h1"], cache["h2"]
    g_w3 = h2.T @ dout
    g_b3 = dout.sum()
    dz2 = np.outer(dout, w3) * (1.0 - h2 * h2)
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    g_W1 = dz1.T @ X
    g_b1 = dz1.sum(axis=0)
    return pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def mse_and_grad(out: np.ndarray, y: np.ndarray) -> Tuple[float, np.ndarray]:
    r = out - y
    return float(np.mean(r * r)), 2.0 * r / r.shape[0]


def adam_step(w, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (bias-corrected moments), returning (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def train(w0, X, y, steps: int, lr: float = 1e-3):
    w, m, v = w0.copy(), np.zeros_like(w0), np.zeros_like(w0)
    losses = []
    for t in range(1, steps + 1):
        out, cache = mlp_forward(w, X)
        loss, dout = mse_and_grad(out, y)
        losses.append(loss)
        g = mlp_backward(w, cache, dout)
        w, m, v = adam_step(w, g, m, v, t, lr)
    return w, np.array(losses)


def screen_mask(n_h: int, pairs: np.ndarray, log_norm: np.ndarray, threshold: float) -> np.ndarray:
    """Symmetric n_h x n_h mask: 1 keeps the pair, 0 drops it (log_norm < log threshold).
    Rows and columns outside the listed pairs (active holes) are always kept."""
    mask = np.ones((n_h, n_h), dtype=np.uint8)
    drop = log_norm < math.log(threshold)
    for (i, j), d in zip(pairs, drop):
        if d:
            mask[i, j] = mask[j, i] = 0
    return mask
