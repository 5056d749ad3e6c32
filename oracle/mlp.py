"""FP64 oracle of the fold-in surrogate network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The surrogate maps a new application's masked profile vector straight to its latent row.
The input of a row with observed set O and values r is x = [r * mask ; mask] (length 2n),
followed by two GELU layers and a linear output layer:

    h1 = GELU(W1 x + b1),  h2 = GELU(W2 h1 + b2),  u_hat = W3 h2 + b3,
    GELU(z) = z/2 (1 + erf(z / sqrt 2)).

Training minimises L = 1/(B k) sum_i |u_hat_i - u_i|^2 against ALS fold-in targets with
Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).  A row whose observed-entry RMS
residual |r - u_hat . v_j| exceeds tau falls back to the ridge fold-in.

Weights are held in float32 and rounded to bfloat16 (round to nearest, ties to even) for
the forward and backward products; this module evaluates in float64 on those rounded
weights.  Dense matrices and numpy matmuls are used throughout: plain and slow.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from . import ridge_rows

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def round_bf16(a) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float64.  NaN stays NaN."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    bits = a32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a32), np.nan, out)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def dense_input(row_ptr, col, val, n) -> np.ndarray:
    """x = [r * mask ; mask] for every CSR row, float64[m, 2n]."""
    m = len(row_ptr) - 1
    X = np.zeros((m, 2 * n))
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    X[rows, col] = np.asarray(val, dtype=np.float64)
    X[rows, n + np.asarray(col)] = 1.0
    return X


def weights_bf16(params, bf16=True):
    """[W1, b1, W2, b2, W3, b3] with the three weight matrices rounded to bfloat16;
    biases stay at their float32 values.  bf16=False keeps every weight as given."""
    W1, b1, W2, b2, W3, b3 = params
    if not bf16:
        return [np.asarray(p, np.float64) for p in params]
    return [round_bf16(W1), np.asarray(b1, np.float64), round_bf16(W2), np.asarray(b2, np.float64),
            round_bf16(W3), np.asarray(b3, np.float64)]


def forward(params, X, bf16=True):
    """Returns (u_hat, cache) for a float64 batch X[B, 2n]."""
    W1, b1, W2, b2, W3, b3 = weights_bf16(params, bf16)
    z1 = X @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    out = h2 @ W3.T + b3
    return out, (X, z1, h1, z2, h2)


def loss_and_grads(params, X, target, bf16=True):
    """Mean-squared loss against target[B, k] and its gradients with respect to
    [W1, b1, W2, b2, W3, b3] (gradients flow through the bfloat16-rounded weights)."""
    W1, b1, W2, b2, W3, b3 = weights_bf16(params, bf16)
    out, (X, z1, h1, z2, h2) = forward(params, X, bf16)
    B, k = out.shape
    diff = out - np.asarray(target, np.float64)
    L = float((diff * diff).sum() / (B * k))
    d_out = 2.0 * diff / (B * k)
    gW3 = d_out.T @ h2
    gb3 = d_out.sum(0)
    d_z2 = (d_out @ W3) * gelu_grad(z2)
    gW2 = d_z2.T @ h1
    gb2 = d_z2.sum(0)
    d_z1 = (d_z2 @ W2) * gelu_grad(z1)
    gW1 = d_z1.T @ X
    gb1 = d_z1.sum(0)
    return L, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Kingma and Ba 2015) at step number t >= 1.
    Returns new (params, m, v) as float64 lists."""
    new_p, new_m, new_v = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        mi = beta1 * mi + (1.0 - beta1) * g
        vi = beta2 * vi + (1.0 - beta2) * g * g
        mhat = mi / (1.0 - beta1 ** t)
        vhat = vi / (1.0 - beta2 ** t)
        new_p.append(np.asarray(p, np.float64) - lr * mhat / (np.sqrt(vhat) + eps))
        new_m.append(mi)
        new_v.append(vi)
    return new_p, new_m, new_v


def residual_rms(row_ptr, col, val, Uhat, V) -> np.ndarray:
    """sqrt(mean over observed j of (r_ij - u_hat_i . v_j)^2) per row (0 for an empty row)."""
    m = len(row_ptr) - 1
    cnt = np.diff(row_ptr)
    rows = np.repeat(np.arange(m), cnt)
    pred = np.einsum("tk,tk->t", np.asarray(Uhat, np.float64)[rows], np.asarray(V, np.float64)[col])
    sq = (np.asarray(val, np.float64) - pred) ** 2
    acc = np.bincount(rows, weights=sq, minlength=m)
    return np.sqrt(np.divide(acc, cnt, out=np.zeros(m), where=cnt > 0))


def surrogate_foldin(params, V, row_ptr, col, val, tau, lam, weighted=True):
    """Network prediction with ridge fallback on rows whose residual exceeds tau.
    Returns (U f64[m,k], used_fallback bool[m], residual f64[m])."""
    n = V.shape[0]
    X = dense_input(row_ptr, col, val, n)
    Uhat, _ = forward(params, X)
    rho = residual_rms(row_ptr, col, val, Uhat, V)
    fall = ~(rho <= tau)
    if fall.any():
        Xr, _ = ridge_rows(row_ptr, col, val, V, lam, weighted)
        Uhat = np.where(fall[:, None], Xr, Uhat)
    return Uhat, fall, rho
