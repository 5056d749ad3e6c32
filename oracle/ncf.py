"""Neural collaborative filtering (Section III-B.1) and its fold-in of new applications, FP64.

TEST INFRASTRUCTURE ONLY: the tests use it to produce expected values; nothing in the GPU
path imports it.

The paper's CF model maps an application index and a power-cap-pair index to embeddings,
concatenates them and passes the joint vector through a SELU multi-layer perceptron to one
scalar, the predicted performance.  A new application, arriving as a sparse row of observed
values, needs its own embedding while everything learned offline stays fixed.  The paper
gives no widths, depth, regulariser or optimiser; the readings taken here are

    x = [e_i ; s_j] (d = 32 each),  h1 = SELU(W1 x + b1),  h2 = SELU(W2 h1 + b2),
    y_ij = w3 . h2 + b3,             hidden layers of 64 units,
    SELU(z) = lam (z if z > 0 else alpha (exp(z) - 1))   (Klambauer et al., 2017),

and the fold-in of row i takes T steps of plain gradient descent from e_i = 0 on

    L_i(e) = (1/q) sum_{j in O_i} (y(e, s_j) - r_ij)^2 + mu |e|^2,   q = |O_i|,

with step eta, the setting embeddings and the network frozen.  Rows with no observation, a
non-finite value or a setting index out of range keep e = 0 and report a status (1, 3, 5).
"""
from __future__ import annotations

import math

import numpy as np

SELU_ALPHA = 1.6732632423543772848170429916717
SELU_LAMBDA = 1.0507009873554804934193349852946


def selu(z):
    return SELU_LAMBDA * np.where(z > 0, z, SELU_ALPHA * np.expm1(np.minimum(z, 0.0)))


def selu_grad(z):
    return SELU_LAMBDA * np.where(z > 0, 1.0, SELU_ALPHA * np.exp(np.minimum(z, 0.0)))


def _f64(p):
    return {k: np.asarray(v, dtype=np.float64) for k, v in p.items()}


def forward(e, S, p):
    """Scores y (float64[q]) of embedding e against setting embeddings S (q x d), with the
    pre-activations (Z1, Z2) kept for the backward pass."""
    q, d = S.shape
    X = np.concatenate([np.broadcast_to(e, (q, d)), S], axis=1)
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = selu(Z1)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = selu(Z2)
    y = H2 @ p["w3"] + p["b3"][0]
    return y, Z1, Z2


def loss(e, S, r, p, mu):
    y, _, _ = forward(e, S, p)
    return float(np.mean((y - r) ** 2) + mu * (e @ e))


def grad(e, S, r, p, mu, flip=None):
    """dL/de by the chain rule, layer by layer backwards.  flip = (layer, obs, unit), when
    given, evaluates SELU's derivative at that one pre-activation on the other side of the
    kink (the right-hand value lam where the left-hand one applies, and the reverse); the
    tests use it to describe a trajectory whose pre-activation sits at 0 within rounding."""
    q, d = S.shape
    y, Z1, Z2 = forward(e, S, p)
    dy = 2.0 * (y - r) / q
    G1, G2 = selu_grad(Z1), selu_grad(Z2)
    if flip is not None:
        layer, o, u = flip
        Z, G = (Z1, G1) if layer == 1 else (Z2, G2)
        z = Z[o, u]
        G[o, u] = SELU_LAMBDA * SELU_ALPHA * math.exp(min(z, 0.0)) if z > 0 else SELU_LAMBDA
    dZ2 = dy[:, None] * p["w3"][None, :] * G2
    dH1 = dZ2 @ p["W2"]
    dZ1 = dH1 * G1
    dX = dZ1 @ p["W1"]
    return dX[:, :d].sum(axis=0) + 2.0 * mu * e


def foldin_row(S_obs, r, p, steps, eta, mu, flip=None):
    """T steps of gradient descent from e = 0.  flip = (step, layer, obs, unit) takes SELU's
    derivative on the other side of the kink at that one evaluation (see grad)."""
    e = np.zeros(S_obs.shape[1])
    for t in range(steps):
        f = flip[1:] if flip is not None and flip[0] == t else None
        e = e - eta * grad(e, S_obs, r, p, mu, f)
    return e


def kink_events(S_obs, r, p, steps, eta, mu, eps):
    """Pre-activations within eps of SELU's kink along the trajectory of foldin_row: a list
    of (|z|, step, layer, obs, unit), nearest first.  Where |z| is below the rounding error
    of a lower-precision evaluation, that evaluation may take SELU's derivative from the other
    side; each event is one such decision."""
    p = _f64(p)
    e = np.zeros(S_obs.shape[1])
    out = []
    for t in range(steps):
        _, Z1, Z2 = forward(e, S_obs, p)
        for layer, Z in ((1, Z1), (2, Z2)):
            for o, u in zip(*np.nonzero(np.abs(Z) < eps)):
                out.append((abs(float(Z[o, u])), t, layer, int(o), int(u)))
        e = e - eta * grad(e, S_obs, r, p, mu)
    return sorted(out)


def foldin(row_ptr, col, val, S, p, steps, eta, mu, rows=None):
    """Embeddings (float64[len(rows), d]), final losses L_i(e_T) and statuses of the listed
    CSR rows (all rows by default)."""
    p = _f64(p)
    S = np.asarray(S, dtype=np.float64)
    n, d = S.shape
    rows = np.arange(len(row_ptr) - 1) if rows is None else np.asarray(rows)
    E = np.zeros((len(rows), d))
    L = np.zeros(len(rows))
    st = np.zeros(len(rows), dtype=np.int32)
    for t, i in enumerate(rows):
        a, b = int(row_ptr[i]), int(row_ptr[i + 1])
        c = np.asarray(col[a:b], dtype=np.int64)
        r = np.asarray(val[a:b], dtype=np.float64)
        if b == a:
            st[t] = 1
            continue
        if ((c < 0) | (c >= n)).any():
            st[t] = 5
            continue
        if not np.isfinite(r).all():
            st[t] = 3
            continue
        E[t] = foldin_row(S[c], r, p, steps, eta, mu)
        L[t] = loss(E[t], S[c], r, p, mu)
    return E, L, st


def loss_rows(row_ptr, col, val, S, p, mu, E, rows=None):
    """L_i(E[t]) for the listed CSR rows (all rows by default), E[t] the embedding of rows[t];
    0 for the rows the fold-in rejects (no entry, index out of range, non-finite value)."""
    p = _f64(p)
    S = np.asarray(S, dtype=np.float64)
    rows = np.arange(len(row_ptr) - 1) if rows is None else np.asarray(rows)
    out = np.zeros(len(rows))
    for t, i in enumerate(rows):
        a, b = int(row_ptr[i]), int(row_ptr[i + 1])
        c = np.asarray(col[a:b], dtype=np.int64)
        if b > a and ((c >= 0) & (c < len(S))).all() and np.isfinite(val[a:b]).all():
            out[t] = loss(np.asarray(E[t], dtype=np.float64), S[c], np.asarray(val[a:b], dtype=np.float64), p, mu)
    return out


def train_loss_and_grads(E, S, p, apps, R):
    """Offline training of the model on the dense offline matrix R (applications x settings,
    every entry observed): the objective on a batch of whole applications (rows `apps` of R,
    every setting of each),

        L = (1/B) sum_{g, j} (y(E[apps[g]], S[j]) - R[apps[g], j])^2,   B = len(apps) * n,

    and its gradient with respect to the application embeddings E, the setting embeddings S
    and every network parameter, by the chain rule layer by layer backwards.  Returns
    (L, {"E", "S", "W1", "b1", "W2", "b2", "w3", "b3"})."""
    p = _f64(p)
    E = np.asarray(E, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    apps = np.asarray(apps, dtype=np.int64)
    n, d = S.shape
    G = len(apps)
    ai = np.repeat(apps, n)                 # application of each batch entry
    sj = np.tile(np.arange(n), G)           # setting of each batch entry
    r = np.asarray(R, dtype=np.float64)[ai, sj]
    X = np.concatenate([E[ai], S[sj]], axis=1)
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = selu(Z1)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = selu(Z2)
    y = H2 @ p["w3"] + p["b3"][0]
    B = len(r)
    L = float(np.mean((y - r) ** 2))
    dy = 2.0 * (y - r) / B
    g = {"w3": H2.T @ dy, "b3": np.array([dy.sum()])}
    dZ2 = dy[:, None] * p["w3"][None, :] * selu_grad(Z2)
    g["W2"], g["b2"] = dZ2.T @ H1, dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * selu_grad(Z1)
    g["W1"], g["b1"] = dZ1.T @ X, dZ1.sum(axis=0)
    dX = dZ1 @ p["W1"]
    g["E"] = np.zeros_like(E)
    np.add.at(g["E"], ai, dX[:, :d])
    g["S"] = np.zeros_like(S)
    np.add.at(g["S"], sj, dX[:, d:])
    return L, g


def ncf_params(S_shape_d=32, hidden=64):
    """Shapes of the network arrays (for documentation and tests)."""
    d = S_shape_d
    return {"W1": (hidden, 2 * d), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,), "w3": (hidden,),
            "b3": (1,)}


assert math.isclose(SELU_LAMBDA * SELU_ALPHA, 1.7580993408473766, rel_tol=1e-15)
