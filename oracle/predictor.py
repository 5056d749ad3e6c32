"""Offline performance predictor (Section III-A.2, "Performance Prediction Model"), FP64.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's checks use it to produce expected
values; nothing in the GPU path imports it.

The paper's predictor is a multi-layer perceptron that maps a profiled run's seven features
(CPU power cap, GPU power cap, memory throughput, IPS, SM clock, DRAM active rate, FP active
rate) to the run's performance normalized to the uncapped run.  The paper gives neither the
widths, the activation nor the input scaling; the readings taken here are two hidden layers
of 64 ReLU units, a linear output unit and per-feature centring and scaling:

    z = (x - mu) * rs,  h1 = max(W1 z + b1, 0),  h2 = max(W2 h1 + b2, 0),  y = w3 . h2 + b3.

W1 and W2 are used rounded to bfloat16 (nearest, ties to even), the model's stored precision;
every other quantity is float64 here.  A run with a non-finite feature has y = NaN.
"""
from __future__ import annotations

import numpy as np

from .mlp import round_bf16


def predict(X, p: dict, hidden: bool = False):
    """y (float64[runs]) for the rows of X (runs x 7).  With hidden=True also returns
    (h1, h2), the hidden activations (runs x 64 each)."""
    X = np.asarray(X, dtype=np.float64)
    mu = np.asarray(p["mu"], dtype=np.float64)
    rs = np.asarray(p["rs"], dtype=np.float64)
    W1 = round_bf16(p["W1"])
    W2 = round_bf16(p["W2"])
    b1 = np.asarray(p["b1"], dtype=np.float64)
    b2 = np.asarray(p["b2"], dtype=np.float64)
    w3 = np.asarray(p["w3"], dtype=np.float64)
    b3 = float(np.asarray(p["b3"], dtype=np.float64).reshape(-1)[0])
    Z = (X - mu) * rs
    H1 = np.maximum(Z @ W1.T + b1, 0.0)
    H2 = np.maximum(H1 @ W2.T + b2, 0.0)
    y = H2 @ w3 + b3
    y[~np.isfinite(X).all(axis=1)] = np.nan
    if hidden:
        return y, H1, H2
    return y
