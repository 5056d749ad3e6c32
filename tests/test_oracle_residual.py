"""Pins of the oracle's observed-entry residual, rho_i = sqrt(mean_{j in O_i}(r_ij - u_i.v_j)^2)
(the fallback test of the fold-in surrogate): rows worked by hand, including an empty row,
and agreement with the surrogate oracle's independent numpy evaluation on random input."""
import math

import numpy as np

import oracle
from oracle import mlp


def test_hand_worked_rows():
    V = np.array([[1.0, 0.0], [0.0, 2.0], [1.0, 1.0]])
    U = np.array([[1.0, 0.5], [7.0, 7.0], [2.0, -1.0], [0.0, 0.0]])
    rp = np.array([0, 2, 2, 3, 6], dtype=np.int64)
    col = np.array([0, 2, 1, 0, 1, 2], dtype=np.int32)
    val = np.array([1.5, 2.0, 0.0, 3.0, 4.0, 0.0])
    rho = oracle.residual(rp, col, val, U, V)
    # row 0: predictions 1 and 1.5, residuals 0.5 and 0.5 -> 0.5
    # row 1: no observed entry -> 0
    # row 2: prediction 2 * (-1) = -2 against 0 -> 2
    # row 3: zero factors, residuals 3, 4, 0 -> sqrt(25 / 3)
    assert rho[0] == 0.5 and rho[1] == 0.0 and rho[2] == 2.0
    assert abs(rho[3] - math.sqrt(25.0 / 3.0)) < 1e-15


def test_agrees_with_numpy_evaluation():
    r = np.random.default_rng(11)
    m, n, k = 300, 50, 8
    cnt = r.integers(0, 12, size=m)
    cnt[::17] = 0
    rp = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    col = np.concatenate([np.sort(r.choice(n, size=c, replace=False)) for c in cnt]).astype(np.int32)
    val = r.uniform(0.4, 1.0, size=rp[-1])
    U, V = r.normal(size=(m, k)), r.normal(size=(n, k))
    a = oracle.residual(rp, col, val, U, V)
    b = mlp.residual_rms(rp, col, val, U, V)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-15)
    assert (a[cnt == 0] == 0).all()
