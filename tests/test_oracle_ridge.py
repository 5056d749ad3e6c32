"""Pins of the oracle's ridge row solve (fold-in; each ALS half-sweep) against facts that
do not depend on the oracle: a scalar closed form, LAPACK least squares on the augmented
system, exact recovery of noiseless rows, and the push-through (dual) identity."""
import numpy as np
import pytest

import oracle


def _random_csr(r, m, n, lo, hi):
    counts = r.integers(lo, hi + 1, size=m)
    rp = np.zeros(m + 1, dtype=np.int64)
    rp[1:] = np.cumsum(counts)
    col = np.concatenate([np.sort(r.choice(n, size=c, replace=False)) for c in counts]).astype(np.int32)
    val = r.uniform(0.4, 1.0, size=int(rp[-1]))
    return rp, col, val


def test_scalar_closed_form():
    # k = 1: u = sum r_j v_j / (sum v_j^2 + lambda w)
    r = np.random.default_rng(1)
    rp, col, val = _random_csr(r, 50, 30, 1, 12)
    V = r.normal(size=(30, 1))
    for weighted in (True, False):
        X, st = oracle.ridge_rows(rp, col, val, V, 0.3, weighted)
        assert (st == 0).all()
        for i in range(50):
            s, e = rp[i], rp[i + 1]
            v = V[col[s:e], 0]
            w = (e - s) if weighted else 1.0
            expect = (val[s:e] * v).sum() / ((v * v).sum() + 0.3 * w)
            assert abs(X[i, 0] - expect) <= 1e-13 * abs(expect)


@pytest.mark.parametrize("k", [8, 32])
@pytest.mark.parametrize("weighted", [True, False])
def test_matches_augmented_least_squares(k, weighted):
    # argmin |V_O u - r|^2 + lambda w |u|^2  ==  lstsq([V_O; sqrt(lambda w) I], [r; 0])
    r = np.random.default_rng(2 + k)
    n = 60
    rp, col, val = _random_csr(r, 40, n, 1, 50)
    V = r.normal(size=(n, k))
    lam = 0.05
    X, st = oracle.ridge_rows(rp, col, val, V, lam, weighted)
    assert (st == 0).all()
    for i in range(40):
        s, e = rp[i], rp[i + 1]
        w = (e - s) if weighted else 1.0
        A = np.vstack([V[col[s:e]], np.sqrt(lam * w) * np.eye(k)])
        b = np.concatenate([val[s:e], np.zeros(k)])
        ref = np.linalg.lstsq(A, b, rcond=None)[0]
        assert np.linalg.norm(X[i] - ref) <= 1e-11 * np.linalg.norm(ref)


def test_exact_recovery_noiseless():
    # r = V_O u* with |O| >= k and a negligible ridge term returns u*
    r = np.random.default_rng(3)
    k, n = 8, 40
    V = r.normal(size=(n, k))
    rp, col, _ = _random_csr(r, 30, n, k + 2, n)
    ustar = r.normal(size=(30, k))
    rows = np.repeat(np.arange(30), np.diff(rp))
    val = np.einsum("tk,tk->t", ustar[rows], V[col])
    X, st = oracle.ridge_rows(rp, col, val, V, 1e-14, True)
    assert (st == 0).all()
    assert np.abs(X - ustar).max() <= 1e-9


def test_dual_form_identity():
    # V_O^T (V_O V_O^T + lambda w I)^-1 r equals the primal solution (push-through identity)
    r = np.random.default_rng(4)
    k, n = 32, 480
    V = r.normal(scale=0.3, size=(n, k))
    rp, col, val = _random_csr(r, 30, n, 4, 24)
    X, _ = oracle.ridge_rows(rp, col, val, V, 0.05, True)
    for i in range(30):
        s, e = rp[i], rp[i + 1]
        Vo = V[col[s:e]]
        alpha = np.linalg.solve(Vo @ Vo.T + 0.05 * (e - s) * np.eye(e - s), val[s:e])
        ref = Vo.T @ alpha
        assert np.linalg.norm(X[i] - ref) <= 1e-11 * np.linalg.norm(ref)


def test_status_codes_and_empty_rows():
    V = np.ones((5, 2))
    V[:, 1] = 0.0  # second latent column never observed: singular without ridge
    rp = np.array([0, 0, 2, 4, 6], dtype=np.int64)
    col = np.array([0, 1, 1, 2, 3, 4], dtype=np.int32)
    val = np.array([0.5, 0.6, 0.7, np.nan, 0.9, 1.0])
    X, st = oracle.ridge_rows(rp, col, val, V, 0.0, True)
    assert st.tolist() == [1, 2, 3, 2]
    assert (X == 0).all()
    X, st = oracle.ridge_rows(rp, col, val, V, 0.1, True)
    assert st.tolist() == [1, 0, 3, 0]
    assert (X[[0, 2]] == 0).all() and (X[[1, 3], 1] == 0).all()


def test_row_permutation_equivariance():
    r = np.random.default_rng(5)
    n, k = 50, 8
    rp, col, val = _random_csr(r, 25, n, 1, 30)
    V = r.normal(size=(n, k))
    X, _ = oracle.ridge_rows(rp, col, val, V, 0.05, True)
    perm = r.permutation(25)
    cnt = np.diff(rp)[perm]
    rp2 = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    col2 = np.concatenate([col[rp[i]:rp[i + 1]] for i in perm]).astype(np.int32)
    val2 = np.concatenate([val[rp[i]:rp[i + 1]] for i in perm])
    X2, _ = oracle.ridge_rows(rp2, col2, val2, V, 0.05, True)
    assert np.array_equal(X2, X[perm])
    Xs, _ = oracle.ridge_subset(perm[:7], rp, col, val, V, 0.05, True)
    assert np.array_equal(Xs, X[perm[:7]])
