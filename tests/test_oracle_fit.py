"""Pins of the oracle's ALS-WR fit and objective: the fully observed case has a closed
form (soft-thresholded truncated SVD), noiseless low-rank matrices are recovered exactly,
every half-sweep lowers the objective, and each half-sweep leaves its factor at a
stationary point of its normal equations."""
import numpy as np
import pytest

import oracle
from paper_2508_07605_amd import synth


def _dense_csr(R):
    m, n = R.shape
    rp = np.arange(0, m * n + 1, n, dtype=np.int64)
    col = np.tile(np.arange(n, dtype=np.int32), m)
    return rp, col, R.reshape(-1).copy()


def _matrix_with_spectrum(r, m, n, sig):
    Q1, _ = np.linalg.qr(r.normal(size=(m, m)))
    Q2, _ = np.linalg.qr(r.normal(size=(n, n)))
    S = np.zeros((m, n))
    S[np.arange(len(sig)), np.arange(len(sig))] = sig
    return Q1 @ S @ Q2.T


@pytest.mark.parametrize("weighted", [True, False])
def test_full_observation_soft_threshold_svd(weighted):
    # weighted: min |R-X|^2 + 2 lambda sqrt(mn) |X|_*  -> threshold tau = lambda sqrt(mn)
    # unweighted: threshold tau = lambda
    r = np.random.default_rng(11)
    m, n, k = 12, 10, 3
    sig = np.array([10.0, 7.0, 4.0, 1.0, 0.6, 0.3, 0.2, 0.1, 0.05, 0.01])
    R = _matrix_with_spectrum(r, m, n, sig)
    lam = 0.5 / np.sqrt(m * n) if weighted else 0.5
    tau = lam * np.sqrt(m * n) if weighted else lam
    rp, col, val = _dense_csr(R)
    U0 = r.normal(scale=0.1, size=(m, k))
    V0 = r.normal(scale=0.1, size=(n, k))
    U, V, obj = oracle.fit(rp, col, val, U0, V0, lam, 300, weighted)
    u, s, vt = np.linalg.svd(R)
    X = (u[:, :k] * (s[:k] - tau)) @ vt[:k]
    assert np.linalg.norm(U @ V.T - X) <= 1e-10 * np.linalg.norm(X)
    # objective value at the optimum: sum_{i>k} s_i^2 + sum_{i<=k} tau (2 s_i - tau)
    fstar = (s[k:] ** 2).sum() + (tau * (2 * s[:k] - tau)).sum()
    assert abs(obj[-1] - fstar) <= 1e-10 * fstar
    assert abs(oracle.objective(rp, col, val, U, V, lam, weighted) - obj[-1]) <= 1e-12 * fstar


def test_exact_recovery_partial_observation():
    r = np.random.default_rng(12)
    m, n, k = 40, 32, 2
    R = r.normal(size=(m, k)) @ r.normal(size=(k, n))
    mask = r.random((m, n)) < 0.7
    rows, cols = np.nonzero(mask)
    rp = np.zeros(m + 1, dtype=np.int64)
    rp[1:] = np.cumsum(mask.sum(1))
    val = R[rows, cols]
    U0 = r.normal(scale=0.1, size=(m, k))
    V0 = r.normal(scale=0.1, size=(n, k))
    U, V, _ = oracle.fit(rp, cols.astype(np.int32), val, U0, V0, 1e-10, 400, True)
    rmse = np.sqrt(((U @ V.T - R) ** 2).mean())
    assert rmse <= 1e-8


@pytest.mark.parametrize("weighted", [True, False])
def test_objective_monotone_and_stationary(weighted):
    grid, _, _, union = synth.tiny_problem(seed=3)
    c = synth.CONFIGS["tiny"]
    U0, V0 = synth.init_factors(c["cfg_id"], union.m, grid.n, c["k"])
    lam = c["lam"]
    U, V, obj = oracle.fit(union.row_ptr, union.col, union.val, U0, V0, lam, c["sweeps"], weighted)
    f0 = oracle.objective(union.row_ptr, union.col, union.val, U0, V0, lam, weighted)
    seq = np.concatenate([[f0], obj])
    assert (seq[1:] <= seq[:-1] * (1 + 1e-12)).all()
    # after the last (column) half-sweep each column solves its normal equations
    rp, ridx, cval = oracle.csr_to_csc(union.row_ptr, union.col, union.val, grid.n)
    for j in range(grid.n):
        s, e = rp[j], rp[j + 1]
        Uo = U[ridx[s:e]]
        w = (e - s) if weighted else 1.0
        lhs = (Uo.T @ Uo + lam * w * np.eye(c["k"])) @ V[j]
        rhs = Uo.T @ cval[s:e]
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * max(1.0, np.linalg.norm(rhs))
    # one more row half-sweep: each row then solves its own normal equations
    U1, _ = oracle.ridge_rows(union.row_ptr, union.col, union.val, V, lam, weighted)
    for i in range(union.m):
        s, e = union.row_ptr[i], union.row_ptr[i + 1]
        Vo = V[union.col[s:e]]
        w = (e - s) if weighted else 1.0
        lhs = (Vo.T @ Vo + lam * w * np.eye(c["k"])) @ U1[i]
        rhs = Vo.T @ union.val[s:e].astype(np.float64)
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * max(1.0, np.linalg.norm(rhs))


def test_csc_transpose_matches_dense():
    r = np.random.default_rng(13)
    m, n = 30, 20
    mask = r.random((m, n)) < 0.3
    R = np.where(mask, r.random((m, n)), 0.0)
    rows, cols = np.nonzero(mask)
    rp = np.zeros(m + 1, dtype=np.int64)
    rp[1:] = np.cumsum(mask.sum(1))
    cp, ridx, cval = oracle.csr_to_csc(rp, cols.astype(np.int32), R[rows, cols], n)
    for j in range(n):
        assert ridx[cp[j]:cp[j + 1]].tolist() == np.nonzero(mask[:, j])[0].tolist()
        assert np.array_equal(cval[cp[j]:cp[j + 1]], R[mask[:, j], j])


def test_tiny_config_fit_and_foldin_accuracy():
    # the tiny configuration end to end: union fit, and dense fit followed by fold-in;
    # both predict the unobserved entries of the 16 online apps against the noiseless truth
    grid, dense, new, union = synth.tiny_problem(seed=0)
    c = synth.CONFIGS["tiny"]
    U0, V0 = synth.init_factors(c["cfg_id"], union.m, grid.n, c["k"])
    U, V, obj = oracle.fit(union.row_ptr, union.col, union.val, U0, V0, c["lam"], c["sweeps"], True)
    T = synth.truth_dense(new.apps, grid)
    obs = np.zeros_like(T, dtype=bool)
    obs[np.repeat(np.arange(new.m), new.counts()), new.col] = True
    pred_union = (U[c["m_dense"]:] @ V.T)[~obs]
    Ud, Vd, _ = oracle.fit(dense.row_ptr, dense.col, dense.val, U0[:c["m_dense"]], V0, c["lam"], c["sweeps"], True)
    Un, st = oracle.ridge_rows(new.row_ptr, new.col, new.val, Vd, c["lam"], True)
    assert (st == 0).all()
    pred_fold = (Un @ Vd.T)[~obs]
    # a weaker predictor: each online app's mean observed value everywhere
    mean = np.array([new.val[new.row_ptr[i]:new.row_ptr[i + 1]].mean() for i in range(new.m)])
    rmse_mean = np.sqrt(((mean[:, None] - T)[~obs] ** 2).mean())
    for pred in (pred_union, pred_fold):
        rmse = np.sqrt(((pred - T[~obs]) ** 2).mean())
        assert rmse < 0.1 and rmse < 0.8 * rmse_mean, (rmse, rmse_mean)
