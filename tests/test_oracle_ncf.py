"""Pins of the NCF fold-in oracle (Section III-B.1 model, Section III-B.2 imputation):
SELU against torch's, the chain-rule gradient against central differences, the whole
gradient-descent trajectory against its closed form where the network is affine in e, the
descent property and the row statuses."""
import numpy as np
import torch

from oracle import ncf
from paper_2508_07605_amd import synth


def rand_params(seed, d=32, h=64):
    r = np.random.default_rng(seed)
    return dict(W1=r.normal(size=(h, 2 * d)) / np.sqrt(2 * d), b1=r.normal(size=h) * 0.1,
                W2=r.normal(size=(h, h)) / np.sqrt(h), b2=r.normal(size=h) * 0.1,
                w3=r.normal(size=h) / np.sqrt(h), b3=np.array([0.7]))


def test_selu_against_torch():
    z = np.concatenate([np.linspace(-20, 5, 1001), [0.0, -0.0, 1e-30, -1e-30]])
    ref = torch.nn.functional.selu(torch.from_numpy(z)).numpy()
    assert np.allclose(ncf.selu(z), ref, rtol=1e-14, atol=1e-15)
    # derivative: central differences away from the kink
    zz = z[np.abs(z) > 1e-3]
    h = 1e-6
    fd = (ncf.selu(zz + h) - ncf.selu(zz - h)) / (2 * h)
    assert np.allclose(ncf.selu_grad(zz), fd, rtol=1e-6, atol=1e-8)


def test_gradient_against_central_differences():
    p = ncf._f64(rand_params(1))
    r = np.random.default_rng(2)
    S = r.normal(size=(17, 32))
    vals = r.uniform(0.4, 1.0, 17)
    e = r.normal(size=32) * 0.5
    g = ncf.grad(e, S, vals, p, 1e-3)
    h = 1e-6
    fd = np.array([(ncf.loss(e + h * u, S, vals, p, 1e-3) - ncf.loss(e - h * u, S, vals, p, 1e-3)) / (2 * h)
                   for u in np.eye(32)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_affine_regime_trajectory_closed_form():
    # non-negative W1[:, :d], W2 and b2 with a large b1 keep every pre-activation positive, so
    # SELU is lam * z and y(e, s_j) = g . e + c_j with g = lam^2 W1e^T W2^T w3 the same for all
    # settings.  Gradient descent from 0 then stays on the line e = alpha g with
    #   alpha_{t+1} = alpha_t - 2 eta ((|g|^2 + mu) alpha_t - mean(r - c)),
    # whose solution is alpha_T = alpha* (1 - (1 - 2 eta (|g|^2 + mu))^T),
    # alpha* = mean(r - c) / (|g|^2 + mu).
    r = np.random.default_rng(3)
    d, h = 32, 64
    p = dict(W1=np.concatenate([r.uniform(0, 0.02, (h, d)), r.normal(size=(h, d)) * 0.1], axis=1),
             b1=np.full(h, 50.0), W2=r.uniform(0, 0.05, (h, h)), b2=r.uniform(0, 1, h),
             w3=r.normal(size=h) * 0.01, b3=np.array([0.2]))
    S = r.normal(size=(9, d))
    vals = r.uniform(0.4, 1.0, 9)
    lam = ncf.SELU_LAMBDA
    W1e, W1s = p["W1"][:, :d], p["W1"][:, d:]
    g = lam * lam * W1e.T @ (p["W2"].T @ p["w3"])
    c = lam * lam * (p["w3"] @ p["W2"]) @ (S @ W1s.T + p["b1"]).T + lam * p["w3"] @ p["b2"] + p["b3"][0]
    mu, eta, T = 1e-3, 0.3, 25
    gg = g @ g + mu
    alpha_star = np.mean(vals - c) / gg
    alpha_T = alpha_star * (1 - (1 - 2 * eta * gg) ** T)
    e = ncf.foldin_row(S, vals, p, T, eta, mu)
    assert np.allclose(e, alpha_T * g, rtol=1e-10, atol=1e-14)
    y, Z1, Z2 = ncf.forward(e, S, p)
    assert (Z1 > 0).all() and (Z2 > 0).all()
    assert np.allclose(y, g @ e + c, rtol=1e-12)


def test_descent_and_statuses():
    grid = synth.grid_of("foldin")
    rows = synth.draw_rows(3, grid, 40, ("uniform", 4, 24), seed=9)
    p = synth.ncf_params(3, grid.n)
    S = p.pop("S")
    E0, L0, _ = ncf.foldin(rows.row_ptr, rows.col, rows.val, S, p, 0, 0.5, 1e-3)
    assert (E0 == 0).all()
    prev = L0
    for T in (5, 10, 30):
        _, L, st = ncf.foldin(rows.row_ptr, rows.col, rows.val, S, p, T, 0.5, 1e-3)
        assert (st == 0).all() and (L <= prev + 1e-12).all()
        prev = L
    # empty row, setting index out of range, non-finite value
    rp = np.array([0, 0, 2, 4, 6])
    col = np.array([1, 2, 3, 480, 5, 6], dtype=np.int32)
    val = np.array([0.5, 0.6, 0.7, 0.8, np.nan, 0.9], dtype=np.float32)
    E, L, st = ncf.foldin(rp, col, val, S, p, 10, 0.5, 1e-3)
    assert st.tolist() == [1, 0, 5, 3]
    assert (E[[0, 2, 3]] == 0).all() and (L[[0, 2, 3]] == 0).all() and L[1] > 0
