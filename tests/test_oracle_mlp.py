"""Pins of the surrogate-network oracle: GELU against math.erf, bfloat16 rounding against
hand-worked ties and torch's conversion, gradients against central finite differences,
one Adam step against hand arithmetic, and the fallback's two limits."""
import math

import numpy as np
import torch

import oracle
from oracle import mlp
from paper_2508_07605_amd import synth


def test_gelu_definition():
    for z in [-6.0, -2.5, -1.0, -1e-3, 0.0, 0.3, 1.0, 2.0, 7.5]:
        ref = 0.5 * z * (1.0 + math.erf(z / math.sqrt(2.0)))
        assert abs(mlp.gelu(np.float64(z)) - ref) <= 1e-15 * max(1.0, abs(ref))
        h = 1e-6
        fd = (0.5 * (z + h) * (1 + math.erf((z + h) / math.sqrt(2))) -
              0.5 * (z - h) * (1 + math.erf((z - h) / math.sqrt(2)))) / (2 * h)
        assert abs(mlp.gelu_grad(np.float64(z)) - fd) <= 1e-8
    assert mlp.gelu(np.float64(0.0)) == 0.0


def test_bf16_rounding():
    one = 1.0
    ulp = 2.0 ** -7  # spacing of bfloat16 in [1, 2)
    x = np.array([one, one + ulp / 2, one + 1.5 * ulp, one + 0.75 * ulp, -(one + ulp / 2), 3.0e38, 1e-40],
                 dtype=np.float32)
    got = mlp.round_bf16(x)
    # ties go to the even mantissa: 1 + ulp/2 -> 1, 1 + 1.5 ulp -> 1 + 2 ulp
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2 * ulp and got[3] == 1.0 + ulp
    assert got[4] == -1.0
    r = np.random.default_rng(31)
    y = (r.normal(size=5000) * np.exp(r.uniform(-20, 20, size=5000))).astype(np.float32)
    ref = torch.from_numpy(y).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.round_bf16(y), ref)
    assert np.array_equal(mlp.round_bf16(x), torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy())


def test_gradients_match_finite_differences():
    r = np.random.default_rng(32)
    n, B, dims = 6, 5, (12, 8, 8, 3)
    params = [p.astype(np.float64) for p in synth.mlp_init(9, dims, seed=1)]
    rp = np.array([0, 2, 5, 5, 9, 12], dtype=np.int64)
    col = np.array([0, 3, 1, 2, 5, 0, 1, 4, 5, 2, 3, 4], dtype=np.int32)
    val = r.uniform(0.4, 1.0, size=12)
    X = mlp.dense_input(rp, col, val, n)
    assert X.shape == (B, 2 * n)
    target = r.normal(size=(B, 3))
    L, grads = mlp.loss_and_grads(params, X, target, bf16=False)
    h = 1e-6
    for pi, (p, g) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        gflat = g.reshape(-1)
        for t in range(flat.size):
            old = flat[t]
            flat[t] = old + h
            lp, _ = mlp.loss_and_grads(params, X, target, bf16=False)
            flat[t] = old - h
            lm, _ = mlp.loss_and_grads(params, X, target, bf16=False)
            flat[t] = old
            fd = (lp - lm) / (2 * h)
            assert abs(gflat[t] - fd) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (pi, t, gflat[t], fd)


def test_dense_input_layout():
    rp = np.array([0, 2, 3], dtype=np.int64)
    col = np.array([1, 3, 0], dtype=np.int32)
    val = np.array([0.5, 0.75, 0.25])
    X = mlp.dense_input(rp, col, val, 4)
    assert X.tolist() == [[0, 0.5, 0, 0.75, 0, 1, 0, 1], [0.25, 0, 0, 0, 1, 0, 0, 0]]


def test_adam_one_step_by_hand():
    p = [np.array([1.0, -2.0])]
    g = [np.array([0.5, -0.25])]
    m = [np.zeros(2)]
    v = [np.zeros(2)]
    newp, newm, newv = mlp.adam_step(p, g, m, v, t=1, lr=1e-3)
    # step 1: m = 0.1 g, v = 0.001 g^2, mhat = g, vhat = g^2 -> p - lr g / (|g| + eps)
    assert np.allclose(newm[0], [0.05, -0.025], rtol=0, atol=1e-16)
    assert np.allclose(newv[0], [0.00025, 0.0000625], rtol=0, atol=1e-18)
    assert abs(newp[0][0] - (1.0 - 1e-3 * 0.5 / (0.5 + 1e-8))) < 1e-16
    assert abs(newp[0][1] - (-2.0 + 1e-3 * 0.25 / (0.25 + 1e-8))) < 1e-16
    # step 2 with the same gradient: mhat = g and vhat = g^2 again (bias correction)
    p2, _, _ = mlp.adam_step(newp, g, newm, newv, t=2, lr=1e-3)
    assert abs(p2[0][0] - (newp[0][0] - 1e-3 * 0.5 / (0.5 + 1e-8))) < 1e-15


def test_fallback_limits():
    grid = synth.cap_grid(6, 5)
    rows = synth.draw_rows(7, grid, 40, ("uniform", 4, 12), seed=2)
    V = synth.setting_factors(7, grid, 8, m_ref=256)
    params = synth.mlp_init(7, (2 * grid.n, 16, 16, 8), seed=3)
    ridge, _ = oracle.ridge_rows(rows.row_ptr, rows.col, rows.val, V, 0.05, True)
    U0, fall0, rho = mlp.surrogate_foldin(params, V, rows.row_ptr, rows.col, rows.val, 0.0, 0.05)
    assert fall0.all() and np.array_equal(U0, ridge)
    Uinf, fallinf, _ = mlp.surrogate_foldin(params, V, rows.row_ptr, rows.col, rows.val, np.inf, 0.05)
    Xd = mlp.dense_input(rows.row_ptr, rows.col, rows.val, grid.n)
    net, _ = mlp.forward(params, Xd)
    assert not fallinf.any() and np.array_equal(Uinf, net)
    # the residual is the RMS over observed entries
    i = 3
    s, e = rows.row_ptr[i], rows.row_ptr[i + 1]
    resid = rows.val[s:e].astype(np.float64) - V[rows.col[s:e]].astype(np.float64) @ net[i]
    assert abs(rho[i] - np.sqrt((resid ** 2).mean())) < 1e-14


def test_forward_worked_by_hand():
    # Pre-activations at least 40 away from 0, where GELU is exactly z or exactly 0 in float64,
    # and weights exact in bfloat16, so the output follows by hand.  W2 is not symmetric: a
    # forward pass that used its transpose gives other numbers.
    W1 = np.array([[64, 0, 20, 0], [0, 50, 41, 0], [0, 0, -60, 45]], dtype=np.float32)
    b1 = np.zeros(3, np.float32)
    W2 = np.array([[1, 2, 5], [3, 4, 7], [0, -1, 2]], dtype=np.float32)
    b2 = np.zeros(3, np.float32)
    W3 = np.array([[1, -1, 2], [0.5, 0, 0.25]], dtype=np.float32)
    b3 = np.array([0.25, -1.0], dtype=np.float32)
    rp = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([0, 1], dtype=np.int32)
    val = np.array([0.5, 1.0])
    X = mlp.dense_input(rp, col, val, 2)  # rows [0.5, 0, 1, 0] and [0, 1, 0, 1]
    out, (_, z1, h1, z2, h2) = mlp.forward([W1, b1, W2, b2, W3, b3], X)
    # row 0: z1 = (52, 41, -60) -> h1 = (52, 41, 0); z2 = (134, 320, -41) -> h2 = (134, 320, 0)
    # row 1: z1 = (0, 50, 45)   -> h1 = (0, 50, 45); z2 = (325, 515, 40)  -> h2 = (325, 515, 40)
    assert h1.tolist() == [[52, 41, 0], [0, 50, 45]]
    assert h2.tolist() == [[134, 320, 0], [325, 515, 40]]
    assert out.tolist() == [[-185.75, 66.0], [-109.75, 171.5]]


def test_forward_invariant_under_relabelling_hidden_units():
    # permuting the units of a hidden layer (rows of its weights and bias, columns of the next
    # layer's weights) leaves the output unchanged; a transposed W2 or W3 in the forward pass
    # breaks this for non-symmetric weights
    r = np.random.default_rng(33)
    n, h, k = 5, 8, 3
    params = [r.normal(size=(h, 2 * n)), r.normal(size=h), r.normal(size=(h, h)), r.normal(size=h),
              r.normal(size=(k, h)), r.normal(size=k)]
    X = r.normal(size=(6, 2 * n))
    base, _ = mlp.forward(params, X)
    p1, p2 = r.permutation(h), r.permutation(h)
    W1, b1, W2, b2, W3, b3 = params
    perm = [W1[p1], b1[p1], W2[p2][:, p1], b2[p2], W3[:, p2], b3]
    out, _ = mlp.forward(perm, X)
    assert np.allclose(out, base, rtol=1e-12, atol=1e-12)
    swapped = [W1, b1, W2.T, b2, W3, b3]
    assert not np.allclose(mlp.forward(swapped, X)[0], base, rtol=1e-3)
