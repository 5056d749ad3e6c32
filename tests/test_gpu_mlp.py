"""GPU parity of the fold-in surrogate network through the C ABI: forward output and every
gradient tensor against the FP64 oracle evaluated on the same bfloat16-rounded weights
(relative Frobenius error <= 1e-2 per tensor, stated), Adam, training progress, and the
ridge fallback at its two limits and in between."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp
from paper_2508_07605_amd import native, synth

pytestmark = pytest.mark.gpu
N, K, H = 480, 32, 256
NAMES = ["W1", "b1", "W2", "b2", "W3", "b3"]


@pytest.fixture(scope="module")
def ctx():
    c = native.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pack(params):
    return np.concatenate([np.asarray(p, np.float32).reshape(-1) for p in params])


def unpack(flat, n=N, k=K, h=H):
    shapes = [(h, 2 * n), (h,), (h, h), (h,), (k, h), (k,)]
    out, o = [], 0
    for s in shapes:
        c = int(np.prod(s))
        out.append(flat[o:o + c].reshape(s))
        o += c
    return out


def fro(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def data():
    grid = synth.grid_of("foldin")
    rows = synth.draw_rows(3, grid, 4099, ("uniform", 4, 24), seed=21)
    V = synth.setting_factors(3, grid, K, m_ref=1024)
    target, _ = oracle.ridge_rows(rows.row_ptr, rows.col, rows.val, V, 0.05, True)
    params = synth.mlp_init(3, (2 * N, H, H, K), seed=1)
    return grid, rows, V, target.astype(np.float32), params


def test_forward_and_gradients(ctx, data):
    grid, rows, V, target, params = data
    net = native.Surrogate(ctx, N, K, H, init=pack(params))
    B = 1024
    rp = rows.row_ptr[:B + 1]
    col, val = rows.col[:rp[-1]], rows.val[:rp[-1]]
    out = net.forward(dev(rp), dev(col), dev(val)).cpu().numpy()
    X = omlp.dense_input(rp, col, val, N)
    ref, _ = omlp.forward(params, X)
    ef = fro(out, ref)
    loss, g = net.loss_grad(dev(rp), dev(col), dev(val), dev(target[:B]))
    Lr, gr = omlp.loss_and_grads(params, X, target[:B].astype(np.float64))
    errs = {nm: fro(a, b) for nm, a, b in zip(NAMES, unpack(g), gr)}
    print("forward rel %.2e  loss %.6g vs %.6g  grads %s" % (ef, loss, Lr, {k: "%.2e" % v for k, v in errs.items()}))
    assert ef <= 1e-2
    assert abs(loss - Lr) <= 1e-2 * Lr
    assert max(errs.values()) <= 1e-2
    net.close()


def test_adam_step(ctx, data):
    grid, rows, V, target, params = data
    net = native.Surrogate(ctx, N, K, H, init=pack(params))
    B = 512
    rp = rows.row_ptr[:B + 1]
    col, val = rows.col[:rp[-1]], rows.val[:rp[-1]]
    w0 = net.get_weights()
    net.train_step(dev(rp), dev(col), dev(val), dev(target[:B]), None, 1e-3)
    w1 = net.get_weights()
    X = omlp.dense_input(rp, col, val, N)
    _, gr = omlp.loss_and_grads(params, X, target[:B].astype(np.float64))
    pr, _, _ = omlp.adam_step(params, gr, [0 * p for p in gr], [0 * p for p in gr], 1, lr=1e-3)
    d_gpu = w1.astype(np.float64) - w0
    d_ref = pack(pr).astype(np.float64) - pack(params)
    # first Adam step moves every weight by ~lr * sign(g); compare where the gradient is not tiny
    gflat = np.concatenate([g.reshape(-1) for g in gr])
    big = np.abs(gflat) > 1e-3 * np.abs(gflat).max()
    cos = d_gpu @ d_ref / (np.linalg.norm(d_gpu) * np.linalg.norm(d_ref))
    print("adam: update cosine %.5f, max |diff| on clear gradients %.2e" % (cos, np.abs(d_gpu - d_ref)[big].max()))
    assert cos > 0.99
    assert np.abs(d_gpu - d_ref)[big].max() <= 2e-5
    net.close()


def test_training_reduces_loss(ctx, data):
    grid, rows, V, target, params = data
    net = native.Surrogate(ctx, N, K, H, init=pack(params))
    drp, dcol, dval, dt = dev(rows.row_ptr), dev(rows.col), dev(rows.val), dev(target)
    gen = torch.Generator(device="cpu").manual_seed(0)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for s in range(300):
        idx = torch.randperm(rows.m, generator=gen)[:512].to(torch.int64).cuda()
        net.train_step(drp, dcol, dval, dt, idx, 1e-3, loss_out=loss)
        if s % 50 == 0 or s == 299:
            hist.append(float(loss.item()))
    print("training loss", hist)
    assert hist[-1] < 0.5 * hist[0]
    net.close()


def test_fallback_limits_and_middle(ctx, data):
    grid, rows, V, target, params = data
    net = native.Surrogate(ctx, N, K, H, init=pack(params))
    drp, dcol, dval, dV = dev(rows.row_ptr), dev(rows.col), dev(rows.val), dev(V)
    als = native.open_foldin(ctx, dV, drp, dcol, dval, 0.05).cpu().numpy()
    fwd = net.forward(drp, dcol, dval).cpu().numpy()
    U0, nf0 = net.foldin(dV, drp, dcol, dval, 0.0, 0.05)
    assert nf0 == rows.m and np.array_equal(U0.cpu().numpy(), als)
    Uinf, nfi = net.foldin(dV, drp, dcol, dval, float("inf"), 0.05)
    assert nfi == 0 and np.array_equal(Uinf.cpu().numpy(), fwd)
    # tau in the middle of the residual distribution: each row takes the branch its residual says
    rho = torch.empty(rows.m, dtype=torch.float32, device="cuda")
    used = torch.empty(rows.m, dtype=torch.uint8, device="cuda")
    _, _ = net.foldin(dV, drp, dcol, dval, float("inf"), 0.05, rho=rho)
    tau = float(np.median(rho.cpu().numpy()))
    Um, nfm = net.foldin(dV, drp, dcol, dval, tau, 0.05, used_fallback=used, rho=rho)
    Um, used, rho = Um.cpu().numpy(), used.cpu().numpy().astype(bool), rho.cpu().numpy()
    assert np.array_equal(used, ~(rho <= tau)) and nfm == used.sum()
    assert np.array_equal(Um[used], als[used]) and np.array_equal(Um[~used], fwd[~used])
    net.close()
