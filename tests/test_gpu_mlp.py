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
    # the kernel's residual is the observed-entry RMS residual of its own output (the network's
    # rows), against the oracle's evaluation of that definition on the same factors
    ref_rho = oracle.residual(rows.row_ptr, rows.col, rows.val, fwd.astype(np.float64), V.astype(np.float64))
    e = np.abs(rho - ref_rho) / np.maximum(ref_rho, 1e-30)
    print("surrogate residual vs oracle: max rel err %.2e" % e.max())
    assert e.max() <= 1e-5
    net.close()


def mix64(z):
    # SplitMix64 output function on uint64 arrays (wrapping arithmetic)
    with np.errstate(over="ignore"):
        z = np.asarray(z, dtype=np.uint64) + np.uint64(0x9e3779b97f4a7c15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xbf58476d1ce4e5b9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94d049bb133111eb)
        return z ^ (z >> np.uint64(31))


def feistel_order(m, seed, epoch):
    # the training order the header defines: four Feistel rounds on 2h-bit integers (4^h >= m),
    # walked along the cycle until the value is below m
    h = 1
    while (1 << (2 * h)) < m:
        h += 1
    with np.errstate(over="ignore"):
        base = mix64(np.uint64(seed)) + np.uint64(4 * epoch)
    keys = [mix64(base + np.uint64(r)) for r in range(4)]
    mask = np.uint64((1 << h) - 1)
    x = np.arange(m, dtype=np.uint64)
    out = np.empty(m, dtype=np.uint64)
    todo = np.arange(m)
    while todo.size:
        L, R = x[todo] >> np.uint64(h), x[todo] & mask
        for kr in keys:
            L, R = R, L ^ (mix64(R ^ kr) & mask)
        y = (L << np.uint64(h)) | R
        x[todo] = y
        done = y < np.uint64(m)
        out[todo[done]] = y[done]
        todo = todo[~done]
    return out.astype(np.int64)


def test_feistel_order_is_a_permutation():
    for m in (1, 2, 3, 5, 1000, 4099, 65537):
        p = feistel_order(m, 7, 3)
        assert np.array_equal(np.sort(p), np.arange(m))
    assert not np.array_equal(feistel_order(4099, 7, 0), feistel_order(4099, 7, 1))


def test_train_equals_its_steps(ctx, data):
    # open_mlp_train (device shuffle, eager first step, graph replays) against the same Adam
    # steps taken one by one through open_mlp_train_step on the order computed here
    grid, rows, V, target, params = data
    drp, dcol, dval, dt = dev(rows.row_ptr), dev(rows.col), dev(rows.val), dev(target)
    B, E, seed = 1000, 3, 11
    a = native.Surrogate(ctx, N, K, H, init=pack(params))
    hist = a.train(drp, dcol, dval, dt, B, 1e-3, E, seed=seed)
    b = native.Surrogate(ctx, N, K, H, init=pack(params))
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    per_epoch = []
    for e in range(E):
        order = feistel_order(rows.m, seed, e)
        ls = []
        for s in range(rows.m // B):
            b.train_step(drp, dcol, dval, dt, dev(order[s * B:(s + 1) * B]), 1e-3, loss_out=loss)
            ls.append(float(loss.item()))
        per_epoch.append(np.mean(np.asarray(ls, np.float64)))
    wa, wb = a.get_weights(), b.get_weights()
    print("train: epoch losses", hist, "steps", np.asarray(per_epoch, np.float32))
    assert np.array_equal(wa, wb)
    assert np.allclose(hist, per_epoch, rtol=1e-6)
    assert hist[-1] < hist[0]
    a.close()
    b.close()


def test_seeded_initial_weights(ctx):
    a = native.Surrogate(ctx, N, K, H, seed=5).get_weights()
    b = native.Surrogate(ctx, N, K, H, seed=5).get_weights()
    c = native.Surrogate(ctx, N, K, H, seed=6).get_weights()
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    for arr, fan in zip(unpack(a), [2 * N, 2 * N, H, H, H, H]):
        bound = 1.0 / np.sqrt(fan)
        assert np.abs(arr).max() <= bound
        assert abs(arr.mean()) < 0.1 * bound and arr.std() > 0.5 * bound  # U(-a, a): sd a/sqrt 3


def test_large_grid_rank64_network_and_fallback(ctx):
    # the large grid's shape: 1920 settings (48 x 40 caps), rank 64, network 3840-256-256-64.
    # Forward against the oracle, the fused inference against the batched forward bit for bit,
    # and the fallback rows against the ridge fold-in, including rows of 1024 or more entries
    # (solved by the primal rank-64 kernel in several chunks).
    grid = synth.grid_of("large")
    n, k = grid.n, 64
    r = np.random.default_rng(64)
    counts = np.concatenate([r.integers(3, 40, size=700), r.integers(33, 400, size=200), [1024, 1500, 1920, 0]])
    r.shuffle(counts)
    rp = np.zeros(len(counts) + 1, np.int64)
    rp[1:] = np.cumsum(counts)
    col = np.concatenate([np.sort(r.choice(n, size=c, replace=False)) for c in counts]).astype(np.int32)
    val = r.uniform(0.4, 1.0, size=int(rp[-1])).astype(np.float32)
    V = synth.setting_factors(5, grid, k, m_ref=1024)
    params = synth.mlp_init(5, (2 * n, H, H, k), seed=2)
    net = native.Surrogate(ctx, n, k, H, init=pack(params))
    drp, dcol, dval, dV = dev(rp), dev(col), dev(val), dev(V)
    fwd = net.forward(drp, dcol, dval).cpu().numpy()
    sub = np.arange(0, len(counts), 7)
    Xs = omlp.dense_input(np.concatenate([[0], np.cumsum(counts[sub])]),
                          np.concatenate([col[rp[i]:rp[i + 1]] for i in sub]),
                          np.concatenate([val[rp[i]:rp[i + 1]] for i in sub]), n)
    ref, _ = omlp.forward(params, Xs)
    ef = fro(fwd[sub], ref)
    print("rank 64 forward rel %.2e" % ef)
    assert ef <= 1e-2
    Uinf, nfi = net.foldin(dV, drp, dcol, dval, float("inf"), 0.05, False)
    assert nfi == 0 and np.array_equal(Uinf.cpu().numpy(), fwd)
    als = native.open_foldin(ctx, dV, drp, dcol, dval, 0.05, False).cpu().numpy()
    rho = torch.empty(len(counts), dtype=torch.float32, device="cuda")
    used = torch.empty(len(counts), dtype=torch.uint8, device="cuda")
    net.foldin(dV, drp, dcol, dval, float("inf"), 0.05, False, rho=rho)
    tau = float(np.median(rho.cpu().numpy()[counts > 0]))
    Um, nfm = net.foldin(dV, drp, dcol, dval, tau, 0.05, False, used_fallback=used, rho=rho)
    Um, used = Um.cpu().numpy(), used.cpu().numpy().astype(bool)
    ref_als, _ = oracle.ridge_rows(rp, col, val, V, 0.05, False)
    e = np.linalg.norm(Um[used] - ref_als[used], axis=1) / np.linalg.norm(ref_als[used], axis=1)
    print("rank 64 fallback rows %d (long rows among them %d): max rel err vs oracle %.2e"
          % (used.sum(), (used & (counts >= 1024)).sum(), e.max()))
    assert e.max() <= 1e-4
    assert np.array_equal(Um[~used], fwd[~used])
    # every row re-solved: the long rows through the fallback path against the oracle
    U0, nf0 = net.foldin(dV, drp, dcol, dval, 0.0, 0.05, False)
    U0 = U0.cpu().numpy()
    assert nf0 == int((counts > 0).sum())
    long_rows = counts >= 1024
    e0 = np.linalg.norm(U0[long_rows] - ref_als[long_rows], axis=1) / np.linalg.norm(ref_als[long_rows], axis=1)
    print("rank 64 rows of 1024+ entries via the fallback: max rel err %.2e" % e0.max())
    assert e0.max() <= 1e-4
    net.close()
