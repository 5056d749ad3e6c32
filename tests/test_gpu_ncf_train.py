"""GPU NCF offline training through the C ABI against the FP64 oracle: the loss and the
gradient of every parameter group on a batch of whole applications (relative Frobenius error
<= 1e-2 per network tensor, <= 3e-2 for the embedding gradients; the products run on
bfloat16 operands), and training: the loss falls and two runs from the same start give the
same parameters bit for bit."""
import numpy as np
import pytest
import torch

from oracle import ncf as oncf
from paper_2508_07605_amd import native, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = native.Context(0)
    yield c
    c.close()


def problem(m_off=64, seed=0):
    grid = synth.grid_of("foldin")
    apps = synth.draw_apps(synth.rng(3, 99, seed), m_off)
    R = synth.truth_dense(apps, grid).astype(np.float32)
    p = synth.ncf_params(3, grid.n, seed=seed)
    S = p.pop("S")
    E = (0.1 * np.random.default_rng(seed).standard_normal((m_off, 32))).astype(np.float32)
    return R, E, S, p


def fro(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300)


def test_batch_gradient_against_oracle(ctx):
    R, E, S, p = problem()
    flat = torch.from_numpy(native.ncf_pack(E, S, p)).cuda()
    apps = np.array([5, 17, 3, 40, 63, 0], dtype=np.int64)
    loss, g = native.open_ncf_loss_grad(ctx, torch.from_numpy(R).cuda(), flat, torch.from_numpy(apps).cuda())
    Lr, gr = oncf.train_loss_and_grads(E, S, p, apps, R)
    gE, gS, gnet = native.ncf_unpack(g, R.shape[0], R.shape[1])
    errs = {"E": fro(gE, gr["E"]), "S": fro(gS, gr["S"])}
    errs.update({k: fro(v, gr[k]) for k, v in gnet.items()})
    print("NCF batch loss %.6g vs %.6g; gradient errors %s" % (loss, Lr, {k: "%.2e" % v for k, v in errs.items()}))
    assert abs(loss - Lr) <= 1e-2 * Lr
    # network tensors within 1e-2.  The embedding gradients pass through three chained
    # bfloat16 products (dZ2, dZ1, dX) and are then sums over every setting (application
    # rows) or every application of the batch (setting rows) with heavy cancellation: a single
    # length-64 bfloat16 dot product of mixed signs already admits about 2^-9 sqrt(64) = 1.6e-2
    # relative error.  They must be within 3e-2 and point the same way (cosine >= 0.999).
    assert max(v for k, v in errs.items() if k not in ("E", "S")) <= 1e-2
    assert errs["E"] <= 3e-2 and errs["S"] <= 3e-2
    for got, ref in ((gE, gr["E"]), (gS, gr["S"])):
        got = np.asarray(got, np.float64).ravel()
        ref = ref.ravel()
        assert got @ ref / (np.linalg.norm(got) * np.linalg.norm(ref)) >= 0.999
    # applications outside the batch have zero gradient
    others = np.setdiff1d(np.arange(R.shape[0]), apps)
    assert not gE[others].any()


def test_training_reduces_loss_and_repeats(ctx):
    R, E, S, p = problem(m_off=256, seed=1)
    dR = torch.from_numpy(R).cuda()
    init = native.ncf_pack(E, S, p)
    a = torch.from_numpy(init.copy()).cuda()
    b = torch.from_numpy(init.copy()).cuda()
    ha = native.open_ncf_train(ctx, dR, a, 8, 1e-3, 6, seed=3)
    hb = native.open_ncf_train(ctx, dR, b, 8, 1e-3, 6, seed=3)
    print("NCF epoch losses", ha)
    assert np.array_equal(ha, hb) and torch.equal(a, b)
    assert ha[-1] < 0.5 * ha[0]
    # the trained parameters drive the fold-in kernel unchanged (views into the flat vector)
    Et, St, net = native.ncf_unpack(a, R.shape[0], R.shape[1])
    rows = synth.draw_rows(3, synth.grid_of("foldin"), 257, ("uniform", 4, 24), seed=5)
    dv = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    E_new = native.open_ncf_foldin(ctx, St, net, dv(rows.row_ptr), dv(rows.col), dv(rows.val), 30, 0.5, 1e-3)
    assert torch.isfinite(E_new).all()
