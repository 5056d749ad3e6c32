"""What the trained surrogate gains over the method without it.  The network (960-256-256-32)
is trained with open_mlp_train on the plain-lambda ALS fold-ins of new apps.  It is then used
with the ridge fallback (observed-entry RMS residual > tau = 0.02) on other new apps, beside
the same network untrained.  Checks: the trained network falls back on far fewer rows and
runs faster, and the predictions of surrogate + fallback stay within an RMSE gap of 1e-3
(unobserved settings, against the noiseless truth) of the FP64 oracle's ALS fold-in."""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_07605_amd import native, synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.timeout(300)
def test_trained_surrogate_gain():
    ctx = native.Context(0)
    c = synth.CONFIGS["surrogate"]
    grid = synth.grid_of("surrogate")
    n, k, lam, wt, tau = grid.n, c["k"], c["lam"], c["weighted"], c["tau"]
    V = synth.setting_factors(c["cfg_id"], grid, k)
    dV = dev(V)
    tr = synth.draw_rows(c["cfg_id"], grid, 500_000, c["counts"], seed=31)
    trp, tcol, tval = dev(tr.row_ptr), dev(tr.col), dev(tr.val)
    target = native.open_foldin(ctx, dV, trp, tcol, tval, lam, wt)
    net = native.Surrogate(ctx, n, k, c["hidden"], seed=4)
    untrained = native.Surrogate(ctx, n, k, c["hidden"], seed=4)
    hist = net.train(trp, tcol, tval, target, c["batch"], c["lr"], 10, seed=5)
    print("epoch losses", hist)
    assert hist[-1] < 0.2 * hist[0]

    ev = synth.draw_rows(c["cfg_id"], grid, 1_000_000, c["counts"], seed=32)
    erp, ecol, evl = dev(ev.row_ptr), dev(ev.col), dev(ev.val)
    U = torch.empty((ev.m, k), dtype=torch.float32, device="cuda")

    def run(model):
        for _ in range(2):
            model.foldin(dV, erp, ecol, evl, tau, lam, wt, U_out=U, count=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            model.foldin(dV, erp, ecol, evl, tau, lam, wt, U_out=U, count=False)
        e1.record()
        torch.cuda.synchronize()
        _, nf = model.foldin(dV, erp, ecol, evl, tau, lam, wt, U_out=U)
        return e0.elapsed_time(e1) / 5, nf / ev.m, U.cpu().numpy().astype(np.float64)

    ms0, f0, _ = run(untrained)
    ms1, f1, Us = run(net)
    print("fallback: trained %.3f untrained %.3f; ms per 1M rows: trained %.3f untrained %.3f" % (f1, f0, ms1, ms0))
    assert f0 > 0.99
    assert f1 < 0.5 and f1 < f0 - 0.4
    assert ms1 < ms0

    sample = np.arange(0, ev.m, 200)
    Uo, st = oracle.ridge_subset(sample, ev.row_ptr, ev.col, ev.val, V, lam, wt)
    assert (st == 0).all()
    T = synth.truth_dense(ev.apps.take(sample), grid)
    obs = np.zeros_like(T, dtype=bool)
    for j, i in enumerate(sample):
        obs[j, ev.col[ev.row_ptr[i]:ev.row_ptr[i + 1]]] = True
    Vd = V.astype(np.float64)
    rmse_s = float(np.sqrt((((Us[sample] @ Vd.T) - T)[~obs] ** 2).mean()))
    rmse_o = float(np.sqrt((((Uo @ Vd.T) - T)[~obs] ** 2).mean()))
    print("RMSE vs truth: surrogate + fallback %.6f, oracle ALS fold-in %.6f, gap %.2e" % (rmse_s, rmse_o,
                                                                                          abs(rmse_s - rmse_o)))
    assert abs(rmse_s - rmse_o) <= 1e-3
    net.close()
    untrained.close()
    ctx.close()
