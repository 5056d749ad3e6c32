"""GPU parity of the batched offline performance predictor (Section III-A.2) against the FP64
oracle, through the C ABI.

Tolerance: the kernel multiplies the bfloat16 weights (the oracle uses the same rounded
weights) by activations split into two bfloat16 parts, exact to 2^-18 relative, and
accumulates in float32.  Each layer therefore adds at most a few 2^-18 of the magnitude it
sums, so |y_gpu - y_ref| <= 3e-5 * S + 1e-7 with S = |b3| + |w3| . (|W2| (|W1| |z| + |b1|) + |b2|),
the output computed with every term replaced by its magnitude."""
import numpy as np
import pytest
import torch

from oracle import predictor
from oracle.mlp import round_bf16
from paper_2508_07605_amd import native, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = native.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def dev_params(p):
    return {k: dev(v) for k, v in p.items()}


def magnitude(X, p):
    Z = np.abs((np.asarray(X, np.float64) - p["mu"]) * p["rs"])
    H = np.abs(round_bf16(p["W1"])) @ Z.T + np.abs(p["b1"].astype(np.float64))[:, None]
    H = np.abs(round_bf16(p["W2"])) @ H + np.abs(p["b2"].astype(np.float64))[:, None]
    return abs(float(p["b3"][0])) + np.abs(p["w3"].astype(np.float64)) @ H


def run(ctx, X, p):
    y = native.open_perf_predict(ctx, dev(X), dev_params(p))
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def check(y, X, p, name):
    ref = predictor.predict(X, p)
    tol = 3e-5 * magnitude(X, p) + 1e-7
    err = np.abs(y - ref)
    print("%s: runs %d  max err %.3e  max err/tol %.3f" % (name, len(y), err.max(), (err / tol).max()))
    assert (err <= tol).all()


def workload(m_runs, seed=0):
    grid = synth.grid_of("foldin")
    setting = np.random.default_rng(seed).integers(0, grid.n, size=m_runs)
    return synth.run_features(3, grid, setting, seed=seed), synth.predictor_params(3, grid)


def test_parity_ragged(ctx):
    # several tiles of 32 runs per wavefront, a ragged tail
    X, p = workload(100_003, seed=1)
    check(run(ctx, X, p), X, p, "predictor 100003")


@pytest.mark.parametrize("n", [1, 31, 32, 33, 65, 4099])
def test_small_sizes(ctx, n):
    X, p = workload(n, seed=n)
    check(run(ctx, X, p), X, p, "predictor n=%d" % n)


def test_hand_worked_network_exact(ctx):
    # the hand-worked network of the oracle's pins: every product and sum is exact in float32,
    # so the kernel must give the hand values bit for bit (and NaN for the non-finite run)
    from test_oracle_predictor import hand_params
    p, X, y = hand_params()
    got = run(ctx, X, p)
    assert np.array_equal(np.isnan(got), np.isnan(y))
    assert np.array_equal(got[~np.isnan(y)], y[~np.isnan(y)])


def test_nonfinite_runs_only_affect_themselves(ctx):
    X, p = workload(1000, seed=5)
    X[[3, 500, 999], [0, 4, 6]] = [np.nan, np.inf, -np.inf]
    y = run(ctx, X, p)
    bad = np.zeros(1000, bool)
    bad[[3, 500, 999]] = True
    assert np.isnan(y[bad]).all() and np.isfinite(y[~bad]).all()
    check(y[~bad], X[~bad], p, "predictor with non-finite runs")


def test_empty_and_invalid(ctx):
    _, p = workload(1)
    X = torch.empty((0, 7), dtype=torch.float32, device="cuda")
    y = torch.full((4,), 7.0, device="cuda")
    native.open_perf_predict(ctx, X, dev_params(p), y=y)  # no runs: nothing written
    torch.cuda.synchronize()
    assert (y == 7.0).all()
    with pytest.raises(ValueError):
        native.open_perf_predict(ctx, torch.zeros((4, 6), device="cuda"), dev_params(p))


def test_deterministic(ctx):
    X, p = workload(50_000, seed=7)
    assert np.array_equal(run(ctx, X, p), run(ctx, X, p))


def test_full_size_sampled(ctx):
    # one predicted value per profiled run of the 1M-app fold-in workload (14.0M runs), in the
    # launch configuration the benchmark times; the oracle recomputes a seeded sample
    c = synth.CONFIGS["foldin"]
    grid = synth.grid_of("foldin")
    rows = synth.draw_rows(c["cfg_id"], grid, c["m"], c["counts"], seed=0)
    X = synth.run_features(c["cfg_id"], grid, rows.col)
    p = synth.predictor_params(c["cfg_id"], grid)
    y = run(ctx, X, p)
    assert np.isfinite(y).all()
    sample = np.sort(np.random.default_rng(9).choice(len(X), size=20_000, replace=False))
    check(y[sample], X[sample], p, "predictor full-size sample")
