"""Pins of the offline-predictor oracle (Section III-A.2): a network worked by hand
(tests/golden/predictor_hand.json), the linear regime against the collapsed affine map, the
all-off regime, invariance under a relabelling of hidden units, and the centring/scaling."""
import json
import os

import numpy as np

from oracle import predictor
from oracle.mlp import round_bf16
from paper_2508_07605_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "predictor_hand.json")


def _num(v):
    return float("nan") if v == "nan" else float(v)


def hand_params():
    g = json.load(open(GOLDEN))
    p = dict(mu=np.array(g["mu"], float), rs=np.array(g["rs"], float), W1=np.zeros((64, 7)), b1=np.zeros(64),
             W2=np.zeros((64, 64)), b2=np.zeros(64), w3=np.zeros(64), b3=np.array([g["b3"]], float))
    for h, f, v in g["W1"]:
        p["W1"][h, f] = v
    for o, i, v in g["W2"]:
        p["W2"][o, i] = v
    for name in ("b1", "b2", "w3"):
        for i, v in g[name]:
            p[name][i] = v
    X = np.array([[_num(v) for v in r] for r in g["runs"]])
    y = np.array([_num(v) for v in g["expected"]])
    return p, X, y


def test_hand_worked_network():
    p, X, y = hand_params()
    got = predictor.predict(X, p)
    assert np.array_equal(np.isnan(got), np.isnan(y))
    ok = ~np.isnan(y)
    assert np.array_equal(got[ok], y[ok])  # every intermediate is a short binary fraction


def positive_params(seed):
    # every weight, bias and centred input positive: no unit is ever cut off
    r = np.random.default_rng(seed)
    return dict(mu=np.zeros(7), rs=r.uniform(0.5, 2.0, 7), W1=r.uniform(0.01, 1.0, (64, 7)),
                b1=r.uniform(0.0, 0.5, 64), W2=r.uniform(0.01, 0.2, (64, 64)), b2=r.uniform(0.0, 0.5, 64),
                w3=r.uniform(-1.0, 1.0, 64), b3=np.array([0.3]))


def test_linear_regime_equals_collapsed_affine_map():
    # with no unit cut off the network is the affine map y = a . x + c with
    # a = rs * (W1^T (W2^T w3)) and c = w3 . (W2 b1 + b2) + b3 (bfloat16 weights), evaluated
    # here right to left as vector products instead of layer by layer
    p = positive_params(1)
    X = np.random.default_rng(2).uniform(0.0, 3.0, (200, 7))
    W1, W2 = round_bf16(p["W1"]), round_bf16(p["W2"])
    v = W2.T @ p["w3"]
    a = p["rs"] * (W1.T @ v)
    c = p["w3"] @ (W2 @ p["b1"] + p["b2"]) + p["b3"][0]
    y = predictor.predict(X, p)
    assert np.allclose(y, X @ a + c, rtol=1e-12, atol=1e-12)


def test_all_first_layer_units_off():
    # b1 far below zero: h1 = 0 for every input, so y = w3 . max(b2, 0) + b3
    p = positive_params(3)
    p["b1"] = np.full(64, -1e6)
    p["b2"] = np.random.default_rng(4).normal(size=64)
    X = np.random.default_rng(5).uniform(0.0, 3.0, (50, 7))
    expect = float(np.sum(p["w3"] * np.maximum(p["b2"], 0.0)) + p["b3"][0])
    assert np.allclose(predictor.predict(X, p), expect, rtol=0, atol=1e-12)


def test_hidden_unit_relabelling_invariance():
    # permuting the units of a hidden layer (rows of the weights into it, entries of its bias,
    # columns of the weights out of it) does not change the output
    grid = synth.grid_of("foldin")
    p = synth.predictor_params(3, grid)
    X = synth.run_features(3, grid, np.arange(300) % grid.n)
    y = predictor.predict(X, p)
    r = np.random.default_rng(6)
    q = {k: v.copy() for k, v in p.items()}
    s1 = r.permutation(64)
    q["W1"], q["b1"], q["W2"] = q["W1"][s1], q["b1"][s1], q["W2"][:, s1]
    s2 = r.permutation(64)
    q["W2"], q["b2"], q["w3"] = q["W2"][s2], q["b2"][s2], q["w3"][s2]
    assert np.allclose(predictor.predict(X, q), y, rtol=1e-12, atol=1e-12)


def test_centring_and_scaling():
    # shifting features and centres together, or scaling features and centres by s and the
    # inverse scales by 1/s, leaves the output unchanged
    grid = synth.grid_of("foldin")
    p = synth.predictor_params(3, grid)
    X = synth.run_features(3, grid, np.arange(300) % grid.n).astype(np.float64)
    y = predictor.predict(X, p)
    d = np.random.default_rng(7).normal(size=7) * 10
    q = dict(p, mu=p["mu"] + d)
    assert np.allclose(predictor.predict(X + d, q), y, rtol=1e-9, atol=1e-12)
    s = np.array([2.0, 0.5, 4.0, 0.25, 8.0, 2.0, 0.5])  # powers of two: exact rescaling
    q = dict(p, mu=p["mu"] * s, rs=p["rs"] / s)
    assert np.allclose(predictor.predict(X * s, q), y, rtol=1e-12, atol=1e-12)
    # the features really matter: moving one centre changes the output
    q = dict(p, mu=p["mu"] + np.eye(7)[3] * 1e10)
    assert not np.allclose(predictor.predict(X, q), y)
