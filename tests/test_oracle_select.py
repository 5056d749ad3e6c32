"""Pins of the oracle's Alg. 2 (energy-efficient cap selection, Section III-B.3):
a hand-worked example and a brute-force re-implementation over every candidate."""
import itertools

import numpy as np

import oracle


def _select_through_identity(p_rows, cap_c, cap_g, base, gamma):
    # U = p, V = I  ->  U V^T = p exactly
    p_rows = np.asarray(p_rows, dtype=np.float64)
    n = p_rows.shape[1]
    return oracle.predict_select(p_rows, np.eye(n), cap_c, cap_g, base, gamma, want_p=True)


def test_hand_example():
    # settings (CPU W, GPU W): 0 (150, 200), 1 (150, 250), 2 (200, 200), 3 (200, 250) = baseline
    cap_c = [150.0, 150.0, 200.0, 200.0]
    cap_g = [200.0, 250.0, 200.0, 250.0]
    p = [[0.90, 0.96, 0.97, 1.00]]
    best, saving, st, P = _select_through_identity(p, cap_c, cap_g, 3, 0.05)
    # (150, 200): loss 0.10 > 0.05, invalid despite the lowest energy bound 350/0.9
    # (200, 200): E = 400/0.97 = 412.37113..., saving = (450 - E)/450 = 0.0836197...
    # (150, 250): E = 400/0.96 = 416.666...,  saving = 0.0740740...
    assert best[0] == 2 and st[0] == 0
    assert abs(saving[0] - (450.0 - 400.0 / 0.97) / 450.0) < 1e-15
    assert abs(saving[0] - 0.08361970217640321) < 1e-12
    # gamma = 0.1 admits (150, 200): E = 388.88..., saving = 0.1358024...
    best, saving, _, _ = _select_through_identity(p, cap_c, cap_g, 3, 0.10)
    assert best[0] == 0 and abs(saving[0] - (450.0 - 350.0 / 0.9) / 450.0) < 1e-15
    # gamma = 0: only settings at least as fast as the baseline; the baseline itself, saving 0
    best, saving, _, _ = _select_through_identity(p, cap_c, cap_g, 3, 0.0)
    assert best[0] == 3 and saving[0] == 0.0


def _brute(p, cap_c, cap_g, base, gamma):
    e_base = cap_c[base] + cap_g[base]
    pb = p[base]
    if not pb > 0:
        return base, 0.0
    cands = []
    for s in range(len(p)):
        if p[s] > 0 and 1.0 - p[s] / pb <= gamma:
            e = (cap_c[s] + cap_g[s]) / p[s]
            cands.append(((e_base - e) / e_base, -s))
    sv, neg_s = max(cands)
    return -neg_s, sv


def test_brute_force_random_grids():
    r = np.random.default_rng(21)
    for trial in range(40):
        nc, ng = r.integers(1, 6), r.integers(1, 6)
        c = np.repeat(np.linspace(100, 250, nc), ng)
        g = np.tile(np.linspace(90, 300, ng), nc)
        base = int(r.integers(0, nc * ng))
        p = r.uniform(-0.1, 1.2, size=(7, nc * ng))
        p[0, base] = -0.5  # a row with a non-positive baseline prediction
        gamma = float(r.choice([0.0, 0.05, 0.15, 0.5]))
        best, saving, st, _ = _select_through_identity(p, c, g, base, gamma)
        for i in range(7):
            b, sv = _brute(p[i], c, g, base, gamma)
            assert best[i] == b and saving[i] == sv
            assert st[i] == (2 if p[i, base] <= 0 else 0)


def test_ties_take_lowest_index():
    # two settings with identical caps and identical predictions: the lower index wins
    c = np.array([200.0, 150.0, 150.0, 200.0])
    g = np.array([250.0, 200.0, 200.0, 200.0])
    p = np.array([[1.0, 0.98, 0.98, 0.99]])
    best, _, _, _ = _select_through_identity(p, c, g, 0, 0.05)
    assert best[0] == 1


def test_low_rank_predictions():
    # p from a genuine factorisation: the oracle's P equals U V^T and selection agrees with brute force
    r = np.random.default_rng(22)
    U = r.normal(0.3, 0.1, size=(20, 4))
    V = r.normal(0.6, 0.2, size=(30, 4))
    c = np.repeat(np.linspace(120, 270, 6), 5)
    g = np.tile(np.linspace(100, 250, 5), 6)
    best, saving, _, P = oracle.predict_select(U, V, c, g, 29, 0.05, want_p=True)
    assert np.allclose(P, U @ V.T, rtol=1e-14, atol=1e-15)
    for i in range(20):
        b, sv = _brute(P[i], c, g, 29, 0.05)
        assert best[i] == b and saving[i] == sv


def test_cartesian_enumeration_order():
    # flat setting index s = a * n_gpu + b enumerates C x G CPU-major
    cpu = [120.0, 195.0, 270.0]
    gpu = [100.0, 250.0]
    pairs = list(itertools.product(cpu, gpu))
    from paper_2508_07605_amd import synth
    grid = synth.cap_grid(3, 2)
    assert [(a, b) for a, b in zip(grid.cpu_w, grid.gpu_w)] == pairs
    assert grid.base == 5 and pairs[grid.base] == (270.0, 250.0)
