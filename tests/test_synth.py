"""Properties of the seeded workload generator (the inputs both sides receive)."""
import numpy as np

from paper_2508_07605_amd import synth


def test_truth_normalised_and_monotone():
    grid = synth.grid_of("fit")
    apps = synth.draw_apps(synth.rng(99, synth.S_APPS), 500)
    T = synth.truth_dense(apps, grid)
    assert np.array_equal(T[:, grid.base], np.ones(500))  # 1 at (Cmax, Gmax) exactly
    assert T.min() >= 0.4 and T.max() <= 1.0
    T3 = T.reshape(500, grid.n_cpu, grid.n_gpu)
    assert (np.diff(T3, axis=1) >= 0).all() and (np.diff(T3, axis=2) >= 0).all()


def test_sets_sorted_unique_and_counts():
    grid = synth.grid_of("foldin")
    rows = synth.draw_rows(3, grid, 5000, ("uniform", 4, 24), seed=7)
    cnt = rows.counts()
    assert cnt.min() >= 4 and cnt.max() <= 24
    for i in range(0, 5000, 97):
        c = rows.col[rows.row_ptr[i]:rows.row_ptr[i + 1]]
        assert (np.diff(c) > 0).all() and c.min() >= 0 and c.max() < grid.n
    # roughly uniform column usage
    hist = np.bincount(rows.col, minlength=grid.n)
    assert hist.min() > 0.6 * hist.mean() and hist.max() < 1.4 * hist.mean()
    # the values are the truth times (1 + small noise)
    t = synth.truth_at(rows.apps, grid, rows.row_ids(), rows.col.astype(np.int64))
    rel = rows.val / t - 1.0
    assert abs(rel.std() - 0.02) < 0.002 and abs(rel.mean()) < 0.002


def test_deterministic_and_seeded():
    grid = synth.grid_of("tiny")
    a = synth.draw_rows(1, grid, 50, ("uniform", 3, 9), seed=4)
    b = synth.draw_rows(1, grid, 50, ("uniform", 3, 9), seed=4)
    c = synth.draw_rows(1, grid, 50, ("uniform", 3, 9), seed=5)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert not np.array_equal(a.val[:10], c.val[:10])


def test_zipf_counts_mean():
    r = synth.rng(2, synth.S_COUNTS)
    c = synth.draw_counts(r, 200_000, 480, ("zipf", 1.2, 3, 480))
    assert c.min() >= 3 and c.max() <= 480
    assert abs(c.mean() - 63.69) < 1.0


def test_setting_factors_span_truth():
    grid = synth.grid_of("foldin")
    V = synth.setting_factors(3, grid, 32)
    assert V.shape == (480, 32) and V.dtype == np.float32
    apps = synth.draw_apps(synth.rng(123, synth.S_APPS), 200)
    T = synth.truth_dense(apps, grid)
    Q, _ = np.linalg.qr(V.astype(np.float64))
    resid = T - (T @ Q) @ Q.T
    assert np.sqrt((resid ** 2).mean()) < 1e-3  # rank 32 captures the truth manifold
