"""GPU parity of the ALS-WR fit path through the C ABI: the column view (exact), the
objective and residual reductions, single half-sweeps from generator inputs, and whole fits
(same initial factors) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_07605_amd import native, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = native.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def fro_rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def fit_rows(name, m=None, seed=0):
    c = synth.CONFIGS[name]
    grid = synth.grid_of(name)
    rows = synth.draw_rows(c["cfg_id"], grid, m or c["m"], c["counts"], seed=seed)
    return c, grid, rows


def test_csc_exact(ctx):
    _, grid, rows = fit_rows("fit", m=30_001)
    cp, ri, cv = native.open_csr_to_csc(ctx, dev(rows.row_ptr), dev(rows.col), dev(rows.val), grid.n)
    rcp, rri, rcv = oracle.csr_to_csc(rows.row_ptr, rows.col, rows.val, grid.n)
    assert np.array_equal(host(cp), rcp)
    assert np.array_equal(host(ri), rri)
    assert np.array_equal(host(cv).astype(np.float64), rcv)


def test_csc_rejects_bad_index(ctx):
    rp = np.array([0, 2, 3], dtype=np.int64)
    col = np.array([0, 9, 1], dtype=np.int32)
    val = np.ones(3, dtype=np.float32)
    with pytest.raises(native.OpenError):
        native.open_csr_to_csc(ctx, dev(rp), dev(col), dev(val), 4)


@pytest.mark.parametrize("k", [8, 32, 64])
def test_objective_and_residual(ctx, k):
    _, grid, rows = fit_rows("fit_d5", m=20_000, seed=3)
    U, V = synth.init_factors(6, rows.m, grid.n, k, std=0.3, seed=3)
    for weighted in (True, False):
        f = native.open_objective(ctx, dev(rows.row_ptr), dev(rows.col), dev(rows.val), dev(U), dev(V), 0.05, weighted)
        ref = oracle.objective(rows.row_ptr, rows.col, rows.val, U, V, 0.05, weighted)
        assert abs(f - ref) <= 1e-6 * ref
    rho = host(native.open_residual(ctx, dev(rows.row_ptr), dev(rows.col), dev(rows.val), dev(U), dev(V)))
    ref = oracle.residual(rows.row_ptr, rows.col, rows.val, U, V)
    assert np.abs(rho - ref).max() <= 1e-5 * ref.max()


@pytest.mark.parametrize("name", ["fit", "fit_d5", "large"])
def test_half_sweeps_from_generator_inputs(ctx, name):
    # one row half-sweep (against V0) and one column half-sweep (against U0), both from the
    # generator's initial factors, compared row by row and column by column
    c, grid, rows = fit_rows(name, m=20_000, seed=5)
    U0, V0 = synth.init_factors(c["cfg_id"], rows.m, grid.n, c["k"], seed=5)
    st = torch.empty(rows.m, dtype=torch.int32, device="cuda")
    Ur = host(native.open_foldin(ctx, dev(V0), dev(rows.row_ptr), dev(rows.col), dev(rows.val), c["lam"], True,
                                 row_status=st)).astype(np.float64)
    ref, ref_st = oracle.ridge_rows(rows.row_ptr, rows.col, rows.val, V0, c["lam"], True)
    assert np.array_equal(host(st), ref_st)
    e = np.linalg.norm(Ur - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print("%s row half-sweep: max %.3e median %.3e" % (name, e.max(), np.median(e)))
    assert e.max() <= 1e-4
    cp, ri, cv = native.open_csr_to_csc(ctx, dev(rows.row_ptr), dev(rows.col), dev(rows.val), grid.n)
    Vc = host(native.open_foldin(ctx, dev(U0), cp, ri, cv, c["lam"], True)).astype(np.float64)
    rcp, rri, rcv = oracle.csr_to_csc(rows.row_ptr, rows.col, rows.val, grid.n)
    refc, _ = oracle.ridge_rows(rcp, rri, rcv, U0, c["lam"], True)
    e = np.linalg.norm(Vc - refc, axis=1) / np.linalg.norm(refc, axis=1)
    print("%s column half-sweep: max %.3e median %.3e" % (name, e.max(), np.median(e)))
    assert e.max() <= 1e-4


@pytest.mark.parametrize("weighted", [True, False])
def test_tiny_config_fit(ctx, weighted):
    # the tiny configuration: 64 dense + 16 sparse apps x 120 settings, rank 8, 20 sweeps
    grid, dense, new, union = synth.tiny_problem(seed=0)
    c = synth.CONFIGS["tiny"]
    U0, V0 = synth.init_factors(c["cfg_id"], union.m, grid.n, c["k"])
    U, V = dev(U0), dev(V0)
    obj = native.open_fit(ctx, dev(union.row_ptr), dev(union.col), dev(union.val), U, V, c["lam"], c["sweeps"],
                          weighted, want_obj=True)
    Ug, Vg = host(U).astype(np.float64), host(V).astype(np.float64)
    Ur, Vr, objr = oracle.fit(union.row_ptr, union.col, union.val, U0, V0, c["lam"], c["sweeps"], weighted)
    pe = fro_rel(Ug @ Vg.T, Ur @ Vr.T)
    fe = max(fro_rel(Ug, Ur), fro_rel(Vg, Vr))
    oe = np.abs(obj - objr).max() / objr.max()
    print("tiny fit w%d: UV^T %.3e  factors %.3e  objective %.3e" % (weighted, pe, fe, oe))
    assert pe <= 1e-4 and oe <= 1e-4
    assert (obj[1:] <= obj[:-1] * (1 + 1e-5)).all()


def test_fit_config_shape(ctx):
    # rank 32, 480 settings, truncated Zipf(1.2) counts, 15 sweeps, at 12k apps
    c, grid, rows = fit_rows("fit", m=12_000, seed=7)
    U0, V0 = synth.init_factors(c["cfg_id"], rows.m, grid.n, c["k"], seed=7)
    U, V = dev(U0), dev(V0)
    obj = native.open_fit(ctx, dev(rows.row_ptr), dev(rows.col), dev(rows.val), U, V, c["lam"], c["sweeps"], True,
                          want_obj=True)
    Ug, Vg = host(U).astype(np.float64), host(V).astype(np.float64)
    Ur, Vr, objr = oracle.fit(rows.row_ptr, rows.col, rows.val, U0, V0, c["lam"], c["sweeps"], True)
    pe = fro_rel(Ug @ Vg.T, Ur @ Vr.T)
    oe = np.abs(obj - objr).max() / objr.max()
    print("fit k32: UV^T %.3e  U %.3e  V %.3e  objective %.3e" % (pe, fro_rel(Ug, Ur), fro_rel(Vg, Vr), oe))
    assert pe <= 1e-4 and oe <= 1e-4


def test_fit_graph_replay_matches_eager(ctx):
    # without an objective history the sweeps after the first replay one recorded HIP graph;
    # with it every launch is eager: the same kernels in the same order give identical factors
    c, grid, rows = fit_rows("fit", m=6_000, seed=9)
    U0, V0 = synth.init_factors(c["cfg_id"], rows.m, grid.n, c["k"], seed=9)
    args = (dev(rows.row_ptr), dev(rows.col), dev(rows.val))
    Ug, Vg = dev(U0), dev(V0)
    native.open_fit(ctx, *args, Ug, Vg, c["lam"], 4, True, want_obj=False)
    Ue, Ve = dev(U0), dev(V0)
    native.open_fit(ctx, *args, Ue, Ve, c["lam"], 4, True, want_obj=True)
    assert torch.equal(Ug, Ue) and torch.equal(Vg, Ve)


@pytest.mark.parametrize("sweeps", [0, 2])
def test_refit_warm_start(ctx, sweeps):
    # offline rows + newly arrived rows: fold-in of the new rows against V, then ALS sweeps on
    # the union from the offline factors, against the oracle doing the same steps in FP64
    c, grid, rows = fit_rows("fit", m=5_000, seed=13)
    m_old = 4_000
    U0, V0 = synth.init_factors(c["cfg_id"], rows.m, grid.n, c["k"], seed=13)
    U, V = dev(U0), dev(V0)
    obj = native.open_refit(ctx, m_old, dev(rows.row_ptr), dev(rows.col), dev(rows.val), U, V, c["lam"], sweeps,
                            True, want_obj=sweeps > 0)
    rp_new = rows.row_ptr[m_old:] - rows.row_ptr[m_old]
    seg = slice(int(rows.row_ptr[m_old]), int(rows.row_ptr[-1]))
    Unew, _ = oracle.ridge_rows(rp_new, rows.col[seg], rows.val[seg], V0, c["lam"], True)
    Ui = np.concatenate([U0[:m_old].astype(np.float64), Unew])
    if sweeps == 0:
        Ur, Vr = Ui, V0.astype(np.float64)
    else:
        Ur, Vr, objr = oracle.fit(rows.row_ptr, rows.col, rows.val, Ui, V0, c["lam"], sweeps, True)
    Ug, Vg = host(U).astype(np.float64), host(V).astype(np.float64)
    pe = fro_rel(Ug @ Vg.T, Ur @ Vr.T)
    print("refit sweeps=%d: UV^T %.3e" % (sweeps, pe))
    assert pe <= 1e-4
    if sweeps > 0:
        assert np.abs(obj - objr).max() / objr.max() <= 1e-4
    else:
        assert np.array_equal(host(U)[:m_old], U0[:m_old])


@pytest.mark.timeout(600)
def test_large_config_fit_sampled(ctx):
    # the large configuration at full size: 2M apps x 1920 settings, ~2 % density, rank 64.
    # One ALS-WR sweep from the generator's initial factors; the oracle recomputes a seeded
    # sample of 10,000 rows from V0 (the input of the row half-sweep) and 64 columns from the
    # GPU's U (the input of the column half-sweep).
    import time
    t0 = time.time()
    c, grid, rows = fit_rows("large")
    U0, V0 = synth.init_factors(c["cfg_id"], rows.m, grid.n, c["k"])
    print("large: %d rows, %d entries generated in %.1f s" % (rows.m, rows.nnz, time.time() - t0), flush=True)
    U, V = dev(U0), dev(V0)
    native.open_fit(ctx, dev(rows.row_ptr), dev(rows.col), dev(rows.val), U, V, c["lam"], 1, True, want_obj=False)
    Ug, Vg = host(U), host(V)
    assert np.isfinite(Ug).all() and np.isfinite(Vg).all()
    r = np.random.default_rng(2025)
    srows = np.sort(r.choice(rows.m, size=10_000, replace=False))
    ref, st = oracle.ridge_subset(srows, rows.row_ptr, rows.col, rows.val, V0, c["lam"], True)
    assert (st == 0).all()
    e = np.linalg.norm(Ug[srows] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    cnt = np.diff(rows.row_ptr)[srows]
    print("large row half-sweep (10,000 rows; %d with more than 32 entries): max %.3e p99 %.3e median %.3e"
          % ((cnt > 32).sum(), e.max(), np.percentile(e, 99), np.median(e)), flush=True)
    assert e.max() <= 1e-4
    rcp, rri, rcv = oracle.csr_to_csc(rows.row_ptr, rows.col, rows.val, grid.n)
    scols = np.sort(r.choice(grid.n, size=64, replace=False))
    refc, stc = oracle.ridge_subset(scols, rcp, rri, rcv, Ug, c["lam"], True)
    assert (stc == 0).all()
    ec = np.linalg.norm(Vg[scols] - refc, axis=1) / np.linalg.norm(refc, axis=1)
    print("large column half-sweep (64 columns, %d-%d entries): max %.3e median %.3e"
          % (np.diff(rcp)[scols].min(), np.diff(rcp)[scols].max(), ec.max(), np.median(ec)), flush=True)
    assert ec.max() <= 1e-4
