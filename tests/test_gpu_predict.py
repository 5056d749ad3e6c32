"""GPU parity of the fused predict + Algorithm 2 selection through the C ABI.

Two checks per case: (1) given the kernel's own float32 predictions (P written on request),
a float32 restatement of the rule reproduces best_idx and best_saving bit for bit; (2)
against the FP64 oracle, P agrees to float32 rounding and the selected setting is optimal
up to near-ties: it is valid and its energy bound is within 1e-5 of the oracle's least."""
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


def mirror_f32(P, cap_c, cap_g, base, gamma):
    """Alg. 2 on float32 predictions with the kernel's float32 operations: validity by the
    correctly rounded 1 - p / p_base <= gamma; the least E = w / p as the greatest key
    p * fl(1 / w) (first index on ties); the saving from E = fl(w / p) of the pick."""
    P = P.astype(np.float32)
    w = (cap_c.astype(np.float32) + cap_g.astype(np.float32)).astype(np.float32)
    iw = (np.float32(1) / w).astype(np.float32)
    pb = P[:, base:base + 1]
    with np.errstate(divide="ignore", invalid="ignore"):
        loss = np.float32(1.0) - (P / pb).astype(np.float32)
        valid = (P > 0) & (pb > 0) & (loss.astype(np.float32) <= np.float32(gamma))
        key = np.where(valid, (P * iw[None, :]).astype(np.float32), np.float32(-np.inf))
    best = np.argmax(key, axis=1).astype(np.int32)  # first index of the maximum
    ok = (pb[:, 0] > 0) & valid.any(axis=1)
    ebase = np.float32(cap_c[base]) + np.float32(cap_g[base])
    with np.errstate(divide="ignore", invalid="ignore"):
        Ebest = (w[best] / P[np.arange(len(P)), best]).astype(np.float32)
    sav = np.where(ok, ((ebase - Ebest) / ebase).astype(np.float32), np.float32(0))
    best = np.where(ok, best, base)
    return best, sav.astype(np.float32), ok


def run(ctx, U, V, cap_c, cap_g, base, gamma, want_p=True):
    m, n = U.shape[0], V.shape[0]
    P = torch.empty((m, n), dtype=torch.float32, device="cuda") if want_p else None
    st = torch.empty(m, dtype=torch.int32, device="cuda")
    bi, bs = native.open_predict(ctx, dev(U), dev(V), dev(cap_c.astype(np.float32)), dev(cap_g.astype(np.float32)),
                                 base, gamma, P=P, row_status=st)
    torch.cuda.synchronize()
    return (P.cpu().numpy() if want_p else None), bi.cpu().numpy(), bs.cpu().numpy(), st.cpu().numpy()


def check_vs_oracle(U, V, cap_c, cap_g, base, gamma, bi, bs, P=None):
    bo, so, sto, Po = oracle.predict_select(U, V, cap_c, cap_g, base, gamma, want_p=True)
    if P is not None:
        scale = np.abs(Po).max()
        assert np.abs(P - Po).max() <= 2e-6 * scale
    Pb = Po[:, base]
    p_sel = Po[np.arange(len(bi)), bi]
    w = cap_c + cap_g
    E_sel = w[bi] / p_sel
    E_or = w[bo] / Po[np.arange(len(bo)), bo]
    good = sto == 0
    # the GPU's pick is (near-)valid and (near-)optimal under the FP64 prediction
    assert (p_sel[good] > 0).all()
    assert (1 - p_sel[good] / Pb[good] <= gamma + 1e-5).all()
    assert (E_sel[good] <= E_or[good] * (1 + 1e-5)).all()
    agree = (bi == bo).mean()
    print("selection agrees with the FP64 oracle on %.5f of rows; saving max abs diff %.2e" %
          (agree, np.abs(bs[bi == bo] - so[bi == bo]).max() if (bi == bo).any() else 0.0))
    assert agree >= 0.99
    return bo


@pytest.mark.parametrize("name,k,m", [("tiny", 8, 3001), ("foldin", 32, 5003), ("large", 64, 4097)])
def test_exact_mirror_and_oracle(ctx, name, k, m):
    grid = synth.grid_of(name)
    c = synth.CONFIGS[name]
    V = synth.setting_factors(c["cfg_id"], grid, k, m_ref=1024)
    U = synth.latent_rows(c["cfg_id"], grid, V, m, seed=3)
    gamma = 0.05
    P, bi, bs, st = run(ctx, U, V, grid.cpu_w, grid.gpu_w, grid.base, gamma)
    mb, ms, ok = mirror_f32(P, grid.cpu_w, grid.gpu_w, grid.base, gamma)
    assert np.array_equal(bi, mb)
    assert np.array_equal(bs, ms)
    assert np.array_equal(st == 0, ok)
    check_vs_oracle(U, V, grid.cpu_w, grid.gpu_w, grid.base, gamma, bi, bs, P)


def test_nonpositive_baseline_and_gamma_limits(ctx):
    grid = synth.grid_of("foldin")
    V = synth.setting_factors(3, grid, 32, m_ref=1024)
    U = synth.latent_rows(3, grid, V, 200, seed=4)
    U[:7] = -U[:7]  # predictions (and the baseline) negative
    P, bi, bs, st = run(ctx, U, V, grid.cpu_w, grid.gpu_w, grid.base, 0.05)
    assert (st[:7] == 4).all() and (bi[:7] == grid.base).all() and (bs[:7] == 0).all()
    assert (st[7:] == 0).all()
    # gamma = 0: only settings predicted at least as fast as the baseline
    P, bi, bs, st = run(ctx, U[7:], V, grid.cpu_w, grid.gpu_w, grid.base, 0.0)
    pb = P[:, grid.base]
    assert (P[np.arange(len(bi)), bi] >= pb).all()
    mb, ms, _ = mirror_f32(P, grid.cpu_w, grid.gpu_w, grid.base, 0.0)
    assert np.array_equal(bi, mb) and np.array_equal(bs, ms)


def test_without_prediction_output_matches(ctx):
    grid = synth.grid_of("foldin")
    V = synth.setting_factors(3, grid, 32, m_ref=1024)
    U = synth.latent_rows(3, grid, V, 1000, seed=5)
    _, bi, bs, _ = run(ctx, U, V, grid.cpu_w, grid.gpu_w, grid.base, 0.05, want_p=True)
    _, bi2, bs2, _ = run(ctx, U, V, grid.cpu_w, grid.gpu_w, grid.base, 0.05, want_p=False)
    assert np.array_equal(bi, bi2) and np.array_equal(bs, bs2)


def test_large_grid_full_size_sampled(ctx):
    # 2M apps x 1920 settings (48 x 40 caps), rank 64: selection for every row, the oracle
    # recomputes a seeded sample
    c = synth.CONFIGS["large"]
    grid = synth.grid_of("large")
    V = synth.setting_factors(c["cfg_id"], grid, c["k"], m_ref=2048)
    U = synth.latent_rows(c["cfg_id"], grid, V, c["m"], seed=6)
    _, bi, bs, st = run(ctx, U, V, grid.cpu_w, grid.gpu_w, grid.base, c["gamma"], want_p=False)
    assert (st == 0).all()
    sample = np.sort(np.random.default_rng(8).choice(c["m"], size=4000, replace=False))
    check_vs_oracle(U[sample], V, grid.cpu_w, grid.gpu_w, grid.base, c["gamma"], bi[sample], bs[sample])
