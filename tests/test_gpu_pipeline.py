"""The online phase end to end on the GPU (Section III-B.2): each new application's profiled
runs go through the offline predictor (Section III-A.2), the predicted normalized performances
become the observed entries of its sparse row, and the row is folded in against the fixed
setting factors.  Compared with the oracle doing the same two steps in FP64.

Tolerance: the predictor's outputs differ from the oracle's by at most a few 1e-6 (its own
parity bound); the ridge fold-in is well conditioned (lambda n_i on the diagonal), so the
per-row relative error of the embedding stays within the fold-in's 1e-4."""
import numpy as np
import pytest
import torch

import oracle
from oracle import predictor
from paper_2508_07605_amd import native, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = native.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_predictor_then_foldin(ctx):
    c = synth.CONFIGS["foldin"]
    grid = synth.grid_of("foldin")
    V = synth.setting_factors(c["cfg_id"], grid, c["k"], m_ref=2048)
    rows = synth.draw_rows(c["cfg_id"], grid, 5003, c["counts"], seed=17)
    X = synth.run_features(c["cfg_id"], grid, rows.col, seed=17)
    p = synth.predictor_params(c["cfg_id"], grid)
    y = native.open_perf_predict(ctx, dev(X), {k: dev(v) for k, v in p.items()})
    st = torch.full((rows.m,), -7, dtype=torch.int32, device="cuda")
    U = native.open_foldin(ctx, dev(V), dev(rows.row_ptr), dev(rows.col), y, c["lam"], True, row_status=st)
    torch.cuda.synchronize()
    y_ref = predictor.predict(X, p)
    U_ref, st_ref = oracle.ridge_rows(rows.row_ptr, rows.col, y_ref, V, c["lam"], True)
    assert np.abs(y.cpu().numpy() - y_ref).max() < 1e-4
    assert np.array_equal(st.cpu().numpy(), st_ref)
    U = U.cpu().numpy().astype(np.float64)
    nrm = np.linalg.norm(U_ref, axis=1)
    e = np.linalg.norm(U - U_ref, axis=1) / np.where(nrm > 0, nrm, 1.0)
    print("predictor -> fold-in: rows %d  max rel err %.3e" % (rows.m, e.max()))
    assert e.max() <= 1e-4
