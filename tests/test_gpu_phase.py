"""GPU Algorithm 1 (phase-transition detection) through the C ABI against the oracle:
bit-exact detection indices (integer result)."""
import numpy as np
import pytest
import torch

from oracle import phase
from paper_2508_07605_amd import native, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = native.Context(0)
    yield c
    c.close()


def run(ctx, P, th=60.0, n=25):
    out = native.open_phase_detect(ctx, torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32)).cuda(), th, n)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_generator_traces_paper_parameters(ctx):
    P = synth.power_traces(7, 600, 1337, seed=1)  # L not a multiple of the 64-reading step
    got = run(ctx, P)
    want = np.array([phase.detect(tr) for tr in P])
    assert np.array_equal(got, want)
    assert (want == -1).any() and (want > 0).any()


@pytest.mark.parametrize("n", [1, 5, 25, 63, 64, 65, 200, 300])
def test_windows_across_steps(ctx, n):
    r = np.random.default_rng(n)
    P = r.choice(np.array([10.0, 59.9, 60.0, 61.0, 150.0], np.float32), size=(300, 700),
                 p=[0.004, 0.004, 0.2, 0.3, 0.492])
    got = run(ctx, P, 60.0, n)
    want = np.array([phase.detect(tr, n_window=n) for tr in P])
    assert np.array_equal(got, want)


def test_edges(ctx):
    # trace length below the window, exactly the window, report at the last reading, NaN
    # readings, the threshold value itself, and an empty batch
    assert run(ctx, np.full((3, 24), 100.0)).tolist() == [-1, -1, -1]
    assert run(ctx, np.full((2, 25), 100.0)).tolist() == [24, 24]
    tr = np.full((1, 90), 100.0)
    tr[0, :65] = 0.0  # the qualifying window is readings 65..89, crossing a 64-reading step
    assert run(ctx, tr).tolist() == [89] == [phase.detect(tr[0])]
    tr = np.full((1, 30), 100.0)
    tr[0, 3] = np.nan
    assert run(ctx, tr).tolist() == [24]
    assert run(ctx, np.full((1, 25), 60.0)).tolist() == [24]
    empty = native.open_phase_detect(ctx, torch.empty((0, 10), dtype=torch.float32, device="cuda"))
    assert empty.numel() == 0


def test_row_stride_through_the_c_abi(ctx):
    # traces of L readings at a row stride ld > L (the binding passes contiguous rows only)
    r = np.random.default_rng(11)
    T, L, ld = 50, 777, 777 + 37
    wide = r.choice(np.array([10.0, 60.0, 150.0], np.float32), size=(T, ld), p=[0.01, 0.3, 0.69])
    dev = torch.from_numpy(wide).cuda()
    out = torch.empty(T, dtype=torch.int64, device="cuda")
    ctx.check(native.lib().open_phase_detect(ctx.handle, dev.data_ptr(), T, L, ld, 60.0, 25, out.data_ptr()))
    torch.cuda.synchronize()
    want = np.array([phase.detect(tr[:L]) for tr in wide])
    assert np.array_equal(out.cpu().numpy(), want)


def test_rejects_bad_arguments(ctx):
    P = torch.ones((2, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(native.OpenError):
        native.open_phase_detect(ctx, P, 60.0, 0)
    with pytest.raises(native.OpenError):
        native.open_phase_detect(ctx, P, float("nan"), 25)
