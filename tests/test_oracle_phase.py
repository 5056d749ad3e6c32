"""Pins of the Algorithm 1 oracle: hand-built traces with known answers, the paper's
parameters (0.2 s sampling, 5 s window, 60 W), brute force over the window definition on
random traces, and the five 1 s intervals of the paper's window checked one by one."""
import numpy as np

from oracle import phase


def test_paper_parameters_hand_traces():
    # 0.2 s sampling, 5 s window -> 25 readings, five 1 s intervals of 5 readings
    assert phase.detect([100.0] * 25) == 24            # the first full buffer qualifies
    assert phase.detect([100.0] * 24) == -1            # never full
    assert phase.detect([30.0] * 40 + [150.0] * 25) == 64
    # a dip inside the window delays the report until the dip leaves the buffer
    tr = [150.0] * 30
    tr[10] = 59.9
    assert phase.detect(tr + [150.0] * 10) == 35
    assert phase.detect([60.0] * 25) == 24              # equal to the threshold is not below it
    assert phase.detect([59.999] * 100) == -1


def test_dip_in_each_interval_position():
    # a single dip at every offset of the last window: the report comes exactly when it leaves
    for off in range(25):
        tr = [200.0] * 25 + [200.0] * 25
        tr[25 + off] = 10.0
        assert phase.detect(tr) == 24  # the first 25 readings already qualify
        tr2 = [10.0] + [200.0] * 60
        tr2[1 + off] = 10.0
        assert phase.detect(tr2) == 1 + off + 25


def test_nan_reading_does_not_break_the_condition():
    tr = [100.0] * 25
    tr[7] = float("nan")
    assert phase.detect(tr) == 24


def test_brute_force_window_definition():
    # the report is the first t >= N-1 whose last N readings are all >= P_th (the interval
    # split cannot change which readings are looked at)
    r = np.random.default_rng(4)
    for _ in range(300):
        L = int(r.integers(1, 120))
        p = r.choice([20.0, 59.0, 60.0, 61.0, 200.0], size=L, p=[0.05, 0.05, 0.1, 0.3, 0.5])
        N = int(r.choice([5, 10, 25]))
        want = -1
        for t in range(N - 1, L):
            if (p[t - N + 1:t + 1] >= 60.0).all():
                want = t
                break
        assert phase.detect(p, n_window=N) == want


def test_interval_split_checks_the_same_readings():
    # the paper tests its window as five 1 s intervals of 5 readings; checking the intervals
    # one by one (stopping at the first interval with a reading below P_th) reports the same
    # index as the run-length evaluation
    r = np.random.default_rng(5)
    for _ in range(200):
        L = int(r.integers(1, 90))
        p = r.choice([10.0, 59.9, 60.0, 75.0, 250.0], size=L, p=[0.04, 0.04, 0.12, 0.3, 0.5])
        want = -1
        for t in range(24, L):
            window = p[t - 24:t + 1]
            if all(not (window[5 * i:5 * i + 5] < 60.0).any() for i in range(5)):
                want = t
                break
        assert phase.detect(p) == want
