"""Phase-transition detection (Algorithm 1), plain Python.

TEST INFRASTRUCTURE ONLY: used by the tests (and nothing in the GPU path) to produce the
expected detection index of each power trace.

Algorithm 1 samples the GPU power every delta seconds into a circular buffer of
N = W / delta readings.  Once the buffer is full, it splits the buffer into W one-second
intervals, and reports a phase transition as soon as no reading in any interval is below
the threshold P_th.  The result here is the 0-based index of the sample whose arrival
triggers the report, or -1 if the trace ends first.  The comparison is the literal
"reading < P_th", so a NaN reading never breaks the condition.
"""
from __future__ import annotations

from collections import deque


def detect(trace, n_window: int = 25, n_intervals: int = 5, threshold: float = 60.0) -> int:
    """Step through one trace as Algorithm 1 does."""
    assert n_window % n_intervals == 0
    per = n_window // n_intervals
    q = deque(maxlen=n_window)  # appending to a full deque drops the oldest reading
    for t, p in enumerate(trace):
        q.append(float(p))
        if len(q) == n_window:
            items = list(q)
            flag = True
            for i in range(n_intervals):
                interval = items[i * per:(i + 1) * per]
                if any(v < threshold for v in interval):
                    flag = False
                    break
            if flag:
                return t
    return -1


def detect_all(traces, n_window: int = 25, n_intervals: int = 5, threshold: float = 60.0):
    return [detect(tr, n_window, n_intervals, threshold) for tr in traces]
