"""Phase-transition detection (Algorithm 1, Section III-B.2), plain Python.

TEST INFRASTRUCTURE ONLY: used by the tests (and nothing in the GPU path) to produce the
expected detection index of each power trace.

The paper samples the GPU power at a fixed interval and declares that the application has
left its CPU-bound start-up phase once every reading of the most recent window (5 s, that
is N = 25 readings at 0.2 s) is at or above the power threshold P_th (60 W).  Splitting that
window into 1 s intervals, as the paper does, cannot change which readings are tested, so the
condition is simply: the last N readings are all >= P_th.  The report comes at the first
reading at which that holds.

Here it is evaluated from the length of the current run of readings that are not below the
threshold: a reading below P_th resets the run, any other reading extends it, and the first
index at which the run reaches N is the result (-1 when the trace ends first).  "Below" is the
literal comparison p < P_th, so a NaN reading does not reset the run.
"""
from __future__ import annotations


def detect(trace, n_window: int = 25, threshold: float = 60.0) -> int:
    """0-based index of the reading that completes the first window of n_window readings
    that are all >= threshold, or -1."""
    assert n_window >= 1
    run = 0
    for t, p in enumerate(trace):
        run = 0 if float(p) < threshold else run + 1
        if run >= n_window:
            return t
    return -1


def detect_all(traces, n_window: int = 25, threshold: float = 60.0):
    return [detect(tr, n_window, threshold) for tr in traces]
