"""Pins of the monitor's step-table oracle (oracle/monitor.py): traces
worked by hand (interval assignment to the first timestamp, half-open
intervals, samples outside every step, NaN metrics, empty steps) and
invariants of any trace (the steps partition the event span; refining an
event splits a step's count, maximum and finite-weighted mean)."""
import math

from oracle import monitor as M


def test_hand_worked_trace():
    # samples every 0.5 s; events start 0, "load" 1.0, "pca" 2.2, stop 3.0
    t = [0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5]
    v = [[0, 10], [10, 10], [20, 30], [40, 50], [60, 70], [90, 80], [100, 100], [5, 5]]
    cnt, mean, mx = M.steps(t, v, [0.0, 1.0, 2.2, 3.0])
    assert cnt == [2, 3, 1]            # [0, 1): 0.0, 0.5; [1, 2.2): 1.0, 1.5, 2.0; [2.2, 3): 2.5
    assert mean[0] == [5.0, 10.0] and mx[0] == [10.0, 10.0]
    assert mean[1] == [40.0, 50.0] and mx[1] == [60.0, 70.0]
    assert mean[2] == [90.0, 80.0] and mx[2] == [90.0, 80.0]


def test_nan_metrics_and_empty_steps():
    nan = math.nan
    t = [0.1, 0.2, 0.3, 5.0]
    v = [[nan, 1.0], [2.0, nan], [4.0, 3.0], [7.0, 7.0]]
    cnt, mean, mx = M.steps(t, v, [0.0, 1.0, 2.0, 4.0])
    assert cnt == [3, 0, 0]            # 5.0 is past the last event
    assert mean[0] == [3.0, 2.0] and mx[0] == [4.0, 3.0]
    assert all(math.isnan(x) for x in mean[1] + mx[1] + mean[2] + mx[2])
    # a sample exactly at an event belongs to the step that event starts
    cnt, _, _ = M.steps([1.0, 2.0], [[1.0], [1.0]], [0.0, 1.0, 2.0, 3.0])
    assert cnt == [0, 1, 1]


def _trace(seed, n=200, f=3, m=7):
    # seeded trace on a 0.1 s grid; events on the same grid, so some samples
    # fall exactly on an event; a few metric values are NaN
    import numpy as np
    rng = np.random.default_rng(seed)
    t = [round(0.1 * i, 1) for i in range(n)]
    v = rng.uniform(-5.0, 50.0, (n, f))
    v[rng.random((n, f)) < 0.1] = math.nan
    ev = sorted(set(round(0.1 * int(x), 1) for x in rng.integers(0, n + 20, m)))
    return t, v.tolist(), ev


def test_counts_partition_the_event_span():
    # the steps are half-open and adjacent: their counts add up to the
    # samples in [first event, last event), each counted once
    for seed in range(20):
        t, v, ev = _trace(seed)
        if len(ev) < 2:
            continue
        cnt, _, _ = M.steps(t, v, ev)
        assert sum(cnt) == sum(1 for x in t if ev[0] <= x < ev[-1])


def test_refining_an_event_splits_a_step():
    # an extra timestamp inside a step splits it in two: counts add up, the
    # maxima combine by max, and the means combine weighted by the finite
    # samples of each part
    for seed in range(20):
        t, v, ev = _trace(seed, f=1)
        if len(ev) < 2 or ev[1] - ev[0] < 0.25:
            continue
        mid = round((ev[0] + ev[1]) / 2, 1)
        c1, m1, x1 = M.steps(t, v, [ev[0], ev[1]])
        c2, m2, x2 = M.steps(t, v, [ev[0], mid, ev[1]])
        assert c1[0] == c2[0] + c2[1]
        fin = [sum(1 for i, x in enumerate(t) if lo <= x < hi and math.isfinite(v[i][0]))
               for lo, hi in ((ev[0], mid), (mid, ev[1]))]
        parts = [(m2[k][0], x2[k][0], fin[k]) for k in range(2) if fin[k]]
        if not parts:
            assert math.isnan(m1[0][0]) and math.isnan(x1[0][0])
            continue
        assert x1[0][0] == max(p[1] for p in parts)
        whole = sum(p[0] * p[2] for p in parts) / sum(p[2] for p in parts)
        assert abs(m1[0][0] - whole) <= 1e-12 * max(1.0, abs(whole))


def test_single_step_is_the_plain_mean_and_max():
    # with all values finite and one step over the whole trace, the table is
    # the ordinary mean and max of the samples
    t = [0.0, 0.25, 0.5, 0.75]
    v = [[3.0, -1.0], [5.0, 2.0], [4.0, 8.0], [0.0, 3.0]]
    cnt, mean, mx = M.steps(t, v, [0.0, 1.0])
    assert cnt == [4]
    assert mean[0] == [3.0, 3.0] and mx[0] == [5.0, 8.0]
