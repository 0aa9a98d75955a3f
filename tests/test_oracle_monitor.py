"""Pins of the monitor's step-table oracle (oracle/monitor.py) on traces
worked by hand: interval assignment to the first timestamp (half-open
intervals), samples outside every step, NaN metrics, empty steps."""
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
