"""Host-side checks of the monitor: the library's step table against the
oracle's on random traces; argument checks; and the sampler itself on the
CPU (no GPU: GPU columns nan, the process columns measured) -- start,
timestamps, stop, the row grid, a busy step's CPU share, parse and plot."""
import ctypes as C
import math
import os
import time

import numpy as np
import pytest

from oracle import monitor as OM
from paper_2605_13928_amd import _lib, monitor


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_steps_match_oracle(seed):
    rng = np.random.default_rng(seed)
    n, f = 400, 5
    t = np.sort(rng.uniform(0, 20, n))
    v = rng.normal(size=(n, f)) * 10
    v[rng.random((n, f)) < 0.1] = np.nan
    v[:, 4] = np.nan  # a field with no value at all
    ev = np.r_[0.5, np.sort(rng.uniform(1, 19, 6)), 19.5]
    ev[3] = ev[2]  # an empty step
    cnt, mean, mx = monitor.steps_table(t, v, ev)
    ocnt, omean, omx = OM.steps(t.tolist(), v.tolist(), ev.tolist())
    np.testing.assert_array_equal(cnt, ocnt)
    np.testing.assert_array_equal(mean, np.array(omean))  # same sums in the same order
    np.testing.assert_array_equal(mx, np.array(omx))


def test_steps_arguments():
    L = _lib.load()
    IA = _lib.TSNE_ERR_INVALID_ARG
    t = np.array([0.0, 1.0, 0.5])
    v = np.zeros((3, 1))
    ev = np.array([0.0, 2.0])
    out = [np.zeros(1, np.int64), np.zeros(1), np.zeros(1)]
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    assert L.tsne_monitor_steps(p(t), p(v), 3, 1, p(ev), 2, *map(p, out)) == IA  # t not ascending
    t[2] = 2.0
    assert L.tsne_monitor_steps(p(t), p(v), 3, 1, p(ev), 1, *map(p, out)) == IA  # one event
    assert L.tsne_monitor_steps(p(t), p(v), 3, 1, p(ev[::-1].copy()), 2, *map(p, out)) == IA
    assert L.tsne_monitor_steps(p(t), p(v), 3, 1, p(ev), 2, *map(p, out)) == 0 and out[0][0] == 2  # [0, 2)
    h = C.c_void_p()
    assert L.tsne_monitor_start(0.0, -1, 0, b"/tmp/x.csv", b"/tmp/y.csv", C.byref(h)) == IA
    assert L.tsne_monitor_start(1.0, -1, 0, b"/nonexistent/dir/x.csv", b"/tmp/y.csv", C.byref(h)) == IA
    assert L.tsne_monitor_timestamp(None, b"x") == IA and L.tsne_monitor_stop(None) == IA


def test_sampler_on_cpu(tmp_path):
    mon = monitor.Monitor(period=0.05, device=-1, directory=str(tmp_path))
    assert not mon.has_gpu
    time.sleep(0.3)
    mon.timestamp("busy, loop")  # the comma becomes '_'
    t_end = time.perf_counter() + 0.4
    x = 0
    while time.perf_counter() < t_end:
        x += 1
    mon.timestamp("idle")
    time.sleep(0.4)
    s = mon.stop()
    names = [e[1] for e in s.events]
    assert names == ["start", "busy_ loop", "idle", "stop"]
    assert np.all(np.diff([e[0] for e in s.events]) >= 0)
    assert len(s.t) >= 10 and np.all(np.diff(s.t) > 0)
    # rows on the 0.05 s grid (the last one is taken at stop); the bounds
    # leave room for a loaded host
    assert abs(np.median(np.diff(s.t[:-1])) - 0.05) < 0.02
    assert np.all(np.isnan(s.data["gfx_pct"])) and np.all(np.isnan(s.data["power_w"]))
    assert np.all(np.isnan(s.data["hip_used_bytes"]))
    assert np.nanmin(s.data["proc_rss_bytes"]) > 1e6
    steps = {r["name"]: r for r in s.steps}
    assert set(steps) == {"start", "busy_ loop", "idle"}
    assert steps["busy_ loop"]["mean_proc_cpu_pct"] > 25.0
    assert steps["idle"]["mean_proc_cpu_pct"] < steps["busy_ loop"]["mean_proc_cpu_pct"]
    assert math.isnan(steps["idle"]["mean_gfx_pct"])
    assert abs(steps["busy_ loop"]["duration_s"] - 0.4) < 0.15
    svg = monitor.plot_usage(s, str(tmp_path / "usage.svg"))
    assert os.path.getsize(svg) > 1000 and open(svg).read().startswith("<svg")
