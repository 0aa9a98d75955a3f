"""The monitor on the GPU: amd-smi columns sampled for the HIP device, and
the step table sees the phases of a workload -- an 8 GB allocation in VRAM
used, the all-pairs gradient kernel in the graphics activity -- with each
sample's cost and the grid of rows checked."""
import time

import numpy as np
import pytest
import torch

from helpers import random_graph_P, say, sparse_to_dev, to_dev
from paper_2605_13928_amd import api, monitor, synth

pytestmark = pytest.mark.gpu


def test_monitor_sees_workload_phases(dev, tmp_path):
    say("monitor phases")
    _, _, _, S = random_graph_P(20_000, 90, 30.0, 3)
    P = sparse_to_dev(S, dev)
    Y = to_dev(synth.random_embedding(20_000, 10.0, 4), dev)
    api.kl_grad(Y, P, 1.0)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # so that the 8 GB below is a new device allocation, not torch's cache
    mon = monitor.Monitor(period=0.05, device=dev.index or 0, directory=str(tmp_path))
    assert mon.has_gpu
    time.sleep(0.5)
    mon.timestamp("alloc")
    x = torch.ones(8 << 30, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    time.sleep(0.5)
    mon.timestamp("compute")
    t_end = time.perf_counter() + 1.5
    while time.perf_counter() < t_end:
        for _ in range(50):
            api.kl_grad(Y, P, 1.0)
        torch.cuda.synchronize()
    mon.timestamp("release")
    del x
    torch.cuda.empty_cache()
    time.sleep(0.5)
    s = mon.stop()
    st = {r["name"]: r for r in s.steps}
    for r in s.steps:
        say(r["name"], f"{r['duration_s']:.2f} s", r["samples"], "samples, gfx mean/max",
            r["mean_gfx_pct"], r["max_gfx_pct"], "VRAM max GB (amd-smi, HIP)", r["max_vram_used_bytes"] / 1e9, r["max_hip_used_bytes"] / 1e9,
            "power mean/max", r["mean_power_w"], r["max_power_w"], "hotspot max", r["max_temp_hotspot_c"])
    say("events", [(round(t, 3), n) for t, n in s.events])
    say("hip_used GB", [(round(float(t), 3), round(float(v) / 1e9, 2)) for t, v in zip(s.t, s.data["hip_used_bytes"])])
    assert [e[1] for e in s.events] == ["start", "alloc", "compute", "release", "stop"]
    assert abs(np.median(np.diff(s.t[:-1])) - 0.05) < 0.01
    assert np.isfinite(s.data["vram_total_bytes"]).all() and s.data["vram_total_bytes"][0] > 200e9
    assert np.isfinite(s.data["gfx_pct"]).all() and np.isfinite(s.data["hip_used_bytes"]).all()
    assert st["alloc"]["max_hip_used_bytes"] >= st["start"]["max_hip_used_bytes"] + 7.5e9
    assert st["release"]["samples"] > 0
    assert s.data["hip_used_bytes"][-1] <= st["alloc"]["max_hip_used_bytes"] - 7.5e9
    # amd-smi's own VRAM figure is recorded too but not checked: it trails
    # frees by seconds (it read 15 GB here while HIP reported 1.8 GB)
    # the device's activity and power are running averages that trail the
    # load by a fraction of a second: the compute phase reaches full activity
    assert st["compute"]["max_gfx_pct"] >= 50.0 and st["compute"]["mean_gfx_pct"] > st["start"]["mean_gfx_pct"]
    assert st["compute"]["max_power_w"] > st["start"]["mean_power_w"]
    p = s.data["power_w"]
    assert np.isfinite(p).any() and np.nanmax(p) > 0
    h = s.data["temp_hotspot_c"]
    assert np.isfinite(h).any() and 0 < np.nanmax(h) < 125
    assert np.median(s.data["sample_us"]) < 20_000  # one sample costs well under the period
