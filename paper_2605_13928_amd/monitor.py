"""Workload monitor on MI355X: start / timestamp / stop / parse / plot.

The analogue of the paper's GPU monitor (Section 2) and of its CPU monitor
of the workload's process (Section 3.2).  Sampling runs in the library's
native thread (amd-smi for the GPU, /proc for the process); the step table
(each interval between consecutive timestamps assigned to the first) is the
library's `tsne_monitor_steps`.  This module opens and reads the CSV files
and draws the usage plot.

    mon = Monitor(period=0.5, device=0)
    mon.timestamp("knn")
    ...                                   # workload
    mon.timestamp("layout")
    ...
    session = mon.stop()                  # parsed: samples, events, steps
    plot_usage(session, "usage.svg")
"""
from __future__ import annotations

import ctypes as C
import os
import tempfile
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from ._lib import check

FIELDS = ("gfx_pct", "umc_pct", "vram_used_bytes", "vram_total_bytes", "temp_edge_c", "temp_hotspot_c",
          "temp_vram_c", "power_w", "proc_cpu_pct", "proc_rss_bytes", "hip_used_bytes", "sample_us")


class Monitor:
    """A running sampler; `stop()` ends it and returns the parsed Session."""

    def __init__(self, period: float = 1.0, device: int = 0, pid: int = 0, directory: str | None = None,
                 prefix: str = "monitor"):
        directory = directory or tempfile.mkdtemp(prefix="tsne_monitor_")
        os.makedirs(directory, exist_ok=True)
        self.samples_csv = os.path.join(directory, f"{prefix}_samples.csv")
        self.events_csv = os.path.join(directory, f"{prefix}_events.csv")
        self._L = _lib.load()
        h = C.c_void_p()
        check("tsne_monitor_start", self._L.tsne_monitor_start(float(period), int(device), int(pid),
                                                               self.samples_csv.encode(), self.events_csv.encode(),
                                                               C.byref(h)))
        self._h = h

    @property
    def has_gpu(self) -> bool:
        return bool(self._L.tsne_monitor_has_gpu(self._h))

    def timestamp(self, name: str) -> None:
        if self._h is None:
            raise RuntimeError("monitor stopped")
        check("tsne_monitor_timestamp", self._L.tsne_monitor_timestamp(self._h, str(name).encode()))

    def stop(self) -> "Session":
        if self._h is not None:
            check("tsne_monitor_stop", self._L.tsne_monitor_stop(self._h))
            self._h = None
        return parse(self.samples_csv, self.events_csv)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()


@dataclass
class Session:
    samples_csv: str
    events_csv: str
    t: np.ndarray                                  # sample times, s
    data: dict = field(default_factory=dict)       # field name -> values per sample
    events: list = field(default_factory=list)     # (t_s, name), "start" first, "stop" last
    steps: list = field(default_factory=list)      # one dict per interval between events


def steps_table(t, values, event_times):
    """(count [m-1], mean [m-1, f], max [m-1, f]) from the library."""
    t = np.ascontiguousarray(t, np.float64)
    values = np.ascontiguousarray(values, np.float64)
    ev = np.ascontiguousarray(event_times, np.float64)
    n, f = values.shape
    m = ev.shape[0]
    count = np.zeros(m - 1, np.int64)
    mean = np.zeros((m - 1, f))
    mx = np.zeros((m - 1, f))
    check("tsne_monitor_steps", _lib.load().tsne_monitor_steps(
        t.ctypes.data_as(C.c_void_p), values.ctypes.data_as(C.c_void_p), n, f, ev.ctypes.data_as(C.c_void_p), m,
        count.ctypes.data_as(C.c_void_p), mean.ctypes.data_as(C.c_void_p), mx.ctypes.data_as(C.c_void_p)))
    return count, mean, mx


def parse(samples_csv: str, events_csv: str) -> Session:
    raw = np.genfromtxt(samples_csv, delimiter=",", skip_header=1, dtype=np.float64, ndmin=2)
    if raw.size == 0:
        raw = np.zeros((0, 1 + len(FIELDS)))
    t = raw[:, 0].copy()
    vals = np.ascontiguousarray(raw[:, 1:])
    events = []
    with open(events_csv) as f:
        next(f)
        for line in f:
            ts, name = line.rstrip("\n").split(",", 1)
            events.append((float(ts), name))
    s = Session(samples_csv, events_csv, t, {k: vals[:, q] for q, k in enumerate(FIELDS)}, events)
    if len(events) >= 2:
        cnt, mean, mx = steps_table(t, vals, [e[0] for e in events])
        for k in range(len(events) - 1):
            row = {"name": events[k][1], "start_s": events[k][0], "end_s": events[k + 1][0],
                   "duration_s": events[k + 1][0] - events[k][0], "samples": int(cnt[k])}
            for q, name in enumerate(FIELDS):
                row[f"mean_{name}"] = float(mean[k, q])
                row[f"max_{name}"] = float(mx[k, q])
            s.steps.append(row)
    return s


def plot_usage(session: Session, path: str, width: int = 900) -> str:
    """GPU activity, VRAM, power and process CPU against time, with the
    timestamps marked, as an SVG file."""
    panels = [("gfx_pct", "GPU activity (%)", 1.0), ("hip_used_bytes", "device memory used (GB)", 1e-9),
              ("power_w", "socket power (W)", 1.0), ("proc_cpu_pct", "process CPU (%)", 1.0)]
    ph, left, top = 120, 70, 20
    height = top + len(panels) * (ph + 30) + 20
    t = session.t
    tmax = max(float(t.max()) if t.size else 1.0, session.events[-1][0] if session.events else 1.0, 1e-9)
    x = lambda v: left + (width - left - 20) * v / tmax
    out = [f'<svg xmlns="http://www.w3.org/2000/svg" width="{width}" height="{height}" font-family="sans-serif" '
           f'font-size="11">']
    for p, (key, label, scale) in enumerate(panels):
        y0 = top + p * (ph + 30)
        v = session.data.get(key, np.zeros(0)) * scale
        ok = np.isfinite(v)
        vmax = float(v[ok].max()) if ok.any() else 1.0
        vmax = vmax if vmax > 0 else 1.0
        y = lambda u: y0 + ph - ph * u / vmax
        out.append(f'<rect x="{left}" y="{y0}" width="{width - left - 20}" height="{ph}" fill="none" stroke="#999"/>')
        out.append(f'<text x="{left}" y="{y0 - 4}">{label}, max {vmax:.3g}</text>')
        pts = " ".join(f"{x(float(a)):.1f},{y(float(b)):.1f}" for a, b, o in zip(t, v, ok) if o)
        if pts:
            out.append(f'<polyline points="{pts}" fill="none" stroke="#c03" stroke-width="1.2"/>')
        for ts, name in session.events:
            out.append(f'<line x1="{x(ts):.1f}" y1="{y0}" x2="{x(ts):.1f}" y2="{y0 + ph}" stroke="#36c" '
                       f'stroke-dasharray="3,3"/>')
            if p == 0:
                out.append(f'<text x="{x(ts) + 2:.1f}" y="{y0 + 12}" fill="#36c">{name}</text>')
    out.append(f'<text x="{left}" y="{height - 4}">time (s), 0 to {tmax:.3g}</text></svg>')
    with open(path, "w") as f:
        f.write("\n".join(out))
    return path
