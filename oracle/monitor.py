"""Reference of the monitor's step table (test infrastructure only: imported
by the tests and nothing else).

The paper's workflow monitor (Section 2, and the caption of Figure 1)
records timestamps between code phases and assigns each interval between
consecutive timestamps to the first of the two: step k runs from event k to
event k + 1.  Per step, over the samples whose time t satisfies
e_k <= t < e_{k+1}: the sample count and, per metric, the mean and the
maximum of the finite values (NaN when there are none, as for a metric the
device does not report).  Samples before the first event or at/after the
last are in no step.  Plain loops over the samples, in order.
"""
from __future__ import annotations

import math


def steps(t, values, events):
    """t: sample times [n] ascending; values: [n][f] rows; events: event
    times [m] ascending.  Returns (count [m-1], mean [m-1][f], max [m-1][f])."""
    m = len(events)
    f = len(values[0]) if len(values) else 0
    counts, means, maxs = [], [], []
    for k in range(m - 1):
        lo, hi = events[k], events[k + 1]
        cnt = 0
        s = [0.0] * f
        c = [0] * f
        mx = [-math.inf] * f
        for i in range(len(t)):
            if lo <= t[i] < hi:
                cnt += 1
                for q in range(f):
                    v = float(values[i][q])
                    if math.isfinite(v):
                        s[q] += v
                        c[q] += 1
                        mx[q] = max(mx[q], v)
        counts.append(cnt)
        means.append([s[q] / c[q] if c[q] else math.nan for q in range(f)])
        maxs.append([mx[q] if c[q] else math.nan for q in range(f)])
    return counts, means, maxs
