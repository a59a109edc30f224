"""Request traces for serving: Poisson arrivals over viewer sessions, each
with its own resolution and a gaze path of saccades plus drift.

A trace is a dict of equal-length NumPy arrays, one entry per frame request,
sorted by arrival time:

* ``t``: scheduled arrival, seconds from the start of the trace;
* ``session``: which viewer the frame belongs to;
* ``h``, ``w``: frame size (the session's resolution);
* ``fix_x``, ``fix_y``: the session's gaze at that moment (pixel-centre
  coordinates);
* ``slope``: the session's ramp slope.

Gaze model: a session starts at a fixation uniform in the central half of its
frame.  Saccades come as a Poisson process (exponential gaps, mean
``saccade_mean_s``) and land uniformly in the central half; between frames the
gaze drifts by an independent normal step (``drift_px`` per axis per frame),
clamped to the frame.
"""
from __future__ import annotations

import numpy as np

from .frames import RESOLUTIONS, central_half_fixation


def poisson_trace(rate_fps: float, seconds: float, seed: int, sessions: int = 16, resolutions=RESOLUTIONS,
                  saccade_mean_s: float = 0.3, drift_px: float = 2.0, slope_range=(0.01, 0.04)):
    rng = np.random.Generator(np.random.PCG64(seed))
    # arrivals: a Poisson process of the total rate, each frame owned by a
    # session drawn uniformly (so every session is Poisson at rate/sessions)
    gaps = rng.exponential(1.0 / rate_fps, size=int(rate_fps * seconds * 1.5) + 64)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    n = t.size
    owner = rng.integers(sessions, size=n)
    res = [resolutions[int(rng.integers(len(resolutions)))] for _ in range(sessions)]
    slope = rng.uniform(slope_range[0], slope_range[1], size=sessions)
    gaze = [list(central_half_fixation(rng, h, w)) for h, w in res]
    next_saccade = rng.exponential(saccade_mean_s, size=sessions)
    out = {k: np.empty(n) for k in ("fix_x", "fix_y", "slope")}
    hs = np.empty(n, np.int64)
    ws = np.empty(n, np.int64)
    for i in range(n):
        s = int(owner[i])
        h, w = res[s]
        if t[i] >= next_saccade[s]:
            while next_saccade[s] <= t[i]:
                next_saccade[s] += rng.exponential(saccade_mean_s)
            gaze[s] = list(central_half_fixation(rng, h, w))
        else:
            dx, dy = rng.normal(0.0, drift_px, size=2)
            gaze[s][0] = min(max(gaze[s][0] + dx, 0.0), w - 1.0)
            gaze[s][1] = min(max(gaze[s][1] + dy, 0.0), h - 1.0)
        out["fix_x"][i], out["fix_y"][i] = gaze[s]
        out["slope"][i] = slope[s]
        hs[i], ws[i] = h, w
    return {"t": t, "session": owner, "h": hs, "w": ws, **out}
