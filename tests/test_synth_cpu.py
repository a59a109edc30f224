"""Properties of the seeded request traces used by the serving benchmark."""
import numpy as np

import synth


def test_poisson_trace_properties():
    tr = synth.poisson_trace(480.0, 4.0, seed=3)
    t = tr["t"]
    n = t.size
    assert np.all(np.diff(t) >= 0) and t[-1] < 4.0
    assert abs(n - 480 * 4) < 5 * np.sqrt(480 * 4)  # Poisson count within 5 sd
    assert set(np.unique(tr["session"])) <= set(range(16))
    res = set(zip(tr["h"].tolist(), tr["w"].tolist()))
    assert res <= set(synth.frames.RESOLUTIONS)
    assert np.all((tr["fix_x"] >= 0) & (tr["fix_x"] <= tr["w"] - 1))
    assert np.all((tr["fix_y"] >= 0) & (tr["fix_y"] <= tr["h"] - 1))
    assert np.all((tr["slope"] >= 0.01) & (tr["slope"] <= 0.04))
    # one resolution and one slope per session
    for s in np.unique(tr["session"]):
        m = tr["session"] == s
        assert len(set(tr["h"][m])) == 1 and len(set(tr["slope"][m])) == 1
    # deterministic for a seed
    tr2 = synth.poisson_trace(480.0, 4.0, seed=3)
    assert all(np.array_equal(tr[k], tr2[k]) for k in tr)


def test_gaze_drift_and_saccades():
    tr = synth.poisson_trace(1920.0, 6.0, seed=5, sessions=1, resolutions=((2160, 3840),))
    step = np.hypot(np.diff(tr["fix_x"]), np.diff(tr["fix_y"]))
    small = step < 20  # drift steps: |N(0, 2^2 I)| rarely exceeds 20 px
    assert 0.9 < small.mean() < 1.0
    # saccades: roughly 6 s / 0.3 s = 20 big jumps
    assert 5 <= int((step > 100).sum()) <= 45
    assert abs(np.std(np.diff(tr["fix_x"])[small]) - 2.0) < 0.3
