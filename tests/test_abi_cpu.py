"""Host-side checks of libfoveate.so: exports, host planner, argument
validation.  No kernel runs here (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from paper_2012_08655_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "foveate.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(foveate_\w+)\s*\(", text)))


def test_library_exports_every_header_symbol():
    lib = N.lib()
    names = header_functions()
    assert "foveate_forward" in names and "foveate_backward" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in N.SIGNATURES, "binding lacks " + name


def test_version_and_error_strings():
    lib = N.lib()
    assert b"gfx950" in lib.foveate_version()
    assert isinstance(lib.foveate_last_error(), bytes)


def test_grid_matches_oracle(orc):
    lib = N.lib()
    for (h, w, B, ox, oy) in [(256, 256, 32, 0, 0), (1080, 1920, 32, 0, 0), (70, 90, 32, -5, -11),
                              (1, 1, 1, 0, 0), (33, 31, 16, -15, 0)]:
        p = synth.params_dict(0, 0, 0, 0, 0, B, ox, oy)
        nbx, nby = ctypes.c_int32(), ctypes.c_int32()
        assert lib.foveate_grid(h, w, ctypes.byref(N.make_params(p)), ctypes.byref(nbx), ctypes.byref(nby)) == 0
        assert (nby.value, nbx.value) == orc.grid(h, w, p)


def host_plan(h, w, p):
    from paper_2012_08655_amd import api
    return api.plan_host(h, w, p)


def test_host_plan_bit_identical_to_oracle(orc):
    # Same reading of the ramp, evaluated independently: sigma must agree to
    # the bit and r exactly (r = ceil(3 sigma) is discontinuous).
    rng = np.random.default_rng(11)
    cases = [(256, 256, synth.params_cfg1()), (1080, 1920, synth.params_cfg2(centred=True))]
    for _ in range(40):
        h, w = int(rng.integers(1, 900)), int(rng.integers(1, 900))
        B = int(rng.choice([1, 7, 16, 32, 64]))
        cases.append((h, w, synth.params_dict(rng.uniform(-50, w + 50), rng.uniform(-50, h + 50),
                                              rng.uniform(-10, 100), rng.uniform(0, 0.3), rng.uniform(0, 25), B,
                                              -int(rng.integers(0, B)), -int(rng.integers(0, B)))))
    for h, w, p in cases:
        s_o, r_o = orc.plan(h, w, p)
        s_h, r_h = host_plan(h, w, p)
        assert np.array_equal(r_o, r_h)
        assert np.array_equal(s_o.view(np.int64), s_h.view(np.int64))


def fake_desc(dtype, n, c, h, w, ptr=0x10000000, layout="NCHW"):
    if layout == "NCHW":
        st = (c * h * w, h * w, w, 1)
    else:
        st = (h * w * c, 1, w * c, c)
    return N.FovTensor(ptr, dtype, n, c, h, w, *st)


def call_fwd(di, do, p, np_=1):
    arr = (N.FovParams * 1)(N.make_params(p))
    return N.lib().foveate_forward(ctypes.byref(di), ctypes.byref(do), arr, np_, None)


P0 = synth.params_dict(10, 10, 5, 0.1, 4)


def test_validation_errors_before_any_device_work():
    L = N.lib()
    a = fake_desc(N.FOV_F32, 1, 3, 64, 64, 0x10000000)
    b = fake_desc(N.FOV_F32, 1, 3, 64, 64, 0x20000000)
    arr = (N.FovParams * 1)(N.make_params(P0))
    assert L.foveate_forward(None, ctypes.byref(b), arr, 1, None) == N.FOV_EINVAL
    assert L.foveate_forward(ctypes.byref(a), ctypes.byref(b), None, 1, None) == N.FOV_EINVAL
    # dtype pairs
    assert call_fwd(fake_desc(N.FOV_F32, 1, 3, 64, 64), fake_desc(N.FOV_U8, 1, 3, 64, 64, 0x20000000), P0) == N.FOV_EDTYPE
    assert call_fwd(fake_desc(7, 1, 3, 64, 64), b, P0) == N.FOV_EDTYPE
    # shapes
    assert call_fwd(a, fake_desc(N.FOV_F32, 1, 3, 64, 63, 0x20000000), P0) == N.FOV_EINVAL
    # aliasing: overlapping ranges
    assert call_fwd(a, fake_desc(N.FOV_F32, 1, 3, 64, 64, 0x10000000 + 4096), P0) == N.FOV_EALIAS
    # negative stride
    bad = fake_desc(N.FOV_F32, 1, 3, 64, 64, 0x20000000)
    bad.sw = -1
    assert call_fwd(a, bad, P0) == N.FOV_ELAYOUT
    # self-overlapping output
    ov = fake_desc(N.FOV_F32, 1, 3, 64, 64, 0x20000000)
    ov.sc = 1
    assert call_fwd(a, ov, P0) == N.FOV_ELAYOUT
    # parameters
    for key, val in [("slope", -1.0), ("cap", float("nan")), ("fix_x", float("inf")), ("block", 0),
                     ("block", 65), ("origin_x", 1), ("origin_y", -32)]:
        p = dict(P0)
        p[key] = val
        assert call_fwd(a, b, p) == N.FOV_EINVAL, key
    msg = L.foveate_last_error().decode()
    assert "origin" in msg
    # np must be n or 1
    a2 = fake_desc(N.FOV_F32, 2, 3, 64, 64, 0x10000000)
    b2 = fake_desc(N.FOV_F32, 2, 3, 64, 64, 0x20000000)
    arr3 = (N.FovParams * 3)(*(N.make_params(P0) for _ in range(3)))
    assert L.foveate_forward(ctypes.byref(a2), ctypes.byref(b2), arr3, 3, None) == N.FOV_EINVAL


def test_empty_views_are_noops():
    for dims in [(0, 3, 8, 8), (2, 0, 8, 8), (2, 3, 0, 8), (2, 3, 8, 0)]:
        a = N.FovTensor(None, N.FOV_F32, *dims, 0, 0, 0, 0)
        b = N.FovTensor(None, N.FOV_F32, *dims, 0, 0, 0, 0)
        assert call_fwd(a, b, P0) == N.FOV_OK


def test_backward_rejects_u8():
    a = fake_desc(N.FOV_U8, 1, 3, 8, 8, 0x10000000)
    b = fake_desc(N.FOV_U8, 1, 3, 8, 8, 0x20000000)
    arr = (N.FovParams * 1)(N.make_params(P0))
    assert N.lib().foveate_backward(ctypes.byref(a), ctypes.byref(b), arr, 1, None) == N.FOV_EDTYPE


def test_tuning_force_validation():
    from paper_2012_08655_amd import _native as N
    lib = N.lib()
    for bad in ((3, 64, 0, 0, 0), (1, 48, 0, 0, 0), (1, 64, 2, 0, 0), (0, 64, 0, 0, 0), (1, 64, 0, 2, 0),
                (2, 64, 0, 1, 0), (1, 64, 0, 0, 2), (1, 64, 0, 0, -1), (2, 64, 0, 0, 1)):
        t = N.FovTuning(*bad, 0.0)
        assert lib.foveate_tuning_force(ctypes.byref(t)) == N.FOV_EINVAL
    t = N.FovTuning(1, 64, 0, 1, 1, 0.0)
    assert lib.foveate_tuning_force(ctypes.byref(t)) == N.FOV_OK
    t = N.FovTuning(2, 32, 1, 0, 0, 0.0)
    assert lib.foveate_tuning_force(ctypes.byref(t)) == N.FOV_OK
    assert lib.foveate_tuning_force(None) == N.FOV_OK


def test_profile_every_validation():
    lib = N.lib()
    assert lib.foveate_profile_every(2) == N.FOV_EINVAL  # no profile window on this thread
    assert lib.foveate_profile_every(0) == N.FOV_EINVAL


def test_tuning_file_roundtrip_and_errors(tmp_path):
    from paper_2012_08655_amd import _native as N
    lib = N.lib()
    n = ctypes.c_int32()
    assert lib.foveate_tuning_clear() == N.FOV_OK
    good = tmp_path / "good.txt"
    good.write_text("# comment\n"
                    "fov-tune-v3 gfx950:sramecc+:xnack- 256 0 0 3 32 6 11 0 : 2 32 1 0 0 87.500\n"
                    "\n"
                    "fov-tune-v3 gfx950:sramecc+:xnack- 256 1 1 1 16 4 8 1 : 1 64 0 1 1 12.000\n")
    assert lib.foveate_tuning_load(str(good).encode()) == N.FOV_OK
    assert lib.foveate_tuning_count(ctypes.byref(n)) == N.FOV_OK and n.value == 2
    out = tmp_path / "out.txt"
    assert lib.foveate_tuning_save(str(out).encode()) == N.FOV_OK
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert sorted(lines) == sorted(l for l in good.read_text().splitlines() if l.startswith("fov"))
    for bad_line in ("fov-tune-v3 gfx950 256 0 0 3 32 6 11 0 : 3 32 1 0 0 1.0",      # split 3
                     "fov-tune-v3 gfx950 256 0 0 3 32 6 11 0 : 2 32 1 0 0",          # missing time
                     "fov-tune-v2 gfx950 256 0 0 3 32 6 11 0 : 2 32 1 0 1.0",        # older format
                     "fov-tune-v3 gfx950 256 0 0 3 32 6 11 0 : 2 32 1 0 0 1.0 junk",  # trailing text
                     "fov-tune-v3 gfx950 256 0 5 3 32 6 11 0 : 2 32 1 0 0 1.0",      # bad dtype
                     "fov-tune-v3 gfx950 256 0 0 3 32 6 11 0 : 2 32 1 1 0 1.0",      # merge with a split
                     "fov-tune-v3 gfx950 256 0 0 3 32 6 11 0 : 2 32 1 0 1 1.0"):     # channel items with a split
        bad = tmp_path / "bad.txt"
        bad.write_text(good.read_text() + bad_line + "\n")
        assert lib.foveate_tuning_load(str(bad).encode()) == N.FOV_EINVAL
        assert b":5:" in lib.foveate_last_error()
        assert lib.foveate_tuning_count(ctypes.byref(n)) == N.FOV_OK and n.value == 2  # unchanged
    assert lib.foveate_tuning_load(str(tmp_path / "missing.txt").encode()) == N.FOV_EINVAL
    assert lib.foveate_tuning_clear() == N.FOV_OK
    assert lib.foveate_tuning_count(ctypes.byref(n)) == N.FOV_OK and n.value == 0


def test_u8_frame_span_limit():
    # 8-bit frames are addressed with 32-bit offsets: a frame spanning 2^31 bytes is refused
    a = fake_desc(N.FOV_U8, 1, 1, 2, 64, 0x10000000)
    a.sh = 1 << 31
    b = fake_desc(N.FOV_U8, 1, 1, 2, 64, 0x10000000 + (1 << 33))
    assert call_fwd(a, b, P0) == N.FOV_EINVAL
    assert "2^31" in N.lib().foveate_last_error().decode()


def test_huge_sigma_is_refused_not_overflowed():
    # 3 sigma beyond the int range must not wrap to a small radius (a frame silently copied):
    # the host plan reports the radius bound, and forward/backward refuse the call with
    # FOV_ERANGE before any device work, for the ramp and for a sigma map (bounded by its cap)
    L = N.lib()
    h, w = 64, 64
    p = synth.params_dict(0, 0, 0, 1e9, 1e12, 32)
    _, r = host_plan(h, w, p)
    assert r.max() == 1 << 20 and r.min() > 0
    a = fake_desc(N.FOV_F32, 1, 1, h, w, 0x10000000)
    b = fake_desc(N.FOV_F32, 1, 1, h, w, 0x20000000)
    for cap in (7.3e8, 1e12, 1e300):
        pr = synth.params_dict(0, 0, 0, 1e9, cap, 32)
        assert call_fwd(a, b, pr) == N.FOV_ERANGE, cap
        arr = (N.FovParams * 1)(N.make_params(pr, sigma_map_ptr=0x30000000))
        assert L.foveate_forward(ctypes.byref(a), ctypes.byref(b), arr, 1, None) == N.FOV_ERANGE, cap
        assert L.foveate_backward(ctypes.byref(a), ctypes.byref(b), arr, 1, None) == N.FOV_ERANGE, cap
        assert b"radius" in L.foveate_last_error()


def test_fragment_shift_matches_oracle(orc):
    L = N.lib()
    rng = np.random.default_rng(21)
    ox, oy = ctypes.c_int32(), ctypes.c_int32()
    for i in range(2000):
        B = int(rng.integers(1, 65))
        fx, fy = rng.uniform(-100, 5000, size=2)
        if i % 3 == 0:
            fx, fy = np.round(fx * 2) / 2, np.round(fy * 2) / 2  # exact halves
        assert L.foveate_fragment_shift(fx, fy, B, ctypes.byref(ox), ctypes.byref(oy)) == N.FOV_OK
        ref = orc.fragment_shift(synth.params_dict(fx, fy, 0, 0.1, 4, B))
        assert (ox.value, oy.value) == (ref["origin_x"], ref["origin_y"]), (fx, fy, B)
    assert L.foveate_fragment_shift(1.0, 1.0, 0, ctypes.byref(ox), ctypes.byref(oy)) == N.FOV_EINVAL
    assert L.foveate_fragment_shift(float("nan"), 1.0, 32, ctypes.byref(ox), ctypes.byref(oy)) == N.FOV_EINVAL
    assert L.foveate_fragment_shift(1.0, 1.0, 32, None, ctypes.byref(oy)) == N.FOV_EINVAL


def test_library_shares_torchs_hip_runtime():
    # Loading the library before torch must not put a second HIP runtime in the process
    # (device pointers and streams come from torch's runtime).
    import subprocess
    import sys
    code = ("import paper_2012_08655_amd as fov; fov.load(); import torch; "
            "m = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_csf_params_reproduce_the_oracle_model(orc):
    L = N.lib()
    rng = np.random.default_rng(31)
    for _ in range(20):
        h, w = int(rng.integers(2, 2200)), int(rng.integers(2, 4000))
        ec, cap = float(rng.uniform(5, 60)), float(rng.uniform(2, 30))
        fmax = float(rng.choice([0.0, rng.uniform(10, 60)]))
        B = int(rng.choice([8, 16, 32]))
        base = synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), 0, 0, 0, B)
        p = N.make_params(base)
        assert L.foveate_csf_params(h, w, ec, fmax, cap, ctypes.byref(p)) == N.FOV_OK
        assert p.e0 < 0
        q = dict(base, e0=p.e0, slope=p.slope, cap=p.cap)
        nby, nbx = orc.grid(h, w, q)
        sig = np.zeros(nby * nbx)
        rad = np.zeros(nby * nbx, np.int32)
        arr = (N.FovParams * 1)(N.make_params(q))
        assert L.foveate_plan_host(h, w, arr, sig.ctypes.data_as(ctypes.c_void_p),
                                   rad.ctypes.data_as(ctypes.c_void_p)) == N.FOV_OK
        ref = orc.csf_sigma_map(h, w, base, ec, fmax, cap).reshape(-1)
        assert np.max(np.abs(sig - ref) / ref) <= 1e-12
        rr = np.ceil(3 * ref)
        near = np.abs(3 * ref - np.round(3 * ref)) < 1e-9
        assert np.all((rad == rr) | near)
    p = N.make_params(P0)
    assert L.foveate_csf_params(1, 1, 10.0, 0.0, 8.0, ctypes.byref(p)) == N.FOV_EINVAL
    assert L.foveate_csf_params(10, 10, 0.0, 0.0, 8.0, ctypes.byref(p)) == N.FOV_EINVAL
    assert L.foveate_csf_params(10, 10, 10.0, 0.0, 0.0, ctypes.byref(p)) == N.FOV_EINVAL
