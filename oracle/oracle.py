"""FP64 CPU oracle for block-wise foveation -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product library never loads it and
shares no code with it.

The arithmetic lives in ``fov_oracle.c`` (plain C, double precision, direct
non-separable 2-D convolution with clamp-to-edge, see its header for the
paper passages it follows).  This module compiles it, loads it with ctypes and
adds two NumPy helpers that are themselves definitions:

* :func:`explicit_matrix` -- the forward map written out as a dense matrix by
  applying it to unit impulses (tiny frames only), so its transpose can be
  compared with :func:`adjoint`.
* :func:`to_u8` -- the 8-bit output rule: round half to even, clip to 0..255.
* :func:`fragment_shift` -- the tiling origin that centres one fragment on
  the fixation (Alg. 1, Sec. 3 "SSIM"), in plain Python.
* :func:`csf_sigma` / :func:`csf_sigma_map` -- the Geisler-Perry blur model
  (Appendix "Choosing the Standard Deviation", Eqs. 2-6) evaluated step by
  step in NumPy, per distance or per fragment midpoint.

Arrays are [c, h, w] (or [n, c, h, w]) float64; frame parameters are plain
dicts with keys fix_x, fix_y, e0, slope, cap, block, origin_x, origin_y.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Mapping, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fov_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Frame(ctypes.Structure):
    _fields_ = [
        ("fix_x", ctypes.c_double),
        ("fix_y", ctypes.c_double),
        ("e0", ctypes.c_double),
        ("slope", ctypes.c_double),
        ("cap", ctypes.c_double),
        ("block", ctypes.c_int32),
        ("origin_x", ctypes.c_int32),
        ("origin_y", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile fov_oracle.c into liboracle.so (gcc, FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        fp = ctypes.POINTER(_Frame)
        lib.orc_grid.argtypes = [ctypes.c_int, ctypes.c_int, fp, ip, ip]
        lib.orc_plan.argtypes = [ctypes.c_int, ctypes.c_int, fp, dp, dp, ip]
        lib.orc_forward.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, dp, ctypes.c_int]
        lib.orc_forward_points.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, dp,
                                           ip, ip, ctypes.c_int, dp, ctypes.c_int]
        lib.orc_adjoint.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, dp, ctypes.c_int]
        lib.orc_forward_per_pixel.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, ctypes.c_int]
        lib.orc_eq7_shared_bytes.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.orc_eq7_shared_bytes.restype = ctypes.c_long
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _frame(p: Mapping) -> _Frame:
    return _Frame(float(p["fix_x"]), float(p["fix_y"]), float(p["e0"]), float(p["slope"]),
                  float(p["cap"]), int(p.get("block", 32)), int(p.get("origin_x", 0)),
                  int(p.get("origin_y", 0)))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _map_arg(sigma_map):
    if sigma_map is None:
        return None, None
    m = np.ascontiguousarray(sigma_map, dtype=np.float64)
    return m, _dptr(m)


def max_threads() -> int:
    return int(_load().orc_max_threads())


def grid(h: int, w: int, p: Mapping) -> tuple[int, int]:
    """(nby, nbx): fragment rows and columns covering an h x w frame."""
    nbx = ctypes.c_int32()
    nby = ctypes.c_int32()
    f = _frame(p)
    _load().orc_grid(h, w, ctypes.byref(f), ctypes.byref(nbx), ctypes.byref(nby))
    return nby.value, nbx.value


def fragment_shift(p: Mapping) -> dict:
    """Parameters with the tiling origin moved so that one fragment is centred
    on the fixation (Alg. 1: the fragment shift; Sec. 3: centring a single
    fragment on the fixation keeps the untouched fovea small and lets the blur
    follow the gaze instead of snapping at fragment boundaries).

    Along each axis the fragment [s, s + B) has its midpoint s + (B - 1)/2
    (pixel-centre coordinates) nearest the fixation f when s is the integer
    nearest to f - (B - 1)/2 (halves round up).  The origin is s reduced into
    (-B, 0], the range the tiling origin takes.
    """
    B = int(p.get("block", 32))
    out = dict(p)
    for axis in ("x", "y"):
        f = float(p["fix_" + axis])
        start = int(np.floor(f - (B - 1) / 2.0 + 0.5))
        o = start % B  # Python's modulo: 0 .. B-1
        out["origin_" + axis] = o - B if o > 0 else 0
    return out


# Contrast-threshold model constants the paper adopts (Eq. 2 and the text after it).
CSF_CT0 = 1.0 / 64.0
CSF_ALPHA = 0.106
CSF_E2 = 2.3


def csf_contrast_threshold(f_cpd, e_deg):
    """Eq. 2: contrast needed to detect a grating of f cycles/degree at
    eccentricity e degrees."""
    return CSF_CT0 * np.exp(CSF_ALPHA * f_cpd * (e_deg + CSF_E2) / CSF_E2)


def csf_cutoff_cpd(e_deg):
    """Eq. 3: the frequency whose threshold is full contrast (CT = 1)."""
    return CSF_E2 / (CSF_ALPHA * (e_deg + CSF_E2)) * np.log(1.0 / CSF_CT0)


def csf_sigma(d_px, h: int, w: int, e_corner: float, f_max: float = 0.0):
    """sigma (pixels) at pixel distance d from the fixation, for an h x w frame
    whose corner is e_corner degrees away (Eqs. 3-6).  f_max <= 0 takes the
    foveal cutoff f_c_deg(0) as the highest resolvable frequency."""
    if f_max <= 0:
        f_max = csf_cutoff_cpd(0.0)
    d_corner = np.hypot((w - 1) / 2.0, (h - 1) / 2.0)  # half-diagonal, pixel-centre coordinates
    e = np.asarray(d_px, dtype=np.float64) / d_corner * e_corner  # Eq. 5
    f_c_deg = csf_cutoff_cpd(e)  # Eq. 3
    f_c_pix = 0.5 * f_c_deg / f_max  # Eq. 4, cycles per pixel
    return 1.0 / (2.0 * np.pi * f_c_pix)  # Eq. 6


def csf_sigma_map(h: int, w: int, p: Mapping, e_corner: float, f_max: float = 0.0, cap: float = 1e6):
    """Per-fragment sigma [nby, nbx] from each fragment midpoint's distance to
    the fixation (midpoints as in the ramp plan), capped at cap."""
    nby, nbx = grid(h, w, p)
    B = int(p.get("block", 32))
    half = (B - 1) / 2.0
    cy = p.get("origin_y", 0) + np.arange(nby) * B + half
    cx = p.get("origin_x", 0) + np.arange(nbx) * B + half
    d = np.hypot(cx[None, :] - p["fix_x"], cy[:, None] - p["fix_y"])
    return np.minimum(csf_sigma(d, h, w, e_corner, f_max), cap)


def plan(h: int, w: int, p: Mapping, sigma_map=None) -> tuple[np.ndarray, np.ndarray]:
    """Per-fragment (sigma [nby, nbx] float64, radius [nby, nbx] int32)."""
    nby, nbx = grid(h, w, p)
    s = np.zeros((nby, nbx), np.float64)
    r = np.zeros((nby, nbx), np.int32)
    f = _frame(p)
    m, mp = _map_arg(sigma_map)
    _load().orc_plan(h, w, ctypes.byref(f), mp, _dptr(s), _iptr(r))
    return s, r


def forward(x: np.ndarray, params, sigma_map=None, nthreads: int = 0) -> np.ndarray:
    """Foveate [c,h,w] (one params dict) or [n,c,h,w] (list of n dicts)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 4:
        plist = params if isinstance(params, Sequence) and not isinstance(params, Mapping) else [params] * x.shape[0]
        maps = sigma_map if isinstance(sigma_map, (list, tuple)) else [sigma_map] * x.shape[0]
        return np.stack([forward(x[i], plist[i], maps[i], nthreads) for i in range(x.shape[0])])
    x = np.ascontiguousarray(x)
    c, h, w = x.shape
    out = np.empty_like(x)
    f = _frame(params)
    m, mp = _map_arg(sigma_map)
    _load().orc_forward(_dptr(x), _dptr(out), c, h, w, ctypes.byref(f), mp, int(nthreads))
    return out


def forward_per_pixel(x: np.ndarray, params: Mapping, nthreads: int = 0) -> np.ndarray:
    """'Perfect' foveation of a [c,h,w] frame: every pixel blurred with the
    ramp's sigma at its own distance from the fixation (Sec. 3, Fig. 3)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    c, h, w = x.shape
    out = np.empty_like(x)
    f = _frame(params)
    _load().orc_forward_per_pixel(_dptr(x), _dptr(out), c, h, w, ctypes.byref(f), int(nthreads))
    return out


def forward_points(x: np.ndarray, params: Mapping, ys, xs, sigma_map=None, nthreads: int = 0) -> np.ndarray:
    """Forward map of a [c,h,w] frame at pixels (ys[k], xs[k]); returns [npts, c]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    c, h, w = x.shape
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    assert ys.shape == xs.shape and ys.ndim == 1
    assert ys.min(initial=0) >= 0 and (len(ys) == 0 or ys.max() < h)
    assert xs.min(initial=0) >= 0 and (len(xs) == 0 or xs.max() < w)
    out = np.empty((len(ys), c), np.float64)
    f = _frame(params)
    m, mp = _map_arg(sigma_map)
    _load().orc_forward_points(_dptr(x), c, h, w, ctypes.byref(f), mp, _iptr(ys), _iptr(xs),
                               len(ys), _dptr(out), int(nthreads))
    return out


def adjoint(g: np.ndarray, params, sigma_map=None, nthreads: int = 0) -> np.ndarray:
    """Transpose of the forward map applied to [c,h,w] (or [n,c,h,w]) g."""
    g = np.asarray(g, dtype=np.float64)
    if g.ndim == 4:
        plist = params if isinstance(params, Sequence) and not isinstance(params, Mapping) else [params] * g.shape[0]
        return np.stack([adjoint(g[i], plist[i], sigma_map, nthreads) for i in range(g.shape[0])])
    g = np.ascontiguousarray(g)
    c, h, w = g.shape
    out = np.empty_like(g)
    f = _frame(params)
    m, mp = _map_arg(sigma_map)
    _load().orc_adjoint(_dptr(g), _dptr(out), c, h, w, ctypes.byref(f), mp, int(nthreads))
    return out


def explicit_matrix(h: int, w: int, params: Mapping, sigma_map=None) -> np.ndarray:
    """Dense (h*w) x (h*w) matrix A of the single-channel forward map.

    Column q is the forward map of the unit impulse at pixel q; tiny frames
    only (h*w <= 4096).
    """
    assert h * w <= 4096, "explicit matrix is for tiny frames"
    n = h * w
    eye = np.eye(n, dtype=np.float64).reshape(n, 1, h, w)
    cols = [forward(eye[q], params, sigma_map).reshape(n) for q in range(n)]
    return np.stack(cols, axis=1)


def to_u8(v: np.ndarray) -> np.ndarray:
    """8-bit output: round half to even, then clip to 0..255."""
    return np.clip(np.rint(v), 0, 255).astype(np.uint8)


def eq7_shared_bytes(frag: int, n_taps: int) -> int:
    """Eq. (7): shared-memory bytes for fragment side ``frag`` and N taps."""
    return int(_load().orc_eq7_shared_bytes(int(frag), int(n_taps)))


def max_filter_taps(frag: int, budget_bytes: int) -> int:
    """Largest filter length N (any parity, as the paper's ceil(6 sigma) may
    be even) whose Eq. (7) footprint fits the budget."""
    n = 1
    while eq7_shared_bytes(frag, n + 1) <= budget_bytes:
        n += 1
    return n
