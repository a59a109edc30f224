"""Pins for the FP64 oracle: checks against things the paper and mathematics
fix, independent of the oracle's own code (CPU only).

Each test names the mistake it would catch.
"""
import math
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def uniform_sigma(sigma, block=32, origin=(0, 0)):
    """Parameters under which every fragment gets the same sigma (= cap)."""
    return synth.params_dict(0.0, 0.0, -1e9, 1.0, sigma, block, origin[0], origin[1])


def scipy_blur(img2d, sigma):
    r = int(math.ceil(3.0 * sigma))
    return ndi.gaussian_filter(img2d, sigma, mode="nearest", radius=r)


def test_eq7_reproduces_printed_max_filter_sizes(orc):
    # Paper, Appendix "Algorithm Limitations": 133 / 174 / 196 px.
    rows = [l.split() for l in open(os.path.join(GOLDEN, "eq7_max_filter.txt")) if l[0] != "#"]
    for frag, taps in rows:
        assert orc.max_filter_taps(int(frag), 48000) == int(taps)


def test_plan_hand_worked_values(orc):
    p = synth.params_cfg1()
    sigma, r = orc.plan(256, 256, p)
    rows = [l.split() for l in open(os.path.join(GOLDEN, "plan_cfg1_worked.txt")) if l[0] != "#"]
    assert rows
    for bx, by, s, rad in rows:
        assert sigma[int(by), int(bx)] == pytest.approx(float(s), rel=1e-13, abs=0)
        assert r[int(by), int(bx)] == int(rad)


def test_plan_shape_and_counts(orc):
    # 256x256 in 32 px fragments: 8x8; centre fixation leaves the four central
    # fragments foveal (their midpoints are 22.6 px < 32 px from the centre).
    s, r = orc.plan(256, 256, synth.params_cfg1())
    assert r.shape == (8, 8)
    assert (r == 0).sum() == 4 and r[3:5, 3:5].max() == 0
    assert r.max() == 19
    # 1920x1080: 60 x 34 fragments (last row 24 px tall); radius capped at 48.
    s2, r2 = orc.plan(1080, 1920, synth.params_cfg2(centred=True))
    assert r2.shape == (34, 60)
    assert r2.max() == 48 and s2.max() == 16.0


def test_plan_radius_is_ceil_three_sigma(orc):
    # r = ceil(3 sigma) exactly, r = 0 iff sigma = 0 (a dropped ceil or a
    # factor 6 instead of 3 would fail).
    rng = np.random.default_rng(5)
    for _ in range(20):
        p = synth.params_dict(rng.uniform(0, 300), rng.uniform(0, 200), rng.uniform(0, 80),
                              rng.uniform(0.005, 0.2), rng.uniform(0.5, 20), int(rng.choice([8, 16, 32])))
        s, r = orc.plan(200, 300, p)
        assert np.all((r == 0) == (s == 0))
        nz = s > 0
        assert np.all(r[nz] == np.ceil(3 * s[nz]).astype(np.int32))
        assert s.max() <= p["cap"]


def test_identity_when_sigma_zero(orc):
    rng = np.random.default_rng(0)
    x = rng.random((3, 37, 53))
    for p in (synth.params_dict(10, 10, 0, 0.1, 0.0), synth.params_dict(10, 10, 1e9, 0.1, 5.0)):
        assert np.array_equal(orc.forward(x, p), x)


def test_constant_image_preserved(orc):
    # Normalisation (Appendix "Methods": filter normalised so luminance is kept).
    x = np.full((2, 70, 90), 173.25)
    for p in (synth.params_cfg1(70, 90), uniform_sigma(5.3, 16)):
        y = orc.forward(x, p)
        assert np.max(np.abs(y - 173.25)) < 1e-11


@pytest.mark.parametrize("sigma", [0.3, 0.7, 1.3, 2.9, 6.0])
@pytest.mark.parametrize("shape", [(13, 17), (40, 29)])
def test_uniform_sigma_matches_scipy(orc, sigma, shape):
    # A uniform sigma reduces block-wise foveation to an ordinary Gaussian blur
    # with truncation radius ceil(3 sigma) and clamp-to-edge ('nearest').
    rng = np.random.default_rng(1)
    img = rng.random(shape)
    y = orc.forward(img[None], uniform_sigma(sigma, block=8))[0]
    ref = scipy_blur(img, sigma)
    assert np.max(np.abs(y - ref)) < 1e-13


def test_each_fragment_is_a_full_frame_blur_restricted(orc):
    # Sec. 2: every fragment uses its own filter over the whole (clamped) frame;
    # a two-valued sigma map must equal two scipy blurs cut to their fragments.
    rng = np.random.default_rng(2)
    h, w, B = 48, 64, 16
    img = rng.random((h, w))
    nby, nbx = 3, 4
    smap = rng.choice([0.0, 0.8, 2.5, 4.0], size=(nby, nbx))
    p = synth.params_dict(0, 0, 0, 0, 10.0, B)
    y = orc.forward(img[None], p, sigma_map=smap)[0]
    for by in range(nby):
        for bx in range(nbx):
            s = smap[by, bx]
            ref = img if s == 0 else scipy_blur(img, s)
            sl = np.s_[by * B:(by + 1) * B, bx * B:(bx + 1) * B]
            assert np.max(np.abs(y[sl] - ref[sl])) < 1e-13


def test_impulse_response_is_outer_product(orc):
    # Separability (Appendix "Methods", Fig. 9): the normalised 2-D window of
    # Eq. (1) equals the outer product of two normalised 1-D windows.
    sigma = 2.2
    r = int(math.ceil(3 * sigma))
    h = w = 4 * r + 9
    x = np.zeros((1, h, w))
    x[0, h // 2, w // 2] = 1.0
    y = orc.forward(x, uniform_sigma(sigma, block=8))[0]
    imp = np.zeros(4 * r + 1)
    imp[2 * r] = 1.0
    k1 = ndi.gaussian_filter1d(imp, sigma, mode="constant", radius=r)[r:3 * r + 1]
    patch = y[h // 2 - r:h // 2 + r + 1, w // 2 - r:w // 2 + r + 1]
    assert np.max(np.abs(patch - np.outer(k1, k1))) < 1e-15
    assert abs(y.sum() - 1.0) < 1e-14


def test_grating_attenuation_matches_transfer_function(orc):
    # A cosine grating away from the edges is scaled by the discrete transfer
    # function H(f) = sum_k w_k cos(2 pi f k) of the normalised 1-D window.
    sigma, f = 3.1, 1.0 / 13.0
    r = int(math.ceil(3 * sigma))
    k = np.arange(-r, r + 1)
    wk = np.exp(-k * k / (2 * sigma * sigma))
    wk /= wk.sum()
    hf = float(np.sum(wk * np.cos(2 * np.pi * f * k)))
    h, w = 16, 160
    xs = np.arange(w)
    img = np.tile(np.cos(2 * np.pi * f * xs + 0.4), (h, 1))
    y = orc.forward(img[None], uniform_sigma(sigma, block=16))[0]
    inner = np.s_[:, r + 1:w - r - 1]
    assert np.max(np.abs(y[inner] - hf * img[inner])) < 1e-13


def test_mirror_symmetry_with_centred_fixation(orc):
    rng = np.random.default_rng(3)
    h, w, B = 96, 128, 32
    x = rng.random((2, h, w))
    p = synth.params_dict((w - 1) / 2, (h - 1) / 2, 20, 0.08, 7, B)
    y = orc.forward(x, p)
    assert np.max(np.abs(orc.forward(x[:, :, ::-1], p) - y[:, :, ::-1])) < 1e-13
    assert np.max(np.abs(orc.forward(x[:, ::-1, :], p) - y[:, ::-1, :])) < 1e-13


def test_linearity(orc):
    rng = np.random.default_rng(4)
    a, b = rng.random((2, 50, 61)), rng.random((2, 50, 61))
    p = synth.params_dict(20.3, 31.7, 5, 0.2, 6, 16)
    lhs = orc.forward(2.5 * a - 1.25 * b, p)
    rhs = 2.5 * orc.forward(a, p) - 1.25 * orc.forward(b, p)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_block_locality(orc):
    # Changing one fragment's sigma leaves every other fragment bitwise equal.
    rng = np.random.default_rng(6)
    img = rng.random((1, 64, 64))
    smap = rng.uniform(0, 3, size=(4, 4))
    p = synth.params_dict(0, 0, 0, 0, 10.0, 16)
    y0 = orc.forward(img, p, sigma_map=smap)
    smap2 = smap.copy()
    smap2[1, 2] = 5.0
    y1 = orc.forward(img, p, sigma_map=smap2)
    mask = np.ones((64, 64), bool)
    mask[16:32, 32:48] = False
    assert np.array_equal(y0[0][mask], y1[0][mask])
    assert not np.array_equal(y0[0][~mask], y1[0][~mask])


def test_forward_points_match_full_frame(orc):
    rng = np.random.default_rng(7)
    x = rng.random((3, 70, 90))
    p = synth.params_dict(30, 40, 8, 0.1, 4, 16, -5, -11)
    y = orc.forward(x, p)
    ys = rng.integers(0, 70, 50)
    xs = rng.integers(0, 90, 50)
    pts = orc.forward_points(x, p, ys, xs)
    assert np.array_equal(pts, y[:, ys, xs].T)


def test_shifted_grid_blocks(orc):
    # Fragment shift (Alg. 1, grid offset): origin (-5, -11) makes the first
    # fragment column 27 px wide and first row 21 px tall.
    p = synth.params_dict(30, 40, 8, 0.1, 4, 32, -5, -11)
    assert orc.grid(70, 90, p) == (3, 3)
    rng = np.random.default_rng(8)
    img = rng.random((70, 90))
    smap = rng.uniform(0.5, 3, size=(3, 3))
    y = orc.forward(img[None], p, sigma_map=smap)[0]
    ref = scipy_blur(img, smap[0, 0])
    assert np.max(np.abs(y[:21, :27] - ref[:21, :27])) < 1e-13
    ref = scipy_blur(img, smap[1, 1])
    assert np.max(np.abs(y[21:53, 27:59] - ref[21:53, 27:59])) < 1e-13


def test_adjoint_equals_explicit_transpose(orc):
    h, w = 20, 26
    p = synth.params_dict(7.2, 13.9, 3, 0.4, 3.5, 8, -3, -2)
    A = orc.explicit_matrix(h, w, p)
    rng = np.random.default_rng(9)
    g = rng.random((1, h, w))
    at = orc.adjoint(g, p)[0].reshape(-1)
    assert np.max(np.abs(at - A.T @ g.reshape(-1))) < 1e-13


def test_adjoint_dot_identity(orc):
    rng = np.random.default_rng(10)
    x, yv = rng.random((3, 45, 67)), rng.random((3, 45, 67))
    p = synth.params_dict(60, 5, 4, 0.3, 5, 16)
    lhs = float(np.sum(orc.forward(x, p) * yv))
    rhs = float(np.sum(x * orc.adjoint(yv, p)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_to_u8_rounds_half_even(orc):
    v = np.array([-3.0, 0.5, 1.5, 2.5, 254.5, 255.49, 300.0])
    assert orc.to_u8(v).tolist() == [0, 0, 2, 2, 254, 255, 255]


# ---- fragment shift (Alg. 1; Sec. 3) ------------------------------------------------------------

def _golden_rows(name):
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


def test_fragment_shift_hand_worked(orc):
    rows = _golden_rows("fragment_shift_worked.txt")
    assert len(rows) == 7
    for fx, fy, B, ox, oy in rows:
        p = orc.fragment_shift(synth.params_dict(float(fx), float(fy), 0, 0.1, 4, int(B)))
        assert (p["origin_x"], p["origin_y"]) == (int(ox), int(oy)), (fx, fy, B)


def test_fragment_shift_centres_a_fragment(orc):
    # brute force over fragments: some midpoint lies within half a pixel of the fixation,
    # and the origin is in (-B, 0]
    rng = np.random.default_rng(12)
    for _ in range(400):
        B = int(rng.integers(1, 65))
        fx, fy = rng.uniform(-50, 3000, size=2)
        if rng.random() < 0.3:  # exact halves
            fx, fy = np.round(fx * 2) / 2, np.round(fy * 2) / 2
        p = orc.fragment_shift(synth.params_dict(fx, fy, 0, 0.1, 4, B))
        for f, o in ((fx, p["origin_x"]), (fy, p["origin_y"])):
            assert -B < o <= 0
            mids = o + np.arange(-4, 3100 // B + 4) * B + (B - 1) / 2.0
            assert np.min(np.abs(mids - f)) <= 0.5 + 1e-12


def _translate_cols(x, k):
    """x shifted right by k columns (the first k columns repeat column 0)."""
    y = np.empty_like(x)
    y[..., k:] = x[..., :-k]
    y[..., :k] = x[..., :1]
    return y


def test_fragment_shift_makes_blur_follow_the_gaze(orc):
    # Translating frame and fixation by k pixels translates the output (away from the borders)
    # when the tiling follows the fixation; with a fixed tiling the fragments stay put and the
    # blur does not follow (Sec. 3: it would snap at fragment boundaries).
    rng = np.random.default_rng(13)
    x = rng.random((1, 80, 120))
    B, k = 16, 5
    base = synth.params_dict(50.25, 40.25, 4.0, 0.1, 2.0, B)  # r <= 6; quarter-pixel fixation
    r = 6
    shifted = dict(base, fix_x=base["fix_x"] + k)
    y0 = orc.forward(x, orc.fragment_shift(base))
    y1 = orc.forward(_translate_cols(x, k), orc.fragment_shift(shifted))
    assert np.max(np.abs(y1[..., r + k:120 - r] - y0[..., r:120 - k - r])) <= 1e-12
    z0 = orc.forward(x, base)
    z1 = orc.forward(_translate_cols(x, k), shifted)
    assert np.max(np.abs(z1[..., r + k:120 - r] - z0[..., r:120 - k - r])) > 1e-3


# ---- Geisler-Perry blur model (Appendix "Choosing the Standard Deviation", Eqs. 2-6) ------------

def test_csf_cutoff_inverts_the_contrast_threshold(orc):
    # Eq. 3 is Eq. 2 solved for CT = 1 (full contrast)
    for e in (0.0, 0.5, 2.3, 10.0, 45.0):
        assert abs(orc.csf_contrast_threshold(orc.csf_cutoff_cpd(e), e) - 1.0) <= 1e-12
    # and a slightly higher frequency needs more than full contrast
    assert orc.csf_contrast_threshold(1.01 * orc.csf_cutoff_cpd(5.0), 5.0) > 1.0


def test_csf_sigma_closed_forms(orc):
    # With f_max = f_c_deg(0): sigma = (e + e2) / (pi e2), so 1/pi at the fixation and
    # (e_corner + e2) / (pi e2) at the half-diagonal; a given f_max scales sigma by f_max / f_c_deg(0).
    h, w, ec = 1080, 1920, 30.0
    dc = math.hypot(959.5, 539.5)
    assert abs(orc.csf_sigma(0.0, h, w, ec) - 1.0 / math.pi) <= 1e-15
    assert abs(orc.csf_sigma(dc, h, w, ec) - (ec + 2.3) / (math.pi * 2.3)) <= 1e-12
    f0 = math.log(64.0) / 0.106
    assert abs(orc.csf_cutoff_cpd(0.0) - f0) <= 1e-12
    assert abs(orc.csf_sigma(dc / 2, h, w, ec, f_max=20.0) / orc.csf_sigma(dc / 2, h, w, ec) - 20.0 / f0) <= 1e-12
    # sigma is affine in the pixel distance (Eq. 5 is linear, Eq. 3 is 1/(e + e2))
    d = np.linspace(0, 1500, 7)
    s = orc.csf_sigma(d, h, w, ec)
    assert np.max(np.abs(np.diff(s, 2))) <= 1e-12


def test_csf_sigma_map_midpoints(orc):
    # 16 px fragments with a shifted grid: columns start at -5, 11, 27 (w = 30) and rows at
    # -3, 13, 29 (h = 40); midpoints worked by hand
    p = synth.params_dict(20.0, 10.0, 0, 0, 0, 16, -5, -3)
    m = orc.csf_sigma_map(40, 30, p, 20.0)
    assert m.shape == (3, 3)
    for by in range(3):
        for bx in range(3):
            cx, cy = -5 + 16 * bx + 7.5, -3 + 16 * by + 7.5
            assert abs(m[by, bx] - orc.csf_sigma(math.hypot(cx - 20.0, cy - 10.0), 40, 30, 20.0)) <= 1e-15
    assert np.all(orc.csf_sigma_map(40, 30, p, 20.0, cap=0.5) <= 0.5)


# ---- per-pixel ("perfect") foveation and SSIM (Sec. 3, Fig. 3) -----------------------------------

def test_per_pixel_equals_blockwise_with_one_pixel_fragments(orc):
    # a fragment of one pixel has its midpoint at the pixel centre
    x = synth.uniform_frames((2, 40, 52), seed=3).astype(np.float64)
    p = synth.params_dict(20.3, 14.8, 3.0, 0.15, 5.0, 1)
    assert np.max(np.abs(orc.forward_per_pixel(x, p) - orc.forward(x, p))) <= 1e-12


def test_per_pixel_uniform_sigma_matches_scipy(orc):
    # the ramp saturated at the cap everywhere: one Gaussian for the whole frame
    x = synth.uniform_frames((1, 37, 45), seed=4).astype(np.float64)
    s = 2.3
    p = synth.params_dict(10.0, 10.0, -1e6, 1.0, s)
    ref = ndi.gaussian_filter(x[0], s, mode="nearest", radius=int(math.ceil(3 * s)))
    assert np.max(np.abs(orc.forward_per_pixel(x, p)[0] - ref)) <= 1e-12


def test_ssim_definition():
    from oracle.ssim import ssim_map
    rng = np.random.default_rng(6)
    a = rng.uniform(0, 255, (40, 50))
    assert np.allclose(ssim_map(a, a), 1.0, atol=1e-12)
    b = np.clip(a + rng.normal(0, 20, a.shape), 0, 255)
    m = ssim_map(a, b)
    assert np.allclose(m, ssim_map(b, a), atol=1e-12) and np.all(m < 1.0)
    # constant images: the variance terms vanish, SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    c1 = (0.01 * 255) ** 2
    m = ssim_map(np.full((20, 20), 100.0), np.full((20, 20), 120.0))
    assert np.allclose(m, (2 * 100 * 120 + c1) / (100 ** 2 + 120 ** 2 + c1), atol=1e-12)
    # brute force at an interior pixel with the explicit 11 x 11 normalised Gaussian window
    y0, x0 = 20, 25
    k = np.exp(-np.arange(-5, 6) ** 2 / (2 * 1.5 ** 2))
    win = np.outer(k, k) / np.outer(k, k).sum()
    pa, pb = a[y0 - 5:y0 + 6, x0 - 5:x0 + 6], b[y0 - 5:y0 + 6, x0 - 5:x0 + 6]
    mx, my = (win * pa).sum(), (win * pb).sum()
    sxx, syy, sxy = (win * pa * pa).sum() - mx * mx, (win * pb * pb).sum() - my * my, (win * pa * pb).sum() - mx * my
    c2 = (0.03 * 255) ** 2
    ref = (2 * mx * my + c1) * (2 * sxy + c2) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    assert abs(ssim_map(a, b)[y0, x0] - ref) <= 1e-10
