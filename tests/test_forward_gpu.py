"""GPU parity of the forward kernel against the FP64 oracle.

Tolerances (written per test):
  f32 compute, values on [0,1]   : max abs error <= 2e-5
  u8 in, f32 out (raw 0..255)    : max abs error <= 2e-5 * 255
  u8 out                         : within 1 LSB
  f64                            : max abs error <= 1e-12
"""
import numpy as np
import pytest
import torch

import synth
from parity import assert_f32_close, assert_u8_close

pytestmark = pytest.mark.gpu

TOL_F32 = 2e-5
TOL_F64 = 1e-12


def run_chw(fov, dev, x, p, **kw):
    y = fov.forward(torch.from_numpy(np.ascontiguousarray(x)).to(dev), p, layout="CHW", **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def random_params(rng, h, w, B=None, shift=True, cap_max=12.0):
    B = int(B or rng.choice([5, 8, 16, 32, 64]))
    ox = -int(rng.integers(0, B)) if shift else 0
    oy = -int(rng.integers(0, B)) if shift else 0
    return synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), rng.uniform(0, 40),
                             rng.uniform(0.01, 0.2), rng.uniform(0.5, cap_max), B, ox, oy)


def test_device_plan_bit_identical_to_oracle(fov, orc, dev):
    rng = np.random.default_rng(21)
    cases = [(256, 256, synth.params_cfg1()), (1080, 1920, synth.params_cfg2(centred=True))]
    for _ in range(60):
        h, w = int(rng.integers(1, 2200)), int(rng.integers(1, 4000))
        cases.append((h, w, random_params(rng, h, w, cap_max=25)))
    for h, w, p in cases:
        s_d, r_d = fov.plan_device(h, w, p, device=dev)
        s_o, r_o = orc.plan(h, w, p)
        assert np.array_equal(r_d.cpu().numpy(), r_o), p
        assert np.array_equal(s_d.cpu().numpy().view(np.int64), s_o.view(np.int64)), p


def test_cfg1_full_frame_f32(fov, orc, dev):
    # 256x256 single-channel float32, U[0,1), 32 px fragments, centre fixation,
    # sigma(e) = 0 below 32 px else 0.05 (e - 32) capped at 8.
    x = synth.uniform_frames((1, 256, 256), seed=0)
    p = synth.params_cfg1()
    y = run_chw(fov, dev, x, p)
    ref = orc.forward(x.astype(np.float64), p)
    assert np.max(np.abs(y - ref)) <= TOL_F32
    # foveal fragments are copied bit for bit
    assert np.array_equal(y[:, 96:160, 96:160], x[:, 96:160, 96:160])


@pytest.mark.parametrize("seed", range(6))
def test_random_shapes_and_grids_f32(fov, orc, dev, seed):
    rng = np.random.default_rng(100 + seed)
    h, w, c = int(rng.integers(1, 180)), int(rng.integers(1, 220)), int(rng.integers(1, 4))
    x = synth.uniform_frames((c, h, w), seed=seed)
    p = random_params(rng, h, w)
    y = run_chw(fov, dev, x, p)
    ref = orc.forward(x.astype(np.float64), p)
    assert np.max(np.abs(y - ref)) <= TOL_F32, (h, w, c, p)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 2, 3), (2, 5, 3), (1, 40, 1), (3, 1, 70)])
def test_degenerate_frames(fov, orc, dev, shape):
    # frames smaller than the window: clamping folds most taps onto the edge
    x = synth.uniform_frames(shape, seed=7)
    p = synth.params_dict(0, 0, 0, 1.0, 9.0, 32)
    y = run_chw(fov, dev, x, p)
    ref = orc.forward(x.astype(np.float64), p)
    assert np.max(np.abs(y - ref)) <= TOL_F32


def test_f64_parity(fov, orc, dev):
    rng = np.random.default_rng(3)
    x = rng.random((3, 97, 141))
    p = synth.params_dict(50.0, 20.0, 10.0, 0.1, 7.0, 16, -3, -9)
    y = run_chw(fov, dev, x, p)
    ref = orc.forward(x, p)
    assert np.max(np.abs(y - ref)) <= TOL_F64


def test_u8_rgb_small_full_frame(fov, orc, dev):
    fr = synth.grating_frame(150, 260, 3, seed=4)
    p = synth.params_dict(120.0, 70.0, 20.0, 0.08, 10.0)
    t = torch.from_numpy(fr).to(dev)
    y8 = fov.forward(t, p, layout="HWC")
    yf = fov.forward(t, p, layout="HWC", out_dtype=torch.float32)
    torch.cuda.synchronize()
    ref = orc.forward(fr.transpose(2, 0, 1).astype(np.float64), p).transpose(1, 2, 0)
    assert np.max(np.abs(yf.cpu().numpy() - ref)) <= TOL_F32 * 255
    d = np.abs(y8.cpu().numpy().astype(np.int32) - orc.to_u8(ref).astype(np.int32))
    assert d.max() <= 1


def sample_points(rng, h, w, B, n):
    """Random pixels plus every fragment corner and the frame border."""
    ys = list(rng.integers(0, h, n))
    xs = list(rng.integers(0, w, n))
    for by in range(0, h, B):
        for bx in range(0, w, B):
            for dy, dx in ((0, 0), (B - 1, 0), (0, B - 1), (B - 1, B - 1)):
                ys.append(min(by + dy, h - 1))
                xs.append(min(bx + dx, w - 1))
    return np.array(ys), np.array(xs)


@pytest.mark.parametrize("fix", ["centre", "rand0", "rand1"])
def test_cfg2_full_size_sampled(fov, orc, dev, fix):
    # 1920x1080 RGB u8 gratings, 32 px fragments, sigma = 0.02 (e - 64) capped
    # at 16, in the launch configuration the benchmark times.
    fr = synth.grating_frame(1080, 1920, 3, seed=1)
    rng = np.random.default_rng({"centre": 0, "rand0": 1, "rand1": 2}[fix])
    p = synth.params_cfg2(rng, centred=(fix == "centre"))
    t = torch.from_numpy(fr).to(dev)
    y8 = fov.forward(t, p, layout="HWC")
    yf = fov.forward(t, p, layout="HWC", out_dtype=torch.float32)
    torch.cuda.synchronize()
    ys, xs = sample_points(rng, 1080, 1920, 32, 1500)
    ref = orc.forward_points(fr.transpose(2, 0, 1).astype(np.float64), p, ys, xs)
    got_f = yf.cpu().numpy()[ys, xs, :]
    assert np.max(np.abs(got_f - ref)) <= TOL_F32 * 255
    got8 = y8.cpu().numpy()[ys, xs, :].astype(np.int32)
    assert np.max(np.abs(got8 - orc.to_u8(ref).astype(np.int32))) <= 1
    # u8 output equals the rounded f32 output of the same kernel
    assert np.array_equal(y8.cpu().numpy(), np.clip(np.rint(yf.cpu().numpy()), 0, 255).astype(np.uint8))


@pytest.mark.parametrize("h", [2048, 2080])
def test_queue_item_count_around_the_held_key_limit(fov, orc, dev, h):
    # The order kernel keeps each work item's key and radius word in LDS between its two passes
    # for up to 4096 items and reads them from memory twice beyond that.  2048x2048 in 32 px
    # fragments is exactly 4096 items, 2080x2048 is 4160; both against the oracle (u8 -> f32
    # within 2e-5 on [0,1], u8 out within 1 LSB and equal to the rounded f32 output).
    fr = synth.grating_frame(h, 2048, 1, seed=h)
    rng = np.random.default_rng(h)
    p = synth.params_cfg2(rng, h=h, w=2048)
    t = torch.from_numpy(fr).to(dev)
    y8 = fov.forward(t, p, layout="HWC")
    yf = fov.forward(t, p, layout="HWC", out_dtype=torch.float32)
    torch.cuda.synchronize()
    ys, xs = sample_points(rng, h, 2048, 32, 1000)
    ref = orc.forward_points(fr.transpose(2, 0, 1).astype(np.float64), p, ys, xs)
    got_f = yf.cpu().numpy()[ys, xs, :]
    assert np.max(np.abs(got_f - ref)) <= TOL_F32 * 255
    got8 = y8.cpu().numpy()[ys, xs, :].astype(np.int32)
    assert np.max(np.abs(got8 - orc.to_u8(ref).astype(np.int32))) <= 1
    assert np.array_equal(y8.cpu().numpy(), np.clip(np.rint(yf.cpu().numpy()), 0, 255).astype(np.uint8))


@pytest.mark.parametrize("fix", ["centre", "rand0"])
def test_cfg2_full_frame(fov, orc, dev, fix):
    # Every pixel of a 1920x1080 RGB u8 frame (32 px fragments, sigma = 0.02 (e - 64) capped
    # at 16) against the oracle: u8 out within 1 LSB, u8 -> f32 out within 2e-5 on [0,1]
    # (2e-5 * 255 raw).  The u8 -> u8 call runs in the launch configuration the autotuner
    # picks for this workload, as the benchmark's timed loop does.
    fr = synth.grating_frame(1080, 1920, 3, seed=1)
    rng = np.random.default_rng({"centre": 0, "rand0": 7}[fix])
    p = synth.params_cfg2(rng, centred=(fix == "centre"))
    t = torch.from_numpy(fr).to(dev)
    y8 = torch.empty_like(t)
    fov.autotune(t, p, out=y8, layout="HWC", reps=2)
    fov.forward(t, p, out=y8, layout="HWC")
    yf = fov.forward(t, p, layout="HWC", out_dtype=torch.float32)
    torch.cuda.synchronize()
    ref = orc.forward(fr.transpose(2, 0, 1).astype(np.float64), p).transpose(1, 2, 0)
    assert_f32_close(yf.cpu().numpy(), ref, TOL_F32 * 255, "1080p u8->f32 " + fix)
    assert_u8_close(y8.cpu().numpy(), orc.to_u8(ref), "1080p u8->u8 " + fix)


def test_identity_and_constant_u8_exact(fov, dev):
    fr = synth.grating_frame(100, 130, 3, seed=5)
    t = torch.from_numpy(fr).to(dev)
    y = fov.forward(t, synth.params_dict(60, 50, 0, 0.5, 0.0), layout="HWC")
    assert torch.equal(y, t)
    const = torch.full((90, 120, 3), 201, dtype=torch.uint8, device=dev)
    y = fov.forward(const, synth.params_dict(0, 0, 0, 0.5, 16.0), layout="HWC")
    assert torch.equal(y, const)


def test_sigma_map(fov, orc, dev):
    rng = np.random.default_rng(12)
    h, w, B = 120, 200, 16
    x = synth.uniform_frames((2, h, w), seed=12)
    p = synth.params_dict(0, 0, 0, 0, 9.0, B)
    nby, nbx = orc.grid(h, w, p)
    smap = rng.uniform(-1, 11, size=(nby, nbx)).astype(np.float32)
    smap[0, 0] = np.nan
    pd = dict(p, sigma_map=torch.from_numpy(smap.reshape(-1)).to(dev))
    y = run_chw(fov, dev, x, pd)
    ref = orc.forward(x.astype(np.float64), p, sigma_map=smap.astype(np.float64))
    assert np.max(np.abs(y - ref)) <= TOL_F32


def test_batch_with_per_frame_params_and_chunking(fov, orc, dev):
    # 40 frames (more than one launch's kernel-argument capacity of 32)
    rng = np.random.default_rng(13)
    n, c, h, w = 40, 2, 70, 90
    x = synth.uniform_frames((n, c, h, w), seed=13)
    plist = [random_params(rng, h, w, B=16) for _ in range(n)]
    y = fov.forward(torch.from_numpy(x).to(dev), plist)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    for i in range(0, n, 7):
        ref = orc.forward(x[i].astype(np.float64), plist[i])
        assert np.max(np.abs(y[i] - ref)) <= TOL_F32, i


def test_layouts_agree_bitwise(fov, dev):
    fr = synth.grating_frame(64, 96, 3, seed=6)
    p = synth.params_dict(20, 30, 5, 0.1, 5)
    hwc = torch.from_numpy(fr).to(dev)
    nchw = hwc.permute(2, 0, 1).contiguous()[None]
    a = fov.forward(hwc, p, layout="HWC")
    b = fov.forward(nchw, p, layout="NCHW")
    # non-contiguous view (every other column of a wider frame)
    wide = torch.zeros((64, 192, 3), dtype=torch.uint8, device=dev)
    wide[:, ::2, :] = hwc
    c = fov.forward(wide[:, ::2, :], p, layout="HWC")
    assert torch.equal(a, b[0].permute(1, 2, 0))
    assert torch.equal(a, c)


def test_large_radius_streams_through_lds(fov, orc, dev):
    # r = 150: the tile no longer fits on chip at once and is staged in strips
    x = synth.uniform_frames((1, 40, 70), seed=14)
    p = synth.params_dict(0, 0, 0, 10.0, 50.0, 32)
    y = run_chw(fov, dev, x, p)
    ref = orc.forward(x.astype(np.float64), p)
    assert np.max(np.abs(y - ref)) <= TOL_F32


def test_radius_beyond_lds_is_refused(fov, dev):
    x = torch.zeros((1, 16, 16), device=dev)
    with pytest.raises(fov.FoveateError) as ei:
        fov.forward(x, synth.params_dict(0, 0, 0, 10.0, 400.0, 32), layout="CHW")
    assert ei.value.status == -10


@pytest.mark.parametrize("B", [64, 1, 3])
def test_extreme_blocks_f32(fov, orc, dev, B):
    # the largest fragment side and degenerate tiny ones
    rng = np.random.default_rng(400 + B)
    h, w, c = 150, 170, 2
    x = synth.uniform_frames((c, h, w), seed=B)
    p = synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), 3.0, 0.1, 12.0, B,
                          -int(rng.integers(0, B)), -int(rng.integers(0, B)))
    y = run_chw(fov, dev, x, p)
    assert np.max(np.abs(y - orc.forward(x.astype(np.float64), p))) <= TOL_F32


def test_u8_every_radius_phase(fov, orc, dev):
    # 8-bit input takes the symmetric horizontal pass, whose register rotation and
    # tail depend on r mod 4 and on (r div 4) mod 3: every radius 1..26 plus a few
    # near the 1080p cap, all fragments at one sigma (cap), ragged tiles, shifted grid.
    fr = synth.grating_frame(70, 100, 3, seed=21)
    t = torch.from_numpy(fr).to(dev)
    x64 = fr.transpose(2, 0, 1).astype(np.float64)
    for r in list(range(1, 27)) + [45, 46, 47, 48, 49, 50]:
        p = synth.params_dict(37.25, 20.5, 0.0, 100.0, (r - 0.5) / 3.0, 32, -5, -9)
        yf = fov.forward(t, p, layout="HWC", out_dtype=torch.float32)
        y8 = fov.forward(t, p, layout="HWC")
        torch.cuda.synchronize()
        ref = orc.forward(x64, p).transpose(1, 2, 0)
        err = np.max(np.abs(yf.cpu().numpy() - ref))
        assert err <= TOL_F32 * 255, (r, err)
        d = np.abs(y8.cpu().numpy().astype(np.int32) - orc.to_u8(ref).astype(np.int32))
        assert d.max() <= 1, r


def test_profile_samples_one_call_in_every(fov, dev):
    # profile_begin(n, every=k) times calls 0, k, 2k, ... of the window
    x = torch.from_numpy(synth.uniform_frames((1, 64, 96), seed=5)).to(dev)
    p = synth.params_dict(40.0, 30.0, 4.0, 0.1, 6.0)
    fov.profile_begin(8, every=3)
    for _ in range(7):
        fov.forward(x, p, layout="CHW")
    ms = fov.profile_end(8)
    assert len(ms) == 3 and np.all(ms > 0)
    fov.profile_begin(8)
    for _ in range(5):
        fov.forward(x, p, layout="CHW")
    assert len(fov.profile_end(8)) == 5
