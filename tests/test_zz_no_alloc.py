"""The allocation-free forward entry point (foveate_forward_noalloc) on the GPU.

It runs the kernels of foveate_forward with the plan workspace in the
library's fixed device array, so its outputs must be bitwise those of
foveate_forward (which the other GPU tests hold to the oracle: u8 within
1 LSB, f32 within 2e-5, f64 within 1e-12).  Calls follow each other on one
stream, each smaller than the one before, so a call that read anything an
earlier, larger call left in the array would show up here; the smallest one is
also compared with the oracle directly.
"""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_2012_08655_amd import _native as N
from paper_2012_08655_amd import api
from parity import assert_f32_close, assert_u8_close

pytestmark = pytest.mark.gpu


def call_noalloc(x, out, params, layout):
    """One call through the C ABI; returns its status."""
    di, do = api.tensor_desc(x, layout), api.tensor_desc(out, layout)
    arr, npar, _keep = api._params_array(params, di.n)
    return N.lib().foveate_forward_noalloc(ctypes.byref(di), ctypes.byref(do), arr, npar,
                                           api._stream_handle(None))


def test_u8_frames_two_calls_second_smaller(fov, orc, dev):
    rng = np.random.default_rng(41)
    big = torch.from_numpy(synth.grating_frame(1080, 1920, 3, seed=41)).to(dev)
    small = torch.from_numpy(synth.grating_frame(480, 640, 3, seed=42)).to(dev)
    p_big = synth.params_cfg2(rng)
    p_small = synth.params_cfg2(rng, h=480, w=640)
    y_big = torch.full_like(big, 7)
    y_small = torch.full_like(small, 7)
    print("noalloc u8: 1080x1920x3 then 480x640x3", flush=True)
    assert call_noalloc(big, y_big, p_big, "HWC") == N.FOV_OK, N.lib().foveate_last_error()
    assert call_noalloc(small, y_small, p_small, "HWC") == N.FOV_OK, N.lib().foveate_last_error()
    ref_big = fov.forward(big, p_big, layout="HWC")
    ref_small = fov.forward(small, p_small, layout="HWC")
    torch.cuda.synchronize()
    assert torch.equal(y_big, ref_big)
    assert torch.equal(y_small, ref_small)
    fr = small.cpu().numpy()
    ref = orc.to_u8(orc.forward(fr.transpose(2, 0, 1).astype(np.float64), p_small)).transpose(1, 2, 0)
    assert_u8_close(y_small.cpu().numpy(), ref, "noalloc 480x640 u8")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_float_batches_two_calls_second_smaller(fov, orc, dev, dtype):
    rng = np.random.default_rng(43)
    x_big = torch.from_numpy(synth.uniform_frames((4, 3, 224, 224), seed=43)).to(dev, dtype)
    x_small = torch.from_numpy(synth.uniform_frames((2, 1, 96, 130), seed=44)).to(dev, dtype)
    p_big = [synth.params_cfg5(rng, 224, 224) for _ in range(4)]
    p_small = [synth.params_dict(60.0, 40.0, 8.0, 0.2, 5.0, 16, -3, -9),
               synth.params_dict(10.0, 90.0, 0.0, 0.1, 3.0, 32)]
    y_big = torch.full_like(x_big, 7.0)
    y_small = torch.full_like(x_small, 7.0)
    print("noalloc %s: 4x3x224x224 then 2x1x96x130" % dtype, flush=True)
    assert call_noalloc(x_big, y_big, p_big, "NCHW") == N.FOV_OK, N.lib().foveate_last_error()
    assert call_noalloc(x_small, y_small, p_small, "NCHW") == N.FOV_OK, N.lib().foveate_last_error()
    ref_big = fov.forward(x_big, p_big, layout="NCHW")
    ref_small = fov.forward(x_small, p_small, layout="NCHW")
    torch.cuda.synchronize()
    assert torch.equal(y_big, ref_big)
    assert torch.equal(y_small, ref_small)
    xs = x_small.cpu().numpy().astype(np.float64)
    tol = 2e-5 if dtype == torch.float32 else 1e-12
    for i in range(2):
        assert_f32_close(y_small[i].cpu().numpy(), orc.forward(xs[i], p_small[i]), tol, "noalloc frame %d" % i)


def test_limits_are_refused_before_any_launch(fov, dev):
    # more than 16 frames
    x = torch.zeros((17, 1, 8, 8), device=dev)
    y = torch.full_like(x, 3.0)
    assert call_noalloc(x, y, synth.params_dict(4.0, 4.0, 0.0, 0.5, 2.0, 4), "NCHW") == N.FOV_EINVAL
    assert b"at most 16 frames" in N.lib().foveate_last_error()
    # a plan workspace beyond the array: 3840x2160 in 4 px fragments (518,400 fragments of taps)
    big = torch.zeros((2160, 3840, 3), dtype=torch.uint8, device=dev)
    out = torch.full_like(big, 9)
    p = synth.params_cfg2(np.random.default_rng(45), h=2160, w=3840)
    p["block"] = 4
    assert call_noalloc(big, out, p, "HWC") == N.FOV_EINVAL
    assert b"bytes of plan workspace" in N.lib().foveate_last_error()
    torch.cuda.synchronize()
    assert bool((y == 3.0).all()) and bool((out == 9).all())  # nothing was launched
    # and the entry point still works afterwards
    x2 = torch.from_numpy(synth.uniform_frames((1, 64, 64), seed=46)).to(dev)
    y2 = torch.empty_like(x2)
    p2 = synth.params_dict(20.0, 30.0, 4.0, 0.3, 4.0, 16)
    assert call_noalloc(x2, y2, p2, "CHW") == N.FOV_OK
    ref2 = fov.forward(x2, p2, layout="CHW")
    torch.cuda.synchronize()
    assert torch.equal(y2, ref2)
