"""Geisler-Perry blur model on the GPU: frames foveated with the ramp that
foveate_csf_params derives match the oracle, which evaluates the paper's
Eqs. 2-6 per fragment and blurs with that sigma map."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("h,w,c,ec,fmax,cap", [(200, 300, 1, 20.0, 0.0, 8.0), (150, 170, 3, 45.0, 25.0, 16.0)])
def test_csf_forward_matches_oracle_f32(fov, orc, dev, h, w, c, ec, fmax, cap):
    rng = np.random.default_rng(h + w)
    x = synth.uniform_frames((c, h, w), seed=h)
    base = synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), 0, 0, 0, 16)
    p = fov.csf_params(h, w, base, ec, fmax, cap)
    y = fov.forward(torch.from_numpy(x).to(dev), p, layout="CHW").cpu().numpy()
    smap = orc.csf_sigma_map(h, w, base, ec, fmax, cap)
    ref = orc.forward(x.astype(np.float64), dict(base, cap=cap), sigma_map=smap)  # a map is clipped to cap
    assert np.abs(y - ref).max() <= 2e-5


def test_csf_forward_u8_1080p_sampled(fov, orc, dev):
    h, w = 1080, 1920
    fr = synth.grating_frame(h, w, 3, seed=9)
    base = synth.params_dict(1100.25, 400.5, 0, 0, 0)
    p = fov.csf_params(h, w, base, 30.0, cap=16.0)
    y = fov.forward(torch.from_numpy(fr).to(dev), p, layout="HWC").cpu().numpy()
    rng = np.random.default_rng(2)
    ys, xs = rng.integers(0, h, 3000), rng.integers(0, w, 3000)
    smap = orc.csf_sigma_map(h, w, base, 30.0, cap=16.0)
    ref = orc.to_u8(orc.forward_points(fr.transpose(2, 0, 1).astype(np.float64), dict(base, cap=16.0), ys, xs,
                                       sigma_map=smap))
    d = np.abs(y[ys, xs].astype(np.int32) - ref.astype(np.int32)).max()
    assert d <= 1
