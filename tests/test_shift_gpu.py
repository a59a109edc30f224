"""Fragment shift on the GPU: with the tiling centred on the fixation, moving
frame and gaze together by k pixels moves the foveated output by k pixels,
bit for bit away from the borders; and shifted tilings match the oracle."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def translate(x, k, axis):
    y = torch.roll(x, k, dims=axis)
    idx = [slice(None)] * x.dim()
    idx[axis] = slice(0, k)
    src = [slice(None)] * x.dim()
    src[axis] = slice(0, 1)
    y[tuple(idx)] = x[tuple(src)]
    return y


@pytest.mark.parametrize("k,axis", [(7, 1), (13, 0), (32, 1)])
def test_blur_follows_the_gaze_bitwise(fov, dev, k, axis):
    h, w = 240, 320
    x = torch.from_numpy(synth.grating_frame(h, w, 3, seed=4)).to(dev)  # HWC u8
    base = synth.params_dict(150.25, 110.75, 20.0, 0.05, 6.0)  # r <= 18, quarter-pixel gaze
    moved = dict(base)
    moved["fix_x" if axis == 1 else "fix_y"] += k
    y0 = fov.forward(x, fov.fragment_shift(base), layout="HWC")
    y1 = fov.forward(translate(x, k, axis), fov.fragment_shift(moved), layout="HWC")
    r = 18
    n = w if axis == 1 else h
    a = y1.narrow(axis, r + k, n - k - 2 * r)
    b = y0.narrow(axis, r, n - k - 2 * r)
    assert torch.equal(a, b)


def test_shifted_tiling_matches_oracle(fov, dev, orc):
    rng = np.random.default_rng(5)
    x = synth.uniform_frames((2, 150, 170), seed=6)
    for _ in range(3):
        p = fov.fragment_shift(synth.params_dict(rng.uniform(0, 169), rng.uniform(0, 149), 8.0, 0.08, 6.0,
                                                 int(rng.choice([8, 16, 32]))))
        assert p == orc.fragment_shift(p)
        got = fov.forward(torch.from_numpy(x).to(dev), p, layout="CHW").cpu().numpy()
        assert np.abs(got - orc.forward(x.astype(np.float64), p)).max() <= 2e-5
