"""Quality of block-wise foveation against per-pixel ("perfect") foveation,
the paper's SSIM comparison (Sec. 3, Fig. 3) on synthetic frames: the GPU's
block-wise output for fragment sizes 8/16/32/64, with and without the
fragment shift, against the oracle's per-pixel foveation, SSIM maps averaged
over several frames with the same central fixation."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle.ssim import ssim_map

pytestmark = pytest.mark.gpu

H, W, NFRAMES = 540, 960, 4


@pytest.fixture(scope="module")
def study(fov, orc, dev):
    base = synth.params_dict((W - 1) / 2.0, (H - 1) / 2.0, 64.0, 0.02, 16.0)
    maps = {}
    for i in range(NFRAMES):
        fr = synth.grating_frame(H, W, 3, seed=40 + i)
        ref = orc.to_u8(orc.forward_per_pixel(fr.transpose(2, 0, 1).astype(np.float64), base))
        x = torch.from_numpy(fr).to(dev)
        for B in (8, 16, 32, 64):
            for shift in (False, True):
                p = dict(base, block=B)
                if shift:
                    p = fov.fragment_shift(p)
                y = fov.forward(x, p, layout="HWC").cpu().numpy().transpose(2, 0, 1)
                m = np.mean([ssim_map(y[c], ref[c]) for c in range(3)], axis=0)
                maps.setdefault((B, shift), []).append(m)
    out = {}
    for key, ms in maps.items():
        avg = np.mean(ms, axis=0)
        out[key] = (float(avg.mean()), float(avg.min()))
    summary = {"%d%s" % (B, "_shift" if s else ""): {"mean": round(v[0], 5), "min_of_average_map": round(v[1], 5)}
               for (B, s), v in sorted(out.items())}
    print("quality", json.dumps(summary))
    dest = os.environ.get("FOV_QUALITY_JSON")  # optional copy of the study's numbers
    if dest:
        with open(dest, "w") as f:
            json.dump({"frames": NFRAMES, "size": [H, W], "params": base, "ssim": summary}, f, indent=1)
    return out


def test_ssim_falls_as_fragments_grow(study):
    means = [study[(B, False)][0] for B in (8, 16, 32, 64)]
    assert all(a > b for a, b in zip(means, means[1:])), means
    assert study[(32, False)][0] >= 0.99


def test_fragment_shift_raises_the_worst_region(study):
    # the shift centres a fragment on the fixation (Sec. 3): the weakest part of the
    # averaged map, near the fovea, improves
    assert study[(32, True)][1] > study[(32, False)][1]
    assert study[(16, True)][1] > study[(16, False)][1]
