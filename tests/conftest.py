import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def dev():
    """The first GPU; skips GPU tests cleanly when none is present."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="session")
def fov(dev):
    """The product's Python binding (HIP library must be built)."""
    import paper_2012_08655_amd as fov
    fov.load()
    return fov


@pytest.fixture(scope="session")
def batch64():
    """The 64-frame mixed-resolution batch (resolutions uniform over 640x480 ..
    3840x2160, gratings + noise, central-half fixation, slope in [0.01, 0.04],
    cap 16, e0 64) and the index of its first 4K frame."""
    import synth
    frames, params = synth.batch_mixed(64, seed=3, unique_content=2)
    i4k = next(i for i, f in enumerate(frames) if f.shape[:2] == (2160, 3840))
    return frames, params, i4k


@pytest.fixture(scope="session")
def oracle_4k(orc, batch64):
    """FP64 oracle of that batch's first 4K frame, u8 HWC (computed once per
    session: about half a minute on 16 cores)."""
    import numpy as np
    frames, params, i4k = batch64
    ref = orc.forward(frames[i4k].transpose(2, 0, 1).astype(np.float64), params[i4k])
    return orc.to_u8(ref).transpose(1, 2, 0)

