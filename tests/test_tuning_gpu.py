"""Launch tuning on the GPU: every configuration (output tile split, strip
height, dispatch mode, merged pairs, per-channel items) gives bitwise the same
output as the default launch, and the autotuner caches a configuration that
later calls use."""
import itertools

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

# (split, strip rows, persistent, merge, channel split).  With 16- and 32-row strips every 8-bit
# strip is one or two 16-row blocks, so its horizontal pass runs as 4-output tasks; with 64-row
# strips most run as 8-output tasks: the bitwise comparison covers both forms.
CONFIGS = [cfg for cfg in itertools.product((1, 2, 4), (16, 32, 64), (0, 1), (0, 1), (0, 1))
           if not ((cfg[3] or cfg[4]) and cfg[0] != 1)]


def run_all_configs(fov, fn):
    base = fn()
    torch.cuda.synchronize()
    for cfg in CONFIGS:
        fov.tuning_force(*cfg)
        try:
            got = fn()
            torch.cuda.synchronize()
        finally:
            fov.tuning_force(None)
        assert torch.equal(got, base), cfg
    return base


@pytest.mark.parametrize("h,w,c,block,dtype", [(1080, 1920, 3, 32, torch.uint8), (200, 333, 1, 32, torch.float32),
                                               (97, 131, 2, 24, torch.float32), (70, 90, 1, 6, torch.float32),
                                               (40, 52, 1, 16, torch.float64)])
def test_every_config_bitwise_equal(fov, dev, orc, h, w, c, block, dtype):
    rng = np.random.default_rng(h * w)
    if dtype == torch.uint8:
        x = torch.from_numpy(synth.grating_frame(h, w, c, seed=3)).to(dev)
        p = synth.params_cfg2(rng, h, w)
    else:
        x = torch.from_numpy(synth.uniform_frames((h, w, c), seed=5, dtype=np.float64)).to(dev, dtype)
        p = synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), 4.0, 0.15, 9.0, block)
    base = run_all_configs(fov, lambda: fov.forward(x, p, layout="HWC"))
    if h * w <= 200 * 333:
        ref = orc.forward(x.double().cpu().numpy().transpose(2, 0, 1), p).transpose(1, 2, 0)
        err = np.abs(base.double().cpu().numpy() - ref).max()
        assert err <= (1e-10 if dtype == torch.float64 else 2e-5), err


def test_every_config_bitwise_equal_batch(fov, dev):
    frames, params = synth.batch_mixed(20, seed=7, resolutions=((48, 64), (120, 90), (200, 333), (31, 17)))
    ins = [torch.from_numpy(f).to(dev) for f in frames]

    def call():
        return torch.cat([o.flatten() for o in fov.forward_batch(ins, params, layout="HWC")])

    run_all_configs(fov, call)


def test_autotune_caches_and_matches(fov, dev, tmp_path):
    fov.tuning_clear()
    x = torch.from_numpy(synth.grating_frame(480, 640, 3, seed=2)).to(dev)
    p = synth.params_cfg2(np.random.default_rng(1), 480, 640)
    ref = fov.forward(x, p, layout="HWC")
    out = torch.empty_like(x)
    best = fov.autotune(x, p, out=out, layout="HWC", reps=3)
    torch.cuda.synchronize()
    assert best["split"] in (1, 2, 4) and best["strip_rows"] in (16, 32, 64) and best["persistent"] in (0, 1)
    assert best["merge"] in (0, 1)
    assert best["time_us"] > 0
    assert torch.equal(out, ref)
    assert fov.tuning_count() == 1
    assert torch.equal(fov.forward(x, p, layout="HWC"), ref)  # served from the cache
    # batch tuning adds a second workload class
    frames, params = synth.batch_mixed(18, seed=3, resolutions=((120, 90), (64, 64)))
    ins = [torch.from_numpy(f).to(dev) for f in frames]
    outs = [torch.empty_like(t) for t in ins]
    bb = fov.autotune_batch(ins, params, outs, layout="HWC", reps=2)
    assert bb["split"] in (1, 2, 4)
    plain = fov.forward_batch(ins, params, layout="HWC")
    assert all(torch.equal(a, b) for a, b in zip(outs, plain))
    assert fov.tuning_count() == 2
    path = tmp_path / "tune.txt"
    fov.tuning_save(str(path))
    fov.tuning_clear()
    assert fov.tuning_count() == 0
    fov.tuning_load(str(path))
    assert fov.tuning_count() == 2
    fov.tuning_clear()


def test_split_large_radius(fov, dev, orc):
    # r = 150 with small strips and split tiles still matches the oracle
    # (sampled pixels: the direct 2-D oracle is slow at this radius)
    x = torch.from_numpy(synth.uniform_frames((1, 400, 420), seed=8)).to(dev)
    p = synth.params_dict(0, 0, 0, 1.0, 50.0)
    rng = np.random.default_rng(4)
    ys, xs = rng.integers(0, 400, 1500), rng.integers(0, 420, 1500)
    ref = orc.forward_points(x.double().cpu().numpy(), p, ys, xs)[:, 0]
    for split, sr in ((2, 16), (4, 32)):
        fov.tuning_force(split, sr, 1)
        try:
            y = fov.forward(x, p, layout="CHW")
        finally:
            fov.tuning_force(None)
        got = y[0].double().cpu().numpy()[ys, xs]
        assert np.abs(got - ref).max() <= 2e-5
