"""GPU tests of the batched launch: frames of mixed sizes in one persistent
launch over a global, cost-ordered fragment queue.

Each frame's result must equal (bitwise) the same frame foveated alone, and
match the FP64 oracle within 1 LSB (u8) / 2e-5 (f32 on [0,1]).
"""
import numpy as np
import pytest
import torch

import synth
from parity import assert_u8_close

pytestmark = pytest.mark.gpu


def small_batch(n, seed):
    rng = np.random.default_rng(seed)
    shapes = [(48, 64), (90, 120), (33, 200), (128, 96), (7, 5)]
    frames, params = [], []
    for i in range(n):
        h, w = shapes[int(rng.integers(len(shapes)))]
        frames.append(synth.grating_frame(h, w, 3, seed=seed * 100 + i))
        params.append(synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), rng.uniform(0, 30),
                                        rng.uniform(0.02, 0.2), rng.uniform(1, 12), int(rng.choice([8, 16, 32]))))
    return frames, params


@pytest.mark.parametrize("n", [3, 16, 40])
def test_batch_matches_alone_and_oracle(fov, orc, dev, n):
    frames, params = small_batch(n, seed=n)
    ins = [torch.from_numpy(f).to(dev) for f in frames]
    outs = fov.forward_batch(ins, params, layout="HWC")
    alone = [fov.forward(t, p, layout="HWC") for t, p in zip(ins, params)]
    torch.cuda.synchronize()
    for i in range(n):
        assert torch.equal(outs[i], alone[i]), i
        if i % 5 == 0:
            ref = orc.to_u8(orc.forward(frames[i].transpose(2, 0, 1).astype(np.float64), params[i]))
            d = np.abs(outs[i].cpu().numpy().astype(np.int32) - ref.transpose(1, 2, 0).astype(np.int32))
            assert d.max() <= 1, i


def test_batch_float_frames(fov, orc, dev):
    rng = np.random.default_rng(5)
    frames = [synth.uniform_frames((2, int(rng.integers(10, 80)), int(rng.integers(10, 90))), seed=i)
              for i in range(20)]
    params = [synth.params_dict(rng.uniform(0, 50), rng.uniform(0, 50), 5, 0.15, 6, 16) for _ in frames]
    ins = [torch.from_numpy(f).to(dev) for f in frames]
    outs = fov.forward_batch(ins, params, layout="CHW")
    torch.cuda.synchronize()
    for i in (0, 7, 19):
        ref = orc.forward(frames[i].astype(np.float64), params[i])
        assert np.max(np.abs(outs[i].cpu().numpy() - ref)) <= 2e-5


def test_batch_rejects_mixed_dtypes_and_overlap(fov, dev):
    a = torch.zeros((16, 16, 3), dtype=torch.uint8, device=dev)
    b = torch.zeros((16, 16, 3), dtype=torch.float32, device=dev)
    p = synth.params_dict(8, 8, 0, 0.1, 3)
    with pytest.raises(fov.FoveateError):
        fov.forward_batch([a, b], [p, p], layout="HWC")
    big = torch.zeros((32, 16, 3), dtype=torch.uint8, device=dev)
    x = torch.zeros((16, 16, 3), dtype=torch.uint8, device=dev)
    with pytest.raises(fov.FoveateError) as ei:
        # frame 1 writes into frame 0's input
        fov.forward_batch([big[:16], x], [p, p], outs=[torch.empty_like(x), big[8:24]], layout="HWC")
    assert ei.value.status == -4


def test_mixed_resolution_batch_of_64(fov, orc, dev, batch64, oracle_4k):
    # 64 frames, resolution uniform over {640x480, 1280x720, 1920x1080,
    # 3840x2160}, gratings + noise, fixation uniform in the central half,
    # slope uniform in [0.01, 0.04], cap 16, e0 64 px.
    frames, params, i4k = batch64
    ins = [torch.from_numpy(f).to(dev) for f in frames]
    outs = fov.forward_batch(ins, params, layout="HWC")
    torch.cuda.synchronize()
    # a whole 4K frame of the mix, element by element against the oracle
    assert_u8_close(outs[i4k].cpu().numpy(), oracle_4k, "4K frame %d in the batch" % i4k)
    rng = np.random.default_rng(0)
    checked = set()
    for i in range(64):
        h, w = frames[i].shape[:2]
        if (h, w) in checked:
            continue
        checked.add((h, w))
        alone = fov.forward(ins[i], params[i], layout="HWC")
        torch.cuda.synchronize()
        assert torch.equal(outs[i], alone), i
        ys, xs = rng.integers(0, h, 300), rng.integers(0, w, 300)
        ref = orc.to_u8(orc.forward_points(frames[i].transpose(2, 0, 1).astype(np.float64), params[i], ys, xs))
        got = outs[i].cpu().numpy()[ys, xs, :]
        assert np.max(np.abs(got.astype(np.int32) - ref.astype(np.int32))) <= 1, (i, h, w)


@pytest.mark.parametrize("chan_split", [0, 1])
def test_batch_mixed_channel_counts(fov, orc, dev, chan_split):
    # frames of 1, 2 and 4 channels in one launch: per-channel items of the small radii go up to
    # the largest channel count, and frames with fewer channels skip the rest
    rng = np.random.default_rng(31)
    frames, params = [], []
    for i, c in enumerate((1, 4, 2, 1, 4, 2, 4)):
        h, w = int(rng.integers(20, 90)), int(rng.integers(20, 110))
        frames.append(synth.uniform_frames((c, h, w), seed=40 + i))
        params.append(synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), 2.0, 0.2, 8.0, 16))
    ins = [torch.from_numpy(f).to(dev) for f in frames]
    fov.tuning_force(1, 64, 0, 0, chan_split)
    try:
        outs = fov.forward_batch(ins, params, layout="CHW")
        alone = [fov.forward(t, p, layout="CHW") for t, p in zip(ins, params)]
        torch.cuda.synchronize()
    finally:
        fov.tuning_force(None)
    for i in range(len(frames)):
        assert torch.equal(outs[i], alone[i]), i
        ref = orc.forward(frames[i].astype(np.float64), params[i])
        assert np.max(np.abs(outs[i].cpu().numpy() - ref)) <= 2e-5, i
