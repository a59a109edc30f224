"""GPU tests of the host-to-host pipeline: distinct frames with their own
sizes and gaze go from host memory through the GPU and back, several frames
in flight, every device slot reused; each host output must equal (bitwise)
foveate_forward of that frame on the device and match the FP64 oracle
(within 1 LSB for u8, 2e-5 on [0,1] for f32), element by element."""
import numpy as np
import pytest
import torch

import synth
from paper_2012_08655_amd.pipeline import HostPipeline
from parity import assert_f32_close, assert_u8_close

pytestmark = pytest.mark.gpu


def frames_and_params(n, seed, shapes):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h, w = shapes[i % len(shapes)]
        fr = synth.grating_frame(h, w, 3, seed=seed * 1000 + i)
        p = synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), rng.uniform(0, 30),
                              rng.uniform(0.02, 0.12), rng.uniform(2, 16))
        out.append((fr, p))
    return out


def oracle_u8(orc, fr, p):
    return orc.to_u8(orc.forward(fr.transpose(2, 0, 1).astype(np.float64), p)).transpose(1, 2, 0)


@pytest.mark.parametrize("depth", [1, 3])
def test_pipeline_distinct_frames(fov, orc, dev, depth):
    # 11 frames of five sizes through `depth` slots: every slot is reused, and frames of
    # different sizes follow each other in one slot
    items = frames_and_params(11, seed=5 + depth, shapes=((120, 160), (200, 333), (64, 64), (31, 47), (240, 320)))
    hin = [torch.from_numpy(f).pin_memory() for f, _ in items]
    cap = max(f.nbytes for f, _ in items)
    with HostPipeline(cap, depth=depth) as pl:
        tickets = [pl.submit(x, p) for x, (_, p) in zip(hin, items)]
        outs = [pl.wait(t) for t in tickets]
    for i, (x, (fr, p)) in enumerate(zip(hin, items)):
        dev_out = fov.forward(x.to(dev), p, layout="HWC")
        torch.cuda.synchronize()
        assert torch.equal(outs[i], dev_out.cpu()), i
        assert_u8_close(outs[i].numpy(), oracle_u8(orc, fr, p), "pipeline frame %d" % i)


def test_pipeline_interleaved_f32_pageable(fov, orc, dev):
    # u8 CHW frames into f32 outputs, pageable (not pinned) host memory, frames waited for
    # in an order other than submission, a query before the wait
    rng = np.random.default_rng(9)
    frames = [synth.grating_frame(int(rng.integers(40, 150)), int(rng.integers(40, 200)), 3, seed=70 + i)
              .transpose(2, 0, 1).copy() for i in range(7)]
    params = [synth.params_dict(rng.uniform(0, f.shape[2] - 1), rng.uniform(0, f.shape[1] - 1), 5.0, 0.1, 9.0, 16)
              for f in frames]
    cap_in = max(f.nbytes for f in frames)
    with HostPipeline(cap_in, 4 * cap_in, depth=2) as pl:
        hin = [torch.from_numpy(f) for f in frames]
        outs = [torch.empty(f.shape, dtype=torch.float32) for f in frames]
        tickets = []
        for i in range(len(frames)):
            tickets.append(pl.submit(hin[i], params[i], out=outs[i], layout="CHW"))
            if i % 3 == 2:
                pl.wait(tickets[i - 1])
        pl.done(tickets[-1])
        for i in reversed(range(len(frames))):
            if i % 3 != 1 or i == len(frames) - 1:
                pl.wait(tickets[i])
    for i, f in enumerate(frames):
        ref = orc.forward(f.astype(np.float64), params[i])
        assert_f32_close(outs[i].numpy(), ref, 2e-5 * 255, "pipeline f32 frame %d" % i)
        d = fov.forward(hin[i].to(dev), params[i], layout="CHW", out_dtype=torch.float32)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], d.cpu()), i


def test_pipeline_errors(fov, dev):
    fr = torch.from_numpy(synth.grating_frame(32, 32, 3, seed=1)).pin_memory()
    p = synth.params_dict(10, 10, 0, 0.1, 3)
    with HostPipeline(fr.numel() // 2, depth=2) as pl:
        with pytest.raises(fov.FoveateError) as ei:
            pl.submit(fr, p)  # larger than the slots
        assert ei.value.status == -1
    with HostPipeline(4 * fr.numel(), depth=2) as pl:
        wide = torch.zeros((32, 64, 3), dtype=torch.uint8).pin_memory()
        with pytest.raises(fov.FoveateError) as ei:
            pl.submit(wide[:, ::2, :], p)  # every other column: not one dense block
        assert ei.value.status == -3
        with pytest.raises(fov.FoveateError) as ei:
            pl.wait(12345)
        assert ei.value.status == -9
        with pytest.raises(ValueError):
            pl.submit(fr.to(dev), p)  # device memory is not a host frame
        t = pl.submit(fr, p)
        out = pl.wait(t)
        assert torch.equal(out, fov.forward(fr.to(dev), p, layout="HWC").cpu())
        with pytest.raises(fov.FoveateError):
            pl.wait(t)  # retired
