"""GPU tests of the serving loop: every served frame equals (bitwise) the
same frame foveated alone with foveate_forward, whether it ran alone or in a
batch with other frames, with and without hipGraph replay."""
import time

import numpy as np
import pytest
import torch

import synth
from paper_2012_08655_amd.server import Server

pytestmark = pytest.mark.gpu


def frames_and_params(n, seed, shapes=((48, 64), (120, 90), (200, 333), (31, 17))):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h, w = shapes[int(rng.integers(len(shapes)))]
        fr = synth.grating_frame(h, w, 3, seed=seed * 1000 + i)
        p = synth.params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), rng.uniform(0, 40),
                              rng.uniform(0.01, 0.1), rng.uniform(1, 16))
        out.append((fr, p))
    return out


@pytest.mark.parametrize("use_graph", [True, False])
def test_served_equals_plain(fov, dev, use_graph):
    items = frames_and_params(40, seed=1 + int(use_graph))
    ins = [torch.from_numpy(f).to(dev) for f, _ in items]
    outs = [torch.empty_like(t) for t in ins]
    params = [p for _, p in items]
    # a 4K blocker first: the small frames arrive while it occupies the device, so the
    # scheduler has to batch them (a frame that finds a stream free launches at once)
    g = torch.Generator(device=dev).manual_seed(5)
    big = torch.randint(0, 256, (2160, 3840, 3), dtype=torch.uint8, device=dev, generator=g)
    ins.insert(0, big)
    outs.insert(0, torch.empty_like(big))
    params.insert(0, synth.params_dict(1919.5, 1079.5, 0.0, 1.0, 16.0))
    plain = [fov.forward(t, p, layout="HWC") for t, p in zip(ins, params)]
    torch.cuda.synchronize()
    with Server(hbm_budget_bytes=256 << 20, max_batch_frames=16, max_inflight_batches=1, max_fragments=20000,
                max_sigma=16.0, use_graph=use_graph) as s:
        tickets = [s.submit(t, o, p) for t, o, p in zip(ins, outs, params)]
        s.drain()
        sizes = []
        for tk in tickets:
            done, tm = s.poll(tk)
            assert done and tm.status == 0
            assert tm.t_submit <= tm.t_admit <= tm.t_launch <= tm.t_done
            sizes.append(tm.batch_frames)
    for i in range(len(ins)):
        assert torch.equal(outs[i], plain[i]), i
    assert sizes[0] == 1 and max(sizes[1:]) > 1  # the blocker alone, later frames batched


@pytest.mark.parametrize("shared", [False, True])
def test_served_overlapping_streams_equal_plain(fov, dev, shared):
    # two batches in flight, arrivals spread out: on two streams they overlap on the device, on
    # one shared stream they queue; results unchanged
    items = frames_and_params(30, seed=11)
    ins = [torch.from_numpy(f).to(dev) for f, _ in items]
    outs = [torch.empty_like(t) for t in ins]
    plain = [fov.forward(t, p, layout="HWC") for t, (_, p) in zip(ins, items)]
    torch.cuda.synchronize()
    with Server(hbm_budget_bytes=256 << 20, max_batch_frames=8, max_inflight_batches=2, max_fragments=20000,
                max_sigma=16.0, use_graph=True, shared_stream=shared) as s:
        tickets = []
        for k, (t, o, (_, p)) in enumerate(zip(ins, outs, items)):
            tickets.append(s.submit(t, o, p))
            if k % 7 == 0:
                time.sleep(0.002)
        s.drain()
        for tk in tickets:
            assert s.poll(tk)[0]
    for i in range(len(items)):
        assert torch.equal(outs[i], plain[i]), i


def test_server_budget_smaller_than_batch(fov, dev):
    # a budget of ~3 frames forces several small batches; results unchanged
    items = frames_and_params(12, seed=9, shapes=((64, 64),))
    ins = [torch.from_numpy(f).to(dev) for f, _ in items]
    outs = [torch.empty_like(t) for t in ins]
    budget = 3 * 2 * 64 * 64 * 3
    with Server(hbm_budget_bytes=budget, max_batch_frames=16, max_fragments=1000, use_graph=True) as s:
        tks = [s.submit(t, o, p) for t, o, (_, p) in zip(ins, outs, items)]
        s.drain()
        assert max(s.poll(tk)[1].batch_frames for tk in tks) <= 3
    for t, o, (_, p) in zip(ins, outs, items):
        assert torch.equal(o, fov.forward(t, p, layout="HWC"))
