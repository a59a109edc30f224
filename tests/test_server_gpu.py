"""GPU tests of the serving loop: every served frame matches the FP64 oracle
(within 1 LSB, element by element) and equals (bitwise) the same frame
foveated alone with foveate_forward, whether it ran alone or in a batch with
other frames, with and without hipGraph replay."""
import time

import numpy as np
import pytest
import torch

import synth
from paper_2012_08655_amd.server import Server
from parity import assert_u8_close

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


def oracle_u8(orc, fr, p):
    """Oracle output of an HWC u8 frame, rounded to u8, HWC."""
    return orc.to_u8(orc.forward(fr.transpose(2, 0, 1).astype(np.float64), p)).transpose(1, 2, 0)


@pytest.mark.parametrize("use_graph", [True, False])
def test_served_equals_plain(fov, orc, dev, use_graph, batch64, oracle_4k):
    items = frames_and_params(40, seed=1 + int(use_graph))
    ins = [torch.from_numpy(f).to(dev) for f, _ in items]
    outs = [torch.empty_like(t) for t in ins]
    params = [p for _, p in items]
    # a 4K blocker first (the first 4K frame of the 64-frame mixed batch): the small frames
    # arrive while it occupies the device, so the scheduler has to batch them (a frame that
    # finds a stream free launches at once)
    bframes, bparams, i4k = batch64
    big = torch.from_numpy(bframes[i4k]).to(dev)
    ins.insert(0, big)
    outs.insert(0, torch.empty_like(big))
    params.insert(0, bparams[i4k])
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
    # every served frame against the oracle, the 4K blocker included
    assert_u8_close(outs[0].cpu().numpy(), oracle_4k, "served 4K blocker")
    for i, (fr, p) in enumerate(items):
        assert_u8_close(outs[i + 1].cpu().numpy(), oracle_u8(orc, fr, p), "served frame %d" % (i + 1))


@pytest.mark.parametrize("shared", [False, True])
def test_served_overlapping_streams_equal_plain(fov, orc, dev, shared):
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
    for i, (fr, p) in enumerate(items):
        assert torch.equal(outs[i], plain[i]), i
        assert_u8_close(outs[i].cpu().numpy(), oracle_u8(orc, fr, p), "served frame %d" % i)


def test_server_budget_smaller_than_batch(fov, orc, dev):
    # a budget of ~3 frames forces several small batches; results unchanged
    items = frames_and_params(12, seed=9, shapes=((64, 64),))
    ins = [torch.from_numpy(f).to(dev) for f, _ in items]
    outs = [torch.empty_like(t) for t in ins]
    budget = 3 * 2 * 64 * 64 * 3
    with Server(hbm_budget_bytes=budget, max_batch_frames=16, max_fragments=1000, use_graph=True) as s:
        tks = [s.submit(t, o, p) for t, o, (_, p) in zip(ins, outs, items)]
        s.drain()
        assert max(s.poll(tk)[1].batch_frames for tk in tks) <= 3
    for t, o, (fr, p) in zip(ins, outs, items):
        assert torch.equal(o, fov.forward(t, p, layout="HWC"))
        assert_u8_close(o.cpu().numpy(), oracle_u8(orc, fr, p), "served under a small budget")


@pytest.mark.parametrize("use_graph", [True, False])
def test_submit_waits_for_the_producer_stream(fov, orc, dev, use_graph):
    # Each input is written on another stream, behind a long matrix product, and submitted
    # at once with that stream as its producer: the served batch must wait for it on the
    # device.  No host synchronisation between producing and submitting.
    items = frames_and_params(6, seed=23, shapes=((120, 90), (200, 333)))
    src = [torch.from_numpy(f).to(dev) for f, _ in items]
    ins = [torch.zeros_like(t) for t in src]
    outs = [torch.empty_like(t) for t in src]
    a = torch.randn(4096, 4096, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    producer = torch.cuda.Stream(device=dev)
    with Server(hbm_budget_bytes=256 << 20, max_batch_frames=4, max_inflight_batches=2, max_fragments=20000,
                max_sigma=16.0, use_graph=use_graph) as s:
        tickets = []
        for t, x, o, (_, p) in zip(src, ins, outs, items):
            with torch.cuda.stream(producer):
                for _ in range(2):
                    torch.mm(a, a, out=b)  # keeps the producer busy well past the submit
                x.copy_(t)
            tickets.append(s.submit(x, o, p, stream=producer))
        s.drain()
        for tk in tickets:
            assert s.poll(tk)[0]
    torch.cuda.synchronize()
    for i, (t, (fr, p)) in enumerate(zip(src, items)):
        assert torch.equal(outs[i], fov.forward(t, p, layout="HWC")), i
        assert_u8_close(outs[i].cpu().numpy(), oracle_u8(orc, fr, p), "frame %d after its producer" % i)
