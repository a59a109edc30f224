"""Forward calls from several host threads on one stream, with frame sizes
that make the shared per-stream workspace grow, give the same results as the
same calls made one at a time."""
import threading

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def test_threads_sharing_a_stream(fov, dev):
    stream = torch.cuda.Stream(device=dev)
    # the 4K frames need a plan workspace of several MiB, so the workspace grows under load
    sizes = [(40, 60), (2160, 3840), (90, 70), (700, 900), (33, 47), (1500, 2600)]
    g = torch.Generator(device=dev).manual_seed(3)
    jobs = []
    for i in range(24):
        h, w = sizes[i % len(sizes)]
        x = torch.randint(0, 256, (h, w, 3), dtype=torch.uint8, device=dev, generator=g)
        p = synth.params_dict(w / 2, h / 2, 5.0, 0.05, 16.0)
        jobs.append((x, p))
    ref = [fov.forward(x, p, layout="HWC") for x, p in jobs]
    torch.cuda.synchronize()
    outs = [torch.empty_like(x) for x, _ in jobs]
    errors = []

    def worker(k):
        try:
            for i in range(k, len(jobs), 4):
                x, p = jobs[i]
                fov.forward(x, p, out=outs[i], layout="HWC", stream=stream)
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    stream.synchronize()
    assert not errors, errors
    for i in range(len(jobs)):
        assert torch.equal(outs[i], ref[i]), i
