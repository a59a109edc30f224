"""Scheduler tests of the serving loop on a fake device (CPU only).

The fake device runs no kernels: each batch "completes" a fixed delay after
launch, so admission, batching, latency accounting and failure handling are
exercised without a GPU.  Buffers are fake device addresses (never touched).
"""
import ctypes
import threading
import time

import pytest

import synth
from paper_2012_08655_amd import _native as N
from paper_2012_08655_amd.server import Server

FRAME_BYTES = 2 * 64 * 64 * 4  # one 64x64 f32 input + output


def desc(i, h=64, w=64):
    base = 0x10000000 * (i + 1)
    din = N.FovTensor(base, N.FOV_F32, 1, 1, h, w, h * w, h * w, w, 1)
    dout = N.FovTensor(base + 0x8000000, N.FOV_F32, 1, 1, h, w, h * w, h * w, w, 1)
    return din, dout


P = N.make_params(synth.params_dict(10, 10, 0, 0.1, 4))


def server(**kw):
    args = dict(hbm_budget_bytes=10 ** 9, in_dtype="f32", out_dtype="f32", test_fake_device_us=3000)
    args.update(kw)
    return Server(**args)


def test_all_done_with_ordered_timestamps():
    with server() as s:
        ts = [s.submit_desc(*desc(i), P) for i in range(20)]
        s.drain()
        for t in ts:
            done, tm = s.poll(t)
            assert done and tm.status == 0
            assert tm.t_submit <= tm.t_admit <= tm.t_launch < tm.t_done


def test_admission_respects_hbm_budget():
    # budget of two frames: never more than two frames admitted and unfinished
    with server(hbm_budget_bytes=2 * FRAME_BYTES, max_inflight_batches=4) as s:
        ts = [s.submit_desc(*desc(i), P) for i in range(12)]
        s.drain()
        tms = [s.poll(t)[1] for t in ts]
    events = sorted([(tm.t_admit, 1) for tm in tms] + [(tm.t_done, -1) for tm in tms], key=lambda e: (e[0], e[1]))
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak <= 2
    assert max(tm.batch_frames for tm in tms) <= 2


def test_continuous_batching_overlaps_batches():
    # frames arriving while a batch runs are launched on the second stream
    with server(test_fake_device_us=40000, max_inflight_batches=2) as s:
        first = s.submit_desc(*desc(0), P)
        time.sleep(0.01)
        later = [s.submit_desc(*desc(1 + i), P) for i in range(5)]
        s.drain()
        t0 = s.poll(first)[1]
        tl = [s.poll(t)[1] for t in later]
    assert t0.batch_frames == 1
    # the scheduler is greedy: the next arrival goes straight to the free
    # stream while the first batch runs; the rest wait and go as one batch
    assert any(t.t_launch < t0.t_done for t in tl)
    assert max(t.batch_frames for t in tl) >= 2
    assert len({round(t.t_launch, 9) for t in tl}) <= 3


def test_batch_limits():
    with server(max_batch_frames=3, max_inflight_batches=1) as s:
        ts = [s.submit_desc(*desc(i), P) for i in range(10)]
        s.drain()
        tms = [s.poll(t)[1] for t in ts]
    assert max(t.batch_frames for t in tms) <= 3
    # fragment limit: 64x64 in 32 px fragments = 4 fragments per frame
    with server(max_fragments=8, max_inflight_batches=1) as s:
        ts = [s.submit_desc(*desc(i), P) for i in range(6)]
        s.drain()
        assert max(s.poll(t)[1].batch_frames for t in ts) <= 2


def test_request_table_full_and_tickets():
    with server(max_requests=3) as s:
        ts = [s.submit_desc(*desc(i), P) for i in range(3)]
        with pytest.raises(N.FoveateError) as ei:
            s.submit_desc(*desc(3), P)
        assert ei.value.status == N.FOV_EAGAIN
        with pytest.raises(N.FoveateError) as ei:
            s.poll(999999)
        assert ei.value.status == N.FOV_ENOTICKET
        s.drain()
        assert s.poll(ts[0])[0]
        with pytest.raises(N.FoveateError) as ei:  # retired by the poll that reported it done
            s.poll(ts[0])
        assert ei.value.status == N.FOV_ENOTICKET
        ts.append(s.submit_desc(*desc(3), P))  # a slot was freed
        s.drain()


def test_injected_batch_failures_are_reported_and_serving_continues():
    with server(test_fail_every=2, max_inflight_batches=1, max_batch_frames=1) as s:
        ts = [s.submit_desc(*desc(i), P) for i in range(6)]
        s.drain()
        failed = 0
        for t in ts:
            try:
                assert s.poll(t)[0]
            except N.FoveateError as e:
                assert e.status == N.FOV_EHIP
                failed += 1
        assert failed == 3
        t = s.submit_desc(*desc(7), P)
        s.drain()


def test_submit_during_shutdown_is_refused():
    s = server(test_fake_device_us=200000)
    s.submit_desc(*desc(0), P)
    result = {}

    def late():
        time.sleep(0.05)
        try:
            s.submit_desc(*desc(1), P)
            result["status"] = 0
        except N.FoveateError as e:
            result["status"] = e.status

    th = threading.Thread(target=late)
    th.start()
    s.close()  # drains the running batch first
    th.join()
    assert result["status"] == N.FOV_ECLOSED


def test_request_validation():
    with server(hbm_budget_bytes=FRAME_BYTES, max_sigma=4.0) as s:
        din, dout = desc(0)
        bad = N.FovTensor(dout.data, N.FOV_U8, 1, 1, 64, 64, 4096, 4096, 64, 1)
        with pytest.raises(N.FoveateError) as ei:
            s.submit_desc(din, bad, P)
        assert ei.value.status == N.FOV_EDTYPE
        with pytest.raises(N.FoveateError) as ei:
            s.submit_desc(*desc(1, 65, 64), P)  # larger than the budget
        assert ei.value.status == N.FOV_EINVAL
        with pytest.raises(N.FoveateError) as ei:
            s.submit_desc(din, dout, N.make_params(synth.params_dict(0, 0, 0, 1.0, 9.0)))
        assert ei.value.status == N.FOV_ERANGE


@pytest.mark.parametrize("field,value", [("hbm_budget_bytes", 0), ("max_batch_frames", 0),
                                         ("max_inflight_batches", 9), ("max_block", 65)])
def test_bad_config(field, value):
    kw = {field: value}
    with pytest.raises(N.FoveateError) as ei:
        server(**kw)
    assert ei.value.status == N.FOV_EINVAL


def test_shared_stream_flag_validated():
    cfg = N.FovServerCfg(10 ** 9, 4, 2, 64, N.FOV_F32, N.FOV_F32, 1000, 32, 4.0, 0, 3000, 0, 2)
    h = ctypes.c_void_p()
    assert N.lib().foveate_server_create(ctypes.byref(cfg), ctypes.byref(h)) == N.FOV_EINVAL
    with server(shared_stream=True, max_inflight_batches=3) as s:
        ts = [s.submit_desc(*desc(i), P) for i in range(10)]
        s.drain()
        assert all(s.poll(t)[0] for t in ts)
