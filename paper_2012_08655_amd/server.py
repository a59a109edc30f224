"""Serving binding: a request loop over the library's continuous-batching
server (HBM-budget admission, batches overlapping on several streams,
optional hipGraph replay).  Argument marshalling only."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _native as N

_DT = {"u8": N.FOV_U8, "f32": N.FOV_F32, "f64": N.FOV_F64}


@dataclass
class Timing:
    t_submit: float
    t_admit: float
    t_launch: float
    t_done: float
    batch_frames: int
    status: int


def now() -> float:
    """The server's monotonic clock (seconds)."""
    return N.lib().foveate_now()


class Server:
    """Frames submitted one at a time are admitted by HBM budget and batched.

    ``submit`` takes device tensors (any object exposing ``data_ptr``,
    ``shape``, ``stride`` and ``dtype`` via ``api.tensor_desc``) and keeps
    references until the ticket is polled done.
    """

    def __init__(self, hbm_budget_bytes: int, max_batch_frames: int = 64, max_inflight_batches: int = 2,
                 max_requests: int = 4096, in_dtype: str = "u8", out_dtype: str = "u8",
                 max_fragments: int = 200000, max_block: int = 32, max_sigma: float = 16.0,
                 use_graph: bool = True, test_fake_device_us: int = 0, test_fail_every: int = 0,
                 shared_stream: bool = False):
        cfg = N.FovServerCfg(int(hbm_budget_bytes), int(max_batch_frames), int(max_inflight_batches),
                             int(max_requests), _DT[in_dtype], _DT[out_dtype], int(max_fragments), int(max_block),
                             float(max_sigma), int(bool(use_graph)), int(test_fake_device_us),
                             int(test_fail_every), int(bool(shared_stream)))
        h = ctypes.c_void_p()
        N.check(N.lib().foveate_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep: dict[int, tuple] = {}
        self._events: dict[int, object] = {}  # ticket -> producer event (until polled done)
        self._free_events: list = []

    def submit_desc(self, din: N.FovTensor, dout: N.FovTensor, params: N.FovParams, keep=(), ready=None) -> int:
        """Queue a frame given as descriptors; ``ready`` is a raw hipEvent_t
        handle (int) the frame's batch waits for, or None."""
        t = ctypes.c_uint64()
        N.check(N.lib().foveate_submit(self._h, ctypes.byref(din), ctypes.byref(dout), ctypes.byref(params),
                                       ctypes.c_void_p(ready) if ready else None, ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def submit(self, x, out, params, layout: str = "HWC", stream=None) -> int:
        """Queue frame ``x`` into ``out``.  The frame's batch waits on the
        device for the work queued so far on ``stream`` (default: torch's
        current stream), where ``x`` was produced and ``out`` last used."""
        import torch
        from . import api
        din, dout = api.tensor_desc(x, layout), api.tensor_desc(out, layout)
        arr, _, k = api._params_array(params, 1)
        ev = self._free_events.pop() if self._free_events else torch.cuda.Event()
        ev.record(stream if stream is not None else torch.cuda.current_stream())
        try:
            tk = self.submit_desc(din, dout, arr[0], keep=(x, out, k), ready=ev.cuda_event)
        except Exception:
            self._free_events.append(ev)
            raise
        self._events[tk] = ev
        return tk

    def poll(self, ticket: int):
        """(done, Timing or None).  Raises FoveateError if the frame failed."""
        done = ctypes.c_int32()
        tm = N.FovTiming()
        st = N.lib().foveate_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(tm))
        if done.value:
            self._keep.pop(ticket, None)
            ev = self._events.pop(ticket, None)
            if ev is not None:
                self._free_events.append(ev)  # the batch has waited for it: free to record again
        N.check(st)
        if not done.value:
            return False, None
        return True, Timing(tm.t_submit, tm.t_admit, tm.t_launch, tm.t_done, tm.batch_frames, tm.status)

    def drain(self):
        N.check(N.lib().foveate_server_drain(self._h))

    def close(self):
        if self._h:
            N.check(N.lib().foveate_server_destroy(self._h))
            self._h = None
            self._keep.clear()
            self._events.clear()
            self._free_events.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
