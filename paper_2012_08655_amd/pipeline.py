"""Host-to-host pipeline binding: frames in (pinned) host memory are
uploaded, foveated and downloaded by libfoveate.so, the copies of one frame
overlapping the foveation of its neighbours.  Argument marshalling only."""
from __future__ import annotations

import ctypes

from . import _native as N


class HostPipeline:
    """Frames in host memory through the GPU and back.

    ``submit`` takes CPU tensors (pinned for overlap: ``pin_memory()``) and
    returns a ticket; ``wait`` blocks until the output tensor holds the
    foveated frame.  References to both tensors are kept until then.
    """

    def __init__(self, max_in_bytes: int, max_out_bytes: int | None = None, depth: int = 3):
        h = ctypes.c_void_p()
        N.check(N.lib().foveate_pipeline_create(int(depth), int(max_in_bytes),
                                                int(max_out_bytes or max_in_bytes), ctypes.byref(h)))
        self._h = h
        self._keep: dict[int, tuple] = {}

    def submit(self, x, params, out=None, layout: str = "HWC", out_dtype=None) -> int:
        """Queue host frame ``x`` (one frame in ``layout``: "HWC", "CHW" or
        "HW"); the result goes to ``out`` (a new pinned tensor like ``x`` when
        None).  Returns the ticket."""
        import torch
        from . import api
        if out is None:
            out = torch.empty(x.shape, dtype=out_dtype or x.dtype, pin_memory=True)
        din, dout = api.tensor_desc(x, layout, host=True), api.tensor_desc(out, layout, host=True)
        arr, _, k = api._params_array(params, 1)
        t = ctypes.c_uint64()
        N.check(N.lib().foveate_pipeline_submit(self._h, ctypes.byref(din), ctypes.byref(dout), arr,
                                                ctypes.byref(t)))
        self._keep[t.value] = (x, out, k)
        return t.value

    def done(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        N.check(N.lib().foveate_pipeline_query(self._h, ctypes.c_uint64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        """Block until the ticket's frame is in its output tensor; returns it."""
        keep = self._keep.get(ticket)
        N.check(N.lib().foveate_pipeline_wait(self._h, ctypes.c_uint64(ticket)))
        self._keep.pop(ticket, None)
        return keep[1] if keep else None

    def close(self):
        if self._h:
            N.check(N.lib().foveate_pipeline_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
