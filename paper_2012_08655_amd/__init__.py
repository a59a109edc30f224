"""Block-wise foveation on AMD MI355X (gfx950): HIP kernels behind a C ABI.

The method is that of Malkin, Deza and Poggio, "CUDA-Optimized real-time
rendering of a Foveated Visual System" (arXiv 2012.08655): fragments of a
frame are blurred with Gaussians whose sigma follows the fragment midpoint's
distance from the fixation point.  ``libfoveate.so`` (built from ``csrc/``)
does all the work; this package only marshals arguments to it.
"""
from ._native import FoveateError, lib  # noqa: F401


def load():
    """Load libfoveate.so (raises ImportError if it is not built)."""
    return lib()


def __getattr__(name):
    # The torch binding is imported lazily so that loading the C library (and
    # checking its exports) does not require torch.
    if name in ("forward", "forward_batch", "backward", "grid", "plan_device", "plan_host", "foveate", "FoveateFn",
                "tensor_desc", "profile_begin", "profile_end", "autotune", "autotune_batch", "tuning_force",
                "tuning_clear", "tuning_count", "tuning_save", "tuning_load", "fragment_shift", "csf_params"):
        from . import api
        return getattr(api, name)
    if name == "HostPipeline":
        from .pipeline import HostPipeline
        return HostPipeline
    if name == "Server":
        from .server import Server
        return Server
    raise AttributeError(name)
