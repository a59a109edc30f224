"""Seeded synthetic inputs for block-wise foveation.

Shared by the test suite, the benchmark and the smoke check.  This package
holds no arithmetic of the method itself: it only draws frames, frame
parameters (fixation, ramp constants) and request traces from NumPy's PCG64
generator.
"""
from .frames import (batch_mixed, grating_frame, params_cfg1, params_cfg2,  # noqa: F401
                     params_cfg5, params_dict, uniform_frames)
from .gaze import poisson_trace  # noqa: F401
