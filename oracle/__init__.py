"""FP64 CPU oracle for block-wise foveation (test infrastructure only).

Imported by the test suite, the smoke check and the benchmark's CPU-baseline
leg; never by the product library.
"""
from .oracle import (adjoint, build, csf_contrast_threshold, csf_cutoff_cpd, csf_sigma,  # noqa: F401
                     csf_sigma_map, eq7_shared_bytes, explicit_matrix, forward, forward_per_pixel, forward_points,
                     fragment_shift, grid, max_filter_taps, max_threads, plan, to_u8)
