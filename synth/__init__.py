"""Seeded synthetic wide-dynamic-range inputs shared by tests, the oracle and the bench.

This module only draws inputs.  It holds none of the tone-mapping arithmetic, so both the
HIP path and the CPU oracle can be fed from it without sharing any of the method's code.
"""
from .wdr import WdrImage, gen_wdr, gen_wdr_row, gen_batch_shapes, gen_upstream_grad, WORKLOADS
from .exposures import exposure_times, gen_exposure_stack, gen_sample_pixels

__all__ = ["WdrImage", "gen_wdr", "gen_wdr_row", "gen_batch_shapes", "gen_upstream_grad", "WORKLOADS",
           "exposure_times", "gen_exposure_stack", "gen_sample_pixels"]
