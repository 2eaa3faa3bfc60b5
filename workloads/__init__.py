"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package draws lattice points and loads only. It holds none of the method's
arithmetic (no kernel values, no sums), so both the GPU path and the CPU oracle can
consume its output without sharing any computation.
"""
from .generators import (  # noqa: F401
    zero_sum_loads,
    uniform_box,
    gaussian_clusters,
    clusters_on_background,
    config_small_uniform,
    config_large_uniform,
    config_clusters,
    config_batched,
    config_batched_instance,
    config_serving_request,
    serving_request_size,
    sample_targets,
    inclusion_bars,
    box_boundary,
    lshape_boundary,
)
