"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds none of the gridding arithmetic: it only draws soundings
(x, y, z as float64 arrays), grid descriptors, sampled seafloor grids with
nodes removed, and request schedules.  Both the
oracle and the HIP path consume exactly these arrays.
"""
from .workloads import (  # noqa: F401
    GridSpec, Soundings, seafloor_depth, uniform_field, swath, workload_cfg1,
    workload_cfg2, workload_cfg3_tiles, workload_cfg4, serving_schedule,
    small_swath, checksum, dem_on_grid, grid_a_case, grid_b_case,
)
