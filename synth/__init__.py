"""Seeded synthetic particle workloads.

This package only draws inputs: original positions, a base-compressor-like
reconstruction and the per-workload parameters (linking length b, error bound
xi, periodic box).  It holds none of the correction method's arithmetic and is
shared by the CPU oracle tests, the GPU tests and the benchmark.
"""
from .generators import (  # noqa: F401
    Workload,
    grid_reconstruction,
    plain_blobs,
    cosmology,
    md_block,
    sph_voids,
    md_batch_sizes,
    served_jobs,
    make_job,
    sub_box,
)
