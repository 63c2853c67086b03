"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only builds input matrices (prescribed spectra, orthonormal
factors, noise, kernel blocks, test-matrix streams).  It holds none of the
randomized-SVD arithmetic: neither the CPU oracle nor the HIP library imports
anything from the other, and both receive their inputs from here.
"""
from .gen import (  # noqa: F401
    CONFIGS,
    WorkloadConfig,
    config,
    gaussian_matrix,
    kernel_block,
    low_rank_matrix,
    orthonormal_factor,
    spectrum,
    batched_blocks,
    selector_item_params,
)
