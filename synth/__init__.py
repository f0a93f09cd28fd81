"""Seeded synthetic workloads shaped like the paper's PQ / inverted-index runs.

This package only draws random numbers: Gaussian mixtures, sample rows and
initial rows.  It holds none of the method's arithmetic (no distances, no
assignment, no centroid updates), so the oracle and the GPU path can both take
their inputs from it without sharing any part of the computation.
"""

from .workloads import (  # noqa: F401
    Workload,
    IvfWorkload,
    BatchedWorkload,
    gaussian_mixture,
    choose_rows,
    init_rows_per_subspace,
    plain_pq,
    integer_pq,
    batched_uneven,
    ivf_adc,
    diff_codebooks,
)
