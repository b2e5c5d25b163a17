"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package only builds inputs (sparse matrices in CSR form, start vectors,
random relabellings).  It holds none of the matrix-power method's arithmetic:
no SpMV, no breadth-first search, no grouping, no schedule.
"""
from .matrices import (  # noqa: F401
    CSR,
    seed_streams,
    stencil_2d,
    stencil_3d,
    star_stencil_3d,
    heat_operator_3d,
    stencil_27pt_random,
    anderson_3d,
    random_geometric,
    banded_random,
    zipf_rows,
    relabel,
    uniform_vector,
    gaussian_block,
    random_phase_state,
    integer_stencil_27pt,
    random_small_csr,
    tuner_matrix,
)
