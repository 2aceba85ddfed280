"""Seeded synthetic inputs for the CSR-k sparse matrix-vector product.

This package only builds input data: stencil and FEM-like sparsity patterns in
CSR form, their values, and dense vectors.  It holds none of the method's
arithmetic (no products, no orderings, no grouping) and imports neither the
oracle nor the library, so both can take their inputs from here.

Every random quantity is drawn from NumPy's PCG64 generator with a seed
derived from ``SeedSequence(seed).spawn(...)``, one child stream per quantity,
so a workload is fully determined by its name and seed.
"""

from .stencils import (  # noqa: F401
    CsrInput,
    stencil_pattern,
    laplacian,
    diag_dominant_values,
    drop_offdiagonals,
    scramble_symmetric,
    uniform_vector,
    random_sparse,
    workload_c1,
    workload_c2,
    workload_c3,
    workload_c4,
    workload_c5,
    tuning_suite,
    WORKLOADS,
)
from .irregular import rmat_matrix, rmat_pattern, workload_irregular  # noqa: E402,F401

WORKLOADS = dict(WORKLOADS, irr=workload_irregular)
