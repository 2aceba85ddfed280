"""Oracle for the CSR-k sparse matrix-vector product — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of what the CSR-k hot path
computes, written from the paper (Lane & Booth, "Heterogeneous Sparse
Matrix-Vector Multiplication via Compressed Sparse Row Format"):

* ``spmv``      — y = A x over CSR in FP64 (Section 1 statement of SpMV;
                  Section 2.1 CSR) and the CSR-k traversal of Section 2.2.
* ``bandk``     — Band-k reordering and super-row / super-super-row grouping
                  (Section 2.2, the Band-k algorithm), in this project's
                  deterministic reading ("BandK-v1").
* ``tune``      — the constant-time size model of Section 4.1.
* ``adjoint``   — grad_x = A^T g and grad_vals = g_i x_j (plain definitions).
* ``precision`` — FP64 -> FP32 -> BF16 rounding and forward error bounds.
* ``stats``     — row-density statistics of Section 5.3.
* ``spmv_ref.c``— the same plain CSR product in C with OpenMP (static
                  schedule, as in Section 5.2), used for host timing.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or execute anything here.  The library under
``paper_2203_05096_amd/`` never imports it and shares no code with it; both
take their inputs from ``gen/``.
"""

from . import spmv, bandk, tune, adjoint, precision, stats  # noqa: F401
