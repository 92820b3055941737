"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *generates inputs*: the Q1 (and Q2) hexahedral elasticity problem (mesh,
coordinates, clamped face, per-element materials, element stiffness blocks as a
blocked COO stream, right-hand sides) and random blocked-sparse fixtures.  It holds
none of the solver's arithmetic (no SpMV, no Galerkin product, no aggregation, no
smoother, no Krylov method), so the CPU oracle and the GPU path can both consume it
without sharing any of the method.
"""
from .q1 import (  # noqa: F401
    Q1Mesh,
    make_mesh,
    reference_element_matrices,
    element_matrix,
    materials,
    homogeneous_materials,
    lame,
    coo_indices,
    coo_values,
    coo_values_torch,
    rhs,
    stream_sizes,
)
from .q2 import make_mesh_q2, reference_element_matrices_q2, shape_functions_q2  # noqa: F401
from .random_bsr import random_bsr, random_spd_bsr, random_coo_stream  # noqa: F401
from .batch import batch_sizes, make_batch, batch_values, batch_values_torch  # noqa: F401
