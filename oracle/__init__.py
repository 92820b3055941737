"""CPU oracle for the blocked smoothed-aggregation AMG solve phase.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the GPU library never calls it and shares no code
with it.  Everything here is plain FP64 numpy/scipy, written for readability rather
than speed:

* `sparse`  - block sparse container, scalar-CSR expansion, SpMV and SpMV-transpose,
              blocked COO assembly, structural products and the Galerkin product
              A_c = P^T A P (paper §2.1, §2.3, §3.4, §3.5, §5).
* `sa`      - smoothed aggregation setup: strength graph and greedy aggregation,
              rigid-body near-null space, tentative prolongator, per-level lambda_max
              estimate by Lanczos, prolongator smoothing (paper §2.2, §2.3).
* `solve`   - point-block Jacobi preconditioned Chebyshev smoother, V-cycle with a
              dense Cholesky coarsest solve, preconditioned CG (paper §2.1, §4.1),
              hierarchy setup and the hot recompute with the prolongators reused
              (paper §3.1).
* `mix`     - the splitmix64 generator used for Lanczos start vectors.

Where the paper is silent the readings are listed in the design doc and repeated at the
function that takes them.  Parity status per function is in each docstring.
"""
