"""Batched solves: independent instances with several right-hand sides each.

By definition a batch is a set of independent problems: instance t has its own
hierarchy (built by `solve.setup` on its own operator, paper §3.1), and each of its
right-hand sides is solved by its own preconditioned CG with its own stopping test
(paper §4.1).  The oracle is that definition written out as loops over the
single-instance oracle, so it is pinned by the single-instance pins.
"""
from __future__ import annotations

import numpy as np

from . import sparse as S
from . import solve


def extract_instance(A: S.Bsr, r0: int, r1: int) -> S.Bsr:
    """Diagonal block of a block-diagonal matrix: rows and columns [r0, r1)."""
    k0, k1 = int(A.rowptr[r0]), int(A.rowptr[r1])
    ci = A.colidx[k0:k1] - r0
    if len(ci) and (ci.min() < 0 or ci.max() >= r1 - r0):
        raise ValueError("matrix is not block diagonal over the instances")
    return S.Bsr(r1 - r0, r1 - r0, A.br, A.bc, A.rowptr[r0:r1 + 1] - k0, ci, A.val[k0:k1])


def setup_batch(A: S.Bsr, row0, coords, dirichlet, opts=None):
    """One hierarchy per instance."""
    return [solve.setup(extract_instance(A, int(row0[t]), int(row0[t + 1])), coords[row0[t]:row0[t + 1]],
                        dirichlet[row0[t]:row0[t + 1]], opts) for t in range(len(row0) - 1)]


def pcg_batch(A: S.Bsr, hierarchies, row0, B, rtol=1e-8, maxit=1000):
    """Solve every (instance, column) system independently.  Returns X [n_dof][nrhs]
    and iterations [n_inst][nrhs]."""
    bs = A.br
    X = np.zeros_like(B)
    its = np.zeros((len(hierarchies), B.shape[1]), dtype=np.int64)
    for t, H in enumerate(hierarchies):
        r0, r1 = int(row0[t]) * bs, int(row0[t + 1]) * bs
        At = extract_instance(A, int(row0[t]), int(row0[t + 1]))
        for q in range(B.shape[1]):
            x, it, _, ok = solve.pcg(At, B[r0:r1, q], lambda r: solve.vcycle(H, r), rtol, maxit)
            X[r0:r1, q] = x
            its[t, q] = it
    return X, its
