"""Block sparse matrices: definitions of SpMV, SpMV-transpose, blocked COO assembly
and the Galerkin triple product, computed by expanding every block to scalars.

A block matrix (paper §2.3) is a CSR structure over dense bs_r x bs_c blocks that
share one (block-row, block-column) index; block values are row-major.  The oracle
never operates on blocks directly: it expands to a scalar CSR matrix entry by entry
and applies textbook sparse algebra (scipy), so it is independent of any blocked
kernel design.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class Bsr:
    nbr: int
    nbc: int
    br: int
    bc: int
    rowptr: np.ndarray  # int64/int32 [nbr+1]
    colidx: np.ndarray  # [nnzb]
    val: np.ndarray     # float64 [nnzb, br, bc]
    _csr: object = field(default=None, repr=False, compare=False)  # memoised expansion

    @property
    def nnzb(self) -> int:
        return int(self.rowptr[-1])

    @property
    def shape(self):
        return (self.nbr * self.br, self.nbc * self.bc)

    def block_rows(self) -> np.ndarray:
        return np.repeat(np.arange(self.nbr, dtype=np.int64), np.diff(self.rowptr))

    def with_values(self, val: np.ndarray) -> "Bsr":
        return Bsr(self.nbr, self.nbc, self.br, self.bc, self.rowptr, self.colidx, val)


def to_scalar_csr(A: Bsr) -> sp.csr_matrix:
    """Scalar expansion: block (I, J) entry (r, c) becomes scalar (I*br + r, J*bc + c).
    The expansion is remembered on the matrix (its values are never mutated in place)."""
    if A._csr is not None:
        return A._csr
    rows_b = A.block_rows()
    r = np.arange(A.br)
    c = np.arange(A.bc)
    rows = (rows_b[:, None, None] * A.br + r[None, :, None]) + 0 * c[None, None, :]
    cols = (A.colidx.astype(np.int64)[:, None, None] * A.bc + c[None, None, :]) + 0 * r[None, :, None]
    M = sp.csr_matrix((A.val.reshape(-1), (rows.reshape(-1), cols.reshape(-1))), shape=A.shape)
    M.sort_indices()
    A._csr = M
    return M


def to_dense(A: Bsr) -> np.ndarray:
    """Dense expansion written block by block (used only on tiny matrices)."""
    D = np.zeros(A.shape)
    for I in range(A.nbr):
        for t in range(A.rowptr[I], A.rowptr[I + 1]):
            J = A.colidx[t]
            D[I * A.br:(I + 1) * A.br, J * A.bc:(J + 1) * A.bc] = A.val[t]
    return D


def spmv(A: Bsr, x: np.ndarray, alpha: float = 1.0, beta: float = 0.0, y=None) -> np.ndarray:
    """y = alpha A x + beta y.  x is [n_cols] or [n_cols, nrhs] (row-major per dof)."""
    out = alpha * (to_scalar_csr(A) @ x)
    if beta != 0.0:
        out = out + beta * y
    return out


def spmv_t(A: Bsr, x: np.ndarray, alpha: float = 1.0, beta: float = 0.0, y=None) -> np.ndarray:
    """y = alpha A^T x + beta y (the restriction with P^T, paper §2.1)."""
    out = alpha * (to_scalar_csr(A).T @ x)
    if beta != 0.0:
        out = out + beta * y
    return out


def symmetric_completion(A: Bsr) -> Bsr:
    """The matrix S with A's pattern, A's diagonal and upper blocks (block column >= block
    row), and each strictly lower block replaced by the transpose of its mirror:
    S_IJ = A_JI^T for J < I.  Defined for square blocks and a symmetric pattern; S = A
    exactly when A is symmetric (the SPD operators CG is applied to, paper §2.1, §4.1).
    Plain loop over the blocks with a dictionary of positions."""
    assert A.br == A.bc and A.nbr == A.nbc, "square blocks and a square matrix"
    pos = {}
    for r in range(A.nbr):
        for k in range(int(A.rowptr[r]), int(A.rowptr[r + 1])):
            pos[(r, int(A.colidx[k]))] = k
    val = A.val.copy()
    for (r, c), k in pos.items():
        if c < r:
            assert (c, r) in pos, "pattern is not symmetric"
            val[k] = A.val[pos[(c, r)]].T
    return A.with_values(val)


def spmv_rows(A: Bsr, x: np.ndarray, rows) -> np.ndarray:
    """(A x) restricted to the given block rows, by the definition sum_J A_IJ x_J."""
    xb = x.reshape(A.nbc, A.bc)
    out = np.zeros((len(rows), A.br))
    for t, I in enumerate(rows):
        for k in range(A.rowptr[I], A.rowptr[I + 1]):
            out[t] += A.val[k] @ xb[A.colidx[k]]
    return out


# ----------------------------------------------------------------------------------
# Blocked COO assembly (paper §3.4 and §5)
# ----------------------------------------------------------------------------------

def coo_plan(nbr: int, nbc: int, i: np.ndarray, j: np.ndarray):
    """Preallocation of a blocked COO stream.

    Reading (the paper is silent): a negative i or j marks an entry to ignore.
    Returns (rowptr, colidx, perm, seg): the sorted unique block pattern, the stable
    order of the valid entries sorted by (row, column, original position), and for
    each stored block t the run perm[seg[t]:seg[t+1]] of entries summed into it.
    """
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    valid = (i >= 0) & (j >= 0)
    if np.any(i[valid] >= nbr) or np.any(j[valid] >= nbc):
        raise ValueError("COO coordinate out of range")
    k = np.nonzero(valid)[0]
    keys = i[k] * nbc + j[k]
    order = np.argsort(keys, kind="stable")
    perm = k[order]
    sk = keys[order]
    first = np.ones(len(sk), dtype=bool)
    first[1:] = sk[1:] != sk[:-1]
    starts = np.nonzero(first)[0]
    seg = np.append(starts, len(sk)).astype(np.int64)
    ukeys = sk[starts]
    rows = ukeys // nbc
    colidx = (ukeys % nbc).astype(np.int64)
    rowptr = np.zeros(nbr + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, colidx, perm, seg


def coo_assemble(nbr: int, nbc: int, i, j, vals: np.ndarray, A: Bsr | None = None,
                 mode: str = "insert") -> Bsr:
    """Sum a block value stream into its block matrix: the block at (I, J) is the sum,
    in stream order, of every valid entry with coordinates (I, J).  `insert` replaces
    the values of A (or creates the matrix), `add` adds to them."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    valid = (i >= 0) & (j >= 0)
    keys = i[valid] * nbc + j[valid]
    ukeys, inv = np.unique(keys, return_inverse=True)
    br, bc = vals.shape[1], vals.shape[2]
    acc = np.zeros((len(ukeys), br, bc))
    np.add.at(acc, inv, vals[valid])
    rows = ukeys // nbc
    rowptr = np.zeros(nbr + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    colidx = ukeys % nbc
    if A is None or mode == "insert":
        return Bsr(nbr, nbc, br, bc, rowptr, colidx, acc)
    if not (np.array_equal(A.rowptr, rowptr) and np.array_equal(A.colidx, colidx)):
        raise ValueError("stream pattern differs from the matrix pattern")
    return A.with_values(A.val + acc)


# ----------------------------------------------------------------------------------
# Structural products and the Galerkin product (paper §2.1, §3.1, §3.5)
# ----------------------------------------------------------------------------------

def _pattern_csr(rowptr, colidx, nrows, ncols) -> sp.csr_matrix:
    data = np.ones(len(colidx), dtype=np.int64)
    return sp.csr_matrix((data, np.asarray(colidx, np.int64), np.asarray(rowptr, np.int64)),
                         shape=(nrows, ncols))


def structural_product(rpA, ciA, nrA, ncA, rpB, ciB, ncB):
    """Block pattern of A*B with no numerical dropping: block (I, K) is present iff
    some J has A_IJ and B_JK stored.  Counts are positive, so nothing cancels."""
    M = _pattern_csr(rpA, ciA, nrA, ncA) @ _pattern_csr(rpB, ciB, ncA, ncB)
    M = sp.csr_matrix(M)
    M.sort_indices()
    return M.indptr.astype(np.int64), M.indices.astype(np.int64)


def transpose_pattern(rp, ci, nr, nc):
    M = _pattern_csr(rp, ci, nr, nc).T.tocsr()
    M.sort_indices()
    return M.indptr.astype(np.int64), M.indices.astype(np.int64)


def reblock(M: sp.spmatrix, nbr: int, nbc: int, br: int, bc: int, rowptr, colidx) -> Bsr:
    """Place the scalar matrix M onto a given block pattern (every scalar nonzero of
    M must fall inside a stored block)."""
    C = sp.coo_matrix(M)
    rows_b = np.repeat(np.arange(nbr, dtype=np.int64), np.diff(rowptr))
    pk = rows_b * nbc + np.asarray(colidx, np.int64)
    key = (C.row.astype(np.int64) // br) * nbc + (C.col.astype(np.int64) // bc)
    pos = np.searchsorted(pk, key)
    ok = (pos < len(pk))
    ok[ok] = pk[pos[ok]] == key[ok]
    if not np.all(ok | (C.data == 0)):
        raise ValueError("scalar entry outside the block pattern")
    val = np.zeros((len(pk), br, bc))
    m = ok
    np.add.at(val, (pos[m], C.row[m] % br, C.col[m] % bc), C.data[m])
    return Bsr(nbr, nbc, br, bc, np.asarray(rowptr, np.int64), np.asarray(colidx, np.int64), val)


def ptap_pattern(A: Bsr, P: Bsr):
    """Patterns of AP and of A_c = P^T (A P) (structural, no dropping)."""
    rpAP, ciAP = structural_product(A.rowptr, A.colidx, A.nbr, A.nbc, P.rowptr, P.colidx, P.nbc)
    rpR, ciR = transpose_pattern(P.rowptr, P.colidx, P.nbr, P.nbc)
    rpC, ciC = structural_product(rpR, ciR, P.nbc, P.nbr, rpAP, ciAP, P.nbc)
    return (rpAP, ciAP), (rpC, ciC)


def ptap(A: Bsr, P: Bsr) -> Bsr:
    """Galerkin coarse operator A_c = P^T A P (paper §2.1, §2.2) on its structural
    pattern, computed in scalar CSR and re-blocked.  No symmetry is exploited."""
    if A.nbr != A.nbc or A.br != A.bc or P.nbr != A.nbc or P.br != A.bc:
        raise ValueError("shape mismatch")
    _, (rpC, ciC) = ptap_pattern(A, P)
    As = to_scalar_csr(A)
    Ps = to_scalar_csr(P)
    Cs = Ps.T.tocsr() @ (As @ Ps)
    return reblock(Cs, P.nbc, P.nbc, P.bc, P.bc, rpC, ciC)


def ptap_block(A: Bsr, P: Bsr, a: int, b: int, Pcol_rows=None) -> np.ndarray:
    """One block of P^T A P by its definition: sum over I, J of P_Ia^T A_IJ P_Jb.
    `Pcol_rows[a]` (block rows of P with a stored block in column a) may be given."""
    def pblock(I, c):
        for t in range(P.rowptr[I], P.rowptr[I + 1]):
            if P.colidx[t] == c:
                return P.val[t]
        return None
    rows_a = Pcol_rows[a] if Pcol_rows is not None else [
        I for I in range(P.nbr) if pblock(I, a) is not None]
    out = np.zeros((P.bc, P.bc))
    for I in rows_a:
        Pia = pblock(I, a)
        for t in range(A.rowptr[I], A.rowptr[I + 1]):
            J = A.colidx[t]
            Pjb = pblock(J, b)
            if Pjb is not None:
                out += Pia.T @ A.val[t] @ Pjb
    return out


def block_diag_inverse(A: Bsr) -> np.ndarray:
    """Inverses of the diagonal blocks A_II (point-block Jacobi, paper §4.1)."""
    D = np.empty((A.nbr, A.br, A.br))
    for I in range(A.nbr):
        row = A.colidx[A.rowptr[I]:A.rowptr[I + 1]]
        hit = np.nonzero(row == I)[0]
        if len(hit) != 1:
            raise ValueError(f"block row {I} has no diagonal block")
        D[I] = A.val[A.rowptr[I] + hit[0]]
    return np.linalg.inv(D)


def block_diag_apply(Dinv: np.ndarray, v: np.ndarray) -> np.ndarray:
    n, bs, _ = Dinv.shape
    if v.ndim == 1:
        return np.einsum("nij,nj->ni", Dinv, v.reshape(n, bs)).reshape(-1)
    return np.einsum("nij,njk->nik", Dinv, v.reshape(n, bs, -1)).reshape(n * bs, -1)
