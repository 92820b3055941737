"""Algorithmic byte and flop models of the hot kernels (what the method must move),
used to turn measured times into achieved bandwidth.

Index type int32 (4 B).  Vectors are read once and written once per call (the ideal
with the gathered vector served from cache).  The per-block accounting follows the
paper's SpMV argument (§4.2: 72 B of FP64 values plus one 4 B index per 3x3 block,
against 9 indices for scalar CSR).
"""
from __future__ import annotations

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (packed)

IDX = 4


def block_bytes(br: int, bc: int, val_size: int, blocked: bool = True) -> int:
    """Bytes of one stored br x bc block: values plus index data."""
    vals = br * bc * val_size
    return vals + (IDX if blocked else br * bc * IDX)


def spmv_bytes(nbr: int, nbc: int, br: int, bc: int, nnzb: int, val_size: int, vec_size: int,
               nrhs: int = 1, beta_read: bool = False) -> int:
    """y = A x: values + column indices + row pointers + x once + y once (+ y read if beta != 0)."""
    b = nnzb * block_bytes(br, bc, val_size) + IDX * (nbr + 1)
    b += vec_size * nrhs * (nbc * bc + nbr * br)
    if beta_read:
        b += vec_size * nrhs * nbr * br
    return b


def spmv_sym_bytes(nbr: int, bs: int, n_upper: int, n_lower: int, val_size: int, vec_size: int) -> int:
    """Symmetric reads of a square-blocked symmetric A (bsr_spmv_sym): the diagonal and
    upper blocks once (values + column index), a column index and a mirror index per
    strictly lower block (its values are the transposed mirror, already read), row
    pointers, x once and y once."""
    b = n_upper * block_bytes(bs, bs, val_size) + n_lower * 2 * IDX + IDX * (nbr + 1)
    return b + vec_size * 2 * nbr * bs


def spmv_flops(nnzb: int, br: int, bc: int, nrhs: int = 1) -> int:
    return 2 * nnzb * br * bc * nrhs


def ptap_bytes(a_nbr: int, a_nnzb: int, bs: int, p_nnzb: int, p_bc: int, c_nbr: int, c_nnzb: int,
               a_val: int, p_val: int) -> int:
    """One level of A_c = P^T A P: read A (values, indices, row pointers) and P once, write
    A_c values and read its pattern."""
    b = a_nnzb * block_bytes(bs, bs, a_val) + IDX * (a_nbr + 1)
    b += p_nnzb * block_bytes(bs, p_bc, p_val) + IDX * (a_nbr + 1)
    b += c_nnzb * (p_bc * p_bc * a_val + IDX) + IDX * (c_nbr + 1)
    return b


def ptap_flops(pairs_ap: int, pairs_rap: int, bs: int, nc: int) -> int:
    """2*bs*bs*nc per (A block, P block) product and 2*nc*bs*nc per (P^T block, AP block)."""
    return 2 * bs * bs * nc * pairs_ap + 2 * nc * bs * nc * pairs_rap


def coo_bytes(n_coo: int, nnzb: int, br: int, bc: int, val_size: int) -> int:
    """Blocked COO assembly: read every stream block and its map entry once, write A once."""
    return n_coo * (br * bc * val_size + IDX) + nnzb * br * bc * val_size + IDX * (nnzb + 1)


def pcg_iteration_bytes(levels, hier_val: int, p_val: int) -> int:
    """One PCG iteration with a Chebyshev(2) V-cycle: the fine FP64 SpMV of CG (A p),
    per smoothed level four operator SpMVs, the prolongation and the restriction and
    about 14 vector passes in the hierarchy's type, plus about 10 fine FP64 vector
    passes of the CG recurrence (the coarsest dense solve is not counted).  levels:
    dicts with nbr, bs, nnzb and p_nnzb (blocks of the prolongator to the next level,
    0 on the coarsest)."""
    f = levels[0]
    n0 = f["nbr"] * f["bs"]
    b = spmv_bytes(f["nbr"], f["nbr"], f["bs"], f["bs"], f["nnzb"], 8, 8) + 10 * 8 * n0
    for l in range(len(levels) - 1):
        d, c = levels[l], levels[l + 1]
        n = d["nbr"] * d["bs"]
        b += 4 * spmv_bytes(d["nbr"], d["nbr"], d["bs"], d["bs"], d["nnzb"], hier_val, hier_val)
        b += 2 * spmv_bytes(d["nbr"], c["nbr"], d["bs"], c["bs"], d["p_nnzb"], p_val, hier_val)
        b += 14 * hier_val * n
    return b
