"""Random blocked-sparse fixtures (seeded) for kernel-level tests.

Only random patterns and values are produced here; no product or reduction of them.
A block matrix is returned as (rowptr int32[nbr+1], colidx int32[nnzb] sorted and
unique within each row, val float64[nnzb, bs_r, bs_c] row-major blocks).
"""
from __future__ import annotations

import numpy as np


def random_bsr(nbr: int, nbc: int, bs_r: int, bs_c: int, seed: int,
               max_per_row: int = 8, empty_row_frac: float = 0.0, dtype=np.float64):
    rng = np.random.default_rng(seed)
    counts = rng.integers(1, max(2, min(max_per_row, nbc) + 1), size=nbr) if nbc > 0 else np.zeros(nbr, int)
    if empty_row_frac > 0:
        counts[rng.random(nbr) < empty_row_frac] = 0
    cols = []
    for r in range(nbr):
        c = rng.choice(nbc, size=int(min(counts[r], nbc)), replace=False) if nbc > 0 else np.zeros(0, int)
        cols.append(np.sort(c))
    rowptr = np.zeros(nbr + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum([len(c) for c in cols])
    colidx = np.concatenate(cols).astype(np.int32) if nbr else np.zeros(0, np.int32)
    val = rng.uniform(-1.0, 1.0, size=(len(colidx), bs_r, bs_c)).astype(dtype)
    return rowptr, colidx, val


def random_spd_bsr(nbr: int, bs: int, seed: int, max_per_row: int = 6):
    """Symmetric positive-definite block matrix with a symmetric random pattern
    (off-diagonal blocks random, diagonal blocks made strongly dominant)."""
    rng = np.random.default_rng(seed)
    pairs = set()
    for r in range(nbr):
        for c in rng.choice(nbr, size=min(max_per_row, nbr), replace=False):
            if c != r:
                pairs.add((r, int(c)))
                pairs.add((int(c), r))
    for r in range(nbr):
        pairs.add((r, r))
    keys = sorted(pairs)
    rows = np.array([k[0] for k in keys], dtype=np.int64)
    cols = np.array([k[1] for k in keys], dtype=np.int64)
    rowptr = np.zeros(nbr + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    val = np.zeros((len(keys), bs, bs))
    pos = {k: t for t, k in enumerate(keys)}
    for t, (r, c) in enumerate(keys):
        if r < c:
            blk = rng.uniform(-1.0, 1.0, size=(bs, bs))
            val[t] = blk
            val[pos[(c, r)]] = blk.T
    rowsum = np.zeros(nbr)
    for t, (r, c) in enumerate(keys):
        if r != c:
            rowsum[r] += np.abs(val[t]).sum()
    for r in range(nbr):
        m = rng.uniform(-0.5, 0.5, size=(bs, bs))
        val[pos[(r, r)]] = 0.5 * (m + m.T) + (rowsum[r] + bs + 1.0) * np.eye(bs)
    return rowptr, cols.astype(np.int32), val


def random_coo_stream(nbr: int, nbc: int, bs_r: int, bs_c: int, n: int, seed: int,
                      neg_frac: float = 0.1, dup_pool: int | None = None):
    """A block COO stream with duplicates and ignored (negative) coordinates.
    `dup_pool` limits the number of distinct (i, j) so that duplicates are frequent."""
    rng = np.random.default_rng(seed)
    if dup_pool:
        pi = rng.integers(0, nbr, size=dup_pool)
        pj = rng.integers(0, nbc, size=dup_pool)
        pick = rng.integers(0, dup_pool, size=n)
        i = pi[pick]
        j = pj[pick]
    else:
        i = rng.integers(0, nbr, size=n)
        j = rng.integers(0, nbc, size=n)
    neg = rng.random(n) < neg_frac
    which = rng.integers(0, 3, size=n)
    i = np.where(neg & (which != 1), -1 - rng.integers(0, 3, size=n), i)
    j = np.where(neg & (which != 0), -1 - rng.integers(0, 3, size=n), j)
    v = rng.uniform(-1.0, 1.0, size=(n, bs_r, bs_c))
    return i.astype(np.int32), j.astype(np.int32), v
