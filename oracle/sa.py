"""Smoothed-aggregation setup (paper §2.2, §2.3, §3.2): strength graph, greedy
aggregation, rigid-body near-null space, tentative prolongator, lambda_max estimate,
damped-Jacobi prolongator smoothing.  Plain loops; FP64.
"""
from __future__ import annotations

import numpy as np

from . import sparse as S
from .mix import splitmix64, start_vector

LANCZOS_SEED = 0x5EED
LUBY_SEED = 0x4D495332


def strength_graph(A: S.Bsr, dirichlet: np.ndarray, eps: float = 0.0):
    """Neighbour lists of the aggregation graph (paper §2.2 strong coupling, §3.2 graph
    over blocks): vertices are the non-Dirichlet block rows; j != i is a neighbour of i
    iff A_ij is stored, j is not Dirichlet and ||A_ij||_F >= eps sqrt(||A_ii||_F ||A_jj||_F).
    Reading: Frobenius block norm; eps = 0 gives the structural graph."""
    n = A.nbr
    rp = A.rowptr
    ci = A.colidx
    if eps > 0.0:
        nrm = np.sqrt((A.val ** 2).sum(axis=(1, 2)))
        dn = np.zeros(n)
        for i in range(n):
            for t in range(rp[i], rp[i + 1]):
                if ci[t] == i:
                    dn[i] = nrm[t]
    nbrs = []
    for i in range(n):
        if dirichlet[i]:
            nbrs.append([])
            continue
        lst = []
        for t in range(rp[i], rp[i + 1]):
            j = int(ci[t])
            if j == i or dirichlet[j]:
                continue
            if eps > 0.0 and nrm[t] < eps * np.sqrt(dn[i] * dn[j]):
                continue
            lst.append(j)
        nbrs.append(lst)
    return nbrs


def aggregate(nbrs, dirichlet: np.ndarray):
    """Greedy disjoint covering (paper §2.2), as greedy distance-2 MIS in natural order.

    Phase 1: visiting i = 0, 1, ... in order, a non-Dirichlet, unaggregated i whose
    neighbours are all unaggregated becomes a root, and {i} plus its neighbours form
    the next aggregate.  Phase 2 (reading; the paper does not say how leftovers are
    placed): an unaggregated non-Dirichlet i joins the phase-1 aggregate that holds the
    most of its neighbours, ties going to the smallest aggregate id; only phase-1
    labels are counted, so the result does not depend on the visiting order.  A node
    with no aggregated neighbour (impossible after phase 1, kept for completeness)
    forms its own aggregate.  Dirichlet nodes stay unaggregated (-1).
    Returns (agg[n] int64, n_agg)."""
    n = len(nbrs)
    agg = [-1] * n
    n_agg = 0
    for i in range(n):
        if dirichlet[i] or agg[i] >= 0:
            continue
        if all(agg[j] < 0 for j in nbrs[i]):
            agg[i] = n_agg
            for j in nbrs[i]:
                agg[j] = n_agg
            n_agg += 1
    phase1 = list(agg)
    for i in range(n):
        if dirichlet[i] or phase1[i] >= 0:
            continue
        count = {}
        for j in nbrs[i]:
            g = phase1[j]
            if g >= 0:
                count[g] = count.get(g, 0) + 1
        if count:
            best = max(count.values())
            agg[i] = min(g for g, c in count.items() if c == best)
        else:
            agg[i] = n_agg
            n_agg += 1
    return np.array(agg, dtype=np.int64), n_agg


def luby_keys(n: int, seed: int) -> list:
    """Priority of vertex i in the parallel aggregation: the high 32 bits of
    splitmix64(seed XOR i) above i + 1 in the low 32 bits, so keys are distinct and
    positive (0 is free to mean "none")."""
    return [((splitmix64(seed ^ i) >> 32) << 32) | (i + 1) for i in range(n)]


def _within2(nbrs, i):
    """Vertices at graph distance 1 or 2 from i (i excluded)."""
    out = set(nbrs[i])
    for j in nbrs[i]:
        out.update(nbrs[j])
    out.discard(i)
    return out


def aggregate_luby(nbrs, dirichlet: np.ndarray, seed: int = LUBY_SEED):
    """Parallel disjoint covering (paper §6, the device MIS coarsener: Luby rounds with
    deterministic hash priorities), in the notation of `aggregate`.

    Distance-2 MIS by rounds: every undecided vertex whose key exceeds the keys of all
    undecided vertices within distance 2 becomes a root; then every undecided vertex
    within distance 2 of a new root is decided (not a root).  Repeat until no vertex is
    undecided.  Roots are numbered in increasing vertex order.  Phase 1: each neighbour
    of a root joins that root's aggregate (roots are at least 3 apart, so the root is
    unique).  Phase 2: a remaining vertex joins the phase-1 aggregate that holds the most
    of its neighbours, ties going to the smallest aggregate id (as in `aggregate`).
    Dirichlet vertices stay unaggregated (-1).  Returns (agg[n] int64, n_agg, rounds)."""
    n = len(nbrs)
    key = luby_keys(n, seed)
    UND, ROOT, OUT = 0, 1, 2
    state = [OUT if dirichlet[i] else UND for i in range(n)]
    rounds = 0
    while any(s == UND for s in state):
        rounds += 1
        new = [i for i in range(n) if state[i] == UND and
               all(not (state[j] == UND and key[j] > key[i]) for j in _within2(nbrs, i))]
        for i in new:
            state[i] = ROOT
        for i in new:
            for j in _within2(nbrs, i):
                if state[j] == UND:
                    state[j] = OUT
    agg = [-1] * n
    n_agg = 0
    for i in range(n):
        if state[i] == ROOT:
            agg[i] = n_agg
            n_agg += 1
    phase1 = list(agg)
    for i in range(n):
        if dirichlet[i] or phase1[i] >= 0:
            continue
        roots = [phase1[j] for j in nbrs[i] if state[j] == ROOT]
        if roots:
            agg[i] = roots[0]
    phase1 = list(agg)
    for i in range(n):
        if dirichlet[i] or phase1[i] >= 0:
            continue
        count = {}
        for j in nbrs[i]:
            g = phase1[j]
            if g >= 0:
                count[g] = count.get(g, 0) + 1
        best = max(count.values())
        agg[i] = min(g for g, c in count.items() if c == best)
    return np.array(agg, dtype=np.int64), n_agg, rounds


def rigid_body_modes(coords: np.ndarray) -> np.ndarray:
    """Near-null space of 3D elasticity (paper §2.2, §2.3): six rigid-body modes per
    node, columns t_x, t_y, t_z, r_z = (-y, x, 0), r_x = (0, -z, y), r_y = (z, 0, -x)
    (reading: this column order and sign).  Shape [n_nodes, 3, 6]."""
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    n = len(coords)
    B = np.zeros((n, 3, 6))
    B[:, 0, 0] = 1.0
    B[:, 1, 1] = 1.0
    B[:, 2, 2] = 1.0
    B[:, 0, 3] = -y
    B[:, 1, 3] = x
    B[:, 1, 4] = -z
    B[:, 2, 4] = y
    B[:, 0, 5] = z
    B[:, 2, 5] = -x
    return B


def tentative_prolongator(agg: np.ndarray, n_agg: int, B: np.ndarray, rank_tol: float = 1e-10):
    """Tentative prolongator (paper §2.2): per aggregate g, stack the near-null-space
    rows of its members in ascending node order, B_g = Q_g R_g (thin QR, reading:
    diag(R_g) > 0 fixes the signs).  Member rows of P~ are the rows of Q_g (one block
    of bs x 6 per fine row, in column g); the coarse near-null space is R_g.
    Returns (P~ as Bsr, B_coarse [n_agg, 6, 6])."""
    nbr, bs, nc = B.shape
    members = [[] for _ in range(n_agg)]
    for i in range(nbr):
        if agg[i] >= 0:
            members[agg[i]].append(i)
    Pval = np.zeros((nbr, bs, nc))
    Bc = np.zeros((n_agg, nc, nc))
    for g in range(n_agg):
        m = members[g]
        Bg = B[m].reshape(len(m) * bs, nc)
        if Bg.shape[0] < nc:
            raise ValueError(f"aggregate {g} too small for the near-null space")
        Q, R = np.linalg.qr(Bg, mode="reduced")
        d = np.diag(R)
        if np.any(np.abs(d) <= rank_tol * max(1.0, np.abs(Bg).max())):
            raise ValueError(f"aggregate {g}: near-null space rank deficient")
        s = np.sign(d)
        Q = Q * s[None, :]
        R = R * s[:, None]
        Pval[m] = Q.reshape(len(m), bs, nc)
        Bc[g] = R
    rows = np.nonzero(agg >= 0)[0]
    rowptr = np.zeros(nbr + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(agg >= 0)
    P = S.Bsr(nbr, n_agg, bs, nc, rowptr, agg[rows].astype(np.int64), Pval[rows])
    return P, Bc


def lanczos_lambda_max(A: S.Bsr, Dinv: np.ndarray, k: int = 10, seed: int = LANCZOS_SEED):
    """Estimate of lambda_max(D^-1 A), D = block diagonal of A (reading; the paper does
    not say how the eigen-estimate is formed): k steps of Lanczos on D^-1 A in the
    D inner product (equivalently on D^-1/2 A D^-1/2), no reorthogonalisation, start
    vector from `mix.start_vector(n, seed)`.  Returns (lambda_hat, alphas, betas)."""
    n = A.nbr * A.br
    Dblk = np.linalg.inv(Dinv)
    As = S.to_scalar_csr(A)
    v = start_vector(n, seed)
    Dv = S.block_diag_apply(Dblk, v)
    nrm = np.sqrt(v @ Dv)
    u = v / nrm
    y = Dv / nrm
    u_prev = np.zeros(n)
    y_prev = np.zeros(n)
    beta_prev = 0.0
    alphas, betas = [], []
    for step in range(k):
        wy = As @ u - beta_prev * y_prev
        alpha = u @ wy
        wy = wy - alpha * y
        wu = S.block_diag_apply(Dinv, wy)
        beta = np.sqrt(max(wu @ wy, 0.0))
        alphas.append(alpha)
        if step == k - 1 or beta == 0.0:
            break
        betas.append(beta)
        u_prev, y_prev = u, y
        u = wu / beta
        y = wy / beta
        beta_prev = beta
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    lam = float(np.linalg.eigvalsh(T).max())
    return lam, np.array(alphas), np.array(betas)


def smooth_prolongator(A: S.Bsr, Pt: S.Bsr, Dinv: np.ndarray, lam: float,
                       omega_scale: float = 4.0 / 3.0, omega: float | None = None) -> S.Bsr:
    """Damped-Jacobi prolongator smoothing (paper §2.2): P = (I - omega D^-1 A) P~ with
    D the block diagonal (reading of "the diagonal" for the blocked method) and
    omega = 4 / (3 lambda_hat) (reading: the classical SA weight), or the weight given
    in `omega` (a weight from another estimate of lambda_max, such as a learned one).
    The pattern of P is the structural pattern of A P~ (no dropping)."""
    rp, ci = S.structural_product(A.rowptr, A.colidx, A.nbr, A.nbc, Pt.rowptr, Pt.colidx, Pt.nbc)
    AP = S.reblock(S.to_scalar_csr(A) @ S.to_scalar_csr(Pt), A.nbr, Pt.nbc, A.br, Pt.bc, rp, ci)
    PtOn = S.reblock(S.to_scalar_csr(Pt), A.nbr, Pt.nbc, A.br, Pt.bc, rp, ci)
    if omega is None:
        omega = omega_scale / lam
    rows = AP.block_rows()
    val = PtOn.val - omega * np.einsum("tij,tjk->tik", Dinv[rows], AP.val)
    return AP.with_values(val)
