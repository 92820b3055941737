"""Solve phase: Chebyshev / point-block-Jacobi smoother, V-cycle, preconditioned CG,
and the smoothed-aggregation hierarchy with its hot recompute (paper §2.1, §3.1, §4.1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import sparse as S
from . import sa


@dataclass
class Options:
    max_levels: int = 10
    coarse_eq_limit: int = 1000     # reading: stop coarsening at <= 1000 dofs
    strength_eps: float = 0.0       # reading: structural strength graph
    cheb_degree: int = 2
    cheb_lo: float = 0.1            # reading: Chebyshev interval [0.1, 1.1] * lambda_hat
    cheb_hi: float = 1.1
    lanczos_steps: int = 10
    lanczos_seed: int = sa.LANCZOS_SEED
    omega_scale: float = 4.0 / 3.0
    agg_mode: str = "greedy"        # "greedy" (natural order) or "luby" (parallel rounds)
    agg_seed: int = sa.LUBY_SEED


@dataclass
class Level:
    A: S.Bsr
    P: S.Bsr | None = None
    Dinv: np.ndarray | None = None
    lam: float | None = None
    agg: np.ndarray | None = None
    n_agg: int = 0


@dataclass
class Hierarchy:
    levels: list = field(default_factory=list)
    chol: np.ndarray | None = None   # lower Cholesky factor of the coarsest operator
    opts: Options = field(default_factory=Options)

    @property
    def n_levels(self) -> int:
        return len(self.levels)


def chebyshev(A: S.Bsr, Dinv: np.ndarray, lam: float, f: np.ndarray, x0=None,
              degree: int = 2, lo: float = 0.1, hi: float = 1.1) -> np.ndarray:
    """Chebyshev acceleration of point-block Jacobi (Saad, Iterative Methods for Sparse
    Linear Systems, 2nd ed., Alg. 12.1, with the residual replaced by D^-1 r) on the
    interval [lo*lam, hi*lam].  x0 = None means a zero initial guess (no SpMV)."""
    a = lo * lam
    b = hi * lam
    theta = 0.5 * (b + a)
    delta = 0.5 * (b - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x0 is None:
        x = np.zeros_like(f)
        r = f.copy()
    else:
        x = x0.copy()
        r = f - S.spmv(A, x)
    d = S.block_diag_apply(Dinv, r) / theta
    for t in range(1, degree + 1):
        x = x + d
        if t < degree:
            r = r - S.spmv(A, d)
            rho1 = 1.0 / (2.0 * sigma - rho)
            d = rho1 * rho * d + (2.0 * rho1 / delta) * S.block_diag_apply(Dinv, r)
            rho = rho1
    return x


def coarse_factor(A: S.Bsr) -> np.ndarray:
    """Dense Cholesky factor (lower) of the coarsest operator."""
    return np.linalg.cholesky(S.to_scalar_csr(A).toarray())


def coarse_solve(L: np.ndarray, f: np.ndarray) -> np.ndarray:
    y = sla.solve_triangular(L, f, lower=True)
    return sla.solve_triangular(L.T, y, lower=False)


def vcycle(H: Hierarchy, f: np.ndarray, level: int = 0) -> np.ndarray:
    """One V-cycle from a zero guess (paper §2.1): pre-smooth, residual, restrict with
    P^T, recurse, prolong and add, post-smooth; the coarsest level is solved exactly.
    The same polynomial smoother before and after makes the preconditioner symmetric."""
    o = H.opts
    if level == H.n_levels - 1:
        return coarse_solve(H.chol, f)
    L = H.levels[level]
    x = chebyshev(L.A, L.Dinv, L.lam, f, None, o.cheb_degree, o.cheb_lo, o.cheb_hi)
    r = f - S.spmv(L.A, x)
    xc = vcycle(H, S.spmv_t(L.P, r), level + 1)
    x = x + S.spmv(L.P, xc)
    x = chebyshev(L.A, L.Dinv, L.lam, f, x, o.cheb_degree, o.cheb_lo, o.cheb_hi)
    return x


class Breakdown(RuntimeError):
    pass


def pcg(A: S.Bsr, b: np.ndarray, precond, rtol: float = 1e-8, maxit: int = 1000):
    """Preconditioned conjugate gradients (the CG accelerator of paper §4.1) from x0 = 0.
    The stopping test uses the unpreconditioned recurrence residual, ||r|| <= rtol ||b||
    (paper §4.1 uses the unpreconditioned norm).  The iteration count is the number of
    solution updates.  Returns (x, iterations, ||r||/||b||, converged)."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0.0, True
    z = precond(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        w = S.spmv(A, p)
        pw = p @ w
        if not pw > 0.0:
            raise Breakdown("p^T A p <= 0")
        alpha = rz / pw
        x = x + alpha * p
        r = r - alpha * w
        it += 1
        rn = np.linalg.norm(r)
        if rn <= rtol * bn:
            return x, it, rn / bn, True
        z = precond(r)
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, it, np.linalg.norm(r) / bn, False


def setup(A0: S.Bsr, coords: np.ndarray, dirichlet: np.ndarray, opts: Options | None = None,
          level_params=None) -> Hierarchy:
    """Cold setup (paper §3.1, §3.2): per level aggregate, build P~ from the near-null
    space, estimate lambda_max, smooth P, form A_c = P^T A P; stop when the level has at
    most `coarse_eq_limit` dofs or `max_levels` is reached; factor the coarsest level.
    `level_params[l] = (lambda_hat, omega)` replaces level l's Lanczos estimate and its
    prolongator-smoothing weight (for a hierarchy whose estimates came from elsewhere,
    such as the learned eigenbound); None keeps the method's own."""
    o = opts or Options()
    H = Hierarchy(opts=o)
    A = A0
    B = sa.rigid_body_modes(coords)
    dmask = np.asarray(dirichlet, dtype=bool)
    lev = 0
    while A.nbr * A.br > o.coarse_eq_limit and lev < o.max_levels - 1:
        nbrs = sa.strength_graph(A, dmask, o.strength_eps)
        if o.agg_mode == "luby":
            agg, n_agg, _ = sa.aggregate_luby(nbrs, dmask, o.agg_seed)
        else:
            agg, n_agg = sa.aggregate(nbrs, dmask)
        if n_agg == 0:
            break
        Pt, Bc = sa.tentative_prolongator(agg, n_agg, B)
        Dinv = S.block_diag_inverse(A)
        if level_params is not None and level_params[lev] is not None:
            lam, omega = level_params[lev]
        else:
            lam, _, _ = sa.lanczos_lambda_max(A, Dinv, o.lanczos_steps, o.lanczos_seed + lev)
            omega = None
        P = sa.smooth_prolongator(A, Pt, Dinv, lam, o.omega_scale, omega)
        H.levels.append(Level(A=A, P=P, Dinv=Dinv, lam=lam, agg=agg, n_agg=n_agg))
        A = S.ptap(A, P)
        B = Bc
        dmask = np.zeros(A.nbr, dtype=bool)
        lev += 1
    H.levels.append(Level(A=A))
    H.chol = coarse_factor(A)
    return H


def recompute(H: Hierarchy, A0_new: S.Bsr) -> Hierarchy:
    """Hot recompute with reused interpolation (paper §3.1, §3.5): the prolongators and
    all patterns stay fixed; A_c = P^T A P is recomputed numerically on every level and
    the smoother data (block-diagonal inverses, lambda_hat) and the coarsest factor
    are refreshed."""
    o = H.opts
    new = Hierarchy(opts=o)
    A = A0_new
    for lev, L in enumerate(H.levels[:-1]):
        Dinv = S.block_diag_inverse(A)
        lam, _, _ = sa.lanczos_lambda_max(A, Dinv, o.lanczos_steps, o.lanczos_seed + lev)
        new.levels.append(Level(A=A, P=L.P, Dinv=Dinv, lam=lam, agg=L.agg, n_agg=L.n_agg))
        Ac = S.ptap(A, L.P)
        old = H.levels[lev + 1].A
        if not (np.array_equal(Ac.rowptr, old.rowptr) and np.array_equal(Ac.colidx, old.colidx)):
            raise ValueError("recompute changed a coarse pattern")
        A = Ac
    new.levels.append(Level(A=A))
    new.chol = coarse_factor(A)
    return new
