"""Pins for the oracle's smoother, V-cycle, coarse solve, PCG and hot recompute."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synth
from oracle import sparse as S
from oracle import sa, solve


def _problem(n, seed=None, clamp=True):
    m = synth.make_mesh(n, clamp=clamp)
    i, j = synth.coo_indices(m)
    E, nu = synth.homogeneous_materials(m.n_elem) if seed is None else synth.materials(m.n_elem, seed)
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, synth.coo_values(m, *synth.lame(E, nu)))
    return m, A


def _dense_D(A):
    D = np.zeros(A.shape)
    for I in range(A.nbr):
        for t in range(A.rowptr[I], A.rowptr[I + 1]):
            if A.colidx[t] == I:
                D[I * A.br:(I + 1) * A.br, I * A.br:(I + 1) * A.br] = A.val[t]
    return D


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_chebyshev_error_polynomial_closed_form(degree):
    """x0 = e_j, f = 0: the smoother returns p_k(D^-1 A) e_j with
    p_k(l) = T_k((b+a-2l)/(b-a)) / T_k((b+a)/(b-a))."""
    m, A = _problem(3, seed=4)
    Dinv = S.block_diag_inverse(A)
    lam = 2.0
    a, b = 0.1 * lam, 1.1 * lam
    Ad, Dd = S.to_dense(A), _dense_D(A)
    w, W = sla.eigh(Ad, Dd)             # D^-1 A = W diag(w) W^T D
    T = np.polynomial.chebyshev.Chebyshev.basis(degree)
    p = T((b + a - 2 * w) / (b - a)) / T((b + a) / (b - a))
    Pm = W @ np.diag(p) @ W.T @ Dd
    n = A.nbr * 3
    for j in (5, 40, n - 1):
        e = np.zeros(n)
        e[j] = 1.0
        got = solve.chebyshev(A, Dinv, lam, np.zeros(n), e, degree)
        assert np.abs(got - Pm[:, j]).max() < 1e-12
    f = np.random.default_rng(0).uniform(-1, 1, n)
    got = solve.chebyshev(A, Dinv, lam, f, None, degree)
    want = (np.eye(n) - Pm) @ np.linalg.solve(Ad, f)
    assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()


def test_coarse_solve_matches_cho_solve():
    m, A = _problem(3, seed=1)
    L = solve.coarse_factor(A)
    f = np.random.default_rng(2).uniform(-1, 1, A.nbr * 3)
    Ad = S.to_dense(A)
    want = sla.cho_solve(sla.cho_factor(Ad, lower=True), f)
    assert np.abs(solve.coarse_solve(L, f) - want).max() < 1e-12 * np.abs(want).max()


def test_vcycle_symmetric_positive():
    m, A = _problem(8, seed=3)
    H = solve.setup(A, m.coords, m.dirichlet)
    rng = np.random.default_rng(7)
    u = rng.standard_normal(m.n_dof)
    v = rng.standard_normal(m.n_dof)
    Mu, Mv = solve.vcycle(H, u), solve.vcycle(H, v)
    assert abs(Mu @ v - u @ Mv) <= 1e-12 * np.linalg.norm(Mu) * np.linalg.norm(v)
    assert u @ Mu > 0 and v @ Mv > 0


def test_level_sizes():
    m, A = _problem(8)
    H = solve.setup(A, m.coords, m.dirichlet)
    assert [L.A.nbr * L.A.br for L in H.levels] == [2187, 162]
    m, A = _problem(16, seed=1)
    H = solve.setup(A, m.coords, m.dirichlet)
    assert [L.A.nbr * L.A.br for L in H.levels] == [14739, 1296, 48]
    assert [L.A.nnzb for L in H.levels] == [110735, 4096, 64]
    assert H.levels[0].P.nnzb == 18954


@pytest.mark.parametrize("n,seed", [(8, None), (10, 5)])
def test_pcg_iterations_match_scipy_cg(n, seed):
    m, A = _problem(n, seed=seed)
    H = solve.setup(A, m.coords, m.dirichlet)
    b = synth.rhs(m, 0)
    x, it, rel, ok = solve.pcg(A, b, lambda r: solve.vcycle(H, r), rtol=1e-8)
    assert ok and rel <= 1e-8
    As = S.to_scalar_csr(A)
    assert np.linalg.norm(b - As @ x) <= 2e-8 * np.linalg.norm(b)
    count = [0]
    M = spla.LinearOperator(As.shape, matvec=lambda r: solve.vcycle(H, r))
    xs, info = spla.cg(As, b, rtol=1e-8, atol=0.0, M=M, maxiter=200,
                       callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert info == 0
    assert abs(count[0] - it) <= 1
    assert np.linalg.norm(xs - x) <= 1e-6 * np.linalg.norm(x)


def test_pcg_zero_rhs_and_breakdown():
    m, A = _problem(3)
    H = solve.setup(A, m.coords, m.dirichlet)
    x, it, rel, ok = solve.pcg(A, np.zeros(m.n_dof), lambda r: solve.vcycle(H, r))
    assert it == 0 and ok and not np.any(x)
    neg = A.with_values(-A.val)
    with pytest.raises(solve.Breakdown):
        solve.pcg(neg, synth.rhs(m, 1), lambda r: r)


def test_recompute_matches_fresh_galerkin_on_fixed_p():
    m, A = _problem(5, seed=8)
    H = solve.setup(A, m.coords, m.dirichlet, solve.Options(coarse_eq_limit=20))
    i, j = synth.coo_indices(m)
    E, nu = synth.materials(m.n_elem, 1008)
    A2 = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, synth.coo_values(m, *synth.lame(E, nu)))
    H2 = solve.recompute(H, A2)
    assert H2.n_levels == H.n_levels
    Ad = S.to_dense(A2)
    for lev in range(H.n_levels - 1):
        P = S.to_dense(H.levels[lev].P)
        Ad = P.T @ Ad @ P
        got = S.to_dense(H2.levels[lev + 1].A)
        assert np.linalg.norm(got - Ad) <= 1e-13 * np.linalg.norm(Ad)
    # recompute on unchanged values reproduces the setup
    H3 = solve.recompute(H, A)
    for L, L3 in zip(H.levels, H3.levels):
        assert np.array_equal(L.A.val, L3.A.val)
        if L.lam is not None:
            assert L.lam == L3.lam
