"""Pins for the oracle's block-sparse definitions (SpMV, COO assembly, PtAP) and for
the assembled elasticity operator."""
import numpy as np
import pytest

import synth
from oracle import sparse as S
from oracle import sa, solve


def _bsr(nbr, nbc, br, bc, seed, **kw):
    rp, ci, v = synth.random_bsr(nbr, nbc, br, bc, seed, **kw)
    return S.Bsr(nbr, nbc, br, bc, rp.astype(np.int64), ci.astype(np.int64), v)


def _dense_loops(A):
    """Dense matrix filled scalar by scalar with explicit loops (independent of numpy
    slicing and of the CSR expansion)."""
    D = np.zeros(A.shape)
    for I in range(A.nbr):
        for t in range(A.rowptr[I], A.rowptr[I + 1]):
            for r in range(A.br):
                for c in range(A.bc):
                    D[I * A.br + r, A.colidx[t] * A.bc + c] += A.val[t, r, c]
    return D


@pytest.mark.parametrize("br,bc", [(3, 3), (3, 6), (6, 6), (6, 3), (1, 1), (2, 5)])
def test_spmv_against_dense(br, bc):
    A = _bsr(17, 11, br, bc, seed=br * 10 + bc, empty_row_frac=0.2)
    D = _dense_loops(A)
    rng = np.random.default_rng(0)
    for nrhs in (None, 3):
        shp = (A.nbc * bc,) if nrhs is None else (A.nbc * bc, nrhs)
        x = rng.uniform(-1, 1, shp)
        y0 = rng.uniform(-1, 1, (A.nbr * br,) if nrhs is None else (A.nbr * br, nrhs))
        y = S.spmv(A, x, 0.7, -1.3, y0)
        assert np.allclose(y, 0.7 * D @ x - 1.3 * y0, rtol=0, atol=1e-13)
        xt = rng.uniform(-1, 1, (A.nbr * br,) if nrhs is None else (A.nbr * br, nrhs))
        assert np.allclose(S.spmv_t(A, xt), D.T @ xt, rtol=0, atol=1e-13)
    rows = [0, 3, 16]
    x = rng.uniform(-1, 1, A.nbc * bc)
    assert np.allclose(S.spmv_rows(A, x, rows).reshape(-1),
                       (D @ x).reshape(A.nbr, br)[rows].reshape(-1), atol=1e-13)


def test_adjoint_identity():
    A = _bsr(40, 25, 3, 6, seed=3)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(A.nbc * 6)
    y = rng.standard_normal(A.nbr * 3)
    assert abs(y @ S.spmv(A, x) - S.spmv_t(A, y) @ x) < 1e-12 * np.abs(y).sum() * np.abs(x).sum()


def test_coo_against_add_at_with_duplicates_and_negatives():
    nbr, nbc = 13, 9
    i, j, v = synth.random_coo_stream(nbr, nbc, 3, 6, 500, seed=4, neg_frac=0.2, dup_pool=40)
    A = S.coo_assemble(nbr, nbc, i, j, v)
    ref = np.zeros((nbr * 3, nbc * 6))
    for k in range(len(i)):
        if i[k] >= 0 and j[k] >= 0:
            ref[i[k] * 3:(i[k] + 1) * 3, j[k] * 6:(j[k] + 1) * 6] += v[k]
    assert np.allclose(_dense_loops(A), ref, atol=1e-14)
    rp, ci, perm, seg = S.coo_plan(nbr, nbc, i, j)
    assert np.array_equal(rp, A.rowptr) and np.array_equal(ci, A.colidx)
    # index map: every valid entry exactly once, sorted by (row, col, position)
    valid = np.nonzero((i >= 0) & (j >= 0))[0]
    assert np.array_equal(np.sort(perm), valid)
    key = [(i[k], j[k], k) for k in perm]
    assert key == sorted(key)
    rows = A.block_rows()
    for t in range(A.nnzb):
        run = perm[seg[t]:seg[t + 1]]
        assert np.all(i[run] == rows[t]) and np.all(j[run] == A.colidx[t])
        assert np.allclose(A.val[t], v[run].sum(axis=0), atol=1e-14)
    # add mode
    A2 = S.coo_assemble(nbr, nbc, i, j, v, A=A, mode="add")
    assert np.allclose(A2.val, 2 * A.val)
    with pytest.raises(ValueError):
        S.coo_plan(nbr, nbc, np.array([nbr]), np.array([0]))


def test_empty_coo_stream():
    A = S.coo_assemble(4, 4, np.array([-1, -1]), np.array([-1, 2]), np.zeros((2, 3, 3)))
    assert A.nnzb == 0 and np.all(A.rowptr == 0)


def test_structural_product_brute_force():
    A = _bsr(12, 10, 1, 1, seed=7)
    B = _bsr(10, 8, 1, 1, seed=8)
    rp, ci = S.structural_product(A.rowptr, A.colidx, 12, 10, B.rowptr, B.colidx, 8)
    DA = _dense_loops(A) != 0
    DB = _dense_loops(B) != 0
    want = (DA.astype(int) @ DB.astype(int)) > 0
    got = np.zeros((12, 8), bool)
    for r in range(12):
        got[r, ci[rp[r]:rp[r + 1]]] = True
        assert np.all(np.diff(ci[rp[r]:rp[r + 1]]) > 0)
    assert np.array_equal(got, want)


def test_ptap_random_rectangular_against_dense():
    rp, ci, v = synth.random_spd_bsr(20, 3, seed=9)
    A = S.Bsr(20, 20, 3, 3, rp.astype(np.int64), ci.astype(np.int64), v)
    P = _bsr(20, 6, 3, 6, seed=10, max_per_row=3)
    C = S.ptap(A, P)
    DA, DP = _dense_loops(A), _dense_loops(P)
    ref = DP.T @ DA @ DP
    assert np.allclose(_dense_loops(C), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # block-by-block definition agrees
    for t in range(C.nnzb):
        a = C.block_rows()[t]
        b = C.colidx[t]
        assert np.allclose(S.ptap_block(A, P, a, b), C.val[t], atol=1e-12)


def _tiny_problem(n, clamp=True, seed=None):
    m = synth.make_mesh(n, clamp=clamp)
    i, j = synth.coo_indices(m)
    if seed is None:
        E, nu = synth.homogeneous_materials(m.n_elem)
    else:
        E, nu = synth.materials(m.n_elem, seed)
    v = synth.coo_values(m, *synth.lame(E, nu))
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v)
    return m, A


def test_assembled_operator_symmetric_and_rigid_modes():
    m, A = _tiny_problem(5, seed=3)
    D = S.to_scalar_csr(A)
    assert abs(D - D.T).max() < 1e-14 * abs(D).max()
    B = sa.rigid_body_modes(m.coords).reshape(-1, 6)
    AB = (D @ B).reshape(m.n_nodes, 3, 6)
    ii = np.rint(m.coords[:, 0] * m.n).astype(int)
    assert np.abs(AB[ii >= 2]).max() < 1e-12
    assert np.abs(AB[ii == 1]).max() > 1e-3      # next to the clamp the modes are not free
    mf, Af = _tiny_problem(4, clamp=False, seed=3)
    Bf = sa.rigid_body_modes(mf.coords).reshape(-1, 6)
    assert np.abs(S.to_scalar_csr(Af) @ Bf).max() < 1e-12


def test_patch_test_linear_field_homogeneous():
    m, A = _tiny_problem(4, clamp=False)
    G = np.array([[0.3, -0.2, 0.1], [0.05, 0.4, -0.3], [0.2, 0.1, -0.1]])
    u = (m.coords @ G.T).reshape(-1)
    r = (S.to_scalar_csr(A) @ u).reshape(-1, 3)
    g = np.rint(m.coords * m.n).astype(int)
    interior = np.all((g > 0) & (g < m.n), axis=1)
    assert np.abs(r[interior]).max() < 1e-13
    assert np.abs(r[~interior]).max() > 1e-3


def test_tiny_pattern_counts_and_galerkin_null_space():
    m, A = _tiny_problem(8)
    assert A.nnzb == 13831
    H = solve.setup(A, m.coords, m.dirichlet)
    P = H.levels[0].P
    (rpAP, ciAP), (rpC, ciC) = S.ptap_pattern(A, P)
    assert (P.nnzb, len(ciAP), len(ciC)) == (2028, 4624, 343)
    assert H.levels[1].A.nbr * 6 == 162
    # floating problem: P~ B_c = B and (A B = 0) => P B_c = B, hence A_c B_c = 0 on
    # every level (the Galerkin product keeps the near-null space)
    mf, A = _tiny_problem(6, clamp=False, seed=2)
    B = sa.rigid_body_modes(mf.coords)
    free = np.zeros(A.nbr, bool)
    for lev in range(2):
        nbrs = sa.strength_graph(A, free)
        agg, n_agg = sa.aggregate(nbrs, free)
        Pt, Bc = sa.tentative_prolongator(agg, n_agg, B)
        assert np.abs(S.spmv(Pt, Bc.reshape(-1, 6)) - B.reshape(-1, 6)).max() < 1e-12 * np.abs(B).max()
        Dinv = S.block_diag_inverse(A)
        lam, _, _ = sa.lanczos_lambda_max(A, Dinv)
        P = sa.smooth_prolongator(A, Pt, Dinv, lam)
        PB = S.spmv(P, Bc.reshape(-1, 6))
        assert np.abs(PB - B.reshape(-1, 6)).max() < 1e-11 * np.abs(B).max()
        Ac = S.ptap(A, P)
        absP = abs(S.to_scalar_csr(P))
        scale = (absP.T @ (abs(S.to_scalar_csr(A)) @ (absP @ np.abs(Bc.reshape(-1, 6))))).max()
        assert np.abs(S.to_scalar_csr(Ac) @ Bc.reshape(-1, 6)).max() < 1e-13 * scale
        A, B, free = Ac, Bc, np.zeros(Ac.nbr, bool)


def test_ptap_tiny_mesh_brute_force_and_symmetry():
    m, A = _tiny_problem(4, seed=6)
    H = solve.setup(A, m.coords, m.dirichlet, solve.Options(coarse_eq_limit=10))
    for lev in range(H.n_levels - 1):
        L = H.levels[lev]
        ref = _dense_loops(L.P).T @ _dense_loops(L.A) @ _dense_loops(L.P)
        got = _dense_loops(H.levels[lev + 1].A)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
        assert np.linalg.norm(got - got.T) <= 1e-14 * np.linalg.norm(got)


def test_symmetric_completion_pins():
    """S keeps the diagonal and upper blocks, its strictly lower part is the transpose of
    the upper part (so dense(S) - dense(S)^T vanishes outside the diagonal blocks), and
    S = A for a symmetric matrix; a pattern without mirrors is refused."""
    rp, ci, v = synth.random_spd_bsr(40, 3, seed=3, max_per_row=5)
    A = S.Bsr(40, 40, 3, 3, rp.astype(np.int64), ci.astype(np.int64), v)
    assert np.array_equal(S.symmetric_completion(A).val, A.val)
    # the same pattern with unrelated values
    W = A.with_values(np.random.default_rng(4).uniform(-1, 1, A.val.shape))
    Sw = S.symmetric_completion(W)
    rows = np.repeat(np.arange(W.nbr), np.diff(W.rowptr))
    up = W.colidx >= rows
    assert np.array_equal(Sw.val[up], W.val[up]) and not np.array_equal(Sw.val[~up], W.val[~up])
    D = S.to_dense(Sw)
    E = D - D.T
    for r in range(W.nbr):
        E[3 * r:3 * r + 3, 3 * r:3 * r + 3] = 0.0
    assert np.abs(E).max() == 0.0
    # x^T S y = y^T S x up to the diagonal blocks' asymmetry
    Dg = np.zeros_like(D)
    for r in range(W.nbr):
        Dg[3 * r:3 * r + 3, 3 * r:3 * r + 3] = D[3 * r:3 * r + 3, 3 * r:3 * r + 3]
    x, y = np.random.default_rng(5).uniform(-1, 1, (2, 120))
    assert abs(x @ S.spmv(Sw, y) - y @ S.spmv(Sw, x) - (x @ Dg @ y - y @ Dg @ x)) <= 1e-12
    # a lower block without its mirror
    bad = S.Bsr(2, 2, 1, 1, np.array([0, 1, 2]), np.array([0, 0]), np.ones((2, 1, 1)))
    with pytest.raises(AssertionError):
        S.symmetric_completion(bad)
