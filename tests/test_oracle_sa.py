"""Pins for the oracle's smoothed-aggregation setup: aggregation closed form,
tentative prolongator, Lanczos estimate, prolongator smoothing, splitmix64."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import sparse as S
from oracle import sa, solve
from oracle.mix import splitmix64, splitmix64_array, start_vector


def _problem(n, seed=None, clamp=True):
    m = synth.make_mesh(n, clamp=clamp)
    i, j = synth.coo_indices(m)
    E, nu = synth.homogeneous_materials(m.n_elem) if seed is None else synth.materials(m.n_elem, seed)
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, synth.coo_values(m, *synth.lame(E, nu)))
    return m, A


def _axis_labels(lo, hi):
    """Greedy distance-2 roots on a path lo..hi sit at lo, lo+3, ...; root q covers
    [lo+3q-1, lo+3q+1]; the single leftover position after the last interval joins it."""
    p = np.arange(lo, hi + 1)
    nr = (hi - lo) // 3 + 1
    return np.minimum((p - lo + 1) // 3, nr - 1), nr


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 10, 11])
def test_aggregation_closed_form_clamped_cube(n):
    m, A = _problem(n)
    agg, n_agg = sa.aggregate(sa.strength_graph(A, m.dirichlet), m.dirichlet)
    qx, nx = _axis_labels(1, n)
    qy, ny = _axis_labels(0, n)
    g = np.rint(m.coords * n).astype(int)
    want = np.full(m.n_nodes, -1)
    free = g[:, 0] >= 1
    want[free] = qx[g[free, 0] - 1] + nx * (qy[g[free, 1]] + ny * qy[g[free, 2]])
    assert n_agg == ((n - 1) // 3 + 1) * (n // 3 + 1) ** 2 == nx * ny * ny
    assert np.array_equal(agg, want)


def test_aggregation_small_graph_by_hand():
    # path 0-1-2-3-4-5-6 : roots 0 and 3 take {0,1} and {2,3,4}; 5 joins {2,3,4}
    # (its only aggregated neighbour is 4); 6 is a root (neighbours 5 unaggregated).
    nbrs = [[1], [0, 2], [1, 3], [2, 4], [3, 5], [4, 6], [5]]
    agg, n = sa.aggregate(nbrs, np.zeros(7, bool))
    assert n == 3
    assert list(agg) == [0, 0, 1, 1, 1, 2, 2]
    # a tie: edges 0-1, 1-2, 2-4, 4-3; roots 0 ({0,1}) and 3 ({3,4}); 2 sees one node
    # of aggregate 0 and one of aggregate 1 -> the smaller id
    nbrs = [[1], [0, 2], [1, 4], [4], [2, 3]]
    agg, n = sa.aggregate(nbrs, np.zeros(5, bool))
    assert list(agg) == [0, 0, 0, 1, 1]
    # Dirichlet vertex stays out (the strength graph never lists it as a neighbour)
    agg, n = sa.aggregate([[], []], np.array([True, False]))
    assert list(agg) == [-1, 0] and n == 1


def test_strength_threshold_drops_weak_blocks():
    rp, ci, v = synth.random_spd_bsr(6, 3, seed=1)
    A = S.Bsr(6, 6, 3, 3, rp.astype(np.int64), ci.astype(np.int64), v)
    full = sa.strength_graph(A, np.zeros(6, bool), 0.0)
    strict = sa.strength_graph(A, np.zeros(6, bool), 10.0)
    assert sum(map(len, full)) == A.nnzb - 6
    assert sum(map(len, strict)) == 0


def test_tentative_prolongator_reproduces_near_null_space():
    m, A = _problem(8)
    agg, n_agg = sa.aggregate(sa.strength_graph(A, m.dirichlet), m.dirichlet)
    assert n_agg == 27
    B = sa.rigid_body_modes(m.coords)
    Pt, Bc = sa.tentative_prolongator(agg, n_agg, B)
    PB = S.spmv(Pt, Bc.reshape(-1, 6)).reshape(-1, 3, 6)
    assert np.abs(PB[~m.dirichlet] - B[~m.dirichlet]).max() < 1e-13
    assert np.all(PB[m.dirichlet] == 0)
    D = S.to_scalar_csr(Pt)
    assert np.abs((D.T @ D).toarray() - np.eye(162)).max() < 1e-13
    assert np.all(np.diagonal(Bc, axis1=1, axis2=2) > 0)
    # translation columns are origin independent
    Pt2, _ = sa.tentative_prolongator(agg, n_agg, sa.rigid_body_modes(m.coords + 3.0))
    assert np.abs(Pt2.val - Pt.val).max() < 1e-10
    with pytest.raises(ValueError):
        sa.tentative_prolongator(np.array([0, 0]), 1, B[:2])


def test_splitmix64_published_outputs():
    # the first two outputs of splitmix64 from state 0
    assert splitmix64(0) == 0xE220A8397B1DCDAF
    assert splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4
    st = np.array([0, 0x9E3779B97F4A7C15, 12345], dtype=np.uint64)
    assert [int(z) for z in splitmix64_array(st)] == [splitmix64(int(s)) for s in st]
    v = start_vector(1000, 0x5EED)
    assert v.min() >= -1 and v.max() < 1 and abs(v.mean()) < 0.1
    assert v[7] == 2.0 * ((splitmix64(0x5EED ^ 7) >> 11) * 2.0 ** -53) - 1.0


def _dense_D(A):
    D = np.zeros(A.shape)
    for I in range(A.nbr):
        for t in range(A.rowptr[I], A.rowptr[I + 1]):
            if A.colidx[t] == I:
                D[I * A.br:(I + 1) * A.br, I * A.br:(I + 1) * A.br] = A.val[t]
    return D


def test_lanczos_bounds_and_symmetric_form_equivalence():
    m, A = _problem(4, seed=5)
    Dinv = S.block_diag_inverse(A)
    lam, al, be = sa.lanczos_lambda_max(A, Dinv, 10)
    Ad = S.to_dense(A)
    Dd = _dense_D(A)
    w = sla.eigh(Ad, Dd, eigvals_only=True)
    lam_max = w.max()
    assert lam <= lam_max * (1 + 1e-12)
    assert lam >= 0.9 * lam_max
    gersh = np.abs(np.linalg.solve(Dd, Ad)).sum(axis=1).max()
    assert lam <= gersh
    # the same recurrence written on S = D^-1/2 A D^-1/2 with q0 = D^1/2 u0
    ev, V = np.linalg.eigh(Dd)
    Dh = V @ np.diag(np.sqrt(ev)) @ V.T
    Dmh = V @ np.diag(1 / np.sqrt(ev)) @ V.T
    Sm = Dmh @ Ad @ Dmh
    u0 = start_vector(A.nbr * 3, sa.LANCZOS_SEED)
    q = Dh @ u0
    q /= np.linalg.norm(q)
    qp = np.zeros_like(q)
    bp = 0.0
    a2, b2 = [], []
    for k in range(10):
        wv = Sm @ q - bp * qp
        a = q @ wv
        wv -= a * q
        b = np.linalg.norm(wv)
        a2.append(a)
        if k < 9:
            b2.append(b)
        qp, q, bp = q, wv / b, b
    assert np.allclose(al, a2, rtol=1e-9) and np.allclose(be, b2, rtol=1e-9)


def test_smoothed_prolongator_dense():
    m, A = _problem(4, seed=2)
    agg, n_agg = sa.aggregate(sa.strength_graph(A, m.dirichlet), m.dirichlet)
    Pt, _ = sa.tentative_prolongator(agg, n_agg, sa.rigid_body_modes(m.coords))
    Dinv = S.block_diag_inverse(A)
    P = sa.smooth_prolongator(A, Pt, Dinv, 2.5)
    Ad, Ptd = S.to_dense(A), S.to_dense(Pt)
    ref = Ptd - (4.0 / 3.0 / 2.5) * np.linalg.solve(_dense_D(A), Ad @ Ptd)
    assert np.abs(S.to_dense(P) - ref).max() < 1e-13
    rp, ci = S.structural_product(A.rowptr, A.colidx, A.nbr, A.nbc, Pt.rowptr, Pt.colidx, Pt.nbc)
    assert np.array_equal(P.rowptr, rp) and np.array_equal(P.colidx, ci)


def test_smoothed_prolongator_given_weight_and_setup_level_params():
    """A weight given directly enters P = P~ - omega D^-1 A P~ as is (dense check), and a
    setup with given (lambda_hat, omega) per level uses them: P on each level equals the
    dense smoothing with that omega, and the smoother keeps that lambda_hat."""
    m, A = _problem(4, seed=2)
    agg, n_agg = sa.aggregate(sa.strength_graph(A, m.dirichlet), m.dirichlet)
    Pt, _ = sa.tentative_prolongator(agg, n_agg, sa.rigid_body_modes(m.coords))
    Dinv = S.block_diag_inverse(A)
    Ad, Ptd = S.to_dense(A), S.to_dense(Pt)
    for om in (0.3, 0.61):
        P = sa.smooth_prolongator(A, Pt, Dinv, 2.5, omega=om)
        ref = Ptd - om * np.linalg.solve(_dense_D(A), Ad @ Ptd)
        assert np.abs(S.to_dense(P) - ref).max() < 1e-13
    m, A = _problem(6, seed=4)
    o = solve.Options(coarse_eq_limit=60)
    H0 = solve.setup(A, m.coords, m.dirichlet, o)
    params = [(1.25 * L.lam, 0.9 * o.omega_scale / L.lam) for L in H0.levels[:-1]]
    H = solve.setup(A, m.coords, m.dirichlet, o, level_params=params)
    assert H.n_levels == H0.n_levels == 3
    Pt, _ = sa.tentative_prolongator(H.levels[0].agg, H.levels[0].n_agg, sa.rigid_body_modes(m.coords))
    ref = S.to_dense(Pt) - params[0][1] * np.linalg.solve(_dense_D(A), S.to_dense(A) @ S.to_dense(Pt))
    assert np.abs(S.to_dense(H.levels[0].P) - ref).max() < 1e-13
    for lev, (lam, om) in enumerate(params):
        L = H.levels[lev]
        assert L.lam == lam
        assert np.array_equal(L.agg, H0.levels[lev].agg)
        # a different weight gives a different prolongator than the method's own
        assert np.abs(S.to_dense(L.P) - S.to_dense(H0.levels[lev].P)).max() > 1e-6
    # level_params entries of None keep the method's estimate on that level
    H1 = solve.setup(A, m.coords, m.dirichlet, o, level_params=[None, params[1]])
    assert H1.levels[0].lam == H0.levels[0].lam
    assert np.array_equal(H1.levels[0].P.val, H0.levels[0].P.val)
    assert H1.levels[1].lam == params[1][0]
