"""Pins for the oracle's trilinear element stiffness (oracle/fe.py): closed forms on
affine elements, the rigid-body null space, and the patch test on distorted meshes,
where the union of the elements is still the unit cube."""
import numpy as np
import pytest

import synth
from oracle import fe
from oracle import sparse as S

OFF = np.array(fe._OFFSETS, dtype=float)


def _rbm(X):
    n = len(X)
    B = np.zeros((n, 3, 6))
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    B[:, 0, 0] = B[:, 1, 1] = B[:, 2, 2] = 1
    B[:, 0, 3], B[:, 1, 3] = -y, x
    B[:, 1, 4], B[:, 2, 4] = -z, y
    B[:, 0, 5], B[:, 2, 5] = z, -x
    return B.reshape(3 * n, 6)


def _energy_density(G, lam, mu):
    eps = 0.5 * (G + G.T)
    return lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)


def test_axis_aligned_cube_matches_generator():
    for h, lam, mu in ((1.0, 0.8, 0.45), (0.125, 2.0, 0.3)):
        K = fe.element_stiffness(OFF * h + 0.3, lam, mu)
        assert np.abs(K - synth.element_matrix(h, lam, mu)).max() <= 1e-13 * np.abs(K).max()


def test_affine_element_uniform_strain_energy():
    """x = A xi + c: J = A everywhere, the volume is |det A|, and u = G x has energy
    |det A| (lam tr(eps)^2 + 2 mu eps:eps)."""
    rng = np.random.default_rng(4)
    for _ in range(3):
        A = np.eye(3) + rng.uniform(-0.3, 0.3, (3, 3))
        X = OFF @ A.T + rng.uniform(-1, 1, 3)
        lam, mu = rng.uniform(0.5, 2.0, 2)
        K = fe.element_stiffness(X, lam, mu)
        G = rng.uniform(-1, 1, (3, 3))
        u = (X @ G.T).reshape(-1)
        exact = abs(np.linalg.det(A)) * _energy_density(G, lam, mu)
        assert abs(u @ K @ u - exact) <= 1e-12 * max(1.0, exact)


def test_distorted_element_symmetric_rank18_rigid_null_space():
    rng = np.random.default_rng(7)
    X = OFF + rng.uniform(-0.2, 0.2, (8, 3))
    K = fe.element_stiffness(X, 0.9, 0.4)
    assert np.allclose(K, K.T, atol=1e-14)
    w = np.linalg.eigvalsh(K)
    assert w.min() > -1e-12 * w.max()
    assert np.sum(w > 1e-10 * w.max()) == 18
    assert np.abs(K @ _rbm(X)).max() < 1e-12


@pytest.mark.parametrize("distort", [0.0, 0.2])
def test_patch_test_on_distorted_mesh(distort):
    """For u = G x on every node, the assembled force K u vanishes at interior nodes
    (2x2x2 Gauss integrates cof(J)^T grad N exactly), and u^T K u equals the unit cube's
    volume times the energy density.  A quadratic field leaves interior forces."""
    n = 3
    m = synth.make_mesh(n, clamp=False, distort=distort, seed=5)
    rng = np.random.default_rng(1)
    lam, mu = 0.7, 0.35
    lam_e, mu_e = np.full(m.n_elem, lam), np.full(m.n_elem, mu)
    i, j = synth.coo_indices(m)
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, fe.stream_values(m.coords, m.elem_nodes, lam_e, mu_e))
    M = n + 1
    idx = np.arange(m.n_nodes)
    ii, jj, kk = idx % M, (idx // M) % M, idx // (M * M)
    inner = (ii > 0) & (ii < n) & (jj > 0) & (jj < n) & (kk > 0) & (kk < n)
    G = rng.uniform(-1, 1, (3, 3))
    u = (m.coords @ G.T).reshape(-1)
    f = S.spmv(A, u).reshape(-1, 3)
    assert np.abs(f[inner]).max() < 1e-13
    assert abs(u @ S.spmv(A, u) - _energy_density(G, lam, mu)) < 1e-12
    q = np.zeros((m.n_nodes, 3))
    q[:, 0] = m.coords[:, 0] ** 2
    assert np.abs(S.spmv(A, q.reshape(-1)).reshape(-1, 3)[inner]).max() > 1e-3


def test_stream_matches_generator_on_regular_mesh():
    m = synth.make_mesh(2)
    lam, mu = synth.lame(*synth.materials(m.n_elem, 3))
    a = fe.stream_values(m.coords, m.elem_nodes, lam, mu, m.n_dirichlet)
    b = synth.coo_values(m, lam, mu)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_distortion_keeps_boundary_and_positive_jacobians():
    m = synth.make_mesh(4, distort=0.2, seed=2)
    r = synth.make_mesh(4)
    moved = np.any(m.coords != r.coords, axis=1)
    on_boundary = np.any((r.coords == 0) | (r.coords == 1), axis=1)
    assert moved.sum() == 27 and not np.any(moved & on_boundary)
    for e in range(m.n_elem):
        X = m.coords[m.elem_nodes[e]]
        for xi in fe._gauss_points():
            assert np.linalg.det(X.T @ fe._ref_gradients(xi)) > 0
