"""Pins for the synthetic Q2 (triquadratic) elasticity generator: shape-function
identities, closed-form strain energies of fields Q2 reproduces exactly, and the
row lengths of the assembled pattern against a lattice count."""
import numpy as np
import pytest

import synth
from oracle import sparse as S
from synth.q2 import Q2_LOCAL_OFFSETS


def _rbm_nodes(X):
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    n = len(X)
    B = np.zeros((n, 3, 6))
    B[:, 0, 0] = B[:, 1, 1] = B[:, 2, 2] = 1
    B[:, 0, 3], B[:, 1, 3] = -y, x
    B[:, 1, 4], B[:, 2, 4] = -z, y
    B[:, 0, 5], B[:, 2, 5] = z, -x
    return B.reshape(3 * n, 6)


def test_shape_functions_kronecker_and_partition_of_unity():
    nodes = Q2_LOCAL_OFFSETS.astype(float) / 2
    V = np.stack([synth.shape_functions_q2(p)[0] for p in nodes])
    assert np.allclose(V, np.eye(27), atol=1e-15)
    rng = np.random.default_rng(3)
    for p in rng.uniform(0, 1, (5, 3)):
        val, grad = synth.shape_functions_q2(p)
        assert abs(val.sum() - 1.0) < 1e-14
        assert np.abs(grad.sum(axis=0)).max() < 1e-13
        # gradient against central differences
        for d in range(3):
            e = np.zeros(3)
            e[d] = 1e-6
            fd = (synth.shape_functions_q2(p + e)[0] - synth.shape_functions_q2(p - e)[0]) / 2e-6
            assert np.abs(fd - grad[:, d]).max() < 1e-8


def test_reference_matrices_symmetric_rank75_and_rigid_null_space():
    Kl, Km = synth.reference_element_matrices_q2()
    for K in (Kl, Km):
        assert np.allclose(K, K.T, atol=1e-14)
    K = 0.7 * Kl + 1.3 * Km
    w = np.linalg.eigvalsh(K)
    assert w.min() > -1e-12 * w.max()
    assert np.sum(w > 1e-10 * w.max()) == 81 - 6
    B = _rbm_nodes(Q2_LOCAL_OFFSETS.astype(float) * 0.5 * 0.37 + 0.2)
    assert np.abs(K @ B).max() < 1e-12


def _element(h, lam, mu):
    Kl, Km = synth.reference_element_matrices_q2()
    return h * (lam * Kl + mu * Km)


@pytest.mark.parametrize("h", [1.0, 0.25])
def test_uniform_strain_energy_closed_form(h):
    """u = G x: u^T K_e u = h^3 (lam tr(eps)^2 + 2 mu eps:eps), eps = sym(G)."""
    rng = np.random.default_rng(6)
    lam, mu = 0.8, 0.45
    K = _element(h, lam, mu)
    X = Q2_LOCAL_OFFSETS.astype(float) * (h / 2) + rng.uniform(-1, 1, 3)
    for _ in range(4):
        G = rng.uniform(-1, 1, (3, 3))
        eps = 0.5 * (G + G.T)
        u = (X @ G.T).reshape(-1)
        exact = h ** 3 * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
        assert abs(u @ K @ u - exact) <= 1e-12 * max(1.0, abs(exact))


def test_quadratic_field_energy_closed_form():
    """Fields of degree 2, which Q1 cannot represent, integrated by hand on [0,1]^3:
    u = (x^2, 0, 0): (lam + 2 mu) int (2x)^2 = 4 (lam + 2 mu) / 3;
    u = (0, x y, 0): int lam x^2 + 2 mu (x^2 + y^2 / 2) = (lam + 3 mu) / 3."""
    lam, mu = 0.8, 0.45
    K = _element(1.0, lam, mu)
    X = Q2_LOCAL_OFFSETS.astype(float) / 2
    u1 = np.zeros((27, 3))
    u1[:, 0] = X[:, 0] ** 2
    u2 = np.zeros((27, 3))
    u2[:, 1] = X[:, 0] * X[:, 1]
    for u, exact in ((u1, 4 * (lam + 2 * mu) / 3), (u2, (lam + 3 * mu) / 3)):
        uu = u.reshape(-1)
        assert abs(uu @ K @ uu - exact) < 1e-13


def test_mesh_counts_and_lattice():
    m = synth.make_mesh_q2(3)
    assert m.order == 2 and m.npe == 27
    assert (m.n_nodes, m.n_elem, m.n_dirichlet) == (7 ** 3, 27, 49)
    sz = synth.stream_sizes(3, order=2)
    i, j = synth.coo_indices(m)
    assert len(i) == sz["n_coo"] == 729 * 27 + 49
    assert sz["n_dof"] == m.n_dof
    # element nodes sit on the lattice at spacing h/2 around the element's corner
    e = 13  # the centre element (1, 1, 1)
    X = m.coords[m.elem_nodes[e]]
    assert np.allclose(X, (np.array([1, 1, 1]) + Q2_LOCAL_OFFSETS / 2) / 3)
    # same dofs as Q1 with twice the elements per edge
    assert synth.make_mesh_q2(4).n_dof == synth.make_mesh(8).n_dof


def test_assembled_row_lengths_match_lattice_count():
    """Block-row lengths of the unclamped assembled pattern: per axis, an element-vertex
    lattice index reaches 5 positions (3 on the boundary), a mid-edge one 3."""
    n = 3
    m = synth.make_mesh_q2(n, clamp=False)
    i, j = synth.coo_indices(m)
    v = synth.coo_values(m, *synth.lame(*synth.homogeneous_materials(m.n_elem)))
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v)
    M = 2 * n + 1

    def reach(t):
        if t % 2:
            return 3
        return 3 if t in (0, M - 1) else 5

    idx = np.arange(m.n_nodes)
    want = np.array([reach(a) * reach(b) * reach(c) for a, b, c in zip(idx % M, (idx // M) % M, idx // (M * M))])
    assert np.array_equal(np.diff(A.rowptr), want)
    assert want.max() == 125 and want.min() == 27


def test_assembled_quadratic_energy_and_rigid_modes():
    """Summed over elements, the stream gives the energy of a global quadratic field
    on the unit cube, and the unclamped operator annihilates the rigid-body modes."""
    lam, mu = synth.lame(1.0, 0.3)
    m = synth.make_mesh_q2(2, clamp=False)
    i, j = synth.coo_indices(m)
    v = synth.coo_values(m, *synth.lame(*synth.homogeneous_materials(m.n_elem)))
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v)
    u = np.zeros((m.n_nodes, 3))
    u[:, 0] = m.coords[:, 0] ** 2
    uu = u.reshape(-1)
    assert abs(uu @ S.spmv(A, uu) - 4 * (lam + 2 * mu) / 3) < 1e-12
    Bm = _rbm_nodes(m.coords)
    for c in range(6):
        assert np.abs(S.spmv(A, Bm[:, c])).max() < 1e-12


def test_torch_values_match_numpy():
    torch = pytest.importorskip("torch")
    m = synth.make_mesh_q2(2)
    lam, mu = synth.lame(*synth.materials(m.n_elem, 9))
    a = synth.coo_values(m, lam, mu)
    b = synth.coo_values_torch(m, lam, mu, "cpu").numpy()
    assert np.array_equal(a, b)
