"""Pins for the synthetic Q1 elasticity generator (the inputs both sides consume)."""
import numpy as np
import pytest

import synth
from synth.q1 import LOCAL_OFFSETS


def _rbm_nodes(X):
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    n = len(X)
    B = np.zeros((n, 3, 6))
    B[:, 0, 0] = B[:, 1, 1] = B[:, 2, 2] = 1
    B[:, 0, 3], B[:, 1, 3] = -y, x
    B[:, 1, 4], B[:, 2, 4] = -z, y
    B[:, 0, 5], B[:, 2, 5] = z, -x
    return B.reshape(3 * n, 6)


def test_reference_matrices_symmetric_rank18_and_rigid_null_space():
    Kl, Km = synth.reference_element_matrices()
    for K in (Kl, Km):
        assert np.allclose(K, K.T, atol=1e-15)
    K = 0.7 * Kl + 1.3 * Km
    w = np.linalg.eigvalsh(K)
    assert np.sum(w > 1e-10 * w.max()) == 18
    B = _rbm_nodes(LOCAL_OFFSETS.astype(float) * 0.37 + 0.2)
    assert np.abs(K @ B).max() < 1e-13


@pytest.mark.parametrize("h", [1.0, 0.125, 1 / 64])
def test_uniform_strain_energy_closed_form(h):
    """u = eps x is reproduced exactly by Q1, so u^T K_e u = h^3 (lam tr(eps)^2 + 2 mu eps:eps)."""
    rng = np.random.default_rng(5)
    lam, mu = 0.8, 0.45
    K = synth.element_matrix(h, lam, mu)
    X = LOCAL_OFFSETS.astype(float) * h + rng.uniform(-1, 1, 3)
    for _ in range(5):
        G = rng.uniform(-1, 1, (3, 3))
        eps = 0.5 * (G + G.T)
        u = (X @ G.T).reshape(-1)        # displacement grad = G (rotation part has no energy)
        energy = u @ K @ u
        exact = h ** 3 * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
        assert abs(energy - exact) <= 1e-12 * max(1.0, abs(exact))


def test_lame_closed_form():
    lam, mu = synth.lame(1.0, 0.25)
    assert lam == pytest.approx(0.4)
    assert mu == pytest.approx(0.4)


def test_tiny_counts():
    m = synth.make_mesh(8)
    assert (m.n_nodes, m.n_dof, m.n_dirichlet) == (729, 2187, 81)
    i, j = synth.coo_indices(m)
    assert len(i) == 64 * 512 + 81 == synth.stream_sizes(8)["n_coo"]
    v = synth.coo_values(m, *synth.lame(*synth.homogeneous_materials(m.n_elem)))
    assert v.shape == (len(i), 3, 3)
    # Dirichlet couplings dropped, identity appended
    assert np.all((i < 0) == (j < 0))
    d = np.nonzero(m.dirichlet)[0]
    assert np.array_equal(i[-81:], d) and np.array_equal(j[-81:], d)
    assert np.all(v[-81:] == np.eye(3))
    assert not np.any(m.dirichlet[i[i >= 0]]) or np.all(i[-81:] == j[-81:])


def test_rhs_zero_on_dirichlet_and_seeded():
    m = synth.make_mesh(3)
    b1 = synth.rhs(m, 7)
    b2 = synth.rhs(m, 7)
    assert np.array_equal(b1, b2)
    assert np.all(b1.reshape(-1, 3)[m.dirichlet] == 0)
    assert np.all(np.abs(b1) <= 1)
    B = synth.rhs(m, 7, nrhs=8)
    assert B.shape == (m.n_dof, 8)


def test_materials_distribution():
    E, nu = synth.materials(200000, 1)
    assert abs(np.log(E).mean()) < 0.01 and abs(np.log(E).std() - 1) < 0.01
    assert nu.min() >= 0.2 and nu.max() < 0.35
