"""Q2 (triquadratic, 27-node hexahedral) variant of the elasticity model problem.

The paper's sensitivity study (§4.6, Table 4) sets the trilinear discretisation (about
78 nonzeros per row) against the triquadratic one (about 180) at matched total
degrees of freedom.  This module generates the triquadratic problem with the same
unit cube, materials, clamped x = 0 face and COO stream layout as the Q1 generator:

* n elements per edge; nodes on the (2n+1)^3 lattice of spacing h/2, node
  i + (2n+1)*(j + (2n+1)*k) at (i, j, k) / (2n); dof = 3*node + component;
* element e = ex + n*(ey + n*ez) owns the 27 lattice nodes (2ex+a, 2ey+b, 2ez+c),
  a, b, c in 0..2, local index a + 3b + 9c;
* shape functions are products of the 1D quadratic Lagrange polynomials with nodes
  0, 1/2, 1; the stiffness uses 3x3x3 Gauss-Legendre quadrature, exact here (the
  integrands have degree at most 4 per axis), so again K_e = h (lambda Kl + mu Km);
* 729 blocks of 3x3 per element in the stream, in (local row, local column) order.

With n elements per edge the problem has as many dofs as the Q1 problem with 2n.
Block rows hold 27 (element-interior node) to 125 (element-corner node) blocks.
"""
from __future__ import annotations

import numpy as np

from .q1 import Q1Mesh

Q2_LOCAL_OFFSETS = np.array([(a, b, c) for c in range(3) for b in range(3) for a in range(3)], dtype=np.int64)


def make_mesh_q2(n: int, clamp: bool = True) -> Q1Mesh:
    """Structured n^3-element triquadratic mesh of the unit cube (`order` = 2)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    m = 2 * n + 1
    idx = np.arange(m ** 3, dtype=np.int64)
    i = idx % m
    j = (idx // m) % m
    k = idx // (m * m)
    coords = np.stack([i, j, k], axis=1).astype(np.float64) / (2 * n)
    dirichlet = (i == 0) if clamp else np.zeros(m ** 3, dtype=bool)
    e = np.arange(n ** 3, dtype=np.int64)
    ex = e % n
    ey = (e // n) % n
    ez = e // (n * n)
    base = 2 * ex + m * (2 * ey + m * 2 * ez)
    off = Q2_LOCAL_OFFSETS[:, 0] + m * (Q2_LOCAL_OFFSETS[:, 1] + m * Q2_LOCAL_OFFSETS[:, 2])
    elem_nodes = base[:, None] + off[None, :]
    return Q1Mesh(n=n, n_nodes=m ** 3, n_elem=n ** 3, coords=coords, dirichlet=dirichlet,
                  elem_nodes=elem_nodes, order=2)


def _lagrange2(x: float) -> tuple[np.ndarray, np.ndarray]:
    """Values and derivatives at x of the quadratics that are 1 at 0, 1/2, 1 respectively
    and 0 at the other two points."""
    v = np.array([2.0 * (x - 0.5) * (x - 1.0), -4.0 * x * (x - 1.0), 2.0 * x * (x - 0.5)])
    d = np.array([4.0 * x - 3.0, 4.0 - 8.0 * x, 4.0 * x - 1.0])
    return v, d


def shape_functions_q2(xi: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Values [27] and gradients [27, 3] of the triquadratic shape functions on [0,1]^3."""
    vx, dx = _lagrange2(xi[0])
    vy, dy = _lagrange2(xi[1])
    vz, dz = _lagrange2(xi[2])
    a, b, c = Q2_LOCAL_OFFSETS[:, 0], Q2_LOCAL_OFFSETS[:, 1], Q2_LOCAL_OFFSETS[:, 2]
    val = vx[a] * vy[b] * vz[c]
    grad = np.stack([dx[a] * vy[b] * vz[c], vx[a] * dy[b] * vz[c], vx[a] * vy[b] * dz[c]], axis=1)
    return val, grad


def reference_element_matrices_q2() -> tuple[np.ndarray, np.ndarray]:
    """Unit-cube element matrices (Kl, Km), each [81, 81], dof order 3*a + c, of the
    bilinear form  int lambda div u div v + 2 mu eps(u):eps(v)  (as for Q1)."""
    s = 0.5 * np.sqrt(3.0 / 5.0)
    gp = np.array([0.5 - s, 0.5, 0.5 + s])
    gw = np.array([5.0, 8.0, 5.0]) / 18.0
    Kl = np.zeros((27, 3, 27, 3))
    Km = np.zeros((27, 3, 27, 3))
    eye = np.eye(3)
    for ix, x in enumerate(gp):
        for iy, y in enumerate(gp):
            for iz, z in enumerate(gp):
                _, G = shape_functions_q2(np.array([x, y, z]))
                wt = gw[ix] * gw[iy] * gw[iz]
                Kl += wt * np.einsum("ac,bd->acbd", G, G)
                Km += wt * (np.einsum("cd,ab->acbd", eye, G @ G.T) + np.einsum("ad,bc->acbd", G, G))
    return Kl.reshape(81, 81), Km.reshape(81, 81)
