"""Trilinear hexahedral element stiffness for linear elasticity, written out from its
definition (test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this package).

For an element with nodes X_a (a = 0..7, local order (0,0,0), (1,0,0), (0,1,0),
(1,1,0), (0,0,1), ... x fastest) the isoparametric map is x(xi) = sum_a X_a N_a(xi)
on the reference cube [0,1]^3 with the trilinear shape functions N_a.  The stiffness
of the bilinear form  int lambda div u div v + 2 mu eps(u):eps(v)  is

    K[(a,c),(b,d)] = sum_q w_q det J_q [ lambda g_a,c g_b,d
                                          + mu (delta_cd g_a . g_b + g_a,d g_b,c) ],

with g_a = J^-T grad_xi N_a at the 2x2x2 Gauss-Legendre points (weights 1/8 on the unit
cube) and J = dx/dxi.  The element matrices reach assembly as blocks K_ab (3x3,
row-major) in (a, b) order, the layout of the blocked COO stream (paper §5: finite-
element assembly is the primitive's immediate use beyond the Galerkin product).
"""
from __future__ import annotations

import numpy as np

_OFFSETS = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1), (1, 1, 1)]


def _ref_gradients(xi):
    """grad_xi N_a at xi, [8, 3]."""
    g = np.zeros((8, 3))
    for a, o in enumerate(_OFFSETS):
        f = [xi[d] if o[d] else 1.0 - xi[d] for d in range(3)]
        s = [1.0 if o[d] else -1.0 for d in range(3)]
        g[a] = [s[0] * f[1] * f[2], f[0] * s[1] * f[2], f[0] * f[1] * s[2]]
    return g


def _gauss_points():
    p = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    return [np.array([p[i], p[j], p[k]]) for k in range(2) for j in range(2) for i in range(2)]


def element_stiffness(X: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """Dense [24, 24] stiffness (dof 3a + c) of the element with node coordinates X [8, 3]."""
    K = np.zeros((8, 3, 8, 3))
    for xi in _gauss_points():
        G = _ref_gradients(xi)          # [8, 3] d N_a / d xi_k
        J = X.T @ G                     # J[r, k] = d x_r / d xi_k
        detJ = np.linalg.det(J)
        g = G @ np.linalg.inv(J)        # g[a, c] = sum_k dN_a/dxi_k (J^-1)[k, c]
        wd = detJ / 8.0
        for a in range(8):
            for b in range(8):
                for c in range(3):
                    for d in range(3):
                        v = lam * g[a, c] * g[b, d] + mu * g[a, d] * g[b, c]
                        if c == d:
                            v += mu * (g[a] @ g[b])
                        K[a, c, b, d] += wd * v
    return K.reshape(24, 24)


def element_blocks(X: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """The same matrix as [8, 8, 3, 3] blocks K_ab."""
    return element_stiffness(X, lam, mu).reshape(8, 3, 8, 3).transpose(0, 2, 1, 3)


def stream_values(coords: np.ndarray, elem_nodes: np.ndarray, lam, mu, n_identity: int = 0) -> np.ndarray:
    """Blocked COO value stream [n_elem * 64 + n_identity, 3, 3]: each element's 64 blocks
    in (a, b) order, then n_identity identity blocks (the Dirichlet diagonal)."""
    ne = len(elem_nodes)
    out = np.zeros((ne * 64 + n_identity, 3, 3))
    for e in range(ne):
        out[64 * e: 64 * (e + 1)] = element_blocks(coords[elem_nodes[e]], lam[e], mu[e]).reshape(64, 3, 3)
    out[64 * ne:] = np.eye(3)
    return out
