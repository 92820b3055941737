"""Q1 (trilinear hexahedral) linear-elasticity model problem on the unit cube.

The paper's model problem is 3D linear elasticity discretised with trilinear hex
elements, block size 3 (paper §4.1, experimental setup).  Its own harness is not
available, so this module generates a stand-in with the same structure:

* n elements per edge, nodes (i, j, k) in 0..n at (i/n, j/n, k/n);
  node = i + (n+1)*(j + (n+1)*k) (x fastest); dof = 3*node + component.
* element e = ex + n*(ey + n*ez); local node order (0,0,0), (1,0,0), (0,1,0),
  (1,1,0), (0,0,1), (1,0,1), (0,1,1), (1,1,1) (x fastest).
* isotropic elasticity, lambda = E nu / ((1+nu)(1-2nu)), mu = E / (2(1+nu));
  element stiffness by 2x2x2 Gauss-Legendre quadrature, exact for axis-aligned
  cubes, so K_e = h * (lambda * Kl + mu * Km) with Kl, Km the unit-cube matrices.
* the x = 0 face is clamped: its nodes are Dirichlet (symmetric elimination; the
  Dirichlet block rows hold only an identity diagonal block, couplings to them are
  not stored, and the right-hand side is zero there).

The element matrices reach the solver as a blocked COO stream (paper §3.4 and §5):
64 blocks of 3x3 per element in (local row, local column) order, with index -1 for
any block that touches a Dirichlet node, followed by one identity block per
Dirichlet node.  This stream is an *input*; summing it into a block matrix is the
method's job and is not done here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LOCAL_OFFSETS = np.array(
    [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1), (1, 1, 1)],
    dtype=np.int64,
)


@dataclass
class Q1Mesh:
    n: int                  # elements per edge
    n_nodes: int
    n_elem: int
    coords: np.ndarray      # [n_nodes, 3] float64
    dirichlet: np.ndarray   # [n_nodes] bool
    elem_nodes: np.ndarray  # [n_elem, npe] int64, local order above (Q2: synth.q2)
    order: int = 1          # 1 trilinear (8 nodes), 2 triquadratic (27 nodes)

    @property
    def npe(self) -> int:
        return self.elem_nodes.shape[1]

    @property
    def n_dof(self) -> int:
        return 3 * self.n_nodes

    @property
    def h(self) -> float:
        """Element side (the Q2 lattice spacing is h/2)."""
        return 1.0 / self.n

    @property
    def n_dirichlet(self) -> int:
        return int(self.dirichlet.sum())


def make_mesh(n: int, clamp: bool = True, distort: float = 0.0, seed: int = 0) -> Q1Mesh:
    """Structured n^3-element mesh of the unit cube; `clamp=False` gives the floating
    (no boundary condition) variant used for null-space checks.  `distort` > 0 moves
    every interior node by U[-distort, distort] * h per coordinate (default_rng(seed)),
    so elements become general trilinear hexahedra while the boundary, and hence the
    union of the elements, stays the unit cube (keep distort below about 0.25)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    idx = np.arange(m ** 3, dtype=np.int64)
    i = idx % m
    j = (idx // m) % m
    k = idx // (m * m)
    coords = np.stack([i, j, k], axis=1).astype(np.float64) / n
    if distort > 0:
        interior = (i > 0) & (i < n) & (j > 0) & (j < n) & (k > 0) & (k < n)
        d = np.random.default_rng(seed).uniform(-distort, distort, (m ** 3, 3)) / n
        coords[interior] += d[interior]
    dirichlet = (i == 0) if clamp else np.zeros(m ** 3, dtype=bool)
    e = np.arange(n ** 3, dtype=np.int64)
    ex = e % n
    ey = (e // n) % n
    ez = e // (n * n)
    base = ex + m * (ey + m * ez)
    off = LOCAL_OFFSETS[:, 0] + m * (LOCAL_OFFSETS[:, 1] + m * LOCAL_OFFSETS[:, 2])
    elem_nodes = base[:, None] + off[None, :]
    return Q1Mesh(n=n, n_nodes=m ** 3, n_elem=n ** 3, coords=coords,
                  dirichlet=dirichlet, elem_nodes=elem_nodes)


def _shape_gradients(xi: np.ndarray) -> np.ndarray:
    """Gradients of the 8 trilinear shape functions on [0,1]^3 at point xi: [8, 3]."""
    g = np.empty((8, 3))
    for a, (ox, oy, oz) in enumerate(LOCAL_OFFSETS):
        f = [xi[d] if o else 1.0 - xi[d] for d, o in enumerate((ox, oy, oz))]
        s = [1.0 if o else -1.0 for o in (ox, oy, oz)]
        g[a, 0] = s[0] * f[1] * f[2]
        g[a, 1] = f[0] * s[1] * f[2]
        g[a, 2] = f[0] * f[1] * s[2]
    return g


def reference_element_matrices() -> tuple[np.ndarray, np.ndarray]:
    """Unit-cube element matrices (Kl, Km), each [24, 24], dof order 3*a + c.

    Entry ((a,c),(b,d)) integrates  dN_a/dx_c dN_b/dx_d  (for lambda) and
    delta_cd grad N_a . grad N_b + dN_a/dx_d dN_b/dx_c  (for mu), i.e. the bilinear
    form  int lambda div u div v + 2 mu eps(u):eps(v).  Two-point Gauss per axis
    integrates the biquadratic integrands exactly.
    """
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    w = 0.5
    Kl = np.zeros((8, 3, 8, 3))
    Km = np.zeros((8, 3, 8, 3))
    eye = np.eye(3)
    for x in gp:
        for y in gp:
            for z in gp:
                G = _shape_gradients(np.array([x, y, z]))
                wt = w * w * w
                Kl += wt * np.einsum("ac,bd->acbd", G, G)
                Km += wt * (np.einsum("cd,ab->acbd", eye, G @ G.T) + np.einsum("ad,bc->acbd", G, G))
    return Kl.reshape(24, 24), Km.reshape(24, 24)


_REF = {}


def _ref_blocks(order: int = 1) -> tuple[np.ndarray, np.ndarray]:
    """Reference matrices of the element of `order` split into [npe, npe, 3, 3] node blocks."""
    if order not in _REF:
        if order == 1:
            Kl, Km = reference_element_matrices()
        else:
            from .q2 import reference_element_matrices_q2
            Kl, Km = reference_element_matrices_q2()
        k = Kl.shape[0] // 3
        _REF[order] = (Kl.reshape(k, 3, k, 3).transpose(0, 2, 1, 3).copy(),
                       Km.reshape(k, 3, k, 3).transpose(0, 2, 1, 3).copy())
    return _REF[order]


def lame(E, nu):
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def element_matrix(h: float, lam: float, mu: float) -> np.ndarray:
    """Dense 24x24 stiffness of one cube element of side h."""
    Kl, Km = reference_element_matrices()
    return h * (lam * Kl + mu * Km)


def materials(n_elem: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Per-element (E, nu): E ~ lognormal(0, 1), nu ~ U[0.2, 0.35], drawn in that order
    from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    E = rng.lognormal(0.0, 1.0, n_elem)
    nu = rng.uniform(0.2, 0.35, n_elem)
    return E, nu


def homogeneous_materials(n_elem: int, E: float = 1.0, nu: float = 0.3):
    return np.full(n_elem, E), np.full(n_elem, nu)


def stream_sizes(n: int, clamp: bool = True, order: int = 1) -> dict:
    m = order * n + 1
    npe = (order + 1) ** 3
    n_dir = m * m if clamp else 0
    return {"n_nodes": m ** 3, "n_dof": 3 * m ** 3, "n_elem": n ** 3,
            "n_dirichlet": n_dir, "n_coo": npe * npe * n ** 3 + n_dir}


def coo_indices(mesh: Q1Mesh) -> tuple[np.ndarray, np.ndarray]:
    """Block coordinates (i, j) of the element stream, int32, length npe^2*n_elem + n_dir
    (npe = 8 nodes per element for Q1, 27 for Q2).

    Entry npe^2*e + npe*a + b couples local nodes a (row) and b (column) of element e;
    it is (-1, -1) if either node is Dirichlet.  The last n_dir entries are the
    diagonal blocks (d, d) of the Dirichlet nodes in ascending order.
    """
    en = mesh.elem_nodes.astype(np.int32)
    k = mesh.npe
    ii = np.repeat(en, k, axis=1)          # [e, k*a+b] -> node a
    jj = np.tile(en, (1, k))               # [e, k*a+b] -> node b
    dmask = mesh.dirichlet
    drop = dmask[ii] | dmask[jj]
    ii[drop] = -1
    jj[drop] = -1
    dn = np.nonzero(dmask)[0].astype(np.int32)
    return (np.concatenate([ii.reshape(-1), dn]), np.concatenate([jj.reshape(-1), dn]))


def coo_values(mesh: Q1Mesh, lam: np.ndarray, mu: np.ndarray, dtype=np.float64) -> np.ndarray:
    """Block values [n_coo, 3, 3] matching `coo_indices` (host numpy)."""
    KlB, KmB = _ref_blocks(mesh.order)
    h = mesh.h
    ne = mesh.n_elem
    k = mesh.npe
    out = np.empty((k * k * ne + mesh.n_dirichlet, 3, 3), dtype=dtype)
    ev = out[: k * k * ne].reshape(ne, k, k, 3, 3)
    chunk = max(1, (1 << 22) // (k * k))
    for s in range(0, ne, chunk):
        e = slice(s, min(ne, s + chunk))
        ev[e] = h * (lam[e, None, None, None, None] * KlB[None] + mu[e, None, None, None, None] * KmB[None])
    out[k * k * ne:] = np.eye(3)
    return out


def coo_values_torch(mesh: Q1Mesh, lam, mu, device, dtype=None):
    """Same stream as `coo_values`, built directly in device memory with torch
    (input generation for large problems; no solver arithmetic)."""
    import torch
    dtype = dtype or torch.float64
    KlB, KmB = _ref_blocks(mesh.order)
    h = mesh.h
    ne = mesh.n_elem
    k = mesh.npe
    out = torch.empty((k * k * ne + mesh.n_dirichlet, 3, 3), dtype=dtype, device=device)
    kl = torch.as_tensor(KlB * h, dtype=torch.float64, device=device)
    km = torch.as_tensor(KmB * h, dtype=torch.float64, device=device)
    lam_t = torch.as_tensor(np.asarray(lam), dtype=torch.float64, device=device)
    mu_t = torch.as_tensor(np.asarray(mu), dtype=torch.float64, device=device)
    ev = out[: k * k * ne].view(ne, k, k, 3, 3)
    chunk = max(1, (1 << 24) // (k * k))
    for s in range(0, ne, chunk):
        e = slice(s, min(ne, s + chunk))
        ev[e] = (lam_t[e, None, None, None, None] * kl[None]
                 + mu_t[e, None, None, None, None] * km[None]).to(dtype)
    out[k * k * ne:] = torch.eye(3, dtype=dtype, device=device)
    return out


def rhs(mesh: Q1Mesh, seed: int, nrhs: int = 1) -> np.ndarray:
    """b ~ U[-1, 1] from default_rng(seed), shape [n_dof] (or [n_dof, nrhs]),
    zero on Dirichlet dofs."""
    rng = np.random.default_rng(seed)
    shape = (mesh.n_dof,) if nrhs == 1 else (mesh.n_dof, nrhs)
    b = rng.uniform(-1.0, 1.0, size=shape)
    dd = np.repeat(mesh.dirichlet, 3)
    b[dd] = 0.0
    return b
