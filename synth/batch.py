"""Seeded batch of independent Q1 elasticity instances (inputs only).

The batch is concatenated into one block-diagonal system: instance t occupies the
block rows [row0_t, row0_t + n_nodes_t), its element stream is the single-instance
stream with node indices shifted by row0_t (negative indices stay negative), and its
right-hand sides fill the matching rows of a [n_dof][nrhs] array.
"""
from __future__ import annotations

import numpy as np

from . import q1


def batch_sizes(count: int = 24, seed: int = 100, lo: int = 16, hi: int = 48) -> np.ndarray:
    """Edge lengths n ~ U{lo..hi} (inclusive) from default_rng(seed)."""
    return np.random.default_rng(seed).integers(lo, hi + 1, count)


def make_batch(sizes, mat_seed0: int = 200, rhs_seed0: int = 300, nrhs: int = 8, homogeneous: bool = False):
    meshes = [q1.make_mesh(int(n)) for n in sizes]
    row0 = np.zeros(len(meshes) + 1, dtype=np.int64)
    row0[1:] = np.cumsum([m.n_nodes for m in meshes])
    ii, jj, mats, bs = [], [], [], []
    for t, m in enumerate(meshes):
        i, j = q1.coo_indices(m)
        off = np.int32(row0[t])
        ii.append(np.where(i >= 0, i + off, i).astype(np.int32))
        jj.append(np.where(j >= 0, j + off, j).astype(np.int32))
        E, nu = q1.homogeneous_materials(m.n_elem) if homogeneous else q1.materials(m.n_elem, mat_seed0 + t)
        mats.append(q1.lame(E, nu))
        bs.append(q1.rhs(m, rhs_seed0 + t, nrhs=nrhs).reshape(m.n_dof, nrhs))
    return {
        "meshes": meshes,
        "row0": row0,
        "i": np.concatenate(ii),
        "j": np.concatenate(jj),
        "mats": mats,
        "b": np.concatenate(bs, axis=0),
        "coords": np.concatenate([m.coords for m in meshes], axis=0),
        "dirichlet": np.concatenate([m.dirichlet for m in meshes]),
        "n_nodes": int(row0[-1]),
    }


def batch_values(batch) -> np.ndarray:
    """Concatenated element value streams (host)."""
    return np.concatenate([q1.coo_values(m, lam, mu) for m, (lam, mu) in zip(batch["meshes"], batch["mats"])])


def batch_values_torch(batch, device):
    import torch
    return torch.cat([q1.coo_values_torch(m, lam, mu, device) for m, (lam, mu) in zip(batch["meshes"], batch["mats"])])
