"""Helpers shared by the GPU tests: move oracle matrices to the device and back."""
import numpy as np
import torch

import synth
from oracle import sparse as S
from paper_2606_24748_amd import blkamg as B

TDT = {B.F64: torch.float64, B.F32: torch.float32, B.BF16: torch.bfloat16}


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def to_device_bsr(A: S.Bsr, dtype=B.F64):
    rp = dev(A.rowptr.astype(np.int32))
    ci = dev(A.colidx.astype(np.int32))
    v = dev(A.val.astype(np.float64)).to(TDT[dtype]).contiguous()
    return B.bsr_create(A.nbr, A.nbc, A.br, A.bc, rp, ci, v), (rp, ci, v)


def from_device_bsr(H) -> S.Bsr:
    inf = H.info()
    rp, ci, v = H.arrays()
    return S.Bsr(inf["nbr"], inf["nbc"], inf["bs_r"], inf["bs_c"], rp.cpu().numpy().astype(np.int64),
                 ci.cpu().numpy().astype(np.int64), v.to(torch.float64).cpu().numpy())


def rel2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def q1_problem(n, mat_seed=None, order=1):
    """Mesh (trilinear, or triquadratic for order 2), oracle operator, and the stream that produced it."""
    m = synth.make_mesh(n) if order == 1 else synth.make_mesh_q2(n)
    i, j = synth.coo_indices(m)
    if mat_seed is None:
        E, nu = synth.homogeneous_materials(m.n_elem)
    else:
        E, nu = synth.materials(m.n_elem, mat_seed)
    v = synth.coo_values(m, *synth.lame(E, nu))
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v)
    return m, i, j, v, A
