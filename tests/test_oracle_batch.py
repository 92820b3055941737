"""Pins of the batched oracle.  A batch is, by definition, independent instances
with independent right-hand sides, so the batched oracle is loops over the
single-instance oracle; these tests pin the plumbing around those loops (the
block-diagonal concatenation, the instance extraction) against independent facts,
and the per-column CG against scipy's textbook CG."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import batch as OB
from oracle import solve as OS
from oracle import sparse as S

SIZES = [3, 4, 2]


@pytest.fixture(scope="module")
def small():
    bt = synth.make_batch(SIZES, nrhs=3)
    A = S.coo_assemble(bt["n_nodes"], bt["n_nodes"], bt["i"], bt["j"], synth.batch_values(bt))
    return bt, A


def test_batch_sizes_recipe():
    s = synth.batch_sizes()
    assert len(s) == 24 and s.min() >= 16 and s.max() <= 48
    assert np.array_equal(s, np.random.default_rng(100).integers(16, 49, 24))


def test_concatenation_is_block_diagonal_copy_of_instances(small):
    bt, A = small
    row0 = bt["row0"]
    for t, m in enumerate(bt["meshes"]):
        i, j = synth.coo_indices(m)
        lam, mu = bt["mats"][t]
        At = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, synth.coo_values(m, lam, mu))
        Ex = OB.extract_instance(A, int(row0[t]), int(row0[t + 1]))
        assert np.array_equal(Ex.rowptr, At.rowptr) and np.array_equal(Ex.colidx, At.colidx)
        assert np.array_equal(Ex.val, At.val)  # same stream, same summation order
        assert np.array_equal(bt["b"][row0[t] * 3:row0[t + 1] * 3], synth.rhs(m, 300 + t, nrhs=3))
    # dense check: nothing outside the diagonal blocks
    D = S.to_dense(A)
    for t in range(len(SIZES)):
        a, b = row0[t] * 3, row0[t + 1] * 3
        D[a:b, a:b] = 0.0
    assert not D.any()


def test_extract_rejects_coupled_instances(small):
    _, A = small
    with pytest.raises(ValueError):
        OB.extract_instance(A, 0, int(small[0]["row0"][1]) - 5)  # cuts instance 0 in two


def test_batched_pcg_columns_match_textbook_cg(small):
    bt, A = small
    o = OS.Options(coarse_eq_limit=100)
    H = OB.setup_batch(A, bt["row0"], bt["coords"], bt["dirichlet"], o)
    X, its = OB.pcg_batch(A, H, bt["row0"], bt["b"], rtol=1e-8)
    row0 = bt["row0"]
    for t in range(len(SIZES)):
        At = OB.extract_instance(A, int(row0[t]), int(row0[t + 1]))
        Ad = S.to_scalar_csr(At)
        a, b = row0[t] * 3, row0[t + 1] * 3
        for q in range(bt["b"].shape[1]):
            bq = bt["b"][a:b, q]
            assert np.linalg.norm(bq - Ad @ X[a:b, q]) <= 2e-8 * np.linalg.norm(bq)
        # scipy's CG with the same preconditioner, first column
        Mop = spla.LinearOperator(Ad.shape, matvec=lambda r, H=H[t]: OS.vcycle(H, r))
        count = [0]
        spla.cg(Ad, bt["b"][a:b, 0], rtol=1e-8, M=Mop, maxiter=1000,
                callback=lambda xk: count.__setitem__(0, count[0] + 1))
        assert abs(count[0] - its[t, 0]) <= 1
