"""Pins for the oracle's parallel (Luby-round) distance-2 aggregation: with fixed
priorities the rounds must give exactly the sequential greedy distance-2 MIS visited
in decreasing priority order (brute force here), and the result must be an
independent, maximal set at distance 2 whose aggregates cover every free vertex."""
import numpy as np
import pytest

import synth
from oracle import sa
from oracle import sparse as S


def _graph(kind, seed=0):
    if kind == "q1":
        m = synth.make_mesh(4)
        i, j = synth.coo_indices(m)
        A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j,
                           synth.coo_values(m, *synth.lame(*synth.homogeneous_materials(m.n_elem))))
        d = m.dirichlet
    elif kind == "spd":
        rp, ci, v = synth.random_spd_bsr(150, 3, seed, max_per_row=4)
        A = S.Bsr(150, 150, 3, 3, rp, ci, v)
        d = np.zeros(A.nbr, dtype=bool)
        d[::17] = True
    else:  # path graph
        n = 40
        ci = []
        rp = [0]
        for v in range(n):
            ci += [u for u in (v - 1, v, v + 1) if 0 <= u < n]
            rp.append(len(ci))
        A = S.Bsr(n, n, 1, 1, np.array(rp), np.array(ci), np.ones((len(ci), 1, 1)))
        d = np.zeros(n, dtype=bool)
    return sa.strength_graph(A, d), d


def _dist_le2(nbrs, i, j):
    return j in nbrs[i] or any(j in nbrs[k] for k in nbrs[i])


@pytest.mark.parametrize("kind,seed", [("q1", 0), ("spd", 1), ("spd", 2), ("path", 0)])
def test_rounds_equal_sequential_greedy_in_key_order(kind, seed):
    nbrs, d = _graph(kind, seed)
    agg, n_agg, rounds = sa.aggregate_luby(nbrs, d, seed=sa.LUBY_SEED + seed)
    key = sa.luby_keys(len(nbrs), sa.LUBY_SEED + seed)
    roots = []
    for i in sorted(range(len(nbrs)), key=lambda v: -key[v]):
        if d[i]:
            continue
        if not any(_dist_le2(nbrs, i, r) for r in roots):
            roots.append(i)
    # roots are numbered in vertex order, so root k is the k-th smallest root, and each
    # root's neighbours share its aggregate
    assert n_agg == len(roots) and rounds >= 1
    for k, r in enumerate(sorted(roots)):
        assert agg[r] == k
        assert all(agg[v] == k for v in nbrs[r])


def _sequential_roots(nbrs, d, key):
    roots = []
    for i in sorted(range(len(nbrs)), key=lambda v: -key[v]):
        if not d[i] and not any(_dist_le2(nbrs, i, r) for r in roots):
            roots.append(i)
    return sorted(roots)


@pytest.mark.parametrize("kind,seed", [("q1", 0), ("spd", 3)])
def test_independent_maximal_and_covering(kind, seed):
    nbrs, d = _graph(kind, seed)
    n = len(nbrs)
    agg, n_agg, _ = sa.aggregate_luby(nbrs, d, seed=7 + seed)
    key = sa.luby_keys(n, 7 + seed)
    assert len(set(key)) == n and min(key) > 0
    roots = _sequential_roots(nbrs, d, key)
    for a in range(len(roots)):
        for b in range(a + 1, len(roots)):
            assert not _dist_le2(nbrs, roots[a], roots[b])       # independent at distance 2
    for v in range(n):
        if d[v]:
            assert agg[v] == -1
            continue
        r = roots[agg[v]]                                         # every free vertex is covered
        assert v == r or _dist_le2(nbrs, v, r)                    # ... within distance 2 of its root
        if any(u in roots for u in nbrs[v]):
            assert r in nbrs[v] or v == r                         # root neighbours join that root


def test_seed_changes_the_roots():
    nbrs, d = _graph("q1")
    a, na, _ = sa.aggregate_luby(nbrs, d, seed=1)
    b, nb, _ = sa.aggregate_luby(nbrs, d, seed=2)
    assert not np.array_equal(a, b)
