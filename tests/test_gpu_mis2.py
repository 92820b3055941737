"""GPU parity of the device distance-2 aggregation (Luby rounds) against the oracle,
bit for bit, and of a hierarchy built on it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import sa, solve  # noqa: E402
from oracle import sparse as S  # noqa: E402
from paper_2606_24748_amd import blkamg as B  # noqa: E402
from tests.gpu_util import dev, from_device_bsr, q1_problem, rel2, to_device_bsr  # noqa: E402


@pytest.mark.parametrize("kind,n,seed", [("q1", 6, 0), ("q1", 12, 5), ("q2", 4, 1), ("spd", 400, 2)])
def test_device_aggregation_matches_oracle(kind, n, seed):
    print(f"mis2 {kind} n={n} seed={seed}", flush=True)
    if kind == "spd":
        rp, ci, v = synth.random_spd_bsr(n, 3, seed, max_per_row=5)
        A = S.Bsr(n, n, 3, 3, rp, ci, v)
        d = np.zeros(n, dtype=bool)
        d[::13] = True
    else:
        m, i, j, vv, A = q1_problem(n, 3, order=2 if kind == "q2" else 1)
        d = m.dirichlet
    H, keep = to_device_bsr(A)
    agg, n_agg, rounds = B.sa_aggregate_device(H, d, seed=B.LUBY_SEED + seed)
    want, n_want, r_want = sa.aggregate_luby(sa.strength_graph(A, d), d, B.LUBY_SEED + seed)
    assert n_agg == n_want and rounds == r_want
    assert np.array_equal(agg.cpu().numpy(), want)


def test_device_aggregation_properties_at_64cube():
    """274,625 vertices: every free vertex aggregated, Dirichlet ones not, ids dense,
    a handful of rounds, and the same result on a second call."""
    m = synth.make_mesh(64)
    i, j = synth.coo_indices(m)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    agg, n_agg, rounds = B.sa_aggregate_device(HA, m.dirichlet)
    a = agg.cpu().numpy()
    assert np.all(a[m.dirichlet] == -1) and np.all(a[~m.dirichlet] >= 0)
    assert set(np.unique(a[a >= 0])) == set(range(n_agg))
    assert 2 <= rounds <= 30
    agg2, n2, r2 = B.sa_aggregate_device(HA, m.dirichlet)
    assert n2 == n_agg and r2 == rounds and torch.equal(agg, agg2)


@pytest.mark.parametrize("n,seed", [(10, 7), (16, 2)])
def test_luby_hierarchy_matches_oracle(n, seed):
    m, i, j, v, A = q1_problem(n, seed)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    o = B.blkamg_opts_default()
    o.agg_mode = B.AGG_LUBY
    M = B.amg_setup(HA, m.coords, m.dirichlet, o)
    H = solve.setup(A, m.coords, m.dirichlet, solve.Options(agg_mode="luby"))
    assert M.num_levels() == H.n_levels
    lam = M.lambdas()
    for l in range(H.n_levels - 1):
        L = H.levels[l]
        assert np.array_equal(M.aggregates(l), L.agg)
        assert abs(lam[l] - L.lam) <= 1e-12 * L.lam
        assert rel2(from_device_bsr(M.level(l)[1]).val, L.P.val) <= 1e-12
        assert rel2(from_device_bsr(M.level(l + 1)[0]).val, H.levels[l + 1].A.val) <= 1e-12
    b = synth.rhs(m, 4)
    _, it_o, _, ok = solve.pcg(A, b, lambda r: solve.vcycle(H, r), rtol=1e-8)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, dev(b), x, rtol=1e-8)
    assert ok and code == B.OK and abs(it - it_o) <= 1


def test_luby_option_errors():
    m, i, j, v, A = q1_problem(4, 1)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    o = B.blkamg_opts_default()
    o.agg_mode = B.AGG_LUBY
    o.strength_eps = 0.05
    with pytest.raises(B.BlkAmgError):
        B.amg_setup(HA, m.coords, m.dirichlet, o)
    o = B.blkamg_opts_default()
    o.agg_mode = 7
    with pytest.raises(B.BlkAmgError):
        B.amg_setup(HA, m.coords, m.dirichlet, o)


def test_device_aggregation_degenerate_graphs():
    """Isolated vertices are their own roots after one round; a fully flagged graph has no
    aggregates and takes no round; both as the oracle says."""
    n = 37
    rp = torch.arange(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.arange(n, dtype=torch.int32, device="cuda")
    v = torch.ones(n * 9, dtype=torch.float64, device="cuda")
    H = B.bsr_create(n, n, 3, 3, rp, ci, v)
    A = S.Bsr(n, n, 3, 3, np.arange(n + 1), np.arange(n), np.ones((n, 3, 3)))
    for d in (np.zeros(n, dtype=bool), np.arange(n) % 5 == 0, np.ones(n, dtype=bool)):
        agg, n_agg, rounds = B.sa_aggregate_device(H, d)
        want, n_want, r_want = sa.aggregate_luby(sa.strength_graph(A, d), d)
        assert (n_agg, rounds) == (n_want, r_want)
        assert np.array_equal(agg.cpu().numpy(), want)
    assert n_agg == 0 and rounds == 0


@pytest.mark.parametrize("n,luby", [(6, False), (12, False), (12, True)])
def test_device_tentative_prolongator_matches_oracle(n, luby):
    """The device QR per aggregate against oracle.sa.tentative_prolongator: P~ values
    and the coarse near-null space within 1e-12, and P~ reproduces the rigid-body
    modes exactly on aggregated rows (P~ B_c = B)."""
    from oracle import sa as OSA
    m = synth.make_mesh(n)
    i, j = synth.coo_indices(m)
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, synth.coo_values(m, *synth.lame(*synth.materials(m.n_elem, 7))))
    nbrs = OSA.strength_graph(A, m.dirichlet)
    if luby:
        agg, n_agg, _ = OSA.aggregate_luby(nbrs, m.dirichlet, OSA.LUBY_SEED)
    else:
        agg, n_agg = OSA.aggregate(nbrs, m.dirichlet)
    Bn = OSA.rigid_body_modes(m.coords)
    Pt_o, Bc_o = OSA.tentative_prolongator(agg, n_agg, Bn)
    pt, bc = B.sa_tentative_device(torch.as_tensor(np.asarray(agg, dtype=np.int32)).cuda(), n_agg,
                                   torch.as_tensor(Bn).cuda())
    pt, bc = pt.cpu().numpy(), bc.cpu().numpy()
    rows = np.nonzero(np.asarray(agg) >= 0)[0]
    assert rel2(pt[rows], Pt_o.val) <= 1e-12
    assert not np.any(pt[np.asarray(agg) < 0])
    assert rel2(bc, Bc_o) <= 1e-12
    recon = np.einsum("nij,njk->nik", pt[rows], bc[np.asarray(agg)[rows]])
    assert np.abs(recon - Bn[rows]).max() <= 1e-12 * np.abs(Bn).max()


def test_device_tentative_prolongator_rejects_small_aggregates():
    agg = torch.tensor([0, 0, 1, 1, 1], dtype=torch.int32, device="cuda")  # aggregate 0: 2 nodes x bs 2 = 4 rows < 6
    Bn = torch.rand(5, 2, 6, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BlkAmgError) as e:
        B.sa_tentative_device(agg, 2, Bn)
    assert e.value.code == B.EINVAL
