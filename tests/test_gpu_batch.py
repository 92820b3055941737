"""GPU parity of the batched hierarchy, V-cycle and CG: several independent Q1
instances of different sizes in one block-diagonal operator, 8 right-hand sides
each, against the per-instance oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import batch as OB  # noqa: E402
from oracle import sparse as S  # noqa: E402
from oracle import solve as OS  # noqa: E402
from paper_2606_24748_amd import blkamg as B  # noqa: E402
from tests.gpu_util import dev, from_device_bsr, rel2  # noqa: E402

# depths 3, 2, 2, 2 and 1: instances end on different levels, the one-level one last
SIZES = [16, 8, 12, 6, 3]
NR = 8


def _sub(A: S.Bsr, r0, r1, c0, c1) -> S.Bsr:
    """Rows [r0, r1) of A whose columns all lie in [c0, c1), columns shifted by c0."""
    k0, k1 = int(A.rowptr[r0]), int(A.rowptr[r1])
    ci = A.colidx[k0:k1] - c0
    assert len(ci) == 0 or (ci.min() >= 0 and ci.max() < c1 - c0)
    return S.Bsr(r1 - r0, c1 - c0, A.br, A.bc, A.rowptr[r0:r1 + 1] - k0, ci, A.val[k0:k1])


@pytest.fixture(scope="module")
def batch():
    print(f"batch sizes={SIZES} nrhs={NR}", flush=True)
    bt = synth.make_batch(SIZES, nrhs=NR)
    n = bt["n_nodes"]
    A = S.coo_assemble(n, n, bt["i"], bt["j"], synth.batch_values(bt))
    plan, HA = B.coo_plan_create(n, n, 3, 3, bt["i"], bt["j"])
    vals = dev(synth.batch_values(bt))
    B.coo_assemble_blocked(plan, vals, B.INSERT, HA)
    H = OB.setup_batch(A, bt["row0"], bt["coords"], bt["dirichlet"])
    X, its = OB.pcg_batch(A, H, bt["row0"], bt["b"], rtol=1e-8)
    torch.cuda.synchronize()
    return dict(bt=bt, A=A, plan=plan, HA=HA, vals=vals, H=H, X=X, its=its)


def _setup(d, hier=B.F64, pdt=B.F64, graph=4):
    o = B.blkamg_opts_default()
    o.hier_dtype, o.p_dtype, o.pcg_graph_iters = hier, pdt, graph
    bt = d["bt"]
    return B.amg_setup_batched(d["HA"], bt["row0"], bt["coords"], bt["dirichlet"], o)


def _check_levels(M, H, lam_tol=1e-12, val_tol=1e-12):
    nl = max(h.n_levels for h in H)
    assert M.num_levels() == nl
    lam = M.lambdas()
    for lev in range(nl):
        r0, nr, st = M.instance_rows(lev)
        HAl, HPl = M.level(lev)
        Al = from_device_bsr(HAl)
        smoothed = st == 1
        # in row order, the level's smoothed instances come before those that end on it
        pres = np.flatnonzero(st > 0)
        in_rows = st[pres[np.argsort(r0[pres], kind="stable")]]
        assert np.all(np.diff(np.where(in_rows == 1, 0, 1)) >= 0)
        agg = M.aggregates(lev) if smoothed.any() else None
        Pl = from_device_bsr(HPl) if HPl is not None else None
        if lev + 1 < nl:
            r0n, _, _ = M.instance_rows(lev + 1)
        for t, h in enumerate(H):
            if lev >= h.n_levels:
                assert st[t] == 0
                continue
            assert st[t] == (1 if lev < h.n_levels - 1 else 2)
            want = h.levels[lev].A
            got = _sub(Al, r0[t], r0[t] + nr[t], r0[t], r0[t] + nr[t])
            assert np.array_equal(got.rowptr, want.rowptr) and np.array_equal(got.colidx, want.colidx)
            assert rel2(got.val, want.val) <= val_tol
            if st[t] != 1:
                continue
            L = h.levels[lev]
            assert abs(lam[lev][t] - L.lam) <= lam_tol * L.lam
            base = r0n[t]
            a = agg[r0[t]:r0[t] + nr[t]]
            assert np.array_equal(a, np.where(L.agg >= 0, L.agg + base, -1))
            P = _sub(Pl, r0[t], r0[t] + nr[t], base, base + L.n_agg)
            assert np.array_equal(P.rowptr, L.P.rowptr) and np.array_equal(P.colidx, L.P.colidx)
            assert rel2(P.val, L.P.val) <= val_tol


def test_batched_hierarchy_matches_per_instance_oracle(batch):
    M = _setup(batch)
    assert M.num_instances() == len(SIZES)
    _check_levels(M, batch["H"])


def test_batched_vcycle_matches_oracle(batch):
    M = _setup(batch)
    bt, H = batch["bt"], batch["H"]
    n_dof = bt["n_nodes"] * 3
    R = np.random.default_rng(5).uniform(-1, 1, (n_dof, NR))
    Z = torch.zeros(n_dof, NR, dtype=torch.float64, device="cuda")
    B.vcycle_apply(M, dev(R), Z, nrhs=NR)
    Z1 = torch.zeros(n_dof, dtype=torch.float64, device="cuda")
    B.vcycle_apply(M, dev(np.ascontiguousarray(R[:, 3])), Z1, nrhs=1)
    Zh, Z1h = Z.cpu().numpy(), Z1.cpu().numpy()
    row0 = bt["row0"]
    for t, h in enumerate(H):
        a, b = row0[t] * 3, row0[t + 1] * 3
        for q in range(NR):
            want = OS.vcycle(h, R[a:b, q])
            assert rel2(Zh[a:b, q], want) <= 1e-11, (t, q)
            if q == 3:
                assert rel2(Z1h[a:b], want) <= 1e-11, t


def test_batched_pcg_matches_oracle(batch):
    M = _setup(batch)
    bt = batch["bt"]
    b = bt["b"]
    x = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
    code, its, rel = B.pcg_solve(batch["HA"], M, dev(b), x, rtol=1e-8, nrhs=NR)
    assert code == B.OK
    assert np.all(np.abs(its - batch["its"]) <= 1), (its, batch["its"])
    assert np.all(rel <= 1e-8)
    xs = x.cpu().numpy()
    row0 = bt["row0"]
    A = batch["A"]
    for t in range(len(SIZES)):
        At = OB.extract_instance(A, int(row0[t]), int(row0[t + 1]))
        a, c = row0[t] * 3, row0[t + 1] * 3
        for q in range(NR):
            bq = b[a:c, q]
            assert np.linalg.norm(bq - S.spmv(At, xs[a:c, q])) <= 2e-8 * np.linalg.norm(bq)
            assert rel2(xs[a:c, q], batch["X"][a:c, q]) <= 1e-6
    print(f"batched pcg its={its.tolist()}", flush=True)


def test_batched_pcg_graph_replays_equal_eager(batch):
    bt = batch["bt"]
    b = dev(bt["b"])
    Mg = _setup(batch, graph=3)
    Me = _setup(batch, graph=0)
    xe = torch.zeros_like(b)
    code, its_e, _ = B.pcg_solve(batch["HA"], Me, b, xe, rtol=1e-8, nrhs=NR)
    assert code == B.OK
    z = torch.zeros_like(b)
    for rep in range(3):  # the graph is captured on the first solve and replayed after
        xg = torch.full_like(b, 7.0)
        code, its_g, _ = B.pcg_solve(batch["HA"], Mg, b, xg, rtol=1e-8, nrhs=NR)
        assert code == B.OK
        assert np.array_equal(its_g, its_e), rep
        assert torch.equal(xg, xe), rep
        B.vcycle_apply(Mg, b, z, nrhs=NR)  # eager work between replays
        torch.cuda.synchronize()


def test_batched_zero_columns_and_maxit(batch):
    M = _setup(batch)
    bt = batch["bt"]
    b = bt["b"].copy()
    b[:, 2] = 0.0
    x = torch.full(b.shape, 3.0, dtype=torch.float64, device="cuda")
    code, its, rel = B.pcg_solve(batch["HA"], M, dev(b), x, rtol=1e-8, nrhs=NR)
    assert code == B.OK
    assert np.all(its[:, 2] == 0) and np.all(rel[:, 2] == 0.0)
    assert float(x[:, 2].abs().max()) == 0.0
    other = [q for q in range(NR) if q != 2]
    assert np.all(np.abs(its[:, other] - batch["its"][:, other]) <= 1)
    x.zero_()
    code, its, _ = B.pcg_solve(batch["HA"], M, dev(bt["b"]), x, rtol=1e-8, maxit=3, nrhs=NR)
    # the one-level instance is solved exactly (1 update); the others stop at maxit
    assert code == B.ENOCONV and np.all(its[:-1] == 3) and np.all(its[-1] == 1)


@pytest.mark.parametrize("pdt", [B.F32, B.BF16])
def test_batched_f32_hierarchy_reaches_fp64_residual(batch, pdt):
    M = _setup(batch, hier=B.F32, pdt=pdt)
    bt = batch["bt"]
    b = bt["b"]
    x = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
    code, its, rel = B.pcg_solve(batch["HA"], M, dev(b), x, rtol=1e-8, nrhs=NR)
    assert code == B.OK and np.all(rel <= 1e-8)
    assert np.all(its <= batch["its"] + 4), (its, batch["its"])
    lam = M.lambdas()
    for t, h in enumerate(batch["H"]):
        for lev in range(h.n_levels - 1):
            assert abs(lam[lev][t] - h.levels[lev].lam) <= 1e-4 * h.levels[lev].lam
    xs = x.cpu().numpy()
    row0 = bt["row0"]
    for t in range(len(SIZES)):
        At = OB.extract_instance(batch["A"], int(row0[t]), int(row0[t + 1]))
        a, c = row0[t] * 3, row0[t + 1] * 3
        for q in range(NR):
            assert np.linalg.norm(b[a:c, q] - S.spmv(At, xs[a:c, q])) <= 2e-8 * np.linalg.norm(b[a:c, q])
    print(f"f32 hierarchy (P dtype {pdt}) its={its.tolist()}", flush=True)


def test_batched_hot_recompute_matches_oracle(batch):
    M = _setup(batch)
    bt = batch["bt"]
    vals2 = []
    for t, m in enumerate(bt["meshes"]):
        E, nu = synth.materials(m.n_elem, 1200 + t)
        vals2.append(synth.coo_values(m, *synth.lame(E, nu)))
    v2 = np.concatenate(vals2)
    n = bt["n_nodes"]
    A2 = S.coo_assemble(n, n, bt["i"], bt["j"], v2)
    B.coo_assemble_blocked(batch["plan"], dev(v2), B.INSERT, batch["HA"])
    B.amg_galerkin_recompute(M)
    B.amg_smoother_refresh(M)
    row0 = bt["row0"]
    H2 = [OS.recompute(h, OB.extract_instance(A2, int(row0[t]), int(row0[t + 1])))
          for t, h in enumerate(batch["H"])]
    _check_levels(M, H2)
    # restore the fixture's operator for the tests that follow
    B.coo_assemble_blocked(batch["plan"], batch["vals"], B.INSERT, batch["HA"])
    torch.cuda.synchronize()


def test_batched_user_lambdas(batch):
    M = _setup(batch)
    lam = M.lambdas()
    B.amg_smoother_refresh(M, lam * 1.25)
    assert np.allclose(M.lambdas(), lam * 1.25, rtol=0, atol=0)


def test_single_instance_eight_columns(batch):
    m = synth.make_mesh(8)
    i, j = synth.coo_indices(m)
    E, nu = synth.materials(m.n_elem, 4)
    v = synth.coo_values(m, *synth.lame(E, nu))
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    M = B.amg_setup(HA, m.coords, m.dirichlet)
    H = OS.setup(A, m.coords, m.dirichlet)
    b = synth.rhs(m, 9, nrhs=NR)
    x = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
    code, its, rel = B.pcg_solve(HA, M, dev(b), x, rtol=1e-8, nrhs=NR)
    assert code == B.OK and its.shape == (1, NR)
    for q in range(NR):
        _, it_o, _, _ = OS.pcg(A, b[:, q], lambda r: OS.vcycle(H, r), rtol=1e-8)
        assert abs(its[0, q] - it_o) <= 1


def test_batched_setup_rejects_bad_layouts(batch):
    bt = batch["bt"]
    o = B.blkamg_opts_default()
    row0 = bt["row0"].copy()
    row0[1] -= 5  # cuts instance 0: its rows now couple to instance 1
    with pytest.raises(B.BlkAmgError) as e:
        B.amg_setup_batched(batch["HA"], row0, bt["coords"], bt["dirichlet"], o)
    assert e.value.code == B.EINVAL
    small = synth.make_batch([3, 8], nrhs=1)  # a one-level instance first
    n = small["n_nodes"]
    plan, HA = B.coo_plan_create(n, n, 3, 3, small["i"], small["j"])
    B.coo_assemble_blocked(plan, dev(synth.batch_values(small)), B.INSERT, HA)
    with pytest.raises(B.BlkAmgError) as e:
        B.amg_setup_batched(HA, small["row0"], small["coords"], small["dirichlet"], o)
    assert e.value.code == B.EINVAL


def test_autotune_keeps_results(batch):
    HA = batch["HA"]
    n_dof = batch["bt"]["n_nodes"] * 3
    X = dev(np.random.default_rng(2).uniform(-1, 1, (n_dof, NR)))
    y0 = torch.zeros_like(X)
    B.bsr_spmv(HA, 1.0, X, 0.0, y0, nrhs=NR)
    code = B.bsr_autotune(HA, B.F64, NR)
    assert code in {8 * 8 + 1, 8 * 8 + 2, 16 * 8 + 1, 16 * 8 + 2, 32 * 8 + 1, 32 * 8 + 2, 64 * 8 + 1, 64 * 8 + 2}
    y1 = torch.zeros_like(X)
    B.bsr_spmv(HA, 1.0, X, 0.0, y1, nrhs=NR)
    assert rel2(y1.cpu().numpy(), y0.cpu().numpy()) <= 1e-14
    print(f"autotuned lane code {code}", flush=True)


# Edge lengths spanning the batching workload's range 16..48: the largest instance has
# four levels and the smallest three, so instances end on different levels at scale.
WIDE = [16, 48, 31]
WIDE_COLS = (0, 7)


@pytest.fixture(scope="module")
def wide():
    print(f"wide batch sizes={WIDE} nrhs={NR}", flush=True)
    bt = synth.make_batch(WIDE, nrhs=NR)
    n = bt["n_nodes"]
    A = S.coo_assemble(n, n, bt["i"], bt["j"], synth.batch_values(bt))
    plan, HA = B.coo_plan_create(n, n, 3, 3, bt["i"], bt["j"])
    B.coo_assemble_blocked(plan, dev(synth.batch_values(bt)), B.INSERT, HA)
    H = OB.setup_batch(A, bt["row0"], bt["coords"], bt["dirichlet"])
    torch.cuda.synchronize()
    return dict(bt=bt, A=A, plan=plan, HA=HA, H=H)


def test_wide_batch_hierarchy_vcycle_and_pcg(wide):
    """Hierarchy per instance (aggregates, P, A_c, lambda_hat), the 8-column V-cycle and
    the 8-column CG against the per-instance oracle on two of the columns."""
    M = _setup(wide)
    _check_levels(M, wide["H"])
    bt, H, A = wide["bt"], wide["H"], wide["A"]
    n_dof = bt["n_nodes"] * 3
    R = np.random.default_rng(6).uniform(-1, 1, (n_dof, NR))
    Z = torch.zeros(n_dof, NR, dtype=torch.float64, device="cuda")
    B.vcycle_apply(M, dev(R), Z, nrhs=NR)
    Zh = Z.cpu().numpy()
    b = bt["b"]
    x = torch.zeros(b.shape, dtype=torch.float64, device="cuda")
    code, its, rel = B.pcg_solve(wide["HA"], M, dev(b), x, rtol=1e-8, nrhs=NR)
    assert code == B.OK and np.all(rel <= 1e-8)
    xs = x.cpu().numpy()
    row0 = bt["row0"]
    for t, h in enumerate(H):
        a, c = row0[t] * 3, row0[t + 1] * 3
        At = OB.extract_instance(A, int(row0[t]), int(row0[t + 1]))
        for q in WIDE_COLS:
            assert rel2(Zh[a:c, q], OS.vcycle(h, R[a:c, q])) <= 1e-11, (t, q)
            _, it_o, _, ok = OS.pcg(At, b[a:c, q], lambda r: OS.vcycle(h, r), rtol=1e-8)
            assert ok and abs(int(its[t, q]) - it_o) <= 1, (t, q, its[t, q], it_o)
        for q in range(NR):
            bq = b[a:c, q]
            assert np.linalg.norm(bq - S.spmv(At, xs[a:c, q])) <= 2e-8 * np.linalg.norm(bq), (t, q)
    print(f"wide batch pcg its={its.tolist()}", flush=True)
