"""GPU parity of the hierarchy, smoother, V-cycle and PCG against the CPU oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import sparse as S  # noqa: E402
from oracle import solve  # noqa: E402
from paper_2606_24748_amd import blkamg as B  # noqa: E402
from tests.gpu_util import dev, from_device_bsr, q1_problem, rel2  # noqa: E402


def _gpu_problem(n, mat_seed=None, hier=B.F64, pdt=B.F64):
    m, i, j, v, A = q1_problem(n, mat_seed)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    vals = dev(v)
    B.coo_assemble_blocked(plan, vals, B.INSERT, HA)
    o = B.blkamg_opts_default()
    o.hier_dtype = hier
    o.p_dtype = pdt
    M = B.amg_setup(HA, m.coords, m.dirichlet, o)
    return m, i, j, A, plan, HA, M


@pytest.mark.parametrize("n,seed", [(8, None), (12, 3)])
def test_setup_matches_oracle(n, seed):
    print(f"setup n={n} seed={seed}", flush=True)
    m, i, j, A, plan, HA, M = _gpu_problem(n, seed)
    H = solve.setup(A, m.coords, m.dirichlet)
    assert M.num_levels() == H.n_levels
    lam = M.lambdas()
    for l in range(H.n_levels - 1):
        L = H.levels[l]
        assert np.array_equal(M.aggregates(l), L.agg)
        assert abs(lam[l] - L.lam) <= 1e-12 * L.lam
        _, HP = M.level(l)
        P = from_device_bsr(HP)
        assert np.array_equal(P.rowptr, L.P.rowptr) and np.array_equal(P.colidx, L.P.colidx)
        assert rel2(P.val, L.P.val) <= 1e-12
        HAc, _ = M.level(l + 1)
        Ac = from_device_bsr(HAc)
        want = H.levels[l + 1].A
        assert np.array_equal(Ac.rowptr, want.rowptr) and np.array_equal(Ac.colidx, want.colidx)
        assert rel2(Ac.val, want.val) <= 1e-12


def test_vcycle_matches_oracle_f64():
    m, i, j, A, plan, HA, M = _gpu_problem(8, 5)
    H = solve.setup(A, m.coords, m.dirichlet)
    r = np.random.default_rng(0).uniform(-1, 1, m.n_dof)
    z = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    B.vcycle_apply(M, dev(r), z)
    assert rel2(z.cpu().numpy(), solve.vcycle(H, r)) <= 1e-11


@pytest.mark.parametrize("n,seed", [(8, None), (16, 1)])
def test_pcg_iterations_and_residual(n, seed):
    print(f"pcg n={n}", flush=True)
    m, i, j, A, plan, HA, M = _gpu_problem(n, seed)
    H = solve.setup(A, m.coords, m.dirichlet)
    b = synth.rhs(m, 2)
    _, it_o, rel_o, ok = solve.pcg(A, b, lambda r: solve.vcycle(H, r), rtol=1e-8)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, dev(b), x, rtol=1e-8)
    assert code == B.OK and ok
    assert abs(it - it_o) <= 1
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - S.spmv(A, xs)) <= 2e-8 * np.linalg.norm(b)
    assert rel <= 1e-8


def test_hot_recompute_matches_oracle():
    m, i, j, A, plan, HA, M = _gpu_problem(10, 7)
    H = solve.setup(A, m.coords, m.dirichlet)
    E, nu = synth.materials(m.n_elem, 1007)
    v2 = synth.coo_values(m, *synth.lame(E, nu))
    B.coo_assemble_blocked(plan, dev(v2), B.INSERT, HA)
    B.amg_galerkin_recompute(M)
    B.amg_smoother_refresh(M)
    A2 = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v2)
    H2 = solve.recompute(H, A2)
    lam = M.lambdas()
    for l in range(H2.n_levels - 1):
        assert abs(lam[l] - H2.levels[l].lam) <= 1e-12 * H2.levels[l].lam
        Ac = from_device_bsr(M.level(l + 1)[0])
        assert rel2(Ac.val, H2.levels[l + 1].A.val) <= 1e-12
    b = synth.rhs(m, 3)
    _, it_o, _, _ = solve.pcg(A2, b, lambda r: solve.vcycle(H2, r), rtol=1e-8)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, dev(b), x)
    assert code == B.OK and abs(it - it_o) <= 1


def test_pcg_zero_rhs_maxit_and_user_lambda():
    m, i, j, A, plan, HA, M = _gpu_problem(6, 2)
    x = torch.ones(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, torch.zeros(m.n_dof, dtype=torch.float64, device="cuda"), x)
    assert code == B.OK and it == 0 and not torch.any(x)
    b = dev(synth.rhs(m, 1))
    code, it, rel = B.pcg_solve(HA, M, b, x, rtol=1e-14, maxit=2)
    assert code == B.ENOCONV and it == 2
    lam = M.lambdas()
    B.amg_smoother_refresh(M, lam * 1.5)
    assert np.allclose(M.lambdas(), lam * 1.5, rtol=1e-15)


@pytest.mark.parametrize("pdt", [B.F32, B.BF16])
def test_f32_hierarchy_converges(pdt):
    m, i, j, A, plan, HA, M = _gpu_problem(12, 4, hier=B.F32, pdt=pdt)
    H = solve.setup(A, m.coords, m.dirichlet)
    b = synth.rhs(m, 5)
    _, it_o, _, _ = solve.pcg(A, b, lambda r: solve.vcycle(H, r), rtol=1e-8)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, dev(b), x, rtol=1e-8)
    assert code == B.OK
    assert it <= it_o + 3
    assert np.linalg.norm(b - S.spmv(A, x.cpu().numpy())) <= 2e-8 * np.linalg.norm(b)
    # the FP32 coarse operators agree with the FP64 oracle to FP32 accuracy
    for l in range(H.n_levels - 1):
        Ac = from_device_bsr(M.level(l + 1)[0])
        assert rel2(Ac.val, H.levels[l + 1].A.val) <= (1e-5 if pdt == B.F32 else 2e-2)


@pytest.mark.parametrize("n", [12, 24])
def test_f32_hierarchy_lambdas_and_recompute(n):
    """FP32 Lanczos estimates agree with the FP64 oracle after setup and after a hot
    recompute, and the V-cycle output stays finite (regression: the first Lanczos
    step must not read the unset previous vector)."""
    m, i, j, A, plan, HA, M = _gpu_problem(n, 6, hier=B.F32, pdt=B.F32)
    H = solve.setup(A, m.coords, m.dirichlet)
    lam = M.lambdas()
    assert np.all(np.isfinite(lam)) and np.all(lam > 0)
    for l in range(H.n_levels - 1):
        assert abs(lam[l] - H.levels[l].lam) <= 1e-4 * H.levels[l].lam
    E, nu = synth.materials(m.n_elem, 1006)
    v2 = synth.coo_values(m, *synth.lame(E, nu))
    B.coo_assemble_blocked(plan, dev(v2), B.INSERT, HA)
    B.amg_galerkin_recompute(M)
    B.amg_smoother_refresh(M)
    H2 = solve.recompute(H, S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v2))
    lam = M.lambdas()
    for l in range(H2.n_levels - 1):
        assert abs(lam[l] - H2.levels[l].lam) <= 1e-4 * H2.levels[l].lam
    r = np.random.default_rng(1).uniform(-1, 1, m.n_dof)
    z = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    B.vcycle_apply(M, dev(r), z)
    zo = solve.vcycle(H2, r)
    assert rel2(z.cpu().numpy(), zo) <= 1e-4


@pytest.mark.parametrize("hier", [B.F64, B.F32])
def test_symmetric_reads_give_identical_vcycle_and_pcg(hier):
    """The hierarchy's symmetric reads (sym_spmv = 1, the default; FP64 operators) against
    full reads (sym_spmv = 0): every level operator is symmetric bit for bit, so the two
    differ only in the grouping of the row sums: lambda_hat and the V-cycle agree to
    roundoff, CG takes the same iterations to the same solution."""
    print(f"symmetric reads hier={hier}", flush=True)
    m, i, j, v, A = q1_problem(14, mat_seed=5)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    out = []
    for sym in (0, 1):
        o = B.blkamg_opts_default()
        o.hier_dtype, o.p_dtype, o.sym_spmv = hier, hier, sym
        M = B.amg_setup(HA, m.coords, m.dirichlet, o)
        B.amg_smoother_refresh(M)
        r = dev(np.random.default_rng(9).uniform(-1, 1, m.n_dof))
        z = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
        B.vcycle_apply(M, r, z)
        b = dev(synth.rhs(m, 4))
        x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
        code, it, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8)
        assert code == B.OK
        out.append((M.lambdas().copy(), z.cpu(), x.cpu(), it))
    tol = 1e-12 if hier == B.F64 else 0.0  # FP32 hierarchies read every block either way
    assert np.all(np.abs(out[0][0] - out[1][0]) <= tol * out[0][0])
    assert rel2(out[1][1].numpy(), out[0][1].numpy()) <= max(tol, 1e-14 if hier == B.F64 else 1e-9)
    assert rel2(out[1][2].numpy(), out[0][2].numpy()) <= 1e-9 and out[0][3] == out[1][3]


@pytest.mark.parametrize("hier", [B.F64, B.F32])
def test_ap_residual_update(hier):
    """ap_residual = 1 (the default): the post-smoothing's first fine residual is updated
    as r - (A P) e_c from the Galerkin pass's A P instead of recomputed as f - A x (0), on
    levels where A P is cheaper to read (every block read: sym_spmv = 0 here, so FP64 takes
    it too).  The same residual up to rounding: the V-cycles differ (A P was used) by
    roundoff only, CG takes the same iterations.  With new values assembled but not yet
    recomputed, A P no longer belongs to A and the V-cycle is that of ap_residual = 0 bit
    for bit; after the recompute A P is used again."""
    print(f"ap residual hier={hier}", flush=True)
    m, i, j, v, A = q1_problem(14, mat_seed=5)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    r = dev(np.random.default_rng(9).uniform(-1, 1, m.n_dof))
    b = dev(synth.rhs(m, 4))
    Ms = []
    for ap in (0, 1):
        o = B.blkamg_opts_default()
        o.hier_dtype, o.p_dtype, o.sym_spmv, o.ap_residual = hier, hier, 0, ap
        M = B.amg_setup(HA, m.coords, m.dirichlet, o)
        B.amg_smoother_refresh(M)
        Ms.append(M)

    def vc(M):
        z = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
        B.vcycle_apply(M, r, z)
        return z.cpu().numpy()

    tol = 1e-12 if hier == B.F64 else 1e-5
    z0, z1 = vc(Ms[0]), vc(Ms[1])
    assert 0.0 < rel2(z1, z0) <= tol
    its = []
    for M in Ms:
        x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
        code, it, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8)
        assert code == B.OK and rel <= 1e-8
        its.append(it)
    assert its[0] == its[1]
    if hier == B.F64:  # both hierarchies read the caller's operator itself
        B.coo_assemble_blocked(plan, dev(1.5 * v), B.INSERT, HA)
        assert np.array_equal(vc(Ms[0]), vc(Ms[1]))
        for M in Ms:
            B.amg_galerkin_recompute(M)
            B.amg_smoother_refresh(M)
        z0, z1 = vc(Ms[0]), vc(Ms[1])
        assert 0.0 < rel2(z1, z0) <= tol


@pytest.mark.parametrize("nrhs", [1, 8])
def test_vcycle_on_fp32_vectors(nrhs):
    """vcycle_apply_ex with FP32 vectors on an F32 hierarchy runs the same FP32 V-cycle
    as the FP64 entry (which rounds its input to FP32 and widens the output): equal bit
    for bit; FP32 vectors on an F64 hierarchy are refused."""
    m, i, j, v, A = q1_problem(10, mat_seed=2)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    o = B.blkamg_opts_default()
    o.hier_dtype, o.p_dtype = B.F32, B.F32
    M = B.amg_setup(HA, m.coords, m.dirichlet, o)
    shape = (m.n_dof,) if nrhs == 1 else (m.n_dof, nrhs)
    r = dev(np.random.default_rng(3).uniform(-1, 1, shape))
    z64 = torch.zeros(shape, dtype=torch.float64, device="cuda")
    B.vcycle_apply(M, r, z64, nrhs=nrhs)
    z32 = torch.zeros(shape, dtype=torch.float32, device="cuda")
    B.vcycle_apply(M, r.float().contiguous(), z32, nrhs=nrhs)
    assert torch.equal(z32.double(), z64)
    M64 = B.amg_setup(HA, m.coords, m.dirichlet)
    with pytest.raises(B.BlkAmgError) as e:
        B.vcycle_apply(M64, r.float().contiguous(), z32, nrhs=nrhs)
    assert e.value.code == B.EINVAL


def test_f32_level0_copy_written_by_the_assembly():
    """A mixed-precision hierarchy's FP32 level-0 operator: after COO assembly of new
    values it is written in the same pass (the recompute then skips its cast); once a
    second hierarchy on the same operator holds the assembly's copy, the first one's
    recompute casts.  Either way it is the FP64 operator rounded to FP32, bit for bit,
    and destroying the second hierarchy changes nothing for the first."""
    m, i, j, v, A = q1_problem(8, mat_seed=4)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    o = B.blkamg_opts_default()
    o.hier_dtype, o.p_dtype = B.F32, B.F32

    def level0_matches(M):
        A0f = M.level(0)[0].arrays()[2]
        return torch.equal(A0f, HA.arrays()[2].float())

    M = B.amg_setup(HA, m.coords, m.dirichlet, o)
    assert level0_matches(M)
    for scale in (1.5, 0.25):
        B.coo_assemble_blocked(plan, dev(v * scale), B.INSERT, HA)
        assert level0_matches(M)  # written by the assembly itself
        B.amg_galerkin_recompute(M)
        assert level0_matches(M)
    M2 = B.amg_setup(HA, m.coords, m.dirichlet, o)  # now the registered copy
    B.coo_assemble_blocked(plan, dev(v * 3.0), B.ADD, HA)  # values 0.25 v + 3 v
    B.amg_galerkin_recompute(M)  # M's copy is no longer written by the assembly: cast
    assert level0_matches(M) and level0_matches(M2)
    del M2
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    B.amg_galerkin_recompute(M)
    assert level0_matches(M)
    b = dev(synth.rhs(m, 1))
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, its, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8)
    assert code == B.OK and rel <= 1e-8
