"""Oracle parity at the 64^3 FP64 problem (823,875 dofs, four levels: 3x3 fine
blocks, 3x6 then 6x6 prolongators, 6x6 coarse operators), the problem the CPU
baseline of the benchmark runs: cold setup on materials seed 1, hot recompute on the
redrawn materials (seed 1001), right-hand side seed 2.  The oracle runs whole on the
host inside the test (about a minute of CPU time)."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import sparse as S  # noqa: E402
from oracle import solve  # noqa: E402
from paper_2606_24748_amd import blkamg as B  # noqa: E402
from tests.gpu_util import dev, from_device_bsr, rel2  # noqa: E402

N = 64
SEEDS = (1, 1001, 2)


@pytest.fixture(scope="module")
def cfg():
    print(f"config S: n={N}, seeds {SEEDS}", flush=True)
    t0 = time.perf_counter()
    m = synth.make_mesh(N)
    i, j = synth.coo_indices(m)
    v0 = synth.coo_values(m, *synth.lame(*synth.materials(m.n_elem, SEEDS[0])))
    v1 = synth.coo_values(m, *synth.lame(*synth.materials(m.n_elem, SEEDS[1])))
    b = synth.rhs(m, SEEDS[2])
    # GPU: cold setup on the first draw, then the hot recompute on the second
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v0), B.INSERT, HA)
    M = B.amg_setup(HA, m.coords, m.dirichlet)
    B.coo_assemble_blocked(plan, dev(v1), B.INSERT, HA)
    B.amg_galerkin_recompute(M)
    B.amg_smoother_refresh(M)
    torch.cuda.synchronize()
    print(f"  gpu setup + recompute done ({time.perf_counter() - t0:.1f}s)", flush=True)
    A0 = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v0)
    H = solve.setup(A0, m.coords, m.dirichlet)
    print(f"  oracle setup done ({time.perf_counter() - t0:.1f}s)", flush=True)
    A1 = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v1)
    H1 = solve.recompute(H, A1)
    print(f"  oracle recompute done ({time.perf_counter() - t0:.1f}s)", flush=True)
    return dict(m=m, b=b, HA=HA, M=M, H=H, H1=H1, A1=A1, plan=plan)


def test_config_s_levels_aggregates_and_patterns(cfg):
    M, H1 = cfg["M"], cfg["H1"]
    assert M.num_levels() == H1.n_levels == 4
    assert [L.A.nbr * L.A.br for L in H1.levels] == [823875, 63888, 3072, 162]
    for l in range(3):
        L = H1.levels[l]
        assert np.array_equal(M.aggregates(l), L.agg), l
        P = from_device_bsr(M.level(l)[1])
        assert np.array_equal(P.rowptr, L.P.rowptr) and np.array_equal(P.colidx, L.P.colidx), l
        Ac = from_device_bsr(M.level(l + 1)[0])
        want = H1.levels[l + 1].A
        assert np.array_equal(Ac.rowptr, want.rowptr) and np.array_equal(Ac.colidx, want.colidx), l


def test_config_s_values_after_hot_recompute(cfg):
    M, H1 = cfg["M"], cfg["H1"]
    lam = M.lambdas()
    for l in range(3):
        L = H1.levels[l]
        assert abs(lam[l] - L.lam) <= 1e-12 * L.lam, (l, lam[l], L.lam)
        P = from_device_bsr(M.level(l)[1])
        assert rel2(P.val, L.P.val) <= 1e-12, l          # P is reused: the setup's values
        Ac = from_device_bsr(M.level(l + 1)[0])
        err = rel2(Ac.val, H1.levels[l + 1].A.val)       # Frobenius norm of the difference
        print(f"  level {l + 1}: A_c rel Frobenius error {err:.2e}", flush=True)
        assert err <= 1e-12, l


def test_config_s_vcycle_and_pcg(cfg):
    m, b, HA, M, H1, A1 = cfg["m"], cfg["b"], cfg["HA"], cfg["M"], cfg["H1"], cfg["A1"]
    r = np.random.default_rng(3).uniform(-1, 1, m.n_dof)
    z = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    B.vcycle_apply(M, dev(r), z)
    assert rel2(z.cpu().numpy(), solve.vcycle(H1, r)) <= 1e-11
    _, it_o, rel_o, ok = solve.pcg(A1, b, lambda q: solve.vcycle(H1, q), rtol=1e-8)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, dev(b), x, rtol=1e-8)
    print(f"  pcg its gpu={it} oracle={it_o}", flush=True)
    assert ok and code == B.OK and abs(it - it_o) <= 1
    res = np.linalg.norm(b - S.spmv(A1, x.cpu().numpy())) / np.linalg.norm(b)
    assert res <= 2e-8
