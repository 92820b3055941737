"""Ablation of the trained eigenbound network on a problem outside its training set
(32^3 elements, material seed 21; training used seeds 1000+): the same FP32
hierarchy refreshed by Lanczos and by the network (deferred guard: CG checks its own
residual).  The network must keep the smoother valid one-sidedly (the Chebyshev
interval's end 1.1 lambda_net covers the 50-step reference lambda_max on every level,
no fallback, no restart), reach the same PCG iteration count as the Lanczos run, and
make refresh + solve faster."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from paper_2606_24748_amd import blkamg as B  # noqa: E402
from paper_2606_24748_amd import train_eigmlp  # noqa: E402


def test_packaged_model_shape_and_report():
    model = train_eigmlp.load_model()
    assert model.shape == (B.MLP_MODEL,) and np.all(np.isfinite(model))
    assert np.all(model[B.MLP_PARAMS + 12:B.MLP_PARAMS + 24] > 0)


def _timed_refresh(M, reps=5):
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        B.amg_smoother_refresh(M)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def test_network_against_lanczos_ablation():
    n = 32
    m = synth.make_mesh(n)
    i, j = synth.coo_indices(m)
    v = synth.coo_values_torch(m, *synth.lame(*synth.materials(m.n_elem, 21)), "cuda")
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, v, B.INSERT, HA)
    b = torch.as_tensor(synth.rhs(m, 22), device="cuda")
    out = {}
    for mode in (B.EIG_LANCZOS, B.EIG_MLP):
        o = B.blkamg_opts_default()
        o.hier_dtype, o.p_dtype, o.eig_mode, o.mlp_guard = B.F32, B.F32, mode, B.GUARD_PCG
        M = B.amg_setup(HA, m.coords, m.dirichlet, o)
        if mode == B.EIG_MLP:
            B.amg_set_eig_model(M, train_eigmlp.load_model())
        B.amg_smoother_refresh(M)
        ms = _timed_refresh(M)
        x = torch.zeros_like(b)
        code, its, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8)
        assert code == B.OK and rel <= 1e-8
        lam = M.lambdas().copy()
        tot = []
        for _ in range(5):  # refresh + solve, end to end
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            B.amg_smoother_refresh(M)
            B.pcg_solve(HA, M, b, x, rtol=1e-8)
            e1.record()
            e1.synchronize()
            tot.append(e0.elapsed_time(e1))
        judge = B.amg_judge_lambdas(M, 50)[:, 0]
        out[mode] = dict(ms=ms, its=its, lam=lam, judge=judge, total=float(np.median(tot)))
        if mode == B.EIG_MLP:
            fb, _, _ = B.amg_eig_status(M)
            assert not fb.any() and B.amg_guard_status(M) == (True, 0)
    lz, nn = out[B.EIG_LANCZOS], out[B.EIG_MLP]
    err_l = lz["lam"] / lz["judge"] - 1
    nn_err = nn["lam"] / nn["judge"] - 1
    print(f"refresh ms lanczos {lz['ms']:.3f} network {nn['ms']:.3f}; refresh + solve {lz['total']:.2f} vs "
          f"{nn['total']:.2f} ms; its {lz['its']} vs {nn['its']}; lambda err lanczos {np.round(err_l, 4).tolist()} "
          f"network {np.round(nn_err, 4).tolist()}", flush=True)
    assert np.all(1.1 * nn["lam"] >= nn["judge"])  # one-sided: the interval covers lambda_max
    assert np.all(np.abs(nn_err) <= 0.15)
    assert nn["its"] == lz["its"]
    assert nn["ms"] < lz["ms"] and nn["total"] < lz["total"]
