"""Ablation of the trained eigenbound network on a problem outside its training set
(32^3 elements, material seed 21; training used seeds 1000+): the same FP32
hierarchy refreshed by Lanczos and by the network.  The network must keep the
smoother valid (no fallback, lambda within 15% of the 50-step reference on every
level), keep PCG's iteration count within 2 of the Lanczos run, and refresh faster."""
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
        o.hier_dtype, o.p_dtype, o.eig_mode = B.F32, B.F32, mode
        M = B.amg_setup(HA, m.coords, m.dirichlet, o)
        if mode == B.EIG_MLP:
            B.amg_set_eig_model(M, train_eigmlp.load_model())
        B.amg_smoother_refresh(M)
        ms = _timed_refresh(M)
        x = torch.zeros_like(b)
        code, its, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8)
        assert code == B.OK and rel <= 1e-8
        judge = B.amg_judge_lambdas(M, 50)[:, 0]
        out[mode] = dict(ms=ms, its=its, lam=M.lambdas().copy(), judge=judge)
        if mode == B.EIG_MLP:
            fb, g, _ = B.amg_eig_status(M)
            assert not fb.any() and np.all(g[:, 0] < 1.0)
    lz, nn = out[B.EIG_LANCZOS], out[B.EIG_MLP]
    err_l = np.abs(lz["lam"] / lz["judge"] - 1)
    err_n = np.abs(nn["lam"] / nn["judge"] - 1)
    print(f"refresh ms lanczos {lz['ms']:.3f} network {nn['ms']:.3f}; its {lz['its']} vs {nn['its']}; "
          f"lambda err lanczos {np.round(err_l, 4).tolist()} network {np.round(err_n, 4).tolist()}", flush=True)
    assert np.all(err_n <= 0.15)
    assert nn["its"] <= lz["its"] + 2
    assert nn["ms"] < lz["ms"]
