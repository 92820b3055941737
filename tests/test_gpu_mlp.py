"""GPU parity of the learned-eigenbound pieces: the MFMA products, the network's
forward pass, loss gradient and Adam step against the FP64 oracle; level features
and the reference Lanczos against the oracle; the growth test and the Lanczos
fallback with crafted models."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import batch as OB  # noqa: E402
from oracle import mlp as ML  # noqa: E402
from oracle import solve as OS  # noqa: E402
from oracle import sparse as S  # noqa: E402
from paper_2606_24748_amd import blkamg as B  # noqa: E402
from tests.gpu_util import dev, from_device_bsr, rel2  # noqa: E402


def f32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("m,n,k,ta,tb", [(1, 1, 1, 0, 0), (16, 16, 4, 0, 0), (17, 33, 5, 0, 0), (37, 3, 130, 1, 0),
                                         (12, 64, 2000, 1, 0), (2000, 64, 12, 0, 0), (2000, 64, 2, 0, 1),
                                         (64, 2, 999, 1, 0), (5, 70, 9, 1, 1)])
def test_mfma_gemm_matches_numpy(m, n, k, ta, tb):
    rng = np.random.default_rng(m * 1000 + n + k)
    a = rng.normal(size=(k, m) if ta else (m, k))
    b = rng.normal(size=(n, k) if tb else (k, n))
    c = torch.full((m, n), 5.0, dtype=torch.float32, device="cuda")
    B.mlp_gemm_f32(f32(a), f32(b), c, trans_a=bool(ta), trans_b=bool(tb))
    want = (a.T if ta else a).astype(np.float32).astype(np.float64) @ (b.T if tb else b).astype(np.float32).astype(
        np.float64)
    assert rel2(c.cpu().numpy(), want) <= 3e-6 * max(1.0, np.sqrt(k) / 8)


def _net_case(seed, n=300):
    rng = np.random.default_rng(seed)
    th = rng.normal(0.0, 0.3, ML.N_PARAMS).astype(np.float32).astype(np.float64)
    X = rng.normal(size=(n, 12)).astype(np.float32).astype(np.float64)
    T = rng.normal(size=(n, 2)).astype(np.float32).astype(np.float64)
    return th, X, T


def test_forward_and_gradient_match_oracle():
    th, X, T = _net_case(7)
    n = X.shape[0]
    h1 = torch.zeros(n, 64, dtype=torch.float32, device="cuda")
    h2 = torch.zeros_like(h1)
    y = torch.zeros(n, 2, dtype=torch.float32, device="cuda")
    tt, xx = f32(th), f32(X)
    B.mlp_forward(tt, xx, h1, h2, y)
    H1, H2, Y = ML.forward(th, X)
    assert rel2(h1.cpu().numpy(), H1) <= 1e-5
    assert rel2(h2.cpu().numpy(), H2) <= 1e-5
    assert rel2(y.cpu().numpy(), Y) <= 1e-5
    work = torch.zeros(130 * n, dtype=torch.float32, device="cuda")
    grad = torch.zeros(ML.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.mlp_loss_grad(tt, xx, h1, h2, y, f32(T), work, grad, loss)
    assert abs(float(loss) - ML.loss(th, X, T)) <= 1e-5 * ML.loss(th, X, T)
    g = ML.backward(th, X, T)
    gg = grad.cpu().numpy()
    assert rel2(gg, g) <= 1e-4
    for name, (a, b) in zip(("W1", "b1", "W2", "b2", "W3", "b3"), zip(ML.unpack(gg).values(), ML.unpack(g).values())):
        assert rel2(a, b) <= 1e-4, name


def test_adam_matches_oracle_and_training_reduces_loss():
    th, X, T = _net_case(8, n=512)
    T = np.stack([X[:, 0] - 0.5 * X[:, 3], np.tanh(X[:, 1])], axis=1)  # learnable targets
    n = X.shape[0]
    tt, xx, tg = f32(th), f32(X), f32(T)
    h1 = torch.zeros(n, 64, dtype=torch.float32, device="cuda")
    h2 = torch.zeros_like(h1)
    y = torch.zeros(n, 2, dtype=torch.float32, device="cuda")
    work = torch.zeros(130 * n, dtype=torch.float32, device="cuda")
    grad = torch.zeros(ML.N_PARAMS, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    mo, vo = np.zeros(ML.N_PARAMS), np.zeros(ML.N_PARAMS)
    for step in range(1, 4):  # three steps: the update against the FP64 oracle's Adam on the same gradient
        B.mlp_forward(tt, xx, h1, h2, y)
        B.mlp_loss_grad(tt, xx, h1, h2, y, tg, work, grad, loss)
        before = tt.cpu().numpy().astype(np.float64)
        gd = grad.cpu().numpy().astype(np.float64)
        B.mlp_adam(tt, grad, m, v, step, 1e-3)
        want, mo, vo = ML.adam_step(before, gd, mo, vo, step, 1e-3)
        assert np.abs(tt.cpu().numpy() - want).max() <= 1e-6 * 1e-3 + 1e-7 * np.abs(want).max(), step
    first = None
    for step in range(4, 400):
        B.mlp_forward(tt, xx, h1, h2, y)
        B.mlp_loss_grad(tt, xx, h1, h2, y, tg, work, grad, loss)
        B.mlp_adam(tt, grad, m, v, step, 3e-3)
        if first is None:
            first = float(loss)
    assert float(loss) <= 0.1 * first, (first, float(loss))


def _q1_gpu(n, seed, hier=B.F64, eig=B.EIG_LANCZOS, guard=B.GUARD_SMOOTHER):
    m = synth.make_mesh(n)
    i, j = synth.coo_indices(m)
    E, nu = synth.materials(m.n_elem, seed)
    v = synth.coo_values(m, *synth.lame(E, nu))
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    o = B.blkamg_opts_default()
    o.hier_dtype = hier
    o.p_dtype = hier
    o.eig_mode = eig
    o.mlp_guard = guard
    M = B.amg_setup(HA, m.coords, m.dirichlet, o)
    return m, A, plan, HA, M


def test_features_and_judge_match_oracle():
    m, A, plan, HA, M = _q1_gpu(10, 3)
    H = OS.setup(A, m.coords, m.dirichlet)
    feat, lev, inst = B.amg_features(M)
    assert list(lev) == list(range(H.n_levels - 1)) and not inst.any()
    F = feat.cpu().numpy()
    lam_j = B.amg_judge_lambdas(M, 50)[:, 0]
    for l in range(H.n_levels - 1):
        L = H.levels[l]
        want = ML.features(L.A, L.Dinv, l)
        assert np.allclose(F[l], want, rtol=2e-6, atol=2e-6), (l, F[l], want)
        lj = ML.judge_lambda(L.A, L.Dinv, 50, L_seed(l))
        assert abs(lam_j[l] - lj) <= 1e-9 * lj, (l, lam_j[l], lj)
        assert lam_j[l] >= L.lam * (1 - 1e-12)  # the 10-step estimate never exceeds it


def L_seed(level):
    return OS.Options().lanczos_seed + level


def test_batched_features_match_per_instance_oracle():
    sizes = [8, 6, 10]
    bt = synth.make_batch(sizes, nrhs=1)
    nn = bt["n_nodes"]
    A = S.coo_assemble(nn, nn, bt["i"], bt["j"], synth.batch_values(bt))
    plan, HA = B.coo_plan_create(nn, nn, 3, 3, bt["i"], bt["j"])
    B.coo_assemble_blocked(plan, dev(synth.batch_values(bt)), B.INSERT, HA)
    M = B.amg_setup_batched(HA, bt["row0"], bt["coords"], bt["dirichlet"])
    H = OB.setup_batch(A, bt["row0"], bt["coords"], bt["dirichlet"])
    feat, lev, inst = B.amg_features(M)
    F = feat.cpu().numpy()
    lam_j = B.amg_judge_lambdas(M, 40)
    seen = set()
    for k in range(len(lev)):
        h = H[inst[k]]
        L = h.levels[lev[k]]
        assert np.allclose(F[k], ML.features(L.A, L.Dinv, lev[k]), rtol=2e-6, atol=2e-6)
        lj = ML.judge_lambda(L.A, L.Dinv, 40, L_seed(lev[k]))
        assert abs(lam_j[lev[k], inst[k]] - lj) <= 1e-9 * lj
        seen.add((int(lev[k]), int(inst[k])))
    assert seen == {(l, t) for t, h in enumerate(H) for l in range(h.n_levels - 1)}


def _const_model(lam, omega=0.5):
    """A model whose prediction is lam for every input: zero weights, the bias on the
    standardised target scale."""
    th = np.zeros(ML.N_PARAMS)
    stats = np.concatenate([np.zeros(12), np.ones(12), [0.0, 0.0], [1.0, 1.0]])
    p = ML.unpack(th)
    p["b3"][:] = [np.log(lam), omega]
    return np.concatenate([ML.pack(p), stats]).astype(np.float32)


def test_mlp_refresh_uses_prediction_and_passes_growth_test():
    m, A, plan, HA, M = _q1_gpu(10, 4, eig=B.EIG_MLP)
    lam_l = M.lambdas().copy()
    B.amg_set_eig_model(M, _const_model(8.0))  # above every level's lambda_max: weak but contracting
    B.amg_smoother_refresh(M)
    fb, g, om = B.amg_eig_status(M)
    assert not fb.any() and np.all(g[:, 0] < 1.0)
    assert np.allclose(M.lambdas(), np.float32(np.exp(np.float32(np.log(8.0)))), rtol=1e-6)
    assert np.allclose(om[:, 0], 0.5)
    H = OS.setup(A, m.coords, m.dirichlet)
    for l in range(H.n_levels - 1):
        L = H.levels[l]
        want = ML.growth(L.A, L.Dinv, float(M.lambdas()[l]), OS.Options(), steps=B.blkamg_opts_default().growth_steps)
        assert abs(g[l, 0] - want) <= 1e-9 * want
    b = synth.rhs(m, 2)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, dev(b), x, rtol=1e-8)
    assert code == B.OK and rel <= 1e-8
    del lam_l


def test_mlp_refresh_falls_back_when_bound_is_too_low():
    m, A, plan, HA, M = _q1_gpu(10, 5, eig=B.EIG_MLP)
    lam_lanczos = M.lambdas().copy()
    lam_true = B.amg_judge_lambdas(M, 50)[:, 0]
    H = OS.setup(A, m.coords, m.dirichlet)
    # the injected value 0.3 lambda_true of level 0 is far too low for every level
    low = 0.3 * lam_true[0]
    for l in range(H.n_levels - 1):
        assert ML.growth(H.levels[l].A, H.levels[l].Dinv, low, OS.Options(), steps=3) > 1.0 or low >= lam_true[l]
    B.amg_set_eig_model(M, _const_model(low))
    B.amg_smoother_refresh(M)
    fb, g, _ = B.amg_eig_status(M)
    assert fb.all() and np.all(g[:, 0] > 1.0)
    assert np.array_equal(M.lambdas(), lam_lanczos)  # Lanczos values, recomputed the same way
    b = synth.rhs(m, 2)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, dev(b), x, rtol=1e-8)
    assert code == B.OK


@pytest.mark.parametrize("hier", [B.F64, B.F32])
def test_deferred_guard_restarts_cg_with_lanczos(hier):
    """mlp_guard = GUARD_PCG: a refresh with a far too low network bound runs no test and
    arms the guard; the next CG sees its preconditioned r.z turn non-positive or its
    residual blow up, refreshes every level by Lanczos and restarts; the restarted solve
    is, bit for bit, the solve of the same hierarchy refreshed by Lanczos."""
    print(f"deferred guard hier={hier}", flush=True)
    m, A, plan, HA, M = _q1_gpu(10, 5, hier=hier, eig=B.EIG_MLP, guard=B.GUARD_PCG)
    lam_lanczos = M.lambdas().copy()
    b = dev(synth.rhs(m, 2))
    xl = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code_l, it_l, _ = B.pcg_solve(HA, M, b, xl, rtol=1e-8)  # no model yet: Lanczos scalars
    lam_true = B.amg_judge_lambdas(M, 50)[:, 0]
    B.amg_set_eig_model(M, _const_model(0.1 * lam_true[0]))
    B.amg_smoother_refresh(M)
    fb, g, _ = B.amg_eig_status(M)
    assert not fb.any() and not g.any()
    assert B.amg_guard_status(M) == (True, 0)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8)
    assert B.amg_guard_status(M) == (False, 1)
    fb, _, _ = B.amg_eig_status(M)
    assert fb.all()
    assert np.array_equal(M.lambdas(), lam_lanczos)
    assert code == code_l == B.OK and it == it_l and torch.equal(x, xl)


def test_deferred_guard_keeps_a_good_bound_and_checks_other_solves():
    """With a bound above every level's lambda_max the armed guard lets CG run (no
    restart, iterations within one of Lanczos); vcycle_apply first runs the deferred
    smoother test, which passes."""
    m, A, plan, HA, M = _q1_gpu(10, 4, eig=B.EIG_MLP, guard=B.GUARD_PCG)
    b = dev(synth.rhs(m, 3))
    xl = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    _, it_l, _ = B.pcg_solve(HA, M, b, xl, rtol=1e-8)
    lam_true = B.amg_judge_lambdas(M, 50)[:, 0]
    B.amg_set_eig_model(M, _const_model(1.05 * lam_true.max()))
    B.amg_smoother_refresh(M)
    assert B.amg_guard_status(M) == (True, 0)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8)
    assert code == B.OK and rel <= 1e-8 and B.amg_guard_status(M) == (True, 0)
    z = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    B.vcycle_apply(M, b, z)
    fb, g, _ = B.amg_eig_status(M)
    assert B.amg_guard_status(M) == (False, 0) and not fb.any() and np.all(g[:, 0] > 0) and np.all(g[:, 0] < 1)
    del it_l


def test_deferred_guard_covers_the_cold_setup():
    """GUARD_PCG with the model given from the cold setup on: the setup keeps the
    network's lambda_hat and omega without a smoother test of its own, even a far too
    low bound, and arms the guard; the first CG sees the failing smoother, refreshes by
    Lanczos and restarts, and converges.  With GUARD_SMOOTHER the setup's test rejects
    the same model."""
    m = synth.make_mesh(10)
    i, j = synth.coo_indices(m)
    v = synth.coo_values(m, *synth.lame(*synth.materials(m.n_elem, 6)))
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    M0 = B.amg_setup(HA, m.coords, m.dirichlet)
    lam_true = B.amg_judge_lambdas(M0, 50)[:, 0]
    bad = _const_model(0.1 * lam_true[0], omega=4.0 / (3.0 * lam_true[0]))
    b = dev(synth.rhs(m, 2))
    for guard in (B.GUARD_PCG, B.GUARD_SMOOTHER):
        o = B.blkamg_opts_default()
        o.eig_mode, o.mlp_guard = B.EIG_MLP, guard
        keep = B.opts_with_model(o, bad)
        M = B.amg_setup(HA, m.coords, m.dirichlet, o)
        del keep
        _, om, learned = B.amg_setup_weights(M)
        if guard == B.GUARD_PCG:
            assert learned.all() and np.allclose(om[:, 0], 4.0 / (3.0 * lam_true[0]), rtol=1e-5)
            assert B.amg_guard_status(M) == (True, 0)
            x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
            code, it, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8)
            assert code == B.OK and rel <= 1e-8 and B.amg_guard_status(M) == (False, 1)
        else:
            assert not learned.any()


def test_model_validation_and_missing_model():
    m, A, plan, HA, M = _q1_gpu(6, 6, eig=B.EIG_MLP)
    bad = _const_model(2.0)
    bad[ML.N_PARAMS + 12] = 0.0  # a zero feature std
    with pytest.raises(B.BlkAmgError) as e:
        B.amg_set_eig_model(M, bad)
    assert e.value.code == B.EINVAL
    B.amg_smoother_refresh(M)  # no model yet: Lanczos
    fb, _, _ = B.amg_eig_status(M)
    assert not fb.any()


def _learned_setup(n, seed, model):
    """FP64 hierarchy whose cold setup takes lambda_hat and omega from `model`."""
    m = synth.make_mesh(n)
    i, j = synth.coo_indices(m)
    v = synth.coo_values(m, *synth.lame(*synth.materials(m.n_elem, seed)))
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v)
    plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
    B.coo_assemble_blocked(plan, dev(v), B.INSERT, HA)
    o = B.blkamg_opts_default()
    o.eig_mode = B.EIG_MLP
    keep = B.opts_with_model(o, model)
    M = B.amg_setup(HA, m.coords, m.dirichlet, o)
    del keep
    return m, A, HA, M


def _compare_setup_with_oracle(m, A, M, lam, om):
    """The oracle's cold setup given the library's (lambda_hat, omega) per level: same
    aggregates and patterns bit for bit, P and A_c within 1e-12."""
    H = OS.setup(A, m.coords, m.dirichlet, level_params=[(float(lam[l, 0]), float(om[l, 0]))
                                                          for l in range(M.num_levels() - 1)])
    assert H.n_levels == M.num_levels()
    for l in range(H.n_levels - 1):
        L = H.levels[l]
        assert np.array_equal(M.aggregates(l), L.agg)
        P = from_device_bsr(M.level(l)[1])
        assert np.array_equal(P.colidx, L.P.colidx) and rel2(P.val, L.P.val) <= 1e-12, l
        Ac = from_device_bsr(M.level(l + 1)[0])
        assert np.array_equal(Ac.colidx, H.levels[l + 1].A.colidx)
        assert rel2(Ac.val, H.levels[l + 1].A.val) <= 1e-12, l
    return H


def test_learned_cold_setup_uses_network_weights_and_matches_oracle():
    """A model predicting lambda_hat = 8 (above every level's lambda_max, so the guard
    passes) and omega = 0.3: the setup smooths every prolongator with omega = 0.3, and
    the oracle's setup given those weights reproduces it; the V-cycle matches too."""
    m, A, HA, M = _learned_setup(10, 4, _const_model(8.0, 0.3))
    lam, om, learned = B.amg_setup_weights(M)
    assert learned.all()
    assert np.allclose(om[:, 0], 0.3, rtol=1e-6) and np.allclose(lam[:, 0], 8.0, rtol=1e-6)
    H = _compare_setup_with_oracle(m, A, M, lam, om)
    r = np.random.default_rng(1).uniform(-1, 1, m.n_dof)
    z = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    B.vcycle_apply(M, dev(r), z)
    assert rel2(z.cpu().numpy(), OS.vcycle(H, r)) <= 1e-11
    # the same problem with Lanczos weights has a different prolongator
    Hl = OS.setup(A, m.coords, m.dirichlet)
    assert rel2(from_device_bsr(M.level(0)[1]).val, Hl.levels[0].P.val) > 1e-3


def test_learned_cold_setup_with_trained_model():
    """The packaged network in the cold setup of a problem outside its training draws:
    every level learned (the guard passes), weights within 25 % of the Lanczos
    setup's, parity with the oracle given those weights, and CG converges."""
    from paper_2606_24748_amd import train_eigmlp
    m, A, HA, M = _learned_setup(16, 31, train_eigmlp.load_model())
    lam, om, learned = B.amg_setup_weights(M)
    print(f"learned setup: lambda {lam[:, 0].tolist()} omega {om[:, 0].tolist()} learned {learned.tolist()}",
          flush=True)
    assert learned.all()
    H0 = OS.setup(A, m.coords, m.dirichlet)
    for l in range(M.num_levels() - 1):
        assert abs(lam[l, 0] / H0.levels[l].lam - 1) <= 0.25, l
    _compare_setup_with_oracle(m, A, M, lam, om)
    b = synth.rhs(m, 2)
    x = torch.zeros(m.n_dof, dtype=torch.float64, device="cuda")
    code, it, rel = B.pcg_solve(HA, M, dev(b), x, rtol=1e-8)
    assert code == B.OK and rel <= 1e-8


def test_learned_cold_setup_falls_back_to_lanczos():
    """A model predicting a far too low lambda_hat fails the growth test on every level:
    the setup then uses Lanczos and omega = 4 / (3 lambda_hat), bit for bit the plain
    setup's prolongators."""
    m, A, HA, M = _learned_setup(10, 5, _const_model(0.05, 0.3))
    lam, om, learned = B.amg_setup_weights(M)
    assert not learned.any()
    o = B.blkamg_opts_default()
    M0 = B.amg_setup(HA, m.coords, m.dirichlet, o)
    lam0, om0, le0 = B.amg_setup_weights(M0)
    assert not le0.any()
    assert np.array_equal(lam, lam0) and np.array_equal(om, om0)
    assert np.allclose(om0[:, 0], (4.0 / 3.0) / lam0[:, 0], rtol=1e-15)
    for l in range(M.num_levels() - 1):
        assert torch.equal(M.level(l)[1].arrays()[2], M0.level(l)[1].arrays()[2])


@pytest.mark.parametrize("lam_scale", [None, 0.3])
def test_mlp_refresh_and_judge_on_a_side_stream(lam_scale):
    """The learned refresh (growth test, fallback decision, host downloads) and the judge
    queued on a non-default stream give bit for bit the results of the default stream:
    the packaged model (no fallback) and a far too low constant bound (every level falls
    back to Lanczos)."""
    from paper_2606_24748_amd import train_eigmlp
    print(f"side stream lam_scale={lam_scale}", flush=True)
    m, A, plan, HA, M = _q1_gpu(12, 8, eig=B.EIG_MLP)
    if lam_scale is None:
        model = train_eigmlp.load_model()
    else:
        model = _const_model(lam_scale * B.amg_judge_lambdas(M, 50)[0, 0])
    B.amg_set_eig_model(M, model)
    res = []
    for side in (False, True):
        torch.cuda.synchronize()
        st = torch.cuda.Stream() if side else torch.cuda.current_stream()
        with torch.cuda.stream(st):
            B.amg_smoother_refresh(M)
            fb, g, om = B.amg_eig_status(M)
            lam = M.lambdas().copy()
            judge = B.amg_judge_lambdas(M, 30)
        st.synchronize()
        res.append((fb.copy(), g.copy(), om.copy(), lam, judge.copy()))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    assert res[0][0].all() == (lam_scale is not None)
