"""Pins of the learned-eigenbound oracle: the network's gradients against central
finite differences and closed forms, Adam's first step, the features against closed
forms and invariances, the judge against a dense eigensolver, the growth test
against the smoother's eigen-decomposition."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import mlp as ML
from oracle import sa
from oracle import solve as OS
from oracle import sparse as S


def _theta(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0.0, scale, ML.N_PARAMS)


def test_param_count_and_packing():
    assert ML.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2 == 5122
    th = _theta(0)
    assert np.array_equal(ML.pack(ML.unpack(th)), th)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(40, 12))
    T = rng.normal(size=(40, 2))
    th = _theta(2)
    g = ML.backward(th, X, T)
    h = 1e-6
    fd = np.empty_like(th)
    for k in range(ML.N_PARAMS):
        e = np.zeros_like(th)
        e[k] = h
        fd[k] = (ML.loss(th + e, X, T) - ML.loss(th - e, X, T)) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-7 * np.linalg.norm(g)


def test_zero_weights_closed_form():
    th = np.zeros(ML.N_PARAMS)
    p = ML.unpack(th)
    p["b3"][:] = [0.5, -2.0]
    th = ML.pack(p)
    X = np.random.default_rng(3).normal(size=(7, 12))
    T = np.random.default_rng(4).normal(size=(7, 2))
    _, _, Y = ML.forward(th, X)
    assert np.array_equal(Y, np.tile([0.5, -2.0], (7, 1)))
    g = ML.unpack(ML.backward(th, X, T))
    assert np.allclose(g["b3"], (np.array([0.5, -2.0]) - T).mean(axis=0), rtol=1e-14, atol=0)
    for k in ("W1", "b1", "W2", "b2", "W3"):
        assert not g[k].any()  # every hidden unit is dead at zero weights


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.5, 1e-3])
    th, m, v = ML.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(th, -0.01 * np.sign(g), rtol=1e-15, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def _tridiag(n):
    rows = []
    for i in range(n):
        c = [j for j in (i - 1, i, i + 1) if 0 <= j < n]
        rows.append(c)
    rowptr = np.concatenate([[0], np.cumsum([len(c) for c in rows])])
    colidx = np.concatenate(rows)
    val = np.array([[[2.0 if j == i else -1.0]] for i, c in enumerate(rows) for j in c])
    return S.Bsr(n, n, 1, 1, rowptr, colidx, val)


def test_features_closed_forms():
    A = _tridiag(10)  # D^-1 A rows: 1.5 at the ends, 2 inside
    f = ML.features(A, S.block_diag_inverse(A), 0)
    assert f[0] == pytest.approx(np.log(2.0), rel=1e-15)
    assert f[1] == pytest.approx(np.log((2 * 1.5 + 8 * 2.0) / 10), rel=1e-15)
    assert f[3] == pytest.approx(np.log1p(1.0), rel=1e-15)      # two off-diagonal 1/2 entries
    assert f[5] == 0.0 and f[6] == pytest.approx(2.8) and f[7] == 3.0
    # block-diagonal operator: D^-1 A = I
    D = S.Bsr(4, 4, 3, 3, np.arange(5), np.arange(4), np.stack([np.eye(3) * (k + 1) for k in range(4)]))
    fd = ML.features(D, S.block_diag_inverse(D), 2)
    assert fd[0] == 0.0 and fd[1] == 0.0 and fd[3] == 0.0 and fd[4] == 0.0
    assert fd[5] == pytest.approx(np.log(4.0)) and fd[9] == 2.0 and fd[10] == 0.5


def test_features_scale_invariance_and_gershgorin_bound():
    m = synth.make_mesh(3)
    i, j = synth.coo_indices(m)
    E, nu = synth.materials(m.n_elem, 5)
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, synth.coo_values(m, *synth.lame(E, nu)))
    Dinv = S.block_diag_inverse(A)
    f = ML.features(A, Dinv, 0)
    A2 = S.Bsr(A.nbr, A.nbc, A.br, A.bc, A.rowptr, A.colidx, A.val * 7.5)
    f2 = ML.features(A2, S.block_diag_inverse(A2), 0)
    assert np.allclose(f, f2, rtol=1e-13, atol=1e-13)
    Ad = S.to_dense(A)
    Dm = np.linalg.inv(sp.block_diag(list(Dinv)).toarray())
    lam = np.linalg.eigvals(np.linalg.solve(Dm, Ad)).real.max()
    assert np.log(lam) <= f[0] + 1e-12


def _q1(n, seed):
    m = synth.make_mesh(n)
    i, j = synth.coo_indices(m)
    E, nu = synth.materials(m.n_elem, seed)
    return S.coo_assemble(m.n_nodes, m.n_nodes, i, j, synth.coo_values(m, *synth.lame(E, nu)))


def _sym_spectrum(A, Dinv):
    Ad = S.to_dense(A)
    Dh = np.linalg.inv(sp.block_diag(list(Dinv)).toarray())
    w, V = np.linalg.eigh(Dh)
    Dm12 = V @ np.diag(w ** -0.5) @ V.T
    Dp12 = V @ np.diag(w ** 0.5) @ V.T
    lam, Q = np.linalg.eigh(Dm12 @ Ad @ Dm12)
    return lam, Q, Dm12, Dp12


def test_judge_matches_dense_eigensolver():
    A = _q1(3, 8)
    Dinv = S.block_diag_inverse(A)
    lam, _, _, _ = _sym_spectrum(A, Dinv)
    lj = ML.judge_lambda(A, Dinv, k=50)
    assert abs(lj - lam.max()) <= 1e-10 * lam.max()
    l10, _, _ = sa.lanczos_lambda_max(A, Dinv, 10)
    assert l10 <= lj * (1 + 1e-12)


def test_growth_matches_eigendecomposition_and_flags_low_bounds():
    A = _q1(3, 9)
    Dinv = S.block_diag_inverse(A)
    o = OS.Options()
    lam, Q, Dm12, Dp12 = _sym_spectrum(A, Dinv)
    lmax = lam.max()

    def p(x, lh):
        a, b = o.cheb_lo * lh, o.cheb_hi * lh
        T2 = lambda y: 2 * y * y - 1  # noqa: E731  (degree 2)
        return T2((b + a - 2 * x) / (b - a)) / T2((b + a) / (b - a))

    from oracle.mix import start_vector
    e0 = start_vector(A.nbr * A.br, ML.GROWTH_SEED)
    Ad = S.to_dense(A)
    for lh, expect_growth in ((lmax, False), (0.3 * lmax, True)):
        e1 = Dm12 @ Q @ np.diag(p(lam, lh)) @ Q.T @ Dp12 @ e0
        closed = np.sqrt((e1 @ Ad @ e1) / (e0 @ Ad @ e0))
        g = ML.growth(A, Dinv, lh, o)
        assert abs(g - closed) <= 1e-10 * closed
        assert (g > 1.0) == expect_growth
        assert g <= np.abs(p(lam, lh)).max() * (1 + 1e-12)
        # power steps: e_k = S^k e_0 in closed form, ratio of the last two A-norms
        for k in (2, 4):
            ek = Dm12 @ Q @ np.diag(p(lam, lh) ** k) @ Q.T @ Dp12 @ e0
            ek1 = Dm12 @ Q @ np.diag(p(lam, lh) ** (k - 1)) @ Q.T @ Dp12 @ e0
            closed_k = np.sqrt((ek @ Ad @ ek) / (ek1 @ Ad @ ek1))
            gk = ML.growth(A, Dinv, lh, o, steps=k)
            assert abs(gk - closed_k) <= 1e-9 * closed_k
            assert gk <= np.abs(p(lam, lh)).max() * (1 + 1e-12)
    # a moderately low bound (1/1.25 of lambda_max) amplifies the top of the spectrum:
    # one application can hide it behind the contracted bulk, power steps show it
    lh = lmax / 1.25
    assert np.abs(p(lam, lh)).max() > 1.0
    assert ML.growth(A, Dinv, lh, o, steps=6) > ML.growth(A, Dinv, lh, o, steps=1)
