"""Learned eigenbound: level features, the 12 -> 64 -> 64 -> 2 network, its
gradients and Adam step, the reference eigen-estimate it is trained on and judged
by, and the smoother-growth check that decides the fallback to Lanczos.

The paper's method estimates lambda_max of D^-1 A per level (it sets the Chebyshev
interval, paper §4.1, and the prolongator-smoothing weight, paper §2.2) with a few
Lanczos steps; here a small network predicts it from cheap block-row statistics and
Lanczos stays as the fallback and as the judge.  Readings (the method's learned part
has no paper text to follow): ReLU activations, mean-squared loss on standardised
(log lambda_max, omega) targets with omega = omega_scale / lambda_max, the twelve
features listed at `features`, the A-norm growth test at `growth`.

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64 numpy throughout.
Parity: the network and its gradients are pinned by central finite differences and
closed forms; the features by invariances and the Gershgorin bound; the judge by a
dense eigensolver; the growth test by the eigen-decomposition of the smoother.
"""
from __future__ import annotations

import numpy as np

from . import sparse as S
from . import solve
from .mix import start_vector

N_IN, N_HID, N_OUT = 12, 64, 2
SHAPES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 5122


def unpack(theta: np.ndarray) -> dict:
    """Flat parameter vector -> named arrays (row-major, in x out weights)."""
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def forward(theta: np.ndarray, X: np.ndarray):
    """X [N][12] (standardised features) -> (H1, H2, Y): H1 = relu(X W1 + b1),
    H2 = relu(H1 W2 + b2), Y = H2 W3 + b3."""
    p = unpack(theta)
    H1 = np.maximum(X @ p["W1"] + p["b1"], 0.0)
    H2 = np.maximum(H1 @ p["W2"] + p["b2"], 0.0)
    Y = H2 @ p["W3"] + p["b3"]
    return H1, H2, Y


def loss(theta: np.ndarray, X: np.ndarray, T: np.ndarray) -> float:
    """L = 1/(2N) sum (Y - T)^2."""
    _, _, Y = forward(theta, X)
    return 0.5 * float(((Y - T) ** 2).sum()) / X.shape[0]


def backward(theta: np.ndarray, X: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Gradient of `loss` by the chain rule, flat like theta."""
    p = unpack(theta)
    H1, H2, Y = forward(theta, X)
    dY = (Y - T) / X.shape[0]
    g = {"W3": H2.T @ dY, "b3": dY.sum(axis=0)}
    dH2 = (dY @ p["W3"].T) * (H2 > 0.0)
    g["W2"] = H1.T @ dH2
    g["b2"] = dH2.sum(axis=0)
    dH1 = (dH2 @ p["W2"].T) * (H1 > 0.0)
    g["W1"] = X.T @ dH1
    g["b1"] = dH1.sum(axis=0)
    return pack(g)


def adam_step(theta, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba, 2015, Algorithm 1), step t >= 1; returns new
    (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# level features
# ---------------------------------------------------------------------------
def row_stats(A: S.Bsr, Dinv: np.ndarray):
    """Per block row i: g_i = max over its scalar rows of the absolute row sum of
    D_i^-1 [A_i1 ... A_in] (the Gershgorin radius plus centre of D^-1 A), h_i = sum over
    j != i of ||D_i^-1 A_ij||_F, d_i = ||A_ii||_F, and the number of stored blocks."""
    n = A.nbr
    g = np.zeros(n)
    h = np.zeros(n)
    d = np.zeros(n)
    nb = np.zeros(n)
    for i in range(n):
        rows = np.zeros(A.br)
        for t in range(A.rowptr[i], A.rowptr[i + 1]):
            j = A.colidx[t]
            M = Dinv[i] @ A.val[t]
            rows += np.abs(M).sum(axis=1)
            if j == i:
                d[i] = np.sqrt((A.val[t] ** 2).sum())
            else:
                h[i] += np.sqrt((M ** 2).sum())
        g[i] = rows.max()
        nb[i] = A.rowptr[i + 1] - A.rowptr[i]
    return g, h, d, nb


def features(A: S.Bsr, Dinv: np.ndarray, level: int) -> np.ndarray:
    """The twelve inputs of the network for one level operator (reading):
    0 log max g, 1 log mean g, 2 log sqrt(mean g^2), 3 log(1 + max h),
    4 log(1 + mean h), 5 log(max d / min d), 6 mean blocks per row,
    7 max blocks per row, 8 log(scalar rows), 9 level index, 10 block size / 6,
    11 log(1 + mean h) - log mean g."""
    g, h, d, nb = row_stats(A, Dinv)
    f = np.empty(N_IN)
    f[0] = np.log(g.max())
    f[1] = np.log(g.mean())
    f[2] = np.log(np.sqrt((g * g).mean()))
    f[3] = np.log1p(h.max())
    f[4] = np.log1p(h.mean())
    f[5] = np.log(d.max() / d.min())
    f[6] = nb.mean()
    f[7] = nb.max()
    f[8] = np.log(A.nbr * A.br)
    f[9] = float(level)
    f[10] = A.br / 6.0
    f[11] = f[4] - f[1]
    return f


# ---------------------------------------------------------------------------
# judge and fallback test
# ---------------------------------------------------------------------------
def judge_lambda(A: S.Bsr, Dinv: np.ndarray, k: int = 50, seed: int = 0x5EED) -> float:
    """lambda_max(D^-1 A) by k steps of Lanczos in the D inner product with full
    reorthogonalisation (classical Gram-Schmidt against every earlier Lanczos vector
    after each step), started like the level's estimate.  Returns the largest Ritz
    value."""
    n = A.nbr * A.br
    Dblk = np.linalg.inv(Dinv)
    As = S.to_scalar_csr(A)
    v = start_vector(n, seed)
    Dv = S.block_diag_apply(Dblk, v)
    nrm = np.sqrt(v @ Dv)
    U = [v / nrm]
    Y = [Dv / nrm]
    alphas, betas = [], []
    for step in range(min(k, n)):
        u, y = U[-1], Y[-1]
        wy = As @ u
        alpha = u @ wy
        alphas.append(alpha)
        if step == min(k, n) - 1:
            break
        wy = wy - alpha * y
        if step > 0:
            wy = wy - betas[-1] * Y[-2]
        wu = S.block_diag_apply(Dinv, wy)
        c = np.array([yj @ wu for yj in Y])  # <u_j, wu>_D
        wu = wu - sum(cj * uj for cj, uj in zip(c, U))
        wy = wy - sum(cj * yj for cj, yj in zip(c, Y))
        beta = np.sqrt(max(wu @ wy, 0.0))
        if beta <= 1e-14 * abs(alpha):
            break
        betas.append(beta)
        U.append(wu / beta)
        Y.append(wy / beta)
    T = np.diag(alphas) + np.diag(betas[:len(alphas) - 1], 1) + np.diag(betas[:len(alphas) - 1], -1)
    return float(np.linalg.eigvalsh(T).max())


GROWTH_SEED = 0xC0FFEE


def growth(A: S.Bsr, Dinv: np.ndarray, lam: float, opts: solve.Options, seed: int = GROWTH_SEED,
           steps: int = 1) -> float:
    """A-norm growth of the level's smoother error propagation S (the smoother's result
    for f = 0) after `steps` applications: e_0 from `start_vector`, e_k = S e_(k-1), and
    the value sqrt(e_k^T A e_k / e_(k-1)^T A e_(k-1)) of the last application.  With the
    Chebyshev interval covering the spectrum of D^-1 A the smoother contracts in the
    A-norm (value < 1); an interval whose upper end is well below lambda_max amplifies
    the top of the spectrum (value > 1).  Repeated applications let the amplified modes
    dominate, so the last ratio approaches the largest |p(lambda)| over the spectrum."""
    n = A.nbr * A.br
    e = start_vector(n, seed)
    a_prev = e @ S.spmv(A, e)
    a_cur = a_prev
    for _ in range(steps):
        a_prev = a_cur
        e = solve.chebyshev(A, Dinv, lam, np.zeros(n), e, opts.cheb_degree, opts.cheb_lo, opts.cheb_hi)
        a_cur = e @ S.spmv(A, e)
    return float(np.sqrt(max(a_cur, 0.0) / a_prev))
