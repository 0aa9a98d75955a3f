"""Pins of the oracle's KL(P||Q), Z and t-SNE gradient.

Definitions followed (van der Maaten & Hinton 2008): Student-t Q (eq. 4),
cost KL(P||Q) (eq. 2 with symmetric P), gradient (eq. 5), early
exaggeration multiplying P (Sec. 3.4).  The pins are finite differences,
an independent library implementation of the dense exact method
(scikit-learn), closed cases and invariants.
"""
import numpy as np
import pytest
import scipy.special
from scipy.spatial.distance import squareform
from sklearn.manifold import _t_sne as skl_tsne

from paper_2605_13928_amd import synth


def make_problem(oracle_mod, n, k, perp, seed, y_std=1.0):
    X, _ = synth.make_points("c1", n=n, seed=seed)
    idx, d2 = oracle_mod.knn(X, k)
    Pc, _, _, _ = oracle_mod.calibrate(d2, perp)
    S = oracle_mod.symmetrize(idx, Pc)
    Y = synth.random_embedding(n, y_std, seed + 100).astype(np.float64)
    return S, Y


def objective(oracle_mod, Y, S, alpha):
    # C_alpha = -alpha sum p ln w + ln Z, assembled from the oracle's KL
    # (sum p ln p - sum p ln w + S ln Z) with S = 1.
    kl, Z = oracle_mod.kl(Y, S)
    plogp = float(np.sum(S.val * np.log(S.val)))
    m_plogw = kl - plogp - S.val.sum() * np.log(Z)
    return alpha * m_plogw + np.log(Z)


@pytest.mark.parametrize("alpha", [1.0, 12.0])
def test_gradient_matches_finite_differences(oracle_mod, alpha):
    S, Y = make_problem(oracle_mod, 120, 30, 10.0, 3)
    g, Z, kl = oracle_mod.kl_grad(Y, S, alpha)
    h = 1e-6
    rng = np.random.default_rng(0)
    for i in rng.choice(120, 12, replace=False):
        for c in range(2):
            Yp = Y.copy(); Yp[i, c] += h
            Ym = Y.copy(); Ym[i, c] -= h
            fd = (objective(oracle_mod, Yp, S, alpha) - objective(oracle_mod, Ym, S, alpha)) / (2 * h)
            assert abs(fd - g[i, c]) <= 1e-6 * max(1.0, np.abs(g).max()), (i, c, fd, g[i, c])


@pytest.mark.parametrize("alpha", [1.0, 12.0])
def test_matches_sklearn_exact_kl_and_gradient(oracle_mod, alpha):
    S, Y = make_problem(oracle_mod, 150, 45, 15.0, 4, y_std=3.0)
    g, Z, kl = oracle_mod.kl_grad(Y, S, alpha)
    D = S.dense()
    n = Y.shape[0]
    kl_sk, g_sk = skl_tsne._kl_divergence(Y.ravel().copy(), squareform(alpha * D, checks=False), 1, n, 2)
    np.testing.assert_allclose(g, g_sk.reshape(n, 2), rtol=1e-10, atol=1e-13 * np.abs(g).max())
    if alpha == 1.0:
        np.testing.assert_allclose(kl, kl_sk, rtol=1e-10)


def test_kl_is_relative_entropy(oracle_mod):
    S, Y = make_problem(oracle_mod, 100, 30, 10.0, 5)
    _, Z, kl = oracle_mod.kl_grad(Y, S, 1.0)
    D = S.dense()
    diff = Y[:, None, :] - Y[None, :, :]
    W = 1.0 / (1.0 + (diff ** 2).sum(-1))
    np.fill_diagonal(W, 0.0)
    Q = W / W.sum()
    assert abs(Z - W.sum()) <= 1e-12 * Z
    ref = scipy.special.rel_entr(D, Q).sum()
    assert abs(kl - ref) <= 1e-12 * max(1.0, abs(ref))
    assert kl > 0


def test_gradient_sums_to_zero(oracle_mod):
    S, Y = make_problem(oracle_mod, 300, 30, 10.0, 6, y_std=5.0)
    for alpha in (1.0, 12.0):
        g, _, _ = oracle_mod.kl_grad(Y, S, alpha)
        assert np.abs(g.sum(0)).max() <= 1e-12 * np.abs(g).sum()


def test_two_points(oracle_mod):
    # n = 2 with p_12 = p_21 = 1/2: Q = P for any Y, so KL = 0 and g = 0.
    S = oracle_mod.CSR(np.array([0, 1, 2]), np.array([1, 0]), np.array([0.5, 0.5]))
    Y = np.array([[0.3, -1.2], [2.0, 0.7]])
    g, Z, kl = oracle_mod.kl_grad(Y, S, 1.0)
    assert abs(kl) < 1e-15
    assert np.abs(g).max() < 1e-15


def test_p_equal_q_is_stationary(oracle_mod):
    # P := Q(Y) on the dense pattern: KL = 0 and the gradient vanishes,
    # which fixes the relative sign and scale of attraction and repulsion.
    n = 60
    Y = synth.random_embedding(n, 2.0, 9).astype(np.float64)
    diff = Y[:, None, :] - Y[None, :, :]
    W = 1.0 / (1.0 + (diff ** 2).sum(-1))
    np.fill_diagonal(W, 0.0)
    Q = W / W.sum()
    r, c = np.nonzero(~np.eye(n, dtype=bool))
    S = oracle_mod.CSR(np.arange(0, n * (n - 1) + 1, n - 1), c, Q[r, c])
    g, Z, kl = oracle_mod.kl_grad(Y, S, 1.0)
    assert abs(kl) < 1e-13
    assert np.abs(g).max() < 1e-14


def test_rotation_and_translation(oracle_mod):
    S, Y = make_problem(oracle_mod, 200, 30, 10.0, 8, y_std=4.0)
    g, Z, kl = oracle_mod.kl_grad(Y, S, 12.0)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    g2, Z2, kl2 = oracle_mod.kl_grad(Y @ R.T + np.array([3.0, -8.0]), S, 12.0)
    np.testing.assert_allclose(g2, g @ R.T, rtol=1e-10, atol=1e-12 * np.abs(g).max())
    assert abs(Z2 - Z) <= 1e-11 * Z
    assert abs(kl2 - kl) <= 1e-10


def test_row_parts_compose_gradient(oracle_mod):
    S, Y = make_problem(oracle_mod, 250, 30, 10.0, 10, y_std=3.0)
    g, Z, _ = oracle_mod.kl_grad(Y, S, 12.0)
    rows = np.arange(250)
    Zr, Rr, Ar = oracle_mod.grad_rows(Y, rows, S)
    assert abs(Zr.sum() - Z) <= 1e-13 * Z
    np.testing.assert_allclose(4 * (12.0 * Ar - Rr / Z), g, rtol=1e-9, atol=1e-12 * np.abs(g).max())


def test_row_term_magnitudes(oracle_mod):
    # The per-row term magnitudes bound the parts they belong to, with
    # equality where every term has one sign: for the point with the smallest
    # x every y_i,x - y_j,x is <= 0, for the one with the largest y every
    # y_i,y - y_j,y >= 0.  A brute-force NumPy evaluation pins the rest.
    S, Y = make_problem(oracle_mod, 200, 20, 6.0, 5)
    n = Y.shape[0]
    rows = np.arange(n)
    _, R, A = oracle_mod.grad_rows(Y, rows, S)
    Ra, Aa = oracle_mod.grad_rows_scale(Y, rows, S)
    assert np.all(np.abs(R) <= Ra * (1 + 1e-12)) and np.all(np.abs(A) <= Aa * (1 + 1e-12))
    i0, i1 = int(np.argmin(Y[:, 0])), int(np.argmax(Y[:, 1]))
    assert abs(-R[i0, 0] - Ra[i0, 0]) <= 1e-12 * Ra[i0, 0]
    assert abs(-A[i0, 0] - Aa[i0, 0]) <= 1e-12 * Aa[i0, 0]
    assert abs(R[i1, 1] - Ra[i1, 1]) <= 1e-12 * Ra[i1, 1]
    D = Y[:, None, :] - Y[None, :, :]
    W = 1.0 / (1.0 + (D ** 2).sum(-1))
    np.fill_diagonal(W, 0.0)
    np.testing.assert_allclose(Ra, ((W ** 2)[:, :, None] * np.abs(D)).sum(1), rtol=1e-12)
    Pd = S.dense()
    np.testing.assert_allclose(Aa, ((Pd * W)[:, :, None] * np.abs(D)).sum(1), rtol=1e-12)
