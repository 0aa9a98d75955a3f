"""Pins of the randomized-PCA oracle (oracle/pca.py) against what linear
algebra fixes: on a matrix of rank <= l the method is exact (its singular
values and components are those of the full SVD of the centred matrix,
numpy.linalg.svd); with a spectral gap and power iterations the leading
singular values converge to the full SVD's; components are orthonormal and
the scores are the centred data projected on them; the mean is the column
mean; the sign convention holds; on a full-rank matrix the estimates
interlace below the true singular values and the rank-k reconstruction
error is at least the (k+1)-th singular value (Eckart-Young)."""
import numpy as np
import pytest

from oracle import pca


def low_rank(n, g, r, seed, noise=0.0):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n, r))
    S = np.geomspace(100.0, 5.0, r)
    V = np.linalg.qr(rng.standard_normal((g, r)))[0]
    X = (U * S) @ V.T + 3.0 + noise * rng.standard_normal((n, g))
    return X


def full_svd(X):
    Xc = X - X.mean(0)
    U, s, Vt = np.linalg.svd(Xc, full_matrices=False)
    return s, Vt


@pytest.mark.parametrize("q", [0, 2])
def test_exact_on_low_rank(q):
    X = low_rank(400, 60, 8, 1)
    Om = np.random.default_rng(2).standard_normal((60, 16))
    sc, comp, s, mu = pca.randomized_pca(X, 8, Om, q=q)
    s_ref, Vt = full_svd(X)
    np.testing.assert_allclose(s, s_ref[:8], rtol=1e-10)
    # components equal up to sign
    np.testing.assert_allclose(np.abs(np.sum(comp * Vt[:8], axis=1)), 1.0, atol=1e-10)
    np.testing.assert_allclose(mu, X.mean(0), rtol=1e-12)


def test_power_iterations_converge_with_gap():
    X = low_rank(500, 80, 10, 3, noise=0.05)
    Om = np.random.default_rng(4).standard_normal((80, 20))
    s_ref, _ = full_svd(X)
    errs = []
    for q in (0, 1, 2):
        _, _, s, _ = pca.randomized_pca(X, 10, Om, q=q)
        errs.append(np.abs(s / s_ref[:10] - 1).max())
    assert errs[2] < 1e-6 and errs[2] <= errs[0], errs


def test_orthonormal_projection_and_signs():
    X = low_rank(300, 50, 12, 5, noise=0.1)
    Om = np.random.default_rng(6).standard_normal((50, 20))
    sc, comp, s, mu = pca.randomized_pca(X, 12, Om, q=2)
    np.testing.assert_allclose(comp @ comp.T, np.eye(12), atol=1e-12)
    np.testing.assert_allclose(sc, (X - mu) @ comp.T, rtol=0, atol=1e-8 * np.abs(sc).max())
    assert np.all(np.diff(s) <= 0)
    for c in range(12):
        assert comp[c, np.argmax(np.abs(comp[c]))] > 0


def test_orth_is_unique_qr_factor():
    Y = np.random.default_rng(7).standard_normal((50, 6))
    Q = pca.orth(Y)
    np.testing.assert_allclose(Q.T @ Q, np.eye(6), atol=1e-13)
    R = Q.T @ Y
    assert np.all(np.diag(R) > 0) and np.abs(np.tril(R, -1)).max() < 1e-12


@pytest.mark.parametrize("q", [0, 1, 2])
def test_singular_values_interlace_and_eckart_young(q):
    # On a full-rank noisy matrix, for any q: the estimates are the singular
    # values of Q^T Xc with Q orthonormal, so s_i(estimate) <= s_i(Xc)
    # (interlacing), and no rank-k reconstruction beats the truncated SVD
    # (Eckart-Young): ||Xc - scores components||_2 >= s_{k+1}(Xc).
    X = low_rank(300, 80, 40, 11, noise=2.0)
    k, l = 10, 16
    Om = np.random.default_rng(3).standard_normal((80, l))
    sc, comp, sv, mu = pca.randomized_pca(X, k, Om, q=q)
    s, _ = full_svd(X)
    assert np.all(sv <= s[:k] * (1 + 1e-12))
    err = np.linalg.norm((X - mu) - sc @ comp, 2)
    assert err >= s[k] * (1 - 1e-12)
