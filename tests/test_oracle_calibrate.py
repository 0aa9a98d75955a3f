"""Pins of the oracle's perplexity calibration.

Definition followed (van der Maaten & Hinton 2008, eq. 1 and eq. 3):
p_{j|i} proportional to exp(-beta_i d_ij) over the k neighbours, with beta_i
chosen so that the Shannon entropy of p_{.|i} is ln(perplexity) nats.
"""
import numpy as np
import pytest
import scipy.optimize
import scipy.stats
from sklearn.manifold import _utils as skl_utils

from paper_2605_13928_amd import synth


@pytest.fixture(scope="module")
def c1_knn(oracle_mod):
    X, _ = synth.make_points("c1")
    return oracle_mod.knn(X, 90)


def test_entropy_hits_target(oracle_mod, c1_knn):
    _, d2 = c1_knn
    P, beta, conv, H = oracle_mod.calibrate(d2, 30.0, tol=1e-5)
    assert conv.all()
    # entropy of the returned distribution, by an independent routine
    Hout = scipy.stats.entropy(P, axis=1)
    assert np.abs(Hout - np.log(30.0)).max() <= 1e-5
    np.testing.assert_allclose(P.sum(1), 1.0, rtol=0, atol=1e-14)
    # the tight setting used elsewhere as the reference
    P2, _, conv2, _ = oracle_mod.calibrate(d2, 30.0)
    assert conv2.all()
    assert np.abs(scipy.stats.entropy(P2, axis=1) - np.log(30.0)).max() <= 1e-11


def test_gaussian_kernel_on_squared_distances(oracle_mod, c1_knn):
    _, d2 = c1_knn
    P, beta, _, _ = oracle_mod.calibrate(d2, 30.0)
    # ln p_j - ln p_0 = -beta (d_j - d_0): the kernel is exp of minus beta
    # times the squared distance, nothing else.
    lhs = np.log(P) - np.log(P[:, :1])
    rhs = -beta[:, None] * (d2 - d2[:, :1])
    np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("m,k,delta,perp", [(1, 90, 3.0, 30.0), (5, 30, 0.25, 10.0), (40, 90, 7.0, 60.0)])
def test_two_level_closed_form(oracle_mod, m, k, delta, perp):
    # m neighbours at distance 0 and k - m at distance delta: the entropy is
    # H(b) = ln(m + r) + b delta r / (m + r), r = (k - m) exp(-b delta).
    def H(b):
        r = (k - m) * np.exp(-b * delta)
        return np.log(m + r) + b * delta * r / (m + r)

    b_ref = scipy.optimize.brentq(lambda b: H(b) - np.log(perp), 1e-12, 1e4 / delta, xtol=1e-15, rtol=1e-15)
    row = np.array([[0.0] * m + [delta] * (k - m)])
    P, beta, conv, _ = oracle_mod.calibrate(row, perp)
    assert conv[0] == 1
    np.testing.assert_allclose(beta[0], b_ref, rtol=1e-9)


def test_matches_sklearn_binary_search(oracle_mod, c1_knn):
    # scikit-learn's perplexity search is an independent implementation of
    # the same definition (its own entropy tolerance is 1e-5).
    _, d2 = c1_knn
    P, _, _, _ = oracle_mod.calibrate(d2, 30.0)
    Psk = skl_utils._binary_search_perplexity(d2.astype(np.float32), 30.0, 0)
    np.testing.assert_allclose(P, Psk, rtol=0, atol=2e-4)


def test_beta_monotone_in_perplexity(oracle_mod, c1_knn):
    _, d2 = c1_knn
    betas = [oracle_mod.calibrate(d2, p)[1] for p in (10.0, 20.0, 30.0, 45.0)]
    for a, b in zip(betas, betas[1:]):
        assert (b < a).all()  # wider kernel for higher perplexity


def test_shift_invariance(oracle_mod, c1_knn):
    # Adding a constant to all distances of a row changes nothing.
    _, d2 = c1_knn
    P0, b0, _, _ = oracle_mod.calibrate(d2[:50], 30.0)
    P1, b1, _, _ = oracle_mod.calibrate(d2[:50] + 17.0, 30.0)
    np.testing.assert_allclose(P1, P0, rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(b1, b0)


def test_degenerate_row_reports_unconverged(oracle_mod):
    # All k distances equal: entropy is ln k for every beta, the target
    # ln 30 < ln 90 is unreachable; P is the uniform limit.
    rows = np.full((2, 90), 5.0)
    P, beta, conv, H = oracle_mod.calibrate(rows, 30.0)
    assert (conv == 0).all()
    np.testing.assert_allclose(P, 1.0 / 90, rtol=1e-14)
    np.testing.assert_allclose(H, np.log(90.0), rtol=1e-14)
