"""GPU parity: tsne_pca (randomized truncated SVD on the FP32 matrix cores)
against the FP64 oracle of the same method (oracle/pca.py) on the same X and
the same test matrix Omega: singular values, the mean, the leading
components and scores; orthonormal components and scores = Xc V^T at any
size; bitwise reproducible."""
import numpy as np
import pytest
import torch

from helpers import say, to_dev
from oracle import pca as opca
from paper_2605_13928_amd import api, synth

pytestmark = pytest.mark.gpu


def run(dev, X, k, Om, q):
    sc, comp, sv, mu = api.pca(to_dev(X, dev), k, to_dev(Om, dev), q)
    return sc.cpu().numpy().astype(np.float64), comp.cpu().numpy().astype(np.float64), sv.cpu().numpy(), \
        mu.cpu().numpy().astype(np.float64)


# (n, g, k, q, latent scale range); ragged n and g against the 128-row and
# 32 / 64-column tiles
CASES = [
    (5000, 300, 50, 2, (100.0, 1.0)),
    (4099, 129, 10, 0, (50.0, 5.0)),
    (1000, 64, 64, 1, (20.0, 2.0)),
    (20011, 517, 32, 2, (100.0, 0.5)),
]


@pytest.mark.parametrize("case", CASES)
def test_pca_matches_oracle(dev, case):
    n, g, k, q, (top, bottom) = case
    say("pca vs oracle", case)
    X = synth.make_expression(n, g, 7 + n, latent=min(64, g), top=top, bottom=bottom)
    Om = synth.make_omega(g, 11 + g)
    sc, comp, sv, mu = run(dev, X, k, Om, q)
    osc, ocomp, osv, omu = opca.randomized_pca(X.astype(np.float64), k, Om.astype(np.float64), q)
    np.testing.assert_allclose(mu, omu, rtol=1e-5, atol=1e-5)
    # singular values: well conditioned, to FP32 accuracy relative to the largest
    assert np.abs(sv - osv).max() <= 2e-5 * osv[0], (sv[:4], osv[:4])
    # components and scores: FP32 rounding in the products is ~3e-6 s_1, so a
    # component's angle error is ~3e-6 s_1 / (gap s_c); checked where the
    # relative gap to both neighbours is >= 2 % and s_c >= 0.05 s_1
    gap = np.minimum(np.abs(np.diff(np.r_[np.inf, osv])), np.abs(np.diff(np.r_[osv, 0.0]))) / osv
    good = np.where((gap[:k] > 0.02) & (osv[:k] >= 0.05 * osv[0]))[0]
    assert good.size >= min(k, 4)
    dots = np.sum(comp[good] * ocomp[good], axis=1)
    assert np.all(dots > 1 - 1e-4), dots.min()
    col_err = np.linalg.norm(sc[:, good] - osc[:, good], axis=0) / np.linalg.norm(osc[:, good], axis=0)
    assert col_err.max() <= 1e-2 and col_err[0] <= 1e-4, col_err
    # properties at any size
    np.testing.assert_allclose(comp @ comp.T, np.eye(k), atol=2e-5)
    # scores = Xc V^T holds as far as Q spans the range of Xc: the GPU's
    # deviation from it matches the oracle's
    Xd = X.astype(np.float64)
    proj = (Xd - mu) @ comp.T
    oproj = (Xd - omu) @ ocomp.T
    dg = np.linalg.norm(sc - proj) / np.linalg.norm(proj)
    do = np.linalg.norm(osc - oproj) / np.linalg.norm(oproj)
    assert dg <= do + 1e-4, (dg, do)
    for c in range(k):
        assert comp[c, np.argmax(np.abs(comp[c]))] > 0


def test_pca_deterministic(dev):
    say("pca determinism")
    X = to_dev(synth.make_expression(30000, 700, 3), dev)
    Om = to_dev(synth.make_omega(700, 4), dev)
    a = api.pca(X, 50, Om, 2)
    b = api.pca(X, 50, Om, 2)
    assert all(torch.equal(x, y) for x, y in zip(a, b))


def test_pca_cells_full_size(dev):
    # 200,000 cells x 2,000 genes (the c3 cell count): full parity with the
    # oracle on the singular values and leading components
    say("pca 200k x 2000")
    n, g, k = 200_000, 2000, 50
    X = synth.make_expression(n, g, 2024)
    Om = synth.make_omega(g, 2025)
    sc, comp, sv, mu = run(dev, X, k, Om, 2)
    osc, ocomp, osv, omu = opca.randomized_pca(X.astype(np.float64), k, Om.astype(np.float64), 2)
    assert np.abs(sv - osv).max() <= 2e-5 * osv[0]
    dots = np.sum(comp[:20] * ocomp[:20], axis=1)
    assert np.all(dots > 1 - 1e-6), dots.min()
    rows = np.random.default_rng(1).choice(n, 2000, replace=False)
    e = np.linalg.norm(sc[rows, :20] - osc[rows, :20]) / np.linalg.norm(osc[rows, :20])
    assert e <= 1e-4, e


def test_pca_rank_deficient(dev):
    # X of rank 5 (plus the offset): the 64-column subspace is rank 5, its
    # Gram matrix singular -- the shifted first CholeskyQR pass must carry
    # it; the 5 nonzero singular values and their components match the
    # oracle, the rest are ~0, and everything stays finite and orthonormal
    say("pca rank 5")
    n, g, k = 3000, 200, 10
    X = synth.make_expression(n, g, 41, latent=5, top=50.0, bottom=5.0, noise=0.0)
    Om = synth.make_omega(g, 42)
    sc, comp, sv, mu = run(dev, X, k, Om, 2)
    osc, ocomp, osv, omu = opca.randomized_pca(X.astype(np.float64), k, Om.astype(np.float64), 2)
    assert np.isfinite(sc).all() and np.isfinite(comp).all() and np.isfinite(sv).all()
    np.testing.assert_allclose(sv[:5], osv[:5], rtol=1e-4)
    assert np.all(sv[5:] <= 1e-3 * sv[0]), sv
    dots = np.abs(np.sum(comp[:5] * ocomp[:5], axis=1))
    assert np.all(dots > 1 - 1e-4), dots
    np.testing.assert_allclose(comp @ comp.T, np.eye(k), atol=1e-3)
