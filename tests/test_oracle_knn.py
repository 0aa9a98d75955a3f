"""Pins of the oracle's exact kNN against brute force and invariants.

Definition followed: squared Euclidean distance, k smallest (d, j) keys with
j != i, ascending (the sparse kNN input of tree-accelerated t-SNE,
van der Maaten 2014, Sec. 4.1).
"""
import numpy as np
import pytest
import torch

from paper_2605_13928_amd import synth


def brute_knn(X, k):
    X = X.astype(np.float64)
    n = X.shape[0]
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    idx = np.empty((n, k), np.int64)
    dd = np.empty((n, k))
    js = np.arange(n)
    for i in range(n):
        m = js != i
        order = np.lexsort((js[m], D[i, m]))[:k]  # primary key d, then index
        idx[i] = js[m][order]
        dd[i] = D[i, m][order]
    return idx, dd


@pytest.mark.parametrize("n,d,k", [(40, 3, 5), (257, 50, 30), (300, 7, 90)])
def test_knn_matches_brute_force(oracle_mod, n, d, k):
    rng = np.random.default_rng(n + d + k)
    X = rng.standard_normal((n, d)).astype(np.float32)
    idx, d2 = oracle_mod.knn(X, k)
    bi, bd = brute_knn(X, k)
    np.testing.assert_array_equal(idx, bi)
    np.testing.assert_allclose(d2, bd, rtol=1e-12, atol=0)


def test_knn_ties_broken_by_index(oracle_mod):
    # Exact duplicates: distance 0 ties between copies, equal distances to any
    # third point; the order must be by (d, j).
    rng = np.random.default_rng(5)
    base = rng.standard_normal((20, 4)).astype(np.float32)
    X = np.concatenate([base, base, base[:7]], axis=0)
    idx, d2 = oracle_mod.knn(X, 10)
    bi, bd = brute_knn(X, 10)
    np.testing.assert_array_equal(idx, bi)
    np.testing.assert_array_equal(d2, bd)
    # row 0 has copies 20 at distance exactly 0 and 40 too
    assert idx[0, 0] == 20 and idx[0, 1] == 40 and d2[0, 0] == 0.0 and d2[0, 1] == 0.0


def test_knn_permutation_equivariance(oracle_mod):
    rng = np.random.default_rng(11)
    X = rng.standard_normal((200, 10)).astype(np.float32)
    perm = rng.permutation(200)
    inv = np.argsort(perm)
    i0, d0 = oracle_mod.knn(X, 15)
    i1, d1 = oracle_mod.knn(X[perm], 15)
    # row r of the permuted problem is original row perm[r]; its neighbour t is original perm[t]
    np.testing.assert_array_equal(perm[i1], i0[perm])
    np.testing.assert_array_equal(d1, d0[perm])
    assert inv.shape == perm.shape


def test_knn_scaling_by_two_is_exact(oracle_mod):
    X, _ = synth.make_points("c1", n=300)
    i0, d0 = oracle_mod.knn(X, 20)
    i1, d1 = oracle_mod.knn(X * np.float32(2), 20)
    np.testing.assert_array_equal(i0, i1)
    np.testing.assert_array_equal(d1, 4.0 * d0)


def test_knn_row_subset(oracle_mod):
    X, _ = synth.make_points("c1", n=500)
    rows = np.array([0, 499, 17, 17, 250])
    i0, d0 = oracle_mod.knn(X, 30)
    i1, d1 = oracle_mod.knn(X, 30, rows=rows)
    np.testing.assert_array_equal(i1, i0[rows])
    np.testing.assert_array_equal(d1, d0[rows])


def test_knn_bf16_points_match_torch_rounding(oracle_mod):
    # The bf16 variant must equal exact kNN on points rounded by an
    # independent RNE implementation (torch's float32 -> bfloat16 cast).
    X, _ = synth.make_points("c3", n=300)
    Xr = torch.from_numpy(X).to(torch.bfloat16).to(torch.float32).numpy()
    i0, d0 = oracle_mod.knn(X, 25, bf16_points=True)
    bi, bd = brute_knn(Xr, 25)
    np.testing.assert_array_equal(i0, bi)
    np.testing.assert_allclose(d0, bd, rtol=1e-12)


def test_pair_d2(oracle_mod):
    X, _ = synth.make_points("c1", n=100)
    qi = np.array([0, 5, 99])
    cj = np.array([1, 5, 0])
    out = oracle_mod.pair_d2(X, qi, cj)
    ref = ((X[qi].astype(np.float64) - X[cj].astype(np.float64)) ** 2).sum(1)
    np.testing.assert_allclose(out, ref, rtol=1e-13)
    assert out[1] == 0.0


def test_knn_rejects_bad_arguments(oracle_mod):
    X = np.zeros((10, 3), np.float32)
    with pytest.raises(ValueError):
        oracle_mod.knn(X, 10)  # k >= n
