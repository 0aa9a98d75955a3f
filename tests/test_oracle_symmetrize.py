"""Pins of the oracle's symmetrisation P = (C + C^T) / (2n).

Definition followed: symmetric joint probabilities (van der Maaten &
Hinton 2008, Sec. 3.1) on the union of the kNN patterns (van der Maaten
2014, Sec. 4.1).
"""
import numpy as np
import pytest
import scipy.sparse
from sklearn.manifold import _t_sne as skl_tsne

from paper_2605_13928_amd import synth


def dense_reference(idx, Pc):
    n, k = idx.shape
    Cd = np.zeros((n, n))
    Cd[np.repeat(np.arange(n), k), idx.ravel()] = Pc.ravel()
    return (Cd + Cd.T) / (2.0 * n)


@pytest.mark.parametrize("n,k,seed", [(30, 5, 1), (200, 20, 2), (64, 63, 3)])
def test_matches_dense_definition(oracle_mod, n, k, seed):
    idx, d2 = synth.random_knn_graph(n, k, seed)
    rng = np.random.default_rng(seed)
    Pc = rng.random((n, k))
    Pc /= Pc.sum(1, keepdims=True)
    S = oracle_mod.symmetrize(idx, Pc)
    D = dense_reference(idx, Pc)
    np.testing.assert_allclose(S.dense(), D, rtol=1e-15, atol=0)
    # pattern is exactly the union of both directions
    assert S.nnz == np.count_nonzero(D)
    assert n * k <= S.nnz <= 2 * n * k


def test_structure_and_tpos(oracle_mod):
    idx, d2 = synth.random_knn_graph(500, 30, 7)
    Pc, _, _, _ = oracle_mod.calibrate(d2, 10.0)
    S = oracle_mod.symmetrize(idx, Pc)
    rows = S.rows()
    assert np.all(S.col != rows)  # no diagonal
    for i in range(S.n):
        c = S.col[S.row_ptr[i]:S.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)  # strictly ascending columns
    # tpos points at the transposed entry, with the same value
    assert np.all(S.col[S.tpos] == rows)
    assert np.all(rows[S.tpos] == S.col)
    np.testing.assert_array_equal(S.val[S.tpos], S.val)  # bitwise symmetric
    assert abs(S.val.sum() - 1.0) < 1e-13


def test_matches_sklearn_joint_probabilities(oracle_mod):
    # scikit-learn's sparse joint probabilities: calibrate on the kNN
    # distances, add the transpose, normalise by the sum (= 2n here).
    X, _ = synth.make_points("c1", n=400)
    idx, d2 = oracle_mod.knn(X, 30)
    Pc, _, _, _ = oracle_mod.calibrate(d2, 10.0)
    S = oracle_mod.symmetrize(idx, Pc)
    n = X.shape[0]
    dist = scipy.sparse.csr_matrix((d2.ravel().astype(np.float32), idx.ravel(), np.arange(0, n * 30 + 1, 30)),
                                   shape=(n, n))
    Psk = skl_tsne._joint_probabilities_nn(dist, 10.0, 0).toarray()
    np.testing.assert_allclose(S.dense(), Psk, rtol=0, atol=3e-6 / n)


def test_rejects_self_and_repeats(oracle_mod):
    idx, _ = synth.random_knn_graph(20, 4, 1)
    Pc = np.full((20, 4), 0.25)
    bad = idx.copy()
    bad[3, 1] = 3
    with pytest.raises(ValueError):
        oracle_mod.symmetrize(bad, Pc)
    bad = idx.copy()
    bad[4, 2] = bad[4, 0]
    with pytest.raises(ValueError):
        oracle_mod.symmetrize(bad, Pc)
