"""GPU parity: tsne_symmetrize against the FP64 oracle (structure bit-exact)."""
import numpy as np
import pytest
import torch

import oracle
from helpers import oracle_problem, random_graph_P, say, to_dev
from paper_2605_13928_amd import api, synth

pytestmark = pytest.mark.gpu


def run_both(dev, idx, Pc):
    Pc32 = Pc.astype(np.float32)
    S = oracle.symmetrize(idx, Pc32.astype(np.float64))
    G = api.symmetrize(to_dev(idx, dev), to_dev(Pc32, dev))
    return S, G


def check(S, G, n):
    np.testing.assert_array_equal(G.row_ptr.cpu().numpy(), S.row_ptr)
    np.testing.assert_array_equal(G.col.cpu().numpy(), S.col)
    np.testing.assert_array_equal(G.tpos.cpu().numpy(), S.tpos)
    v = G.val.cpu().numpy()
    np.testing.assert_allclose(v, S.val, rtol=2e-7, atol=0)
    np.testing.assert_array_equal(v[G.tpos.cpu().numpy()], v)  # bitwise symmetric
    assert abs(v.astype(np.float64).sum() - S.val.sum()) <= 1e-6
    return v


def test_symmetrize_c1_knn_graph(dev):
    say("symmetrize c1")
    X, labels, idx, d2, Pc, S0 = oracle_problem("c1", 1500, 90, 30.0)
    S, G = run_both(dev, idx, Pc)
    v = check(S, G, 1500)
    assert abs(v.astype(np.float64).sum() - 1.0) <= 1e-5


@pytest.mark.parametrize("n,k,seed", [(2, 1, 1), (65, 64, 2), (777, 30, 3), (5003, 7, 4), (20_000, 90, 5)])
def test_symmetrize_random_graphs(dev, n, k, seed):
    say("symmetrize", n, k)
    idx, d2, Pc, _ = random_graph_P(n, k, min(10.0, k - 0.5), seed)
    S, G = run_both(dev, idx, Pc)
    check(S, G, n)


@pytest.mark.parametrize("n,k,hubs", [(3000, 20, {5: 300, 7: 900, 11: 2999}), (9000, 3, {0: 8999, 1: 5000})])
def test_symmetrize_hub_rows(dev, n, k, hubs):
    # hubs with in-lists of ~300, ~900, ~3000, ~5000 and ~9000 entries: long
    # runs of one target in the radix sort of the transposed lists, spanning
    # many of its 2048-item blocks
    say("symmetrize hubs", n, k)
    rng = np.random.default_rng(9)
    idx = np.empty((n, k), np.int32)
    for i in range(n):
        row = [h for h, deg in hubs.items() if h != i and (deg == n - 1 or rng.random() < deg / n)][:k]
        while len(row) < k:
            j = int(rng.integers(n))
            if j != i and j not in hubs and j not in row:
                row.append(j)
        idx[i] = row
    Pc = rng.random((n, k))
    Pc /= Pc.sum(1, keepdims=True)
    S, G = run_both(dev, idx, Pc)
    check(S, G, n)
    deg = np.diff(S.row_ptr)
    for h, d in hubs.items():
        if d == n - 1:
            assert deg[h] >= n - 1
        else:
            assert 0.7 * d < deg[h] < 1.3 * d


def test_symmetrize_rejects_invalid_lists(dev):
    say("symmetrize invalid")
    idx, _ = synth.random_knn_graph(100, 5, 1)
    Pc = np.full((100, 5), 0.2, np.float32)
    bad = idx.copy()
    bad[10, 2] = 10  # self
    with pytest.raises(ValueError):
        api.symmetrize(to_dev(bad, dev), to_dev(Pc, dev))
    bad = idx.copy()
    bad[11, 3] = bad[11, 0]  # repeat
    with pytest.raises(ValueError):
        api.symmetrize(to_dev(bad, dev), to_dev(Pc, dev))
    bad = idx.copy()
    bad[12, 1] = 100  # out of range
    with pytest.raises(ValueError):
        api.symmetrize(to_dev(bad, dev), to_dev(Pc, dev))
