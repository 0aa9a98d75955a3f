"""GPU parity: the UMAP entry points against the FP64 oracle of the same
steps (oracle/umap.py) on the same seeded inputs -- smoothed kNN weights,
the fuzzy union (structure bit-exact), and layout epochs (same sampled
entries and negative draws on both sides, so the embeddings agree to FP32
arithmetic); determinism; a whole GPU run separates a mixture; the union
and an epoch at 10^6 points."""
import numpy as np
import pytest
import torch

import oracle
from helpers import say, to_dev
from oracle import umap as U
from paper_2605_13928_amd import api, synth

pytestmark = pytest.mark.gpu


def oracle_graph(X, k):
    """kNN (oracle), weights and union (oracle) of the points X: the inputs
    the GPU steps get, with their oracle results."""
    idx, d2 = oracle.knn(X, k)
    d2f = d2.astype(np.float32)
    rho, sigma, w = U.smooth_knn(np.sqrt(d2f.astype(np.float64)))
    return idx, d2f, rho, sigma, w


def union_inputs(idx, w):
    wf = w.astype(np.float32)
    rp, col, val = U.fuzzy_union(idx, wf.astype(np.float64), idx.shape[0])
    return wf, rp, col, val


def gpu_union(dev, idx, wf):
    return api.umap_fuzzy_union(to_dev(idx, dev), to_dev(wf, dev))


def mixture(n, d, seed, dup=0):
    X, _ = synth.make_points("c1", n=n, seed=seed)
    X = X[:, :d].copy()
    if dup:  # dup + 1 copies of one point: rows whose k distances are all 0
        X[1:dup + 1] = X[0]
        X[dup + 1:dup + 4] = X[dup + 5]  # a few exact duplicates elsewhere
    return np.ascontiguousarray(X, np.float32)


@pytest.mark.parametrize("n,d,k,dup", [(3001, 50, 15, 20), (1500, 20, 90, 0), (700, 10, 1, 0), (2048, 50, 64, 3)])
def test_umap_weights_match_oracle(dev, n, d, k, dup):
    say("umap weights", n, d, k, dup)
    X = mixture(n, d, 31 + n, dup)
    idx, d2f, rho, sigma, w = oracle_graph(X, k)
    g_rho, g_sigma, g_w = (t.cpu().numpy().astype(np.float64) for t in api.umap_weights(to_dev(d2f, dev)))
    np.testing.assert_allclose(g_rho, rho, rtol=6e-8, atol=0)
    np.testing.assert_allclose(g_sigma, sigma, rtol=2e-7, atol=0)
    np.testing.assert_allclose(g_w, w, rtol=2e-7, atol=1e-30)
    if dup >= k:  # rows whose k neighbours all coincide with them
        assert np.all(g_w[:dup + 1] == 1.0) and np.all(g_sigma[:dup + 1] == np.float32(1e-3))


@pytest.mark.parametrize("n,k,seed", [(3001, 15, 1), (2000, 90, 2), (513, 1, 3)])
def test_umap_union_matches_oracle(dev, n, k, seed):
    say("umap union", n, k, seed)
    idx, _ = synth.random_knn_graph(n, k, seed)
    w = np.random.default_rng(seed).random((n, k))
    wf, rp, col, val = union_inputs(idx, w)
    G = gpu_union(dev, idx, wf)
    np.testing.assert_array_equal(G.row_ptr.cpu().numpy(), rp)
    np.testing.assert_array_equal(G.col.cpu().numpy(), col)
    gv = G.val.cpu().numpy()
    np.testing.assert_allclose(gv.astype(np.float64), val, rtol=1.2e-7, atol=0)
    B = U.to_scipy(rp, col, gv, n)
    assert (B != B.T).nnz == 0  # the same FP32 value in rows i and j


def layout_case(dev, n, k, seed):
    X = mixture(n, 20, seed)
    idx, d2f, rho, sigma, w = oracle_graph(X, k)
    wf, rp, col, val = union_inputs(idx, w)
    valf = val.astype(np.float32)
    G = api.SparseP(to_dev(rp, dev), to_dev(col, dev), to_dev(valf, dev), None, n)
    return G, rp, col, valf


def step_tol(Y0, Yo):
    return 2e-6 * np.abs(Yo).max() + 2e-5 * np.abs(Yo - Y0).max()


# Several epochs are compared where the learning rate is moderate: at
# alpha ~ 1 close repulsive encounters (coefficient ~ 1 / (eps + d^2))
# amplify the FP32-vs-FP64 differences of one epoch in the next, so from
# epoch 0 the range split is checked over two epochs only.
@pytest.mark.parametrize("t0,t1,neg", [(0, 1, 5), (0, 2, 5), (100, 101, 5), (40, 43, 0), (150, 155, 5),
                                       (198, 200, 12)])
def test_umap_epochs_match_oracle(dev, t0, t1, neg):
    say("umap epochs", t0, t1, neg)
    n, k, n_epochs = 2500, 15, 200
    G, rp, col, valf = layout_case(dev, n, k, 5)
    a, b = U.fit_ab(0.5)
    Y0 = synth.umap_init(n, 77)
    Yg = to_dev(Y0, dev)
    mid = (t0 + t1) // 2
    api.umap_layout(Yg, G, a, b, n_epochs, 1.0, neg, seed=123, epochs=(t0, mid))   # two calls: the epoch
    api.umap_layout(Yg, G, a, b, n_epochs, 1.0, neg, seed=123, epochs=(mid, t1))   # range splits cleanly
    Yo = U.layout(Y0.astype(np.float64), rp, col, valf, n_epochs, a, b, 1.0, neg, 123, epochs=(t0, t1))
    e = np.abs(Yg.cpu().numpy() - Yo).max()
    tol = step_tol(Y0, Yo) * (t1 - t0)
    assert e <= tol, (e, tol)
    # the scattering path gives the same bits on this symmetric graph
    Ys = api.umap_layout(to_dev(Y0, dev), G, a, b, n_epochs, 1.0, neg, seed=123, epochs=(t0, t1), symmetric=False)
    assert torch.equal(Ys, Yg)


def test_umap_epochs_directed_graph(dev):
    # a graph that is not symmetric (the directed kNN lists themselves):
    # only the scattering path applies; each entry moves both of its ends
    say("umap epochs, directed graph")
    n, k, n_epochs = 3000, 10, 100
    idx, _ = synth.random_knn_graph(n, k, 13)
    order = np.argsort(idx, axis=1, kind="stable")
    col = np.take_along_axis(idx, order, 1).ravel().astype(np.int32)
    valf = np.take_along_axis(np.random.default_rng(13).random((n, k)).astype(np.float32), order, 1).ravel()
    rp = np.arange(0, n * k + 1, k, dtype=np.int64)
    G = api.SparseP(to_dev(rp, dev), to_dev(col, dev), to_dev(valf, dev), None, n)
    Y0 = synth.umap_init(n, 14)
    a, b = 1.2, 0.95
    Yg = api.umap_layout(to_dev(Y0, dev), G, a, b, n_epochs, 0.5, 5, seed=15, epochs=(30, 32), symmetric=False)
    Yo = U.layout(Y0.astype(np.float64), rp, col, valf, n_epochs, a, b, 0.5, 5, 15, epochs=(30, 32))
    e = np.abs(Yg.cpu().numpy() - Yo).max()
    assert e <= 2 * step_tol(Y0, Yo), (e, step_tol(Y0, Yo))


def test_umap_layout_deterministic(dev):
    say("umap determinism")
    n = 20_000
    idx, _ = synth.random_knn_graph(n, 15, 9)
    w = np.random.default_rng(9).random((n, 15)).astype(np.float32)
    G = gpu_union(dev, idx, w)
    Y0 = to_dev(synth.umap_init(n, 10), dev)
    A, B = Y0.clone(), Y0.clone()
    api.umap_layout(A, G, 1.5, 0.9, 50, epochs=(0, 10))
    api.umap_layout(B, G, 1.5, 0.9, 50, epochs=(0, 10))
    assert torch.equal(A, B) and not torch.equal(A, Y0)


def test_umap_gpu_pipeline_separates_mixture(dev):
    # every step on the GPU: kNN (k = 15), weights, union, 200 epochs
    say("umap pipeline")
    X, lab = synth.make_points("c1")
    n = X.shape[0]
    idx, d2 = api.knn(to_dev(X, dev), 15)
    _, _, w = api.umap_weights(d2)
    G = api.umap_fuzzy_union(idx, w)
    a, b = api.umap_fit_ab(0.5)
    Y = api.umap_layout(to_dev(synth.umap_init(n, 3), dev), G, a, b, 200, seed=4).cpu().numpy().astype(np.float64)
    D = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(D, np.inf)
    nn = np.argsort(D, axis=1)[:, :10]
    purity = (lab[nn] == lab[:, None]).mean()
    say("10-NN label purity", purity)
    assert purity >= 0.95


def test_umap_union_and_epoch_full_size(dev):
    # 10^6 points, k = 15 (the pipeline's neighbour count): the whole union
    # against the oracle's, then one mid-schedule epoch against the oracle's
    say("umap 1M")
    n, k = 1_000_000, 15
    idx, _ = synth.random_knn_graph(n, k, 21)
    w = np.random.default_rng(21).random((n, k))
    wf, rp, col, val = union_inputs(idx, w)
    G = gpu_union(dev, idx, wf)
    np.testing.assert_array_equal(G.row_ptr.cpu().numpy(), rp)
    np.testing.assert_array_equal(G.col.cpu().numpy(), col)
    valf = val.astype(np.float32)
    np.testing.assert_allclose(G.val.cpu().numpy(), valf, rtol=1.2e-7, atol=0)
    G = api.SparseP(G.row_ptr, G.col, to_dev(valf, dev), None, n)
    Y0 = synth.umap_init(n, 22)
    Yg = api.umap_layout(to_dev(Y0, dev), G, 0.583, 1.334, 200, 1.0, 5, seed=5, epochs=(150, 151))
    Yo = U.layout_epoch(Y0.astype(np.float64), rp, col, valf, 150, 200, 0.583, 1.334, 1.0, 5, 5)
    e = np.abs(Yg.cpu().numpy() - Yo).max()
    assert e <= step_tol(Y0, Yo), (e, step_tol(Y0, Yo))
    Ys = api.umap_layout(to_dev(Y0, dev), G, 0.583, 1.334, 200, 1.0, 5, seed=5, epochs=(150, 151), symmetric=False)
    assert torch.equal(Ys, Yg)


def test_umap_gather_epochs_equal_scatter_large(dev):
    # 300,000 points, six epochs: the gather path (each vertex takes its own
    # attractive steps twice) gives the scattering path's result bit for bit
    say("umap gather vs scatter, 300k")
    n, k = 300_000, 15
    idx, _ = synth.random_knn_graph(n, k, 31)
    w = np.random.default_rng(31).random((n, k)).astype(np.float32)
    G = gpu_union(dev, idx, w)
    Y0 = to_dev(synth.umap_init(n, 32), dev)
    A = api.umap_layout(Y0.clone(), G, 0.583, 1.334, 200, epochs=(0, 6), seed=3, symmetric=True)
    B = api.umap_layout(Y0.clone(), G, 0.583, 1.334, 200, epochs=(0, 6), seed=3, symmetric=False)
    assert torch.equal(A, B) and not torch.equal(A, Y0)


def test_umap_smallest_graph_and_most_negatives(dev):
    # n = 3, k = 2 (the smallest kNN graph), and neg_rate at its maximum of 64
    say("umap n=3, neg 64")
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0]], np.float32)
    idx, d2 = oracle.knn(X, 2)
    d2f = d2.astype(np.float32)
    rho, sigma, w = U.smooth_knn(np.sqrt(d2f.astype(np.float64)))
    g_rho, g_sigma, g_w = (t.cpu().numpy().astype(np.float64) for t in api.umap_weights(to_dev(d2f, dev)))
    # k = 2: the target sum log2(2) = 1 leaves the second weight ~1e-49,
    # below FP32's smallest subnormal, so the GPU stores 0 there
    np.testing.assert_allclose(g_w, w, rtol=2e-7, atol=1e-30)
    wf, rp, col, val = union_inputs(idx, w)
    G = gpu_union(dev, idx, wf)
    np.testing.assert_array_equal(G.col.cpu().numpy(), col)
    Y0 = synth.umap_init(3, 5)
    valf = val.astype(np.float32)
    Gd = api.SparseP(to_dev(rp, dev), to_dev(col, dev), to_dev(valf, dev), None, 3)
    Yg = api.umap_layout(to_dev(Y0, dev), Gd, 1.5, 0.9, 20, 1.0, 64, seed=7, epochs=(10, 12))
    Yo = U.layout(Y0.astype(np.float64), rp, col, valf, 20, 1.5, 0.9, 1.0, 64, 7, epochs=(10, 12))
    assert np.abs(Yg.cpu().numpy() - Yo).max() <= 2 * step_tol(Y0, Yo)
