"""GPU parity: tsne_knn (FP32 exact and BF16 + re-rank) against the FP64 oracle.

Neighbour indices are compared exactly; a difference is accepted only at a
documented near-tie (within 1e-5 of the oracle's k-th distance).  The BF16
path must reach >= 99.9 % agreement after re-ranking.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import check_knn, oracle_problem, say, to_dev
from paper_2605_13928_amd import api, synth

pytestmark = pytest.mark.gpu


def gpu_knn(dev, X, k, prec="fp32", n_cand=None):
    idx, d2 = api.knn(to_dev(X, dev), k, prec, n_cand=n_cand)
    return idx.cpu().numpy(), d2.cpu().numpy()


def test_knn_fp32_c1(dev):
    say("knn fp32 c1")
    X, labels, idx, d2, Pc, S = oracle_problem("c1", 1500, 90, 30.0)
    gi, gd = gpu_knn(dev, X, 90)
    raw, adj = check_knn(X, np.arange(1500), gi, gd, idx, d2)
    assert adj == 1.0


@pytest.mark.parametrize("n,d,k", [(2, 1, 1), (65, 3, 5), (777, 50, 30), (1000, 100, 129), (600, 17, 256),
                                   (3001, 64, 90)])
def test_knn_fp32_shapes(dev, n, d, k):
    say("knn fp32", n, d, k)
    rng = np.random.default_rng(n + d)
    X = (rng.standard_normal((n, d)) * rng.uniform(0.5, 2.0, d)).astype(np.float32)
    oi, od = oracle.knn(X, k)
    gi, gd = gpu_knn(dev, X, k)
    check_knn(X, np.arange(n), gi, gd, oi, od)


def test_knn_fp32_exact_ties(dev):
    say("knn fp32 ties")
    rng = np.random.default_rng(2)
    base = rng.standard_normal((300, 8)).astype(np.float32)
    X = np.concatenate([base, base, base[:50]], axis=0)
    oi, od = oracle.knn(X, 12)
    gi, gd = gpu_knn(dev, X, 12)
    # duplicates at distance exactly 0 come first, smaller index first
    np.testing.assert_array_equal(gi[:, 0], oi[:, 0])
    check_knn(X, np.arange(X.shape[0]), gi, gd, oi, od)


def test_knn_massive_ties(dev):
    # 8 distinct points, each repeated 500 times in shuffled order: every
    # query has 499 neighbours at distance 0, more than a candidate buffer
    # can keep at its threshold, which takes the sort branch of the
    # compaction.  FP32: the k smallest indices among the duplicates, as the
    # oracle's (d, j) order gives.  BF16: which duplicates survive the
    # candidate stage depends on BF16 rounding, so only validity is checked.
    say("knn massive ties")
    rng = np.random.default_rng(5)
    base = (rng.standard_normal((8, 50)) * 5).astype(np.float32)
    lab = rng.permutation(np.repeat(np.arange(8), 500))
    X = base[lab]
    k = 90
    oi, od = oracle.knn(X, k)
    gi, gd = gpu_knn(dev, X, k)
    np.testing.assert_array_equal(gi, oi)
    assert (gd == 0).all()
    bi, bd = gpu_knn(dev, X, k, "bf16", n_cand=180)
    n = X.shape[0]
    assert (bd == 0).all()
    assert (lab[bi] == lab[:, None]).all()
    assert (bi != np.arange(n)[:, None]).all()
    assert all(len(set(r)) == k for r in bi.tolist())


# 20,000 (the c2 workload) runs 32-row blocks, 30,000 (c2 shape) 64-row ones
@pytest.mark.parametrize("n", [20_000, 30_000])
def test_knn_fp32_c2_sampled_rows(dev, n):
    say("knn fp32 c2 shape", n)
    X, _ = synth.make_points("c2", n=n)
    gi, gd = gpu_knn(dev, X, 90)
    rows = np.random.default_rng(2).choice(X.shape[0], 400, replace=False)
    oi, od = oracle.knn(X, 90, rows=rows)
    check_knn(X, rows, gi[rows], gd[rows], oi, od)


@pytest.mark.parametrize("n", [300, 5000])
def test_knn_bf16_small(dev, n):
    say("knn bf16", n)
    X, _ = synth.make_points("c3", n=n)
    k = 90
    oi, od = oracle.knn(X, k)
    gi, gd = gpu_knn(dev, X, k, "bf16", n_cand=180)
    raw, adj = check_knn(X, np.arange(n), gi, gd, oi, od, min_agree=0.999)
    say("bf16 agreement", n, raw, adj)


@pytest.mark.parametrize("n,d,k", [(3, 2, 1), (65, 3, 5), (333, 58, 20), (1000, 17, 64)])
def test_knn_bf16_shapes(dev, n, d, k):
    # dimensions from 2 to the largest the BF16 layout takes (58: the six
    # norm slots end at element 63), ragged n (partial candidate tiles read
    # the padding row, partial query blocks hold queries past n)
    say("knn bf16 shape", n, d, k)
    X = (np.random.default_rng(n + d).standard_normal((n, d)) * 3).astype(np.float32)
    nc = min(2 * k, n - 1)
    oi, od = oracle.knn(X, k)
    gi, gd = gpu_knn(dev, X, k, "bf16", n_cand=nc)
    raw, adj = check_knn(X, np.arange(n), gi, gd, oi, od, min_agree=0.99)
    say("bf16 agreement", n, d, raw, adj)


def test_knn_bf16_candidates_are_rounded_point_neighbours(dev):
    # With n_cand = k the re-rank only reorders, so the set is the BF16
    # candidate set itself: the k nearest of the bf16-rounded points, which
    # the oracle computes exactly.
    say("knn bf16 candidate stage")
    X, _ = synth.make_points("c3", n=2000)
    k = 40
    oi, od = oracle.knn(X, k, bf16_points=True)
    gi, gd = gpu_knn(dev, X, k, "bf16", n_cand=k)
    hits = np.mean([len(set(a) & set(b)) / k for a, b in zip(gi.tolist(), oi.tolist())])
    assert hits >= 0.999, hits


def test_knn_bf16_c3_sampled_rows(dev):
    say("knn bf16 c3 full")
    X, _ = synth.make_points("c3")
    gi, gd = gpu_knn(dev, X, 90, "bf16", n_cand=180)
    rows = np.random.default_rng(3).choice(X.shape[0], 200, replace=False)
    oi, od = oracle.knn(X, 90, rows=rows)
    raw, adj = check_knn(X, rows, gi[rows], gd[rows], oi, od, min_agree=0.999)
    say("bf16 c3 agreement", raw, adj)


def separated_clusters(n, d, clusters, seed):
    """Far-apart Gaussian clusters (centres N(0, 30^2 I), unit noise): most
    candidate tiles of a query block lie in other clusters, far beyond its
    thresholds, so the BF16 sweep skips them."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((clusters, d)) * 30.0
    lab = rng.integers(0, clusters, n)
    return (centres[lab] + rng.standard_normal((n, d))).astype(np.float32)


@pytest.mark.parametrize("n,d,clusters", [(20001, 40, 16), (12345, 7, 10)])
def test_knn_bf16_tile_skipping(dev, n, d, clusters):
    # Candidate tiles whose box bound exceeds every threshold of a query
    # block are not evaluated; the result must still be the exact kNN (all
    # rows against the oracle) and, with n_cand = k, the candidate set the
    # kNN of the bf16-rounded points.  d = 7 leaves box coordinates past d.
    say("knn bf16 tile skipping", n, d, clusters)
    X = separated_clusters(n, d, clusters, n + d)
    k = 30
    oi, od = oracle.knn(X, k)
    gi, gd = gpu_knn(dev, X, k, "bf16", n_cand=2 * k)
    raw, adj = check_knn(X, np.arange(n), gi, gd, oi, od, min_agree=0.999)
    say("bf16 agreement with skipping", raw, adj)
    ri, _ = oracle.knn(X, k, bf16_points=True)
    ci, _ = gpu_knn(dev, X, k, "bf16", n_cand=k)
    hits = np.mean([len(set(a) & set(b)) / k for a, b in zip(ci.tolist(), ri.tolist())])
    assert hits >= 0.999, hits


def test_knn_bf16_tile_skipping_nonfinite_rows(dev):
    # Rows with a NaN or an infinite coordinate in several tiles: the boxes
    # leave NaN out and stretch to infinity, and the finite rows still get
    # their exact neighbours among the finite points.
    say("knn bf16 tile skipping with non-finite rows")
    n, d, k = 16000, 24, 20
    X = separated_clusters(n, d, 12, 99)
    rng = np.random.default_rng(100)
    bad = rng.choice(n, 40, replace=False)
    for t, r in enumerate(bad):
        X[r, rng.integers(0, d)] = [np.nan, np.inf, -np.inf][t % 3]
    fin = np.setdiff1d(np.arange(n), bad)
    Xf = X[fin]
    gi, gd = gpu_knn(dev, X, k, "bf16", n_cand=2 * k)
    rows = rng.choice(fin.size, 2000, replace=False)
    oi, od = oracle.knn(Xf, k, rows=rows)
    g = gi[fin[rows]]
    assert np.isin(g, fin).all()  # no non-finite point is a neighbour of a finite row
    back = np.searchsorted(fin, g)
    raw, adj = check_knn(Xf, rows, back.astype(np.int32), gd[fin[rows]], oi, od, min_agree=0.999)
    say("bf16 agreement, finite rows", raw, adj)
