"""Shared helpers of the GPU parity tests.

Inputs come from the seeded generators; expected values come from the FP64
oracle only (never from the HIP path).
"""
from __future__ import annotations

import functools
import sys

import numpy as np
import torch

import oracle
from paper_2605_13928_amd import api, synth

NEAR_TIE = 1e-5  # relative slack on the k-th distance that counts as a tie


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def to_dev(a, dev, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


@functools.lru_cache(maxsize=8)
def oracle_problem(workload: str, n: int, k: int, perplexity: float):
    """X from the workload recipe, then the oracle's exact kNN, calibration and P."""
    X, labels = synth.make_points(workload, n=n)
    idx, d2 = oracle.knn(X, k)
    Pc, beta, conv, H = oracle.calibrate(d2, perplexity)
    S = oracle.symmetrize(idx, Pc)
    return X, labels, idx, d2, Pc, S


@functools.lru_cache(maxsize=4)
def random_graph_P(n: int, k: int, perplexity: float, seed: int):
    """P from a seeded random neighbour graph through the oracle's calibration and symmetrisation."""
    idx, d2 = synth.random_knn_graph(n, k, seed)
    Pc, _, _, _ = oracle.calibrate(d2, perplexity)
    S = oracle.symmetrize(idx, Pc)
    return idx, d2, Pc, S


def sparse_to_dev(S: "oracle.CSR", dev, dtype=torch.float32) -> api.SparseP:
    return api.SparseP(to_dev(S.row_ptr, dev), to_dev(S.col, dev), to_dev(S.val, dev, dtype),
                       None if S.tpos is None else to_dev(S.tpos, dev), S.n)


def check_knn(X, rows, g_idx, g_d2, o_idx, o_d2, tie=NEAR_TIE, min_agree=1.0, d2_rtol=2e-5):
    """Compare GPU neighbour lists with the oracle's on the given query rows.

    Unique parts must match exactly; a mismatch is allowed only as a near
    tie (both the missing and the extra neighbour within `tie` of the
    oracle's k-th distance, distances recomputed in FP64).  Returns
    (raw agreement, tie-adjusted agreement).
    """
    m, k = o_idx.shape
    assert g_idx.shape == (m, k)
    # GPU lists are sorted by their own distances and hold distinct, non-self indices
    assert np.all(np.diff(g_d2, axis=1) >= 0)
    assert np.all(g_idx != rows[:, None])
    assert all(len(set(r)) == k for r in g_idx.tolist())
    # GPU distances are the FP32 distances of the pairs they name
    true_g = oracle.pair_d2(X, np.repeat(rows, k), g_idx.ravel()).reshape(m, k)
    np.testing.assert_allclose(g_d2, true_g, rtol=d2_rtol, atol=1e-6)
    hits = 0
    tie_ok = 0
    for r in range(m):
        gs, os_ = set(g_idx[r].tolist()), set(o_idx[r].tolist())
        inter = len(gs & os_)
        hits += inter
        dk = o_d2[r, k - 1]
        extra = np.array(sorted(gs - os_), dtype=np.int64)
        missing = [j for j in os_ - gs]
        ok = True
        if extra.size:
            de = oracle.pair_d2(X, np.full(extra.size, rows[r]), extra)
            ok &= bool(np.all(de <= dk * (1 + tie)))
        if missing:
            dm = o_d2[r][np.isin(o_idx[r], missing)]
            ok &= bool(np.all(dm >= dk / (1 + tie)))
        tie_ok += inter + (k - inter if ok else 0)
    raw = hits / (m * k)
    adj = tie_ok / (m * k)
    assert adj >= min_agree, (raw, adj)
    return raw, adj
