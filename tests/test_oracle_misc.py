"""Pins of the oracle's differentiation form, optimiser step and the
composed t-SNE run; plus the seeded input generators."""
import json
import os

import numpy as np
import pytest

from paper_2605_13928_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def general_problem(oracle_mod, n=80, k=20, seed=1):
    # Symmetric pattern, but values perturbed independently per entry so that
    # neither P = P^T nor sum P = 1 holds (what gradcheck explores).
    idx, d2 = synth.random_knn_graph(n, k, seed)
    Pc, _, _, _ = oracle_mod.calibrate(d2, 7.0)
    S = oracle_mod.symmetrize(idx, Pc)
    rng = np.random.default_rng(seed)
    S.val = S.val * rng.uniform(0.5, 1.5, S.nnz)
    Y = synth.random_embedding(n, 2.0, seed + 7).astype(np.float64)
    return S, Y


def test_backward_dY_matches_finite_differences(oracle_mod):
    S, Y = general_problem(oracle_mod)
    dY, dP = oracle_mod.kl_backward(Y, S, gC=1.0)
    h = 1e-6
    for i in (0, 3, 41, 79):
        for c in range(2):
            Yp = Y.copy(); Yp[i, c] += h
            Ym = Y.copy(); Ym[i, c] -= h
            fd = (oracle_mod.kl(Yp, S)[0] - oracle_mod.kl(Ym, S)[0]) / (2 * h)
            assert abs(fd - dY[i, c]) <= 1e-7 * max(1.0, np.abs(dY).max()), (i, c, fd, dY[i, c])


def test_backward_dP_matches_finite_differences(oracle_mod):
    S, Y = general_problem(oracle_mod, seed=2)
    dY, dP = oracle_mod.kl_backward(Y, S, gC=1.0)
    rng = np.random.default_rng(3)
    for e in rng.choice(S.nnz, 10, replace=False):
        h = 1e-4 * S.val[e]
        Sp = oracle_mod.CSR(S.row_ptr, S.col, S.val.copy()); Sp.val[e] += h
        Sm = oracle_mod.CSR(S.row_ptr, S.col, S.val.copy()); Sm.val[e] -= h
        fd = (oracle_mod.kl(Y, Sp)[0] - oracle_mod.kl(Y, Sm)[0]) / (2 * h)
        assert abs(fd - dP[e]) <= 1e-6 * max(1.0, abs(dP[e])), (e, fd, dP[e])


def test_backward_scales_with_gC_and_reduces_to_tsne_gradient(oracle_mod):
    X, _ = synth.make_points("c1", n=150)
    idx, d2 = oracle_mod.knn(X, 30)
    Pc, _, _, _ = oracle_mod.calibrate(d2, 10.0)
    S = oracle_mod.symmetrize(idx, Pc)
    Y = synth.random_embedding(150, 3.0, 4).astype(np.float64)
    g, Z, kl = oracle_mod.kl_grad(Y, S, 1.0)
    dY, dP = oracle_mod.kl_backward(Y, S, gC=1.0)
    np.testing.assert_allclose(dY, g, rtol=1e-10, atol=1e-13 * np.abs(g).max())
    dY2, dP2 = oracle_mod.kl_backward(Y, S, gC=-2.5)
    np.testing.assert_allclose(dY2, -2.5 * dY, rtol=1e-14)
    np.testing.assert_allclose(dP2, -2.5 * dP, rtol=1e-14)


def test_step_golden_cases(oracle_mod):
    with open(os.path.join(GOLDEN, "step_cases.json")) as f:
        spec = json.load(f)
    prm = spec["params"]
    for case in spec["cases"]:
        Y = np.array([[case["y"], 0.0]])
        U = np.array([[case["update"], 0.0]])
        G = np.array([[case["gain"], 1.0]])
        g = np.array([[case["grad"], 0.0]])
        oracle_mod.step(Y, U, G, g, prm["lr"], case["momentum"], prm["gain_inc"], prm["gain_dec"], prm["min_gain"])
        assert Y[0, 0] == pytest.approx(case["y_new"], rel=1e-12, abs=1e-12), case["why"]
        assert U[0, 0] == pytest.approx(case["update_new"], rel=1e-12, abs=1e-12), case["why"]
        assert G[0, 0] == pytest.approx(case["gain_new"], rel=1e-12), case["why"]


def run_oracle_tsne(oracle_mod, w, n=None):
    X, labels = synth.make_points(w, n=n)
    idx, d2 = oracle_mod.knn(X, w.k)
    Pc, _, conv, _ = oracle_mod.calibrate(d2, w.perplexity)
    S = oracle_mod.symmetrize(idx, Pc)
    Y = synth.make_init(w, n=n).astype(np.float64)
    U = np.zeros_like(Y)
    G = np.ones_like(Y)
    kls = {}
    for t in range(w.iters):
        a, m = oracle_mod.tsne_schedule(t, w.exaggeration, w.exaggeration_iters, w.momentum_early, w.momentum_late)
        g, Z, kl = oracle_mod.kl_grad(Y, S, a, want_kl=(t % 50 == 49))
        if kl is not None:
            kls[t] = kl
        oracle_mod.step(Y, U, G, g, w.lr, m)
    return X, labels, S, Y, kls


def test_oracle_tsne_c1_separates_clusters(oracle_mod):
    w = synth.WORKLOADS["c1"]
    X, labels, S, Y, kls = run_oracle_tsne(oracle_mod, w)
    # 10 nearest embedding neighbours mostly share the point's cluster
    idx, _ = oracle_mod.knn(Y.astype(np.float32), 10)
    agree = (labels[idx] == labels[:, None]).mean()
    assert agree >= 0.95, agree
    assert kls[249] < kls[99]


def test_synth_deterministic_and_shaped():
    X1, l1 = synth.make_points("c2", n=5000)
    X2, l2 = synth.make_points("c2", n=5000)
    assert synth.sha256(X1) == synth.sha256(X2) and np.array_equal(l1, l2)
    assert X1.dtype == np.float32 and X1.shape == (5000, 50) and X1.flags.c_contiguous
    assert len(np.unique(l1)) <= 20
    Xp, lp = synth.make_points("c5", n=200_000)
    v = Xp.var(0)
    assert v[0] > 5 * v[-1]  # variance decays with the dimension index
    Y = synth.make_init("c1")
    assert Y.shape == (1500, 2) and abs(Y.std() - 0.01) < 0.002
    idx, d2 = synth.random_knn_graph(100, 10, 3)
    assert all(len(set(r)) == 10 and i not in r for i, r in enumerate(idx.tolist()))
    assert np.all(np.diff(d2, axis=1) >= 0)
