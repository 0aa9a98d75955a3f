"""Pins of the interpolation oracle (oracle/interp.py) against what the
mathematics fixes: Lagrange interpolation reproduces polynomials of degree
< p; the FFT convolution equals the dense double sum; weights are one-hot at
the nodes; the interpolated repulsion converges to the exact all-pairs sums
(the C oracle) at third order in the box side for p = 3; the attraction
equals the C oracle's."""
import numpy as np
import pytest

import oracle
from oracle import interp as I


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_lagrange_reproduces_polynomials(p):
    u = np.random.default_rng(p).random(64)
    t = (np.arange(p) + 0.5) / p
    L = I.lagrange_weights(u, p)
    for m in range(p):
        np.testing.assert_allclose(L @ (t ** m), u ** m, rtol=0, atol=1e-13)
    # degree p is not reproduced (the interpolation error term is nonzero)
    assert np.abs(L @ (t ** p) - u ** p).max() > 1e-6


def test_weights_one_hot_at_nodes():
    p = 3
    t = (np.arange(p) + 0.5) / p
    L = I.lagrange_weights(t, p)
    np.testing.assert_allclose(L, np.eye(p), atol=1e-15)


@pytest.mark.parametrize("N,F,which", [(6, 16, 1), (18, 64, 2), (18, 36, 1), (25, 64, 2)])
def test_fft_convolution_equals_direct_sum(N, F, which):
    W = np.random.default_rng(N + F).standard_normal((2, N, N))
    a = I.potentials(W, 0.29, which, "direct")
    b = I.potentials(W, 0.29, which, "fft", F)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_grid_params_clamps_and_edges():
    Y = np.array([[0.0, 0.0], [10.0, 3.0]], dtype=np.float32)
    lo, h, B, N, F, c = I.grid_params(Y, p=3, min_boxes=4, max_box_width=1.0, max_fft=2048)
    assert (lo, B, N, F, c) == (0.0, 10, 30, 64, 5.0) and h == 1.0
    # min_boxes and the FFT-size cap
    assert I.grid_params(Y, 3, 50, 1.0, 2048)[2] == 50
    assert I.grid_params(Y, 3, 4, 0.001, 256)[2] == 256 // 6
    # the largest coordinate falls in the last box at u = 1
    b, u = I.boxes(Y.astype(np.float64), lo, h, B)
    assert b[1, 0] == B - 1 and u[1, 0] == 1.0


def test_spread_at_node_and_interpolate_back():
    p, B = 3, 4
    lo, h = 0.0, 1.0
    # a point exactly on node (box 2, local node 1) in x and (box 0, node 2) in y
    Y = np.array([[2.0 + 0.5, 0.0 + 2.5 / 3.0]])
    W = I.spread(Y, np.array([[1.0]]), lo, h, B, p)
    gx, gy = 2 * p + 1, 0 * p + 2
    assert abs(W[0, gx, gy] - 1.0) < 1e-12 and abs(W.sum() - 1.0) < 1e-12
    Phi = np.random.default_rng(1).standard_normal((1, p * B, p * B))
    v = I.interpolate(Y, Phi, lo, h, B, p)
    assert abs(v[0, 0] - Phi[0, gx, gy]) < 1e-12


def _exact(Y):
    Zr, Rr, _ = oracle.grad_rows(Y.astype(np.float64), np.arange(Y.shape[0]))
    return Rr, Zr.sum()


def test_converges_to_exact_repulsion_third_order():
    Y = (np.random.default_rng(0).standard_normal((400, 2)) * 3).astype(np.float32)
    Rr, Zex = _exact(Y)
    errs = []
    for mw in (1.0, 0.5, 0.25):
        R, Z = I.repulsion(Y, p=3, min_boxes=1, max_box_width=mw, max_fft=4096)
        errs.append((np.linalg.norm(R - Rr) / np.linalg.norm(Rr), abs(Z - Zex) / Zex))
    for a, b in zip(errs, errs[1:]):
        assert b[0] < a[0] / 5 and b[1] < a[1] / 5, errs
    assert errs[-1][0] < 1e-3 and errs[-1][1] < 1e-5, errs


def test_attraction_and_gradient_against_c_oracle():
    X, _ = __import__("paper_2605_13928_amd.synth", fromlist=["synth"]).make_points("c1", n=300)
    idx, d2 = oracle.knn(X, 20)
    Pc, _, _, _ = oracle.calibrate(d2, 6.0)
    P = oracle.symmetrize(idx, Pc)
    Y = (np.random.default_rng(3).standard_normal((300, 2)) * 4).astype(np.float32)
    Yd = Y.astype(np.float64)
    _, _, Ar = oracle.grad_rows(Yd, np.arange(300), P)
    np.testing.assert_allclose(I.attraction(Yd, P), Ar, rtol=1e-12, atol=1e-18)
    g_ex, Z_ex, kl_ex = oracle.kl_grad(Yd, P, 12.0)
    g, Z, kl = I.kl_grad(Y, P, 12.0, p=3, min_boxes=1, max_box_width=0.125, max_fft=4096)
    assert np.linalg.norm(g - g_ex) / np.linalg.norm(g_ex) < 1e-5
    assert abs(Z - Z_ex) / Z_ex < 1e-6
    assert abs(kl - kl_ex) / abs(kl_ex) < 1e-6
