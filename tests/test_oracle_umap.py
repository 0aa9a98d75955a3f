"""Pins of the UMAP oracle (oracle/umap.py) against what the definitions and
the mathematics fix: the a, b fit is a least-squares minimum; the smoothed
kNN weights meet their defining sum and are invariant to scaling and to a
shift of a row's distances; the fuzzy union equals a dense evaluation of
A + A^T - A o A^T; the generator reproduces published SplitMix64 outputs;
the schedule samples an entry floor(n_epochs r) times; the step
coefficients are the derivatives of log Phi and log(1 - Phi); one epoch on
two points has a closed form; a whole layout separates a mixture."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import umap as U

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("min_dist", [0.1, 0.5])
def test_fit_ab_is_least_squares_minimum(min_dist):
    a, b = U.fit_ab(min_dist)
    f0 = U.fit_objective(a, b, min_dist)
    h = 1e-5
    ga = (U.fit_objective(a + h, b, min_dist) - U.fit_objective(a - h, b, min_dist)) / (2 * h)
    gb = (U.fit_objective(a, b + h, min_dist) - U.fit_objective(a, b - h, min_dist)) / (2 * h)
    assert abs(ga) < 1e-6 and abs(gb) < 1e-6, (ga, gb)
    for da, db in ((1e-3, 0), (-1e-3, 0), (0, 1e-3), (0, -1e-3)):
        assert U.fit_objective(a + da, b + db, min_dist) > f0
    # Phi falls through 1/2 past min_dist, as Psi does
    x = np.linspace(0, 3, 3001)
    phi = 1.0 / (1.0 + a * x ** (2 * b))
    assert np.all(np.diff(phi) <= 0) and min_dist < x[np.argmin(np.abs(phi - 0.5))] < min_dist + 1.5


def _rows(seed, n=40, k=15):
    rng = np.random.default_rng(seed)
    return np.sort(rng.gamma(2.0, 1.0, (n, k)) + 0.05, axis=1)


def test_smooth_knn_defining_sum_and_nearest_weight():
    d = _rows(1)
    rho, sigma, w = U.smooth_knn(d)
    np.testing.assert_allclose(w.sum(1), np.log2(15), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(rho, d.min(1))
    np.testing.assert_array_equal(w[:, 0], 1.0)
    assert np.all(np.diff(w, axis=1) <= 0) and np.all(w > 0) and np.all(w <= 1)


def test_smooth_knn_scale_and_shift_invariance():
    d = _rows(2)
    rho, sigma, w = U.smooth_knn(d)
    r2, s2, w2 = U.smooth_knn(3.5 * d)
    np.testing.assert_allclose(r2, 3.5 * rho, rtol=1e-14)
    np.testing.assert_allclose(s2, 3.5 * sigma, rtol=1e-10)
    np.testing.assert_allclose(w2, w, rtol=0, atol=1e-12)
    r3, s3, w3 = U.smooth_knn(d + 2.0)
    np.testing.assert_allclose(r3, rho + 2.0, rtol=1e-14)
    np.testing.assert_allclose(s3, sigma, rtol=1e-9)
    np.testing.assert_allclose(w3, w, rtol=0, atol=1e-12)


def test_smooth_knn_degenerate_rows():
    k = 15
    d = np.vstack([np.zeros(k), np.r_[np.full(5, 0.7), np.linspace(1, 3, k - 5)], np.r_[0.0, np.linspace(1, 2, k - 1)]])
    rho, sigma, w = U.smooth_knn(d)
    # all coincident: every weight 1, sigma at the 1e-3 floor
    assert rho[0] == 0 and sigma[0] == 1e-3 and np.all(w[0] == 1)
    # five ties at rho >= log2(15) = 3.9: the floor already meets the target
    assert rho[1] == 0.7 and sigma[1] == pytest.approx(1e-3 * d[1].mean(), rel=1e-15)
    assert np.all(w[1, :5] == 1) and w[1, 5:].max() < 1e-80  # exp(-0.3 / 1.567e-3)
    # a zero distance (duplicate point) is not rho; its weight is 1
    assert rho[2] == 1.0 and w[2, 0] == 1.0 and w[2].sum() == pytest.approx(np.log2(k), abs=1e-12)


def test_fuzzy_union_matches_dense():
    rng = np.random.default_rng(3)
    n, k = 30, 4
    nbr = np.array([rng.choice(np.delete(np.arange(n), i), k, replace=False) for i in range(n)], np.int32)
    w = rng.random((n, k))
    rp, col, val = U.fuzzy_union(nbr, w, n)
    A = np.zeros((n, n))
    for i in range(n):
        for a in range(k):
            A[i, nbr[i, a]] = w[i, a]
    B = A + A.T - A * A.T
    D = U.to_scipy(rp, col, val, n).toarray()
    np.testing.assert_allclose(D, B, rtol=0, atol=1e-15)
    pattern = (A > 0) | (A.T > 0)
    assert rp[-1] == pattern.sum()
    for i in range(n):
        cols = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0) and set(cols) == set(np.nonzero(pattern[i])[0])
    assert np.all(D >= np.maximum(A, A.T) - 1e-15) and np.all(D <= 1.0)


def test_splitmix64_published_outputs_and_counter_form():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64_seed1234567.json")))
    assert [int(v) for v in U.splitmix64(g["seed"], np.arange(5))] == g["outputs"]
    assert U.splitmix64_sequence(g["seed"], 5) == g["outputs"]
    for seed in (0, 42, 2**63 + 5):
        assert [int(v) for v in U.splitmix64(seed, np.arange(64))] == U.splitmix64_sequence(seed, 64)


def test_draws_uniform():
    n = 10
    c = U.draw_vertex(U.splitmix64(7, np.arange(200_000)), n).astype(np.int64)
    assert c.min() == 0 and c.max() == n - 1
    counts = np.bincount(c, minlength=n)
    chi2 = ((counts - 20_000) ** 2 / 20_000).sum()
    assert chi2 < 30.0, chi2  # 9 degrees of freedom: p < 5e-4 beyond 30


def test_schedule_counts():
    rng = np.random.default_rng(4)
    val = rng.random(500).astype(np.float32)
    val[0] = 1.5
    n_epochs = 200
    total = sum(U.sample_mask(val, t).astype(int) for t in range(n_epochs))
    r = val / np.float32(val.max())
    np.testing.assert_array_equal(total, np.floor(np.float32(n_epochs) * r).astype(int))
    assert total[0] == n_epochs


def test_step_coefficients_are_derivatives():
    rng = np.random.default_rng(5)
    for a, b in ((1.577, 0.895), (0.583, 1.334)):
        yi, yj = rng.normal(size=2), rng.normal(size=2)
        h = 1e-6

        def num_grad(f):
            g = np.zeros(2)
            for q in range(2):
                e = np.zeros(2)
                e[q] = h
                g[q] = (f(yi + e) - f(yi - e)) / (2 * h)
            return g

        def logphi(y):
            return -np.log1p(a * np.sum((y - yj) ** 2) ** b)

        def log1mphi(y):
            s = a * np.sum((y - yj) ** 2) ** b
            return np.log(s / (1.0 + s))

        d2 = np.sum((yi - yj) ** 2)
        np.testing.assert_allclose(U.attraction_coef(d2, a, b) * (yi - yj), num_grad(logphi), rtol=1e-6)
        np.testing.assert_allclose(U.repulsion_coef(d2, a, b, eps=0.0) * (yi - yj), num_grad(log1mphi), rtol=1e-6)


def test_epoch_two_points_closed_form():
    # one edge each way, weight 1: both sampled in every epoch
    rp, col, val = np.array([0, 1, 2]), np.array([1, 0], np.int32), np.array([1.0, 1.0])
    Y0 = np.array([[0.0, 0.0], [2.0, 0.0]])
    a, b, alpha0, n_epochs = 1.0, 1.0, 0.1, 10
    # no negatives: each edge moves both ends by alpha * clip(c (y_i - y_j)),
    # c = -2ab d2^(b-1) / (1 + a d2^b) = -2 / 5 at d2 = 4
    Y1 = U.layout_epoch(Y0, rp, col, val, 0, n_epochs, a, b, alpha0, neg_rate=0)
    np.testing.assert_allclose(Y1, [[0.16, 0.0], [1.84, 0.0]], rtol=0, atol=1e-15)
    # with negatives: every draw that is not i itself is the other point,
    # repelling by 2b / ((1e-3 + d2)(1 + a d2^b)) (y_i - y_j)
    t, neg = 3, 5
    alpha = alpha0 * (1 - t / n_epochs)
    ctr = (np.uint64(t) * np.uint64(2) + np.arange(2, dtype=np.uint64)[:, None]) * np.uint64(neg) + \
        np.arange(neg, dtype=np.uint64)[None, :]
    c = U.draw_vertex(U.splitmix64(11, ctr), 2).astype(int)
    m = (c != np.array([[0], [1]])).sum(1)  # draws of the other point, per row
    ca, cr = -2.0 / 5.0, 2.0 / ((1e-3 + 4.0) * 5.0)
    step0 = alpha * (2 * ca * (-2.0) + m[0] * cr * (-2.0))
    step1 = alpha * (2 * ca * 2.0 + m[1] * cr * 2.0)
    Y = U.layout_epoch(Y0, rp, col, val, t, n_epochs, a, b, alpha0, neg_rate=neg, seed=11)
    np.testing.assert_allclose(Y, [[step0, 0.0], [2.0 + step1, 0.0]], rtol=1e-14, atol=1e-15)
    assert m.sum() > 0


def test_epoch_translation_and_reflection():
    rng = np.random.default_rng(6)
    n, k = 60, 5
    nbr = np.array([rng.choice(np.delete(np.arange(n), i), k, replace=False) for i in range(n)], np.int32)
    rp, col, val = U.fuzzy_union(nbr, rng.random((n, k)), n)
    Y = rng.normal(size=(n, 2)) * 3
    Y1 = U.layout_epoch(Y, rp, col, val, 4, 50, 1.2, 0.9, 1.0, 5, 3)
    np.testing.assert_allclose(U.layout_epoch(Y + [5.0, -2.0], rp, col, val, 4, 50, 1.2, 0.9, 1.0, 5, 3),
                               Y1 + [5.0, -2.0], atol=1e-12)
    np.testing.assert_allclose(U.layout_epoch(-Y, rp, col, val, 4, 50, 1.2, 0.9, 1.0, 5, 3), -Y1, atol=1e-12)


def test_layout_separates_mixture():
    rng = np.random.default_rng(8)
    n_per, d, k = 150, 10, 15
    centres = rng.normal(size=(3, d)) * 8
    X = np.vstack([c + rng.normal(size=(n_per, d)) for c in centres]).astype(np.float32)
    lab = np.repeat(np.arange(3), n_per)
    n = X.shape[0]
    idx, d2 = oracle.knn(X, k)
    rho, sigma, w = U.smooth_knn(np.sqrt(d2))
    rp, col, val = U.fuzzy_union(idx, w, n)
    a, b = U.fit_ab(0.5)
    Y0 = rng.uniform(-10, 10, size=(n, 2))
    Y = U.layout(Y0, rp, col, val, 200, a, b, 1.0, 5, 9)
    D = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(D, np.inf)
    nn = np.argsort(D, axis=1)[:, :10]
    assert (lab[nn] == lab[:, None]).mean() >= 0.95


def _mixture_graph(seed, ncl=5, n_per=60, d=10, k=15, spread=6.0):
    rng = np.random.default_rng(seed)
    centres = rng.normal(size=(ncl, d)) * spread
    X = np.vstack([c + rng.normal(size=(n_per, d)) for c in centres]).astype(np.float32)
    lab = np.repeat(np.arange(ncl), n_per)
    idx, d2 = oracle.knn(X, k)
    _, _, w = U.smooth_knn(np.sqrt(d2))
    rp, col, val = U.fuzzy_union(idx, w, X.shape[0])
    return rng, lab, rp, col, val


def test_synchronous_epoch_is_first_order_in_the_step():
    # The published layout is sequential SGD: each step moves the points at
    # once.  The oracle's epoch evaluates every step at the epoch's start.
    # Both apply the same steps, so they differ only through the steps taken
    # earlier in the same epoch: by O(alpha^2), while one epoch moves the
    # points by O(alpha).  Halving the learning rate must quarter the gap.
    rng, lab, rp, col, val = _mixture_graph(20)
    a, b = U.fit_ab(0.1)
    Y0 = rng.uniform(-10, 10, size=(lab.size, 2))
    Ymid = U.layout(Y0, rp, col, val, 200, a, b, 1.0, 5, 9, epochs=(0, 60))
    for t in (60, 61):
        gaps, moves = [], []
        for alpha0 in (4e-3, 2e-3, 1e-3):
            Ys = U.layout_epoch(Ymid, rp, col, val, t, 200, a, b, alpha0, 5, 9)
            Yq = U.layout_epoch_sequential(Ymid, rp, col, val, t, 200, a, b, alpha0, 5, 9)
            gaps.append(np.linalg.norm(Ys - Yq))
            moves.append(np.linalg.norm(Yq - Ymid))
        for g0, g1, m0, m1 in zip(gaps, gaps[1:], moves, moves[1:]):
            assert 3.0 <= g0 / g1 <= 5.0, gaps  # second order in alpha
            assert 1.8 <= m0 / m1 <= 2.2, moves  # the move itself is first order
        assert gaps[-1] <= 0.03 * moves[-1], (gaps, moves)


@pytest.mark.parametrize("case", [0, 1])
def test_synchronous_layout_reaches_sequential_objective(case):
    # Whole layouts (200 epochs, alpha0 = 1): the synchronous form ends at
    # the same value of the objective the layout minimises, the fuzzy-set
    # cross-entropy over all pairs, within 8 % of the sequential form's
    # (mean over three negative-sampling seeds; the sequential runs
    # themselves spread by about 4 %), and at the same 10-NN label purity.
    rng, lab, rp, col, val = _mixture_graph(20 + case, spread=6.0 if case == 0 else 4.0)
    a, b = U.fit_ab(0.1)
    Y0 = rng.uniform(-10, 10, size=(lab.size, 2))

    def purity(Y):
        D = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
        np.fill_diagonal(D, np.inf)
        nn = np.argsort(D, axis=1)[:, :10]
        return (lab[nn] == lab[:, None]).mean()

    ce_s, ce_q = [], []
    for seed in (9, 10, 11):
        Ys = U.layout(Y0, rp, col, val, 200, a, b, 1.0, 5, seed)
        Yq = U.layout_sequential(Y0, rp, col, val, 200, a, b, 1.0, 5, seed)
        ce_s.append(U.fuzzy_cross_entropy(Ys, rp, col, val, a, b))
        ce_q.append(U.fuzzy_cross_entropy(Yq, rp, col, val, a, b))
        assert purity(Ys) >= 0.98 and purity(Yq) >= 0.98
    assert abs(np.mean(ce_s) - np.mean(ce_q)) <= 0.08 * np.mean(ce_q), (ce_s, ce_q)


def test_fuzzy_cross_entropy_definition():
    # three points, hand-evaluated terms: stored pair (0, 1) with v = 0.6,
    # pairs (0, 2) and (1, 2) absent (v = 0)
    rp = np.array([0, 1, 2, 2])
    col = np.array([1, 0], np.int32)
    val = np.array([0.6, 0.6])
    Y = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0]])
    a, b = 1.5, 0.8
    phi = lambda d2: 1.0 / (1.0 + a * d2 ** b)  # noqa: E731
    want = (0.6 * np.log(0.6 / phi(1.0)) + 0.4 * np.log(0.4 / (1 - phi(1.0)))
            + np.log(1.0 / (1 - phi(4.0))) + np.log(1.0 / (1 - phi(5.0))))
    assert abs(U.fuzzy_cross_entropy(Y, rp, col, val, a, b) - want) <= 1e-12 * abs(want)
