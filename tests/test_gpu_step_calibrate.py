"""GPU parity: tsne_step and tsne_calibrate_P against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from helpers import oracle_problem, random_graph_P, say, to_dev
from paper_2605_13928_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 63, 1000, 100_003])
def test_step_matches_oracle(dev, n):
    say("step", n)
    rng = np.random.default_rng(n)
    Y = rng.standard_normal((n, 2)).astype(np.float32)
    U = rng.standard_normal((n, 2)).astype(np.float32)
    G = rng.uniform(0.005, 3.0, (n, 2)).astype(np.float32)
    g = rng.standard_normal((n, 2)).astype(np.float32)
    g[rng.random((n, 2)) < 0.1] = 0.0  # zero-gradient case
    U[rng.random((n, 2)) < 0.1] = 0.0  # zero-update case
    for lr, mom in ((200.0, 0.5), (200.0, 0.8)):
        tY, tU, tG, tg = (to_dev(a, dev) for a in (Y, U, G, g))
        api.step(tY, tU, tG, tg, lr, mom)
        oY, oU, oG = Y.astype(np.float64), U.astype(np.float64), G.astype(np.float64)
        oracle.step(oY, oU, oG, g.astype(np.float64), lr, mom)
        np.testing.assert_allclose(tG.cpu().numpy(), oG, rtol=1e-6)
        scale = np.abs(oU) + 200.0 * np.abs(oG * g) + 1e-30
        assert np.all(np.abs(tU.cpu().numpy() - oU) <= 2e-6 * scale)
        assert np.all(np.abs(tY.cpu().numpy() - oY) <= 2e-6 * (np.abs(oY) + np.abs(oU) + np.abs(Y) + 1e-30))


def entropy64(d2_row, beta):
    s = d2_row - d2_row.min()
    e = np.exp(-beta * s)
    S = e.sum()
    return np.log(S) + beta * (e * s).sum() / S


# The kernel stops its FP32 search TSNE_CALIB_H_MARGIN inside tol, so the
# entropy at the returned beta, recomputed in FP64, must be within tol.


def test_calibrate_c1(dev):
    say("calibrate c1")
    X, labels, idx, d2, Pc, S = oracle_problem("c1", 1500, 90, 30.0)
    d2f = d2.astype(np.float32)
    P, beta, conv, nun = api.calibrate_P(to_dev(d2f, dev), 30.0, tol=1e-5)
    P, beta, conv = P.cpu().numpy(), beta.cpu().numpy(), conv.cpu().numpy()
    assert conv.all() and int(nun.item()) == 0
    d64 = d2f.astype(np.float64)
    H = np.array([entropy64(d64[i], float(beta[i])) for i in range(d64.shape[0])])
    assert np.abs(H - np.log(30.0)).max() <= 1e-5
    np.testing.assert_allclose(P.sum(1), 1.0, atol=2e-6)
    Po, _, _, _ = oracle.calibrate(d64, 30.0)
    assert np.abs(P - Po).max() <= 2e-5 * Po.max()


@pytest.mark.parametrize("n,k,perp", [(1, 5, 2.0), (37, 36, 10.0), (1001, 64, 20.0), (999, 100, 30.0),
                                      (513, 256, 80.0), (20_000, 90, 30.0)])
def test_calibrate_shapes(dev, n, k, perp):
    say("calibrate", n, k, perp)
    rng = np.random.default_rng(k)
    d2 = np.sort(rng.chisquare(50, (n, k)) * 2.0, axis=1).astype(np.float32)
    rng.permuted(d2, axis=1, out=d2)  # any order within a row
    P, beta, conv, nun = api.calibrate_P(to_dev(d2, dev), perp)
    P, beta, conv = P.cpu().numpy(), beta.cpu().numpy(), conv.cpu().numpy()
    assert conv.all() and int(nun.item()) == 0
    d64 = d2.astype(np.float64)
    H = np.array([entropy64(d64[i], float(beta[i])) for i in range(n)])
    assert np.abs(H - np.log(perp)).max() <= 1e-5
    Po, _, _, _ = oracle.calibrate(d64, perp)
    assert np.abs(P - Po).max() <= 2e-5 * Po.max()


def test_calibrate_degenerate_rows(dev):
    say("calibrate degenerate")
    d2 = np.full((10, 90), 4.0, np.float32)
    d2[3] = np.linspace(1, 50, 90)
    P, beta, conv, nun = api.calibrate_P(to_dev(d2, dev), 30.0, max_iter=60)
    conv = conv.cpu().numpy()
    assert conv.tolist() == [0, 0, 0, 1, 0, 0, 0, 0, 0, 0]
    assert int(nun.item()) == 9
    np.testing.assert_allclose(P.cpu().numpy()[0], 1.0 / 90, rtol=1e-6)


def test_calibrate_unreachable_rows_default_max_iter(dev):
    # Rows whose nearest distance is shared by more than `perplexity`
    # neighbours never bracket the target (H > ln 30 for every beta): all 90
    # distances equal (H = ln 90), and 40 tied minima before 50 larger
    # distances (H -> ln 40).  At the default 200 evaluations beta must stay
    # finite and P must be the limit the FP64 oracle reaches: uniform over the
    # tied neighbours.  Two ordinary rows ride along.
    say("calibrate unreachable rows, max_iter 200")
    rng = np.random.default_rng(40)
    d2 = np.sort(rng.chisquare(50, (6, 90)) * 2.0, axis=1).astype(np.float32)
    d2[0] = 4.0
    d2[2, :40] = 1.5
    d2[2, 40:] = np.linspace(2.0, 30.0, 50)
    d2[4, :31] = 0.0  # 31 duplicates of the query: one more than the perplexity
    d2[4, 31:] = np.linspace(0.5, 9.0, 59)
    d2[5] = rng.permutation(d2[2])  # the tied minima in any order
    P, beta, conv, nun = api.calibrate_P(to_dev(d2, dev), 30.0)
    P, beta, conv = P.cpu().numpy(), beta.cpu().numpy(), conv.cpu().numpy()
    Po, _, convo, _ = oracle.calibrate(d2.astype(np.float64), 30.0, tol=1e-5)
    assert conv.tolist() == convo.tolist() == [0, 1, 0, 1, 0, 0]
    assert int(nun.item()) == 4
    assert np.isfinite(P).all() and np.isfinite(beta).all()
    np.testing.assert_allclose(P, Po, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(P[0], 1.0 / 90, rtol=1e-6)
    np.testing.assert_allclose(P[2, :40], 1.0 / 40, rtol=1e-6)
    assert (P[2, 40:] == 0).all()
    np.testing.assert_allclose(P[4, :31], 1.0 / 31, rtol=1e-6)
