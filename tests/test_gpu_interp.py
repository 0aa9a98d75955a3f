"""GPU parity: tsne_kl_grad_fft (repulsion and Z by FFT-accelerated
interpolation) against the FP64 oracle of the same scheme
(oracle/interp.py) -- near-exact agreement, since both take the same grid,
boxes and weights -- and against the exact gradient within the scheme's
approximation error, which falls with the box side."""
import numpy as np
import pytest
import torch

import oracle
from helpers import random_graph_P, rel, say, sparse_to_dev, to_dev
from oracle import interp as I
from paper_2605_13928_amd import api, synth

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-4  # FP32 output and FP32 attraction terms, as for tsne_kl_grad


def widen(S):
    return oracle.CSR(S.row_ptr, S.col, S.val.astype(np.float32).astype(np.float64), S.tpos)


def gpu_fft(dev, Y, So, alpha, **kw):
    g, Z, kl = api.kl_grad_fft(to_dev(Y, dev), sparse_to_dev(So, dev), alpha, want_Z=True, want_kl=True, **kw)
    return g.cpu().numpy().astype(np.float64), Z.item(), kl.item()


# (n, Y std, alpha, p, min_boxes, max_box_width, max_fft)
CASES = [
    (500, 3.0, 12.0, 3, 50, 1.0, 2048),
    (2000, 10.0, 1.0, 2, 20, 0.5, 1024),
    (3001, 20.0, 1.0, 4, 10, 1.0, 2048),
    (4000, 40.0, 1.0, 5, 8, 2.0, 512),      # B capped at max_fft / (2 p) = 51
    (1500, 0.01, 12.0, 3, 50, 1.0, 2048),   # the scale of early iterations: B = min_boxes
    (777, 5.0, 1.0, 3, 1, 0.25, 64),        # the smallest FFT: B = 10, F = 64
]


@pytest.mark.parametrize("case", CASES)
def test_fft_grad_matches_interp_oracle(dev, case):
    n, ystd, alpha, p, mb, mw, mf = case
    say("fft grad vs interp oracle", case)
    _, _, _, S = random_graph_P(n, 30, 10.0, 7)
    So = widen(S)
    Y = synth.random_embedding(n, ystd, 3000 + n)
    g, Z, kl = gpu_fft(dev, Y, So, alpha, n_interp=p, min_boxes=mb, max_box_width=mw, max_fft=mf)
    go, Zo, klo = I.kl_grad(Y, So, alpha, p=p, min_boxes=mb, max_box_width=mw, max_fft=mf)
    e = rel(g, go)
    assert e <= GRAD_RTOL, e
    assert abs(Z - Zo) <= 1e-9 * Zo
    assert abs(kl - klo) <= 1e-5 * max(1.0, abs(klo))


def test_fft_grad_deterministic(dev):
    say("fft grad determinism")
    n = 20_000
    _, _, _, S = random_graph_P(n, 90, 30.0, 2)
    P = sparse_to_dev(widen(S), dev)
    Y = to_dev(synth.random_embedding(n, 15.0, 4100), dev)
    a, Za, _ = api.kl_grad_fft(Y, P, 1.0, want_Z=True)
    b, Zb, _ = api.kl_grad_fft(Y, P, 1.0, want_Z=True)
    assert torch.equal(a, b) and torch.equal(Za, Zb)


def test_fft_grad_same_bits_in_either_row_order(dev):
    """The attraction pass takes the rows in box order unless the KL is asked
    for (then in index order); a row's sum must not depend on which rows
    share its block, so the gradient and Z come out bit for bit the same.
    With k = 90 a block's 16 rows hold about 2,900 entries, so rows straddle
    the 2,048-entry chunks in both orders."""
    say("fft grad: box order vs index order")
    n = 20_000
    _, _, _, S = random_graph_P(n, 90, 30.0, 3)
    P = sparse_to_dev(widen(S), dev)
    Y = to_dev(synth.random_embedding(n, 15.0, 4101), dev)
    a, Za, _ = api.kl_grad_fft(Y, P, 1.0, want_Z=True)
    b, Zb, klb = api.kl_grad_fft(Y, P, 1.0, want_Z=True, want_kl=True)
    assert torch.equal(a, b) and torch.equal(Za, Zb)
    assert torch.isfinite(klb).all()


def test_fft_grad_close_to_exact_c2(dev):
    # the approximation against the exact gradient at 20k points: about 1e-2
    # relative at box side 1 (the method's default), third order below it
    say("fft grad vs exact c2")
    n = 20_000
    _, _, _, S = random_graph_P(n, 90, 30.0, 2)
    P = sparse_to_dev(widen(S), dev)
    for ystd, alpha in ((0.01, 12.0), (20.0, 1.0)):
        Y = to_dev(synth.random_embedding(n, ystd, 4000 + int(ystd)), dev)
        ge, Ze, _, _ = api.kl_grad(Y, P, alpha, want_Z=True)
        ge = ge.cpu().numpy()
        errs = []
        for mw in (1.0, 0.5, 0.25):
            gf, Zf, _ = api.kl_grad_fft(Y, P, alpha, max_box_width=mw, max_fft=4096, want_Z=True)
            errs.append((rel(gf.cpu().numpy(), ge), abs(Zf.item() - Ze.item()) / Ze.item()))
        say("errors vs exact", ystd, errs)
        assert errs[0][0] <= 5e-2 and errs[0][1] <= 2e-3, errs
        assert errs[-1][0] <= 2e-3 and errs[-1][1] <= 1e-4, errs
        if ystd > 1.0:  # (a tiny embedding has B = min_boxes for every width)
            assert errs[-1][0] < errs[0][0] / 8, errs


def test_fft_grad_degenerate(dev):
    say("fft grad degenerate inputs")
    # all points at one position: R = 0, Z = n (n - 1), A = 0
    n = 300
    _, _, _, S = random_graph_P(n, 10, 3.0, 9)
    P = sparse_to_dev(widen(S), dev)
    Y = to_dev(np.full((n, 2), 1.25, np.float32), dev)
    g, Z, kl = api.kl_grad_fft(Y, P, 1.0, want_Z=True, want_kl=True)
    assert torch.isfinite(g).all() and g.abs().max().item() < 1e-6
    assert abs(Z.item() - n * (n - 1)) <= 1e-6 * n * n
    # two points: for P = [[0, 1/2], [1/2, 0]] the attraction and the
    # repulsion cancel up to the interpolation error, so the gradient is a
    # small difference of two terms; compare it on the scale of those terms
    S2 = oracle.CSR(np.array([0, 1, 2]), np.array([1, 0], np.int32), np.array([0.5, 0.5]))
    Y2 = np.array([[0.3, -1.2], [2.0, 0.7]], np.float32)
    g2, Z2, kl2 = api.kl_grad_fft(to_dev(Y2, dev), sparse_to_dev(S2, dev), 1.0, want_Z=True, want_kl=True)
    go, Zo, klo = I.kl_grad(Y2, S2, 1.0)
    scale = 4.0 * np.abs(I.attraction(Y2, S2)).max()
    assert np.abs(g2.cpu().numpy() - go).max() <= 1e-6 * scale
    assert abs(Z2.item() - Zo) <= 1e-9 * Zo


def test_fft_grad_c5_full_size(dev):
    # n = 1,000,000 (the c5 size): the whole repulsion against the oracle of
    # the same scheme, the attraction on a seeded sample of rows against the
    # C oracle's exact sums
    say("fft grad c5")
    n = 1_000_000
    _, _, _, S = random_graph_P(n, 90, 30.0, 5)
    So = widen(S)
    Y = synth.random_embedding(n, 30.0, 2005)
    g, Z, _ = gpu_fft(dev, Y, So, 1.0)
    Ro, Zo = I.repulsion(Y)
    assert abs(Z - Zo) <= 1e-9 * Zo
    rows = np.random.default_rng(5).choice(n, 192, replace=False)
    _, _, Ao = oracle.grad_rows(Y.astype(np.float64), rows, So)
    go = 4.0 * (Ao - Ro[rows] / Zo)
    e = rel(g[rows], go)
    assert e <= GRAD_RTOL, e


def test_fft_grad_clustered_embedding(dev):
    # 95% of 200,000 points in one tight cluster, the rest spread: most
    # points share a few boxes, whose node sums are split into chunks
    say("fft grad clustered")
    n = 200_000
    _, _, _, S = random_graph_P(n, 30, 10.0, 17)
    So = widen(S)
    rng = np.random.default_rng(18)
    Y = np.where(rng.random((n, 1)) < 0.95, rng.normal(0.0, 0.01, (n, 2)), rng.normal(0.0, 20.0, (n, 2)))
    Y = Y.astype(np.float32)
    g, Z, kl = gpu_fft(dev, Y, So, 1.0)
    go, Zo, klo = I.kl_grad(Y, So, 1.0)
    assert rel(g, go) <= GRAD_RTOL, rel(g, go)
    assert abs(Z - Zo) <= 1e-9 * Zo
    g2, Z2, _ = gpu_fft(dev, Y, So, 1.0)
    assert np.array_equal(g, g2) and Z == Z2
