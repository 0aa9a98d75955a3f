"""GPU parity of the differentiation form: KLDivergence forward/backward.

FP64 gradcheck at n = 64 (sparse k = 30 with perplexity 10, and dense
k = 63) and FP32 forward/backward against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import random_graph_P, rel, say, sparse_to_dev, to_dev
from paper_2605_13928_amd import api, synth
from paper_2605_13928_amd.autograd import KLDivergence

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,perp", [(30, 10.0), (63, 20.0)])
def test_gradcheck_fp64_n64(dev, k, perp):
    say("gradcheck n=64", k)
    X, _ = synth.make_points("c4", n=64)
    idx, d2 = oracle.knn(X, k)
    Pc, _, _, _ = oracle.calibrate(d2, perp)
    S = oracle.symmetrize(idx, Pc)
    P = sparse_to_dev(S, dev, torch.float64)
    # general positive values on the symmetric pattern, of order 1/nnz, so
    # the absolute FD step stays far below every value
    rng = np.random.default_rng(k)
    vals = rng.uniform(0.5, 1.5, S.nnz) / S.nnz
    val = torch.tensor(vals, dtype=torch.float64, device=dev, requires_grad=True)
    Y = torch.tensor(synth.random_embedding(64, 1.0, k), dtype=torch.float64, device=dev, requires_grad=True)
    assert torch.autograd.gradcheck(lambda y, v: KLDivergence.apply(y, v, P), (Y, val), eps=1e-7, atol=1e-6,
                                    rtol=1e-5)


def forward_backward(dev, S, Y32, gC=1.0, perturb_seed=None, dtype=torch.float32):
    vals = S.val if perturb_seed is None else S.val * np.random.default_rng(perturb_seed).uniform(0.5, 1.5, S.nnz)
    v32 = vals.astype(np.float32) if dtype == torch.float32 else vals
    P = sparse_to_dev(S, dev, dtype)
    Yt = to_dev(Y32, dev, dtype).requires_grad_(True)
    vt = to_dev(v32, dev, dtype).requires_grad_(True)
    C = KLDivergence.apply(Yt, vt, P)
    C.backward(torch.tensor(gC, dtype=dtype, device=dev))
    So = oracle.CSR(S.row_ptr, S.col, v32.astype(np.float64), S.tpos)
    Co, Zo = oracle.kl(Y32.astype(np.float64), So)
    dYo, dPo = oracle.kl_backward(Y32.astype(np.float64), So, gC)
    return C.item(), Co, Yt.grad.cpu().numpy(), dYo, vt.grad.cpu().numpy(), dPo


@pytest.mark.parametrize("n", [500, 3001])
def test_fp32_forward_backward_vs_oracle(dev, n):
    say("autograd fp32", n)
    idx, d2, Pc, S = random_graph_P(n, 30, 10.0, n)
    Y = synth.random_embedding(n, 3.0, n)
    C, Co, dY, dYo, dP, dPo = forward_backward(dev, S, Y, gC=0.7, perturb_seed=1)
    assert abs(C - Co) <= 1e-5 * max(1.0, abs(Co))
    assert rel(dY, dYo) <= 1e-4
    assert rel(dP, dPo) <= 1e-5


def test_fp32_c4_full_size(dev):
    # n = 50,000, Y ~ N(0, I), P on a k = 90 pattern
    say("autograd c4 full")
    n = 50_000
    idx, d2, Pc, S = random_graph_P(n, 90, 30.0, 4)
    Y = synth.make_init("c4")
    C, Co, dY, dYo, dP, dPo = forward_backward(dev, S, Y)
    assert abs(C - Co) <= 1e-5 * max(1.0, abs(Co))
    assert rel(dY, dYo) <= 1e-4
    assert rel(dP, dPo) <= 1e-5
    # symmetric, normalised P: dC/dY is the t-SNE gradient
    g, _, _ = oracle.kl_grad(Y.astype(np.float64), oracle.CSR(S.row_ptr, S.col, S.val.astype(np.float32).astype(np.float64)), 1.0, want_kl=False)
    assert rel(dY, g) <= 1e-4


def test_fp64_forward_backward_tight(dev):
    say("autograd fp64")
    n = 700
    idx, d2, Pc, S = random_graph_P(n, 30, 10.0, 7)
    Y = synth.random_embedding(n, 2.0, 7).astype(np.float64)
    C, Co, dY, dYo, dP, dPo = forward_backward(dev, S, Y, gC=-1.3, perturb_seed=2, dtype=torch.float64)
    assert abs(C - Co) <= 1e-10 * max(1.0, abs(Co))
    assert rel(dY, dYo) <= 1e-10
    assert rel(dP, dPo) <= 1e-10


@pytest.mark.parametrize("n", [3001, 40_000, 70_001])
def test_fp32_forward_Z_and_kl_match_the_gradient_pass(dev, n):
    # The FP32 forward takes Z from the Z-only symmetric pass; the gradient
    # pass sums the same weights with its own kernel.  Sizes cover the three
    # superblock widths (256, 512, 1024 points) with ragged last superblocks.
    say("autograd fp32 Z vs gradient pass", n)
    idx, d2, Pc, S = random_graph_P(n, 30, 10.0, 7 + n % 13)
    P = sparse_to_dev(S, dev)
    Y = to_dev(synth.random_embedding(n, 4.0, 11 + n % 7), dev)
    C, Zf = api.kl_forward(Y, P.val, P)
    _, Zg, klg, _ = api.kl_grad(Y, P, 1.0, want_Z=True, want_kl=True)
    assert abs(Zf.item() - Zg.item()) <= 1e-6 * Zg.item()
    assert abs(C.item() - klg.item()) <= 1e-5 * max(1.0, abs(klg.item()))
