"""tsne_kl_grad_noalloc (the gradient on the library's static device scratch)
against tsne_kl_grad (the same kernels on a caller workspace): identical
bits for the gradient, Z, KL and per-row Z, over consecutive calls whose
sizes shrink, so the later calls run on scratch that still holds the
earlier calls' contents.  The first call is at the largest size the scratch
takes with per-row Z requested."""
import numpy as np
import pytest
import torch

from helpers import random_graph_P, say, sparse_to_dev, to_dev
from paper_2605_13928_amd import _lib, api, synth

pytestmark = pytest.mark.gpu

# (n, alpha, per-row Z): n = 53,248 is the scratch's limit with per-row Z
CALLS = [(53_248, 12.0, True), (20_000, 1.0, False), (4_225, 1.0, True), (3, 12.0, False)]


def test_noalloc_equals_workspace_entry_point(dev):
    for n, alpha, zrow in CALLS:
        say("kl_grad_noalloc", n, alpha, zrow)
        k = min(30, n - 1)
        _, _, _, S = random_graph_P(n, k, min(10.0, k - 0.5), 500 + n)
        P = sparse_to_dev(S, dev)
        Y = to_dev(synth.random_embedding(n, 5.0, 900 + n), dev)
        g0, Z0, kl0, Zr0 = api.kl_grad(Y, P, alpha, want_Z=True, want_kl=True, want_Zrow=zrow)
        g1 = torch.full_like(Y, float("nan"))
        Z1 = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
        kl1 = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
        Zr1 = torch.full((n,), float("nan"), dtype=torch.float64, device=dev) if zrow else None
        nf = api.nonfinite_counter(dev)
        api.kl_grad_noalloc(Y, P, alpha, grad=g1, Z=Z1, kl=kl1, Zrow=Zr1, nonfinite=nf)
        torch.cuda.synchronize()
        assert torch.equal(g0, g1), f"gradient differs at n={n}"
        assert torch.equal(Z0, Z1) and torch.equal(kl0, kl1)
        if zrow:
            assert torch.equal(Zr0, Zr1)
        assert int(nf.item()) == 0
        assert torch.isfinite(g1).all()


def test_noalloc_rejects_problems_beyond_its_scratch(dev):
    n = 92_161  # one point past the limit without per-row Z
    Y = torch.zeros((n, 2), dtype=torch.float32, device=dev)
    P = api.SparseP(torch.zeros(n + 1, dtype=torch.int64, device=dev), torch.zeros(1, dtype=torch.int32, device=dev),
                    torch.zeros(1, dtype=torch.float32, device=dev), None, n)
    with pytest.raises(_lib.TsneError) as e:
        api.kl_grad_noalloc(Y, P, 1.0)
    assert e.value.status == _lib.TSNE_ERR_SCRATCH
