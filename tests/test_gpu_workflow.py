"""The embedding stages end to end (pipeline.run): PCA -> kNN graph -> t-SNE
and UMAP under the monitor, on a small synthetic expression matrix; every
stage appears in the table, the embeddings are finite and have spread out."""
import math

import pytest
import torch

from helpers import say
from paper_2605_13928_amd import pipeline

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("gradient", ["fft", "exact"])
def test_workflow_small(dev, gradient):
    say("workflow", gradient)
    # 300 iterations: the 100 of early exaggeration (which contract the
    # embedding) and 200 in which it spreads out
    out = pipeline.run(cells=6000, genes=300, tsne_iters=300, gradient=gradient, umap_epochs=30, period=0.02,
                       device=dev.index or 0)
    t = out["table"]
    say({k: round(v["seconds"], 4) for k, v in t.items()})
    assert list(t) == ["pca", "knn_graph", "tsne", "umap"]
    assert all(v["seconds"] > 0 for v in t.values())
    assert out["nnz_P"] >= 6000 * 90 and out["nnz_umap_graph"] >= 6000 * 15
    for Y in (out["Y_tsne"], out["Y_umap"]):
        assert torch.isfinite(Y).all() and Y.std().item() > 0.1
    assert out["top_singular_values"][0] > out["top_singular_values"][2] > 0
    assert not math.isnan(out["total_seconds"])
