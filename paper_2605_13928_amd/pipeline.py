"""The workflow's embedding stages on one MI355X, end to end.

Stages 5 to 7 of the single-cell workflow that the paper monitors (its
Table 1): PCA of a cells x genes matrix, the kNN graph of the PCA scores,
then t-SNE and UMAP of that graph.  Each stage is marked on the resource
monitor, whose step table gives the stage's time, device memory, GPU
activity and power -- the columns of the paper's table, measured here.

Orchestration only: every stage is C-ABI calls (tsne_pca; tsne_knn, BF16
candidates with an FP32 re-rank; tsne_calibrate_P and tsne_symmetrize;
tsne_kl_grad_fft with tsne_step, or tsne_optimize for the exact gradient;
tsne_umap_*).  UMAP's k = 15 graph is the first 15 columns of t-SNE's
k = 90 lists (they are sorted by distance, so that is the 15-NN graph).

    python -m paper_2605_13928_amd.pipeline --cells 1000000 --genes 2000
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np
import torch

from . import api, monitor, synth, tsne


def run(cells: int = 1_000_000, genes: int = 2000, pcs: int = 50, k: int = 90, k_umap: int = 15,
        perplexity: float = 30.0, tsne_iters: int = 1000, gradient: str = "fft", umap_epochs: int = 200,
        min_dist: float = 0.5, seed: int = 0, period: float = 0.1, device: int = 0) -> dict:
    """Runs the stages on synthetic expression data; returns the per-stage
    table and the two embeddings."""
    if gradient not in ("fft", "exact"):
        raise ValueError("gradient must be 'fft' or 'exact'")
    dev = torch.device("cuda", device)
    X = torch.from_numpy(synth.make_expression(cells, genes, seed)).to(dev)
    om = torch.from_numpy(synth.make_omega(genes, seed + 1)).to(dev)
    w = synth.Workload("pipeline", 0, n=cells, clusters=1, iters=tsne_iters, k=k, perplexity=perplexity)
    ws = api.Workspace()
    torch.cuda.synchronize()
    mon = monitor.Monitor(period=period, device=device)

    def stage(name):
        torch.cuda.synchronize()
        mon.timestamp(name)

    stage("pca")
    scores, _, sv, _ = api.pca(X, pcs, om, q=2, ws=ws)
    del X
    stage("knn_graph")
    idx, d2 = api.knn(scores, k, "bf16", n_cand=2 * k, ws=ws)
    stage("tsne")
    P_cond, _, _, _ = api.calibrate_P(d2, perplexity)
    P = api.symmetrize(idx, P_cond, ws=ws)
    st = tsne.State.start(torch.from_numpy(synth.random_embedding(cells, w.init_std, seed + 2)).to(dev))
    if gradient == "exact":
        tsne.iterate(st, P, w, tsne_iters, ws=ws)
    else:
        wsf = api.Workspace()
        for t in range(tsne_iters):
            alpha, mom = tsne.schedule(w, t)
            api.kl_grad_fft(st.Y, P, alpha, grad=st.grad, ws=wsf)
            api.step(st.Y, st.update, st.gains, st.grad, w.lr, mom)
    stage("umap")
    _, _, wu = api.umap_weights(d2[:, :k_umap].contiguous())
    G = api.umap_fuzzy_union(idx[:, :k_umap].contiguous(), wu, ws=ws)
    a, b = api.umap_fit_ab(min_dist)
    Yu = torch.from_numpy(synth.umap_init(cells, seed + 3)).to(dev)
    api.umap_layout(Yu, G, a, b, umap_epochs, seed=seed, ws=ws)
    torch.cuda.synchronize()
    ses = mon.stop()

    def clean(v):
        return None if isinstance(v, float) and not math.isfinite(v) else v

    table = {r["name"]: {"seconds": r["duration_s"], "samples": r["samples"],
                         "peak_device_memory_gb": clean(r["max_hip_used_bytes"] / 1e9),
                         "mean_gpu_activity_pct": clean(r["mean_gfx_pct"]),
                         "max_power_w": clean(r["max_power_w"])}
             for r in ses.steps if r["name"] != "start"}
    return {"cells": cells, "genes": genes, "pcs": pcs, "k": k, "k_umap": k_umap, "tsne_gradient": gradient,
            "tsne_iters": tsne_iters, "umap_epochs": umap_epochs, "table": table,
            "total_seconds": sum(v["seconds"] for v in table.values()),
            "top_singular_values": [float(v) for v in sv[:3].cpu()], "nnz_P": P.nnz, "nnz_umap_graph": G.nnz,
            "Y_tsne": st.Y, "Y_umap": Yu, "session": ses}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--cells", type=int, default=1_000_000)
    ap.add_argument("--genes", type=int, default=2000)
    ap.add_argument("--tsne-iters", type=int, default=1000)
    ap.add_argument("--gradient", choices=("fft", "exact"), default="fft")
    ap.add_argument("--umap-epochs", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--plot", default=None, help="write the usage plot (SVG) here")
    args = ap.parse_args(argv)
    out = run(args.cells, args.genes, tsne_iters=args.tsne_iters, gradient=args.gradient,
              umap_epochs=args.umap_epochs, seed=args.seed)
    if args.plot:
        monitor.plot_usage(out["session"], args.plot)
    ok = bool(torch.isfinite(out["Y_tsne"]).all() and torch.isfinite(out["Y_umap"]).all())
    rec = {k: v for k, v in out.items() if k not in ("Y_tsne", "Y_umap", "session")}
    rec["embeddings_finite"] = ok
    print(json.dumps(rec), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    raise SystemExit(main())
