"""Seeded synthetic inputs for the t-SNE hot path.

This module draws random numbers only: point clouds shaped like the
single-cell workloads (PCA scores of a clustered cell population), initial
embeddings, and random neighbour graphs used as inputs to the calibration
and symmetrisation stages.  It holds none of the method's arithmetic, so
both the HIP path and the FP64 CPU oracle can take their inputs from it.

The paper profiles t-SNE on PCA scores of 1M mouse-brain cells (Section 3.3,
Data; Table 1, row 7); that dataset is not available, so every workload is a
seeded Gaussian mixture of the same shape instead.  All draws use NumPy's
PCG64 generator.  Data seed = 1000 + c, embedding-init seed = 2000 + c for
workload number c.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "make_points",
    "make_init",
    "random_embedding",
    "random_knn_graph",
    "make_expression",
    "make_omega",
    "sha256",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One workload: point cloud recipe plus the t-SNE schedule run on it."""

    name: str
    number: int
    n: int
    d: int = 50
    clusters: int = 10
    weights: str = "equal"  # "equal" | "dirichlet" | "lognormal"
    shape: str = "isotropic"  # "isotropic" | "pca" (variance decaying as 1/d)
    perplexity: float = 30.0
    k: int = 90
    iters: int = 1000
    lr: float = 200.0
    exaggeration: float = 12.0
    exaggeration_iters: int = 100
    momentum_early: float = 0.5
    momentum_late: float = 0.8
    init_std: float = 0.01  # N(0, 1e-4 I): standard deviation 0.01
    knn: str = "fp32"  # "fp32" exact | "bf16" MFMA candidates + FP32 re-rank
    candidates: int = 180

    @property
    def data_seed(self) -> int:
        return 1000 + self.number

    @property
    def init_seed(self) -> int:
        return 2000 + self.number


WORKLOADS = {
    # Plain exact t-SNE on a small balanced mixture.
    "c1": Workload("c1", 1, n=1_500, clusters=10, iters=250),
    # FP32 exact t-SNE, uneven cluster sizes.
    "c2": Workload("c2", 2, n=20_000, clusters=20, weights="dirichlet", iters=1000),
    # Precision form: BF16 candidate kNN re-ranked in FP32.
    "c3": Workload("c3", 3, n=200_000, clusters=30, knn="bf16", iters=0),
    # Differentiation form: embedding drawn N(0, I).
    "c4": Workload("c4", 4, n=50_000, clusters=30, iters=0, init_std=1.0),
    # Full scale: PCA-score-like spectrum, log-normal cluster sizes.
    "c5": Workload("c5", 5, n=1_000_000, clusters=30, weights="lognormal", shape="pca",
                   knn="bf16", iters=1000),
}


def _weights(w: Workload, rng: np.random.Generator) -> np.ndarray:
    if w.weights == "equal":
        return np.full(w.clusters, 1.0 / w.clusters)
    if w.weights == "dirichlet":
        return rng.dirichlet(np.ones(w.clusters))
    if w.weights == "lognormal":
        z = rng.standard_normal(w.clusters)
        e = np.exp(z)
        return e / e.sum()
    raise ValueError(f"unknown weights {w.weights!r}")


def make_points(w: Workload | str, n: int | None = None, seed: int | None = None):
    """Return (X float32 [n, d] C-contiguous, labels int32 [n]).

    Cluster centres are N(0, 25 I) and noise N(0, I) for the isotropic shape;
    for the "pca" shape dimension j (1-based) has centre variance 25/j and
    noise variance 1/j.  Labels are drawn i.i.d. from the cluster weights, so
    row order is random with respect to cluster.  `n` overrides the
    workload's point count (same recipe, fewer points) for small tests.
    """
    if isinstance(w, str):
        w = WORKLOADS[w]
    n = w.n if n is None else int(n)
    rng = np.random.Generator(np.random.PCG64(w.data_seed if seed is None else seed))
    pi = _weights(w, rng)
    if w.shape == "isotropic":
        centre_sd = np.full(w.d, 5.0)
        noise_sd = np.ones(w.d)
    elif w.shape == "pca":
        j = np.arange(1, w.d + 1, dtype=np.float64)
        centre_sd = np.sqrt(25.0 / j)
        noise_sd = np.sqrt(1.0 / j)
    else:
        raise ValueError(f"unknown shape {w.shape!r}")
    centres = rng.standard_normal((w.clusters, w.d)) * centre_sd
    labels = rng.choice(w.clusters, size=n, p=pi).astype(np.int32)
    X = centres[labels] + rng.standard_normal((n, w.d)) * noise_sd
    return np.ascontiguousarray(X, dtype=np.float32), labels


def make_init(w: Workload | str, n: int | None = None, seed: int | None = None) -> np.ndarray:
    """Initial 2-D embedding Y0 ~ N(0, init_std^2 I), float32 [n, 2]."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    n = w.n if n is None else int(n)
    rng = np.random.Generator(np.random.PCG64(w.init_seed if seed is None else seed))
    Y = rng.standard_normal((n, 2)) * w.init_std
    return np.ascontiguousarray(Y, dtype=np.float32)


def random_embedding(n: int, std: float, seed: int) -> np.ndarray:
    """Y ~ N(0, std^2 I), float32 [n, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.standard_normal((n, 2)) * std, dtype=np.float32)


def random_knn_graph(n: int, k: int, seed: int, scale: float = 100.0):
    """A random directed k-regular graph shaped like a kNN result.

    Returns (nbr_idx int32 [n, k], nbr_d2 float32 [n, k]): each row lists k
    distinct neighbours j != i and non-decreasing positive "squared
    distances" (sorted chi-square-like draws).  Used as seeded input for the
    calibration and symmetrisation stages at sizes where an exact kNN on the
    host would take too long.
    """
    if k >= n:
        raise ValueError("need k < n")
    rng = np.random.Generator(np.random.PCG64(seed))
    # Draw k offsets in [1, n) per row, i.e. neighbours (i + off) mod n != i;
    # rows that drew a repeated offset are redrawn until all are distinct.
    off = rng.integers(1, n, size=(n, k))
    while True:
        s = np.sort(off, axis=1)
        bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
        if bad.size == 0:
            break
        for i in bad:
            off[i] = rng.choice(np.arange(1, n), size=k, replace=False)
    idx = (np.arange(n, dtype=np.int64)[:, None] + off) % n
    d2 = np.sort(rng.chisquare(50, size=(n, k)) * (scale / 50.0), axis=1)
    return np.ascontiguousarray(idx, dtype=np.int32), np.ascontiguousarray(d2, dtype=np.float32)


def umap_init(n: int, seed: int, half_width: float = 10.0) -> np.ndarray:
    """A random 2-D starting layout for UMAP: uniform on [-half_width, half_width]^2, float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-half_width, half_width, size=(n, 2)).astype(np.float32)


def make_expression(n: int, g: int, seed: int, latent: int = 64, top: float = 100.0, bottom: float = 1.0,
                    noise: float = 0.05, offset: float = 2.0) -> np.ndarray:
    """Expression-like X [n, g] float32 (the input of the PCA step): cells with
    `latent` hidden factors of geometrically decaying scale (top .. bottom),
    mapped to g genes by an orthonormal loading matrix, plus i.i.d. N(0,
    noise^2) and a constant offset; a smooth spectrum over a noise floor."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scales = np.geomspace(top, bottom, latent)
    Lat = (rng.standard_normal((n, latent)) * scales).astype(np.float32)
    F = np.linalg.qr(rng.standard_normal((g, latent)))[0].T.astype(np.float32)  # latent x g, orthonormal rows
    X = Lat @ F
    X += offset
    X += (rng.standard_normal((n, g)) * noise).astype(np.float32)
    return np.ascontiguousarray(X, dtype=np.float32)


def make_omega(g: int, seed: int, width: int = 64) -> np.ndarray:
    """Gaussian test matrix Omega [g, width] float32 of the randomized PCA."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.standard_normal((g, width)), dtype=np.float32)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
