"""FP64 reference of principal components by randomized truncated SVD (test
infrastructure only: imported by the tests and nothing else).

Method: randomized subspace iteration with re-orthonormalisation, then the
direct SVD of the small projected matrix (Halko, Martinsson and Tropp 2011,
"Finding structure with randomness", SIAM Review 53, Algorithm 4.4 and
Algorithm 5.1), applied to the column-centred matrix Xc = X - 1 mu^T:

1. Y = Xc Omega (Omega: g x l test matrix, passed in), Q = orth(Y).
2. q times: Q~ = orth(Xc^T Q), Q = orth(Xc Q~).
3. B = Q^T Xc (l x g); B B^T = U diag(s^2) U^T (symmetric eigenproblem,
   eigenvalues in descending order).
4. components V = B^T U diag(1/s) (g x l, orthonormal columns), scores
   Q U diag(s) (n x l) = Xc V when Q spans the range of Xc.

orth(Y) is the Q factor of Y = Q R with R's diagonal positive (unique for
full column rank), here from Householder QR with the signs normalised.
Sign convention of the output (a reading: singular vectors are defined up
to sign): each component is flipped so that its entry of largest magnitude
is positive (the first such entry on ties).
"""
from __future__ import annotations

import numpy as np


def orth(Y):
    """Q of Y = Q R with diag(R) > 0 (n x l, full column rank)."""
    Q, R = np.linalg.qr(np.asarray(Y, dtype=np.float64))
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def randomized_pca(X, k, Omega, q=2):
    """(scores [n, k], components [k, g], singular values [k], mean [g]) of X [n, g]."""
    X = np.asarray(X, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    mu = X.mean(axis=0)
    Xc = X - mu
    Q = orth(Xc @ Omega)
    for _ in range(q):
        Q = orth(Xc @ orth(Xc.T @ Q))
    B = Q.T @ Xc
    w, U = np.linalg.eigh(B @ B.T)
    order = np.argsort(-w, kind="stable")
    w, U = w[order], U[:, order]
    s = np.sqrt(np.maximum(w, 0.0))
    V = (B.T @ U) / s
    scores = Q @ (U * s)
    for c in range(V.shape[1]):
        j = int(np.argmax(np.abs(V[:, c])))
        if V[j, c] < 0:
            V[:, c] = -V[:, c]
            scores[:, c] = -scores[:, c]
    return scores[:, :k], V[:, :k].T, s[:k], mu
