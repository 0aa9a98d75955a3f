"""FP64 reference of the interpolation-accelerated t-SNE gradient (test
infrastructure only: imported by the tests and nothing else).

Method: FFT-accelerated polynomial interpolation of the repulsive sums
(Linderman, Rachh, Hoskins, Steinerberger and Kluger 2019, "Fast
interpolation-based t-SNE for improved visualization of single-cell RNA-seq
data", Nat. Methods 16, 243-245), written here from the method's steps:

1. The square domain [lo, lo + B h]^2 around the points is cut into B x B
   boxes of side h; each box holds p x p interpolation nodes at the
   equispaced local positions (k + 1/2) / p, so the nodes of all boxes form
   one uniform grid of N = p B nodes per axis with spacing h / p.
2. Every point spreads its charges q onto the p x p nodes of its box with
   the tensor-product Lagrange weights L_kx(u_x) L_ky(u_y) of its local
   position u in [0, 1]^2.
3. The node potentials are the kernel sums over all node pairs:
   Phi[a] = sum_b K(x_a - x_b) W[b].  The plain definition is the dense
   double sum (`potentials(..., method="direct")`); the same sum as a
   circular convolution of the zero-padded grids by FFT is the fast form
   (`method="fft"`), pinned to the direct one in the tests.
4. Each point interpolates the node potentials back with the same weights.

For t-SNE (van der Maaten and Hinton 2008, eq. 5) the sums needed are
phi1_i = sum_j w_ij and, with centred coordinates z = y - c,
phi2_i = sum_j w_ij^2, phi3_i = sum_j w_ij^2 z_j, so that
R_i = sum_j w_ij^2 (y_i - y_j) = z_i phi2_i - phi3_i and Z = sum_i phi1_i - n
(the j = i terms: w_ii = 1 in phi1; they cancel exactly in R).  Kernels:
K1(d) = 1 / (1 + |d|^2), K2 = K1^2; charges 1 and z_x, z_y.

Grid parameters (readings of the method's settings):
lo = min over both coordinates, range = max - lo (both in the points'
precision), B = clamp(ceil(range / max_box_width), min_boxes, max_fft // (2 p)),
h = range / B (in FP64; range 0 is replaced by 1e-3), box index
b = min(floor((y - lo) / h), B - 1), u = (y - lo) / h - b, FFT size
F = smallest power of two >= 2 N.  The centre is c = lo + range / 2.
"""
from __future__ import annotations

import math

import numpy as np


def grid_params(Y, p=3, min_boxes=50, max_box_width=1.0, max_fft=2048):
    """(lo, h, B, N, F, c) of the interpolation grid for points Y [n, 2]."""
    Y = np.asarray(Y)
    lo = float(min(Y[:, 0].min(), Y[:, 1].min()))
    hi = float(max(Y[:, 0].max(), Y[:, 1].max()))
    rng = hi - lo
    if not rng > 0.0:
        rng = 1e-3
    B = int(math.ceil(rng / max_box_width))
    B = max(B, int(min_boxes))
    B = min(B, int(max_fft) // (2 * p))
    h = rng / B
    N = p * B
    F = 1
    while F < 2 * N:
        F *= 2
    return lo, h, B, N, F, lo + 0.5 * rng


def lagrange_weights(u, p):
    """L_k(u) for the p equispaced local nodes t_k = (k + 1/2) / p; u [m] -> [m, p]."""
    u = np.asarray(u, dtype=np.float64)
    t = (np.arange(p) + 0.5) / p
    L = np.ones((u.shape[0], p))
    for k in range(p):
        for m in range(p):
            if m != k:
                L[:, k] *= (u - t[m]) / (t[k] - t[m])
    return L


def boxes(Y, lo, h, B):
    """Box indices [n, 2] and local positions u [n, 2] of the points."""
    t = (np.asarray(Y, dtype=np.float64) - lo) / h
    b = np.minimum(np.floor(t), B - 1).astype(np.int64)
    b = np.maximum(b, 0)
    return b, t - b


def spread(Y, q, lo, h, B, p):
    """Node charges W [c, N, N] from point charges q [n, c]."""
    n = Y.shape[0]
    N = p * B
    b, u = boxes(Y, lo, h, B)
    Lx = lagrange_weights(u[:, 0], p)
    Ly = lagrange_weights(u[:, 1], p)
    q = np.asarray(q, dtype=np.float64).reshape(n, -1)
    W = np.zeros((q.shape[1], N, N))
    for kx in range(p):
        for ky in range(p):
            gx = p * b[:, 0] + kx
            gy = p * b[:, 1] + ky
            wgt = Lx[:, kx] * Ly[:, ky]
            for c in range(q.shape[1]):
                np.add.at(W[c], (gx, gy), wgt * q[:, c])
    return W


def kernel_values(dx, dy, delta, which):
    """K1 = 1 / (1 + r^2) or K2 = K1^2 at node offsets (dx, dy) * delta."""
    k1 = 1.0 / (1.0 + (delta * dx) ** 2 + (delta * dy) ** 2)
    return k1 if which == 1 else k1 * k1


def potentials(W, delta, which, method="direct", F=None):
    """Phi [c, N, N] = sum over node pairs of K(x_a - x_b) W[c, b]."""
    C, N, _ = W.shape
    if method == "direct":
        g = np.arange(N)
        ax, ay = np.meshgrid(g, g, indexing="ij")
        ax, ay = ax.ravel(), ay.ravel()
        K = kernel_values(ax[:, None] - ax[None, :], ay[:, None] - ay[None, :], delta, which)
        return np.stack([(K @ W[c].ravel()).reshape(N, N) for c in range(C)])
    # circular convolution of the zero-padded grids (F >= 2 N - 1)
    F = F or 2 * N
    off = np.arange(F)
    d = np.where(off < N, off, np.where(off > F - N, off - F, 0))
    valid = (off < N) | (off > F - N)
    dx, dy = np.meshgrid(d, d, indexing="ij")
    Kg = kernel_values(dx, dy, delta, which) * (valid[:, None] & valid[None, :])
    Kf = np.fft.fft2(Kg)
    out = []
    for c in range(C):
        Wp = np.zeros((F, F))
        Wp[:N, :N] = W[c]
        out.append(np.real(np.fft.ifft2(np.fft.fft2(Wp) * Kf))[:N, :N])
    return np.stack(out)


def interpolate(Y, Phi, lo, h, B, p):
    """Point values [n, c] of node potentials Phi [c, N, N]."""
    b, u = boxes(Y, lo, h, B)
    Lx = lagrange_weights(u[:, 0], p)
    Ly = lagrange_weights(u[:, 1], p)
    out = np.zeros((Y.shape[0], Phi.shape[0]))
    for kx in range(p):
        for ky in range(p):
            gx = p * b[:, 0] + kx
            gy = p * b[:, 1] + ky
            out += (Lx[:, kx] * Ly[:, ky])[:, None] * Phi[:, gx, gy].T
    return out


def repulsion(Y, p=3, min_boxes=50, max_box_width=1.0, max_fft=2048, method="fft"):
    """Interpolated (R [n, 2], Z) of the t-SNE repulsion; Y [n, 2] (any float type)."""
    Y32 = np.asarray(Y)
    lo, h, B, N, F, c = grid_params(Y32, p, min_boxes, max_box_width, max_fft)
    Y = Y32.astype(np.float64)
    n = Y.shape[0]
    z = Y - c
    delta = h / p
    W = spread(Y, np.column_stack([np.ones(n), z]), lo, h, B, p)   # charges 1, z_x, z_y
    P1 = potentials(W[:1], delta, 1, method, F)                     # K1 * 1
    P2 = potentials(W, delta, 2, method, F)                         # K2 * (1, z_x, z_y)
    v = interpolate(Y, np.concatenate([P1, P2]), lo, h, B, p)
    phi1, phi2, phi3 = v[:, 0], v[:, 1], v[:, 2:4]
    R = z * phi2[:, None] - phi3
    Z = float(phi1.sum() - n)
    return R, Z


def attraction(Y, P):
    """A_i = sum over stored entries (i, j) of p_ij w_ij (y_i - y_j) (CSR P)."""
    Y = np.asarray(Y, dtype=np.float64)
    n = Y.shape[0]
    rows = np.repeat(np.arange(n), np.diff(P.row_ptr))
    d = Y[rows] - Y[P.col]
    w = 1.0 / (1.0 + (d * d).sum(1))
    A = np.zeros((n, 2))
    np.add.at(A, rows, (P.val * w)[:, None] * d)
    return A


def kl_grad(Y, P, alpha=1.0, p=3, min_boxes=50, max_box_width=1.0, max_fft=2048, method="fft"):
    """(grad [n, 2], Z, KL) with the interpolated repulsion: g = 4 (alpha A - R / Z),
    KL = sum p ln p - sum p ln w + S ln Z over the stored entries."""
    R, Z = repulsion(Y, p, min_boxes, max_box_width, max_fft, method)
    A = attraction(Y, P)
    g = 4.0 * (alpha * A - R / Z)
    Yd = np.asarray(Y, dtype=np.float64)
    rows = np.repeat(np.arange(Yd.shape[0]), np.diff(P.row_ptr))
    d = Yd[rows] - Yd[P.col]
    lnw = -np.log1p((d * d).sum(1))
    pv = P.val
    plp = np.where(pv > 0, pv * np.log(np.where(pv > 0, pv, 1.0)), 0.0).sum()
    kl = float(plp - (pv * lnw).sum() + pv.sum() * math.log(Z))
    return g, Z, kl
