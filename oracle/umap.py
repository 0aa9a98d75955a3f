"""FP64 reference of the UMAP steps on a kNN graph (test infrastructure only:
imported by the tests and nothing else).

Method: McInnes, Healy & Melville 2018, "UMAP: Uniform Manifold
Approximation and Projection for Dimension Reduction", arXiv:1802.03426
[MHM18].

* Local fuzzy simplicial sets (Sec. 3.1): for point i with neighbour
  distances d_i1..d_ik (Euclidean, self excluded), rho_i = the smallest
  positive d_ij, sigma_i solves sum_j exp(-max(0, d_ij - rho_i) / sigma_i)
  = log2(k), and the directed weight is w_ij = exp(-max(0, d_ij - rho_i) /
  sigma_i).  Reading for degenerate rows (the method does not treat them):
  sigma_i is at least 1e-3 times the mean of the row's distances (1e-3 when
  they are all zero), and stays at that floor when the floor already meets
  the target.
* Fuzzy union (Sec. 3.1): B = A + A^T - A o A^T on the union of the kNN
  patterns (the probabilistic t-conorm), kept as a structural pattern.
* Low-dimensional similarity (Sec. 3.2): Phi(x, y) = (1 + a |x - y|^{2b})^-1
  with a, b the least-squares fit to Psi(d) = 1 for d <= min_dist,
  exp(-(d - min_dist)) beyond.  Reading: the fit uses 300 equispaced d in
  [0, 3].
* Layout (Sec. 3.2, the embedding optimisation): per sampled 1-simplex
  (i, j) an attractive step along d/dy_i log Phi for y_i and the opposite
  step for y_j, and for each of `neg_rate` vertices c drawn uniformly a
  repulsive step along d/dy_i log(1 - Phi) with eps = 1e-3 added to the
  squared distance; every coordinate of a step clipped to [-4, 4]; learning
  rate alpha0 (1 - t / n_epochs) in epoch t.

Readings of the data-parallel epoch (the published algorithm is sequential
SGD, written out as layout_epoch_sequential; these make one epoch a
deterministic function of the epoch's start, and the tests check that both
forms reach the same fuzzy-set cross-entropy and neighbourhood purity):
  - every step of epoch t is evaluated at the positions Y_t and the steps
    are summed: Y_{t+1} = Y_t + sum of steps;
  - schedule: with r_e = w_e / w_max in FP32, stored entry e is sampled in
    epoch t (0-based) when floor((t + 1) r_e) > floor(t r_e), both products
    in FP32, so an entry is sampled floor(n_epochs r_e) times in all;
  - negatives: the p-th draw of entry e in epoch t is vertex
    ((z >> 32) * n) >> 32 with z the SplitMix64 output for counter
    (t nnz + e) neg_rate + p (Steele, Lea & Flood 2014, "Fast splittable
    pseudorandom number generators", OOPSLA: z = mix(seed + (ctr + 1) *
    0x9E3779B97F4A7C15)); a draw equal to i is skipped, as is a coincident
    point (no repulsion at distance 0).
"""
from __future__ import annotations

import numpy as np
from scipy import optimize, sparse

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
EPS_REP = 1e-3
CLIP = 4.0


# --- fitted similarity curve -------------------------------------------------

def psi(d, min_dist):
    """Target membership curve of Sec. 3.2 (spread 1)."""
    d = np.asarray(d, np.float64)
    return np.where(d <= min_dist, 1.0, np.exp(-(d - min_dist)))


def fit_ab(min_dist):
    """(a, b) minimising sum over the 300 fit points of (Phi - Psi)^2."""
    x = np.linspace(0.0, 3.0, 300)
    y = psi(x, min_dist)
    (a, b), _ = optimize.curve_fit(lambda d, a, b: 1.0 / (1.0 + a * d ** (2.0 * b)), x, y, p0=(1.0, 1.0),
                                   maxfev=10000, xtol=1e-14, ftol=1e-14)
    return float(a), float(b)


def fit_objective(a, b, min_dist):
    x = np.linspace(0.0, 3.0, 300)
    return float(np.sum((1.0 / (1.0 + a * x ** (2.0 * b)) - psi(x, min_dist)) ** 2))


# --- local fuzzy simplicial sets ---------------------------------------------

def smooth_knn(dist, k=None):
    """rho [n], sigma [n], w [n, k] from the neighbour distances dist [n, k]
    (Euclidean, FP64)."""
    dist = np.asarray(dist, np.float64)
    n, kk = dist.shape
    k = kk if k is None else k
    target = np.log2(k)
    rho = np.zeros(n)
    sigma = np.zeros(n)
    w = np.zeros((n, kk))
    for i in range(n):
        d = dist[i]
        pos = d[d > 0.0]
        rho[i] = pos.min() if pos.size else 0.0
        x = np.maximum(d - rho[i], 0.0)
        mean = d.mean()
        floor = 1e-3 * mean if mean > 0.0 else 1e-3

        def f(s):
            return np.exp(-x / s).sum() - target

        if f(floor) >= 0.0:
            s = floor
        else:
            hi = max(2.0 * floor, x.max() if x.max() > 0 else 1.0)
            while f(hi) < 0.0:
                hi *= 2.0
            s = optimize.brentq(f, floor, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)
        sigma[i] = s
        w[i] = np.exp(-x / s)
    return rho, sigma, w


# --- fuzzy union ---------------------------------------------------------------

def fuzzy_union(nbr, w, n):
    """CSR (row_ptr int64, col int32, val FP64) of B = A + A^T - A o A^T on the
    union of the kNN patterns, columns ascending."""
    nbr = np.asarray(nbr, np.int64)
    kk = nbr.shape[1]
    rows = np.repeat(np.arange(n, dtype=np.int64), kk)
    cols = nbr.ravel()
    vals = np.asarray(w, np.float64).ravel()
    key = rows * n + cols
    tkey = cols * n + rows
    keys = np.union1d(key, tkey)
    order = np.argsort(key)
    sk, sv = key[order], vals[order]

    def lookup(q):
        pos = np.searchsorted(sk, q)
        pos = np.minimum(pos, sk.size - 1)
        hit = sk[pos] == q
        return np.where(hit, sv[pos], 0.0)

    r, c = keys // n, keys % n
    a = lookup(keys)            # A[r, c]
    at = lookup(c * n + r)      # A[c, r]
    val = a + at - a * at
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, c.astype(np.int32), val


# --- counter-based generator -------------------------------------------------

def splitmix64(seed, ctr):
    """SplitMix64 output number ctr (0-based) of the sequence seeded with seed
    (vectorised over ctr, uint64 wrap-around arithmetic)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(ctr, np.uint64) + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def splitmix64_sequence(seed, count):
    """The same outputs by the generator's sequential definition (state +=
    gamma, output = mix(state))."""
    out = []
    s = int(seed)
    m = (1 << 64) - 1
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & m
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
        out.append(z ^ (z >> 31))
    return out


def draw_vertex(z, n):
    return ((np.asarray(z, np.uint64) >> np.uint64(32)) * np.uint64(n)) >> np.uint64(32)


# --- layout ------------------------------------------------------------------

def sample_mask(val, t):
    """Entries sampled in epoch t; the decision in FP32 (see the module notes)."""
    v = np.asarray(val, np.float32)
    r = v / np.float32(v.max())
    lo = np.floor(np.float32(t) * r)
    hi = np.floor(np.float32(t + 1) * r)
    return hi > lo


def attraction_coef(d2, a, b):
    """c with d/dy_i log Phi(y_i, y_j) = c (y_i - y_j); 0 at d2 = 0."""
    d2 = np.asarray(d2, np.float64)
    safe = np.where(d2 > 0.0, d2, 1.0)
    c = -2.0 * a * b * safe ** (b - 1.0) / (1.0 + a * safe ** b)
    return np.where(d2 > 0.0, c, 0.0)


def repulsion_coef(d2, a, b, eps=EPS_REP):
    """c with d/dy_i log(1 - Phi(y_i, y_c)) ~= c (y_i - y_c), eps added to the
    squared distance; 0 at d2 = 0."""
    d2 = np.asarray(d2, np.float64)
    safe = np.where(d2 > 0.0, d2, 1.0)
    c = 2.0 * b / ((eps + safe) * (1.0 + a * safe ** b))
    return np.where(d2 > 0.0, c, 0.0)


def layout_epoch(Y, row_ptr, col, val, t, n_epochs, a, b, alpha0=1.0, neg_rate=5, seed=0):
    """Y_{t+1} from Y_t [n, 2] for epoch t."""
    Y = np.asarray(Y, np.float64)
    n = Y.shape[0]
    nnz = col.shape[0]
    alpha = alpha0 * (1.0 - t / n_epochs)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    e = np.nonzero(sample_mask(val, t))[0]
    i, j = rows[e], col[e].astype(np.int64)
    delta = np.zeros_like(Y)
    d = Y[i] - Y[j]
    g = np.clip(attraction_coef((d * d).sum(1), a, b)[:, None] * d, -CLIP, CLIP)
    np.add.at(delta, i, alpha * g)
    np.add.at(delta, j, -alpha * g)
    for p in range(neg_rate):
        ctr = (np.uint64(t) * np.uint64(nnz) + e.astype(np.uint64)) * np.uint64(neg_rate) + np.uint64(p)
        c = draw_vertex(splitmix64(seed, ctr), n).astype(np.int64)
        keep = c != i
        ii, cc = i[keep], c[keep]
        d = Y[ii] - Y[cc]
        g = np.clip(repulsion_coef((d * d).sum(1), a, b)[:, None] * d, -CLIP, CLIP)
        np.add.at(delta, ii, alpha * g)
    return Y + delta


def layout(Y0, row_ptr, col, val, n_epochs, a, b, alpha0=1.0, neg_rate=5, seed=0, epochs=None):
    """Epochs [t0, t1) (all of them by default) from Y0."""
    t0, t1 = (0, n_epochs) if epochs is None else epochs
    Y = np.asarray(Y0, np.float64)
    for t in range(t0, t1):
        Y = layout_epoch(Y, row_ptr, col, val, t, n_epochs, a, b, alpha0, neg_rate, seed)
    return Y


def layout_epoch_sequential(Y, row_ptr, col, val, t, n_epochs, a, b, alpha0=1.0, neg_rate=5, seed=0):
    """Epoch t of the layout as the published sequential SGD [MHM18] Sec. 3.2:
    the sampled 1-simplices are visited one after another in storage order,
    and every step moves the points at once, so a later step sees the
    positions the earlier ones left.  Per sampled entry (i, j): the
    attractive step on y_i and its opposite on y_j, then the neg_rate
    repulsive steps of y_i against uniformly drawn vertices.  Sampling
    schedule, draws, coefficients and clipping are those of layout_epoch.
    Plain Python loops: for small graphs only."""
    Y = np.array(Y, np.float64)
    n = Y.shape[0]
    nnz = col.shape[0]
    alpha = alpha0 * (1.0 - t / n_epochs)
    mask = sample_mask(val, t)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    es = np.nonzero(mask)[0]
    ctr = ((np.uint64(t) * np.uint64(nnz) + es.astype(np.uint64))[:, None] * np.uint64(neg_rate)
           + np.arange(neg_rate, dtype=np.uint64)[None, :])
    negs = draw_vertex(splitmix64(seed, ctr), n).astype(np.int64)
    y = Y.tolist()

    def clip(v):
        return min(CLIP, max(-CLIP, v))

    for q, e in enumerate(es.tolist()):
        i, j = int(rows[e]), int(col[e])
        dx, dy = y[i][0] - y[j][0], y[i][1] - y[j][1]
        d2 = dx * dx + dy * dy
        if d2 > 0.0:
            c = -2.0 * a * b * d2 ** (b - 1.0) / (1.0 + a * d2 ** b)
            gx, gy = clip(c * dx), clip(c * dy)
            y[i][0] += alpha * gx
            y[i][1] += alpha * gy
            y[j][0] -= alpha * gx
            y[j][1] -= alpha * gy
        for cv in negs[q].tolist():
            if cv == i:
                continue
            dx, dy = y[i][0] - y[cv][0], y[i][1] - y[cv][1]
            d2 = dx * dx + dy * dy
            if d2 > 0.0:
                c = 2.0 * b / ((EPS_REP + d2) * (1.0 + a * d2 ** b))
                y[i][0] += alpha * clip(c * dx)
                y[i][1] += alpha * clip(c * dy)
    return np.array(y, np.float64)


def layout_sequential(Y0, row_ptr, col, val, n_epochs, a, b, alpha0=1.0, neg_rate=5, seed=0):
    """Every epoch of the sequential form from Y0."""
    Y = np.asarray(Y0, np.float64)
    for t in range(n_epochs):
        Y = layout_epoch_sequential(Y, row_ptr, col, val, t, n_epochs, a, b, alpha0, neg_rate, seed)
    return Y


def fuzzy_cross_entropy(Y, row_ptr, col, val, a, b):
    """The objective the layout minimises [MHM18] Sec. 3.2: the fuzzy-set
    cross-entropy between the graph's membership v (0 off the stored
    pattern) and Phi of the embedding, summed over all unordered pairs
    {i, j}, i != j (a pair stored in both rows counts once, with the value
    of row min(i, j)):
      C = sum v ln(v / Phi) + (1 - v) ln((1 - v) / (1 - Phi)),  0 ln 0 = 0.
    Dense over the n (n - 1) / 2 pairs: small n only.  Phi is kept inside
    [1e-12, 1 - 1e-12] so that a pair at distance 0 or far apart stays
    finite."""
    Y = np.asarray(Y, np.float64)
    n = Y.shape[0]
    V = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    V[rows, col.astype(np.int64)] = np.asarray(val, np.float64)
    iu = np.triu_indices(n, 1)
    v = V[iu]
    d2 = ((Y[iu[0]] - Y[iu[1]]) ** 2).sum(1)
    phi = np.clip(1.0 / (1.0 + a * d2 ** b), 1e-12, 1.0 - 1e-12)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(v > 0.0, v * np.log(np.where(v > 0.0, v, 1.0) / phi), 0.0)
        t2 = np.where(v < 1.0, (1.0 - v) * np.log(np.where(v < 1.0, 1.0 - v, 1.0) / (1.0 - phi)), 0.0)
    return float((t1 + t2).sum())


def to_scipy(row_ptr, col, val, n):
    return sparse.csr_matrix((val, col, row_ptr), shape=(n, n))
