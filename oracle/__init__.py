"""FP64 CPU oracle for the exact t-SNE hot path (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It wraps `liboracle.so`, built from
`tsne_oracle.c` by `oracle/build.py`, through ctypes on NumPy arrays.  It
shares no code with the HIP library under test.

Each wrapper cites the definition it evaluates; the definitions themselves
are written out in `tsne_oracle.c`.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def _opt(p):
    """Nullable pointer argument: ctypes.c_void_p of a C-contiguous array or None."""
    return None if p is None else p.ctypes.data_as(C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b

            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.oracle_num_threads.restype = C.c_int
        L.oracle_knn.argtypes = [_f32p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_int64, _i32p, _f64p]
        L.oracle_knn_bf16_points.argtypes = L.oracle_knn.argtypes
        L.oracle_pair_d2.argtypes = [_f32p, C.c_int64, C.c_int32, _i64p, _i64p, C.c_int64, _f64p]
        L.oracle_calibrate.argtypes = [_f64p, C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_int32, _f64p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_symmetrize.argtypes = [_i32p, _f64p, C.c_int64, C.c_int32, _i64p, _i32p, _f64p, C.c_void_p,
                                        C.c_void_p]
        L.oracle_kl_grad.argtypes = [_f64p, C.c_int64, _i64p, _i32p, _f64p, C.c_double, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
        L.oracle_grad_rows.argtypes = [_f64p, C.c_int64, _i64p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_grad_rows_scale.argtypes = [_f64p, C.c_int64, _i64p, C.c_int64, C.c_void_p, C.c_void_p,
                                             C.c_void_p, _f64p, _f64p]
        L.oracle_kl.argtypes = [_f64p, C.c_int64, _i64p, _i32p, _f64p, C.c_void_p, C.c_void_p]
        L.oracle_kl_backward.argtypes = [_f64p, C.c_int64, _i64p, _i32p, _f64p, C.c_double, C.c_void_p, C.c_void_p]
        L.oracle_step.argtypes = [_f64p, _f64p, _f64p, _f64p, C.c_int64, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_double]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def knn(X, k, rows=None, bf16_points=False):
    """Exact kNN by FP64 direct differences; keys (d, j) ascending, self excluded.

    Returns (idx int32 [m, k], d2 float64 [m, k]) for the query rows `rows`
    (all rows when None).  bf16_points=True evaluates the same definition on
    the points rounded to bfloat16 (round-to-nearest-even).
    """
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    if rows is None:
        m, rp = n, None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        m, rp = rows.shape[0], rows
    idx = np.empty((m, k), dtype=np.int32)
    d2 = np.empty((m, k), dtype=np.float64)
    f = lib().oracle_knn_bf16_points if bf16_points else lib().oracle_knn
    _check(f(X, n, d, k, _opt(rp), m, idx, d2), "knn")
    return idx, d2


def pair_d2(X, qi, cj):
    """FP64 squared distances of the (qi[t], cj[t]) pairs."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    qi = np.ascontiguousarray(qi, dtype=np.int64).ravel()
    cj = np.ascontiguousarray(cj, dtype=np.int64).ravel()
    out = np.empty(qi.shape[0], dtype=np.float64)
    _check(lib().oracle_pair_d2(X, X.shape[0], X.shape[1], qi, cj, qi.shape[0], out), "pair_d2")
    return out


def calibrate(nbr_d2, perplexity, tol=1e-13, max_iter=200):
    """Per-row beta with entropy ln(perplexity) nats, by bisection.

    Returns (P_cond float64 [n, k], beta float64 [n], converged uint8 [n],
    H float64 [n]).
    """
    d = np.ascontiguousarray(nbr_d2, dtype=np.float64)
    n, k = d.shape
    P = np.empty((n, k), dtype=np.float64)
    beta = np.empty(n, dtype=np.float64)
    conv = np.empty(n, dtype=np.uint8)
    H = np.empty(n, dtype=np.float64)
    _check(lib().oracle_calibrate(d, n, k, perplexity, tol, max_iter, P, _opt(beta), _opt(conv), _opt(H)),
           "calibrate")
    return P, beta, conv, H


class CSR:
    """Symmetric sparse P: row_ptr int64 [n+1], col int32, val float64, tpos int32."""

    def __init__(self, row_ptr, col, val, tpos=None):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.tpos = None if tpos is None else np.ascontiguousarray(tpos, dtype=np.int32)

    @property
    def n(self):
        return self.row_ptr.shape[0] - 1

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def rows(self):
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def dense(self):
        D = np.zeros((self.n, self.n))
        D[self.rows(), self.col] = self.val
        return D


def symmetrize(nbr_idx, P_cond):
    """P = (C + C^T) / (2n) on the union pattern; CSR with sorted columns and tpos."""
    idx = np.ascontiguousarray(nbr_idx, dtype=np.int32)
    Pc = np.ascontiguousarray(P_cond, dtype=np.float64)
    n, k = idx.shape
    cap = 2 * n * k
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(cap, dtype=np.int32)
    val = np.empty(cap, dtype=np.float64)
    tpos = np.empty(cap, dtype=np.int32)
    nnz = np.zeros(1, dtype=np.int64)
    _check(lib().oracle_symmetrize(idx, Pc, n, k, row_ptr, col, val, _opt(tpos), _opt(nnz)), "symmetrize")
    m = int(nnz[0])
    return CSR(row_ptr, col[:m].copy(), val[:m].copy(), tpos[:m].copy())


def kl_grad(Y, P: CSR, alpha=1.0, want_grad=True, want_kl=True):
    """t-SNE gradient 4 sum_j (alpha p_ij - q_ij) w_ij (y_i - y_j), plus Z and KL(P||Q).

    Returns (grad float64 [n, 2] or None, Z, KL or None).
    """
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    n = Y.shape[0]
    grad = np.empty((n, 2), dtype=np.float64) if want_grad else None
    Z = np.zeros(1)
    kl = np.zeros(1) if want_kl else None
    _check(lib().oracle_kl_grad(Y, n, P.row_ptr, P.col, P.val, alpha, _opt(grad), _opt(Z), _opt(kl)), "kl_grad")
    return grad, float(Z[0]), (None if kl is None else float(kl[0]))


def grad_rows(Y, rows, P: CSR | None = None):
    """Per-row Z_i, R_i = sum_j w^2 (y_i - y_j) and A_i = sum_row p w (y_i - y_j) for `rows`."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    m = rows.shape[0]
    Zr = np.empty(m)
    Rr = np.empty((m, 2))
    Ar = np.empty((m, 2))
    rp = None if P is None else P.row_ptr
    cl = None if P is None else P.col
    vl = None if P is None else P.val
    _check(lib().oracle_grad_rows(Y, Y.shape[0], rows, m, _opt(rp), _opt(cl), _opt(vl), _opt(Zr), _opt(Rr),
                                  _opt(Ar)), "grad_rows")
    return Zr, Rr, Ar


def grad_rows_scale(Y, rows, P: CSR | None = None):
    """Per-row, per-coordinate term magnitudes (Rabs, Aabs), float64 [m, 2]:
    sum_j w^2 |y_i - y_j| and sum_row |p| w |y_i - y_j|, the scale of the
    rounding error of R_i and A_i in any summation order."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    m = rows.shape[0]
    Ra = np.empty((m, 2))
    Aa = np.empty((m, 2))
    rp = None if P is None else P.row_ptr
    cl = None if P is None else P.col
    vl = None if P is None else P.val
    _check(lib().oracle_grad_rows_scale(Y, Y.shape[0], rows, m, _opt(rp), _opt(cl), _opt(vl), Ra, Aa),
           "grad_rows_scale")
    return Ra, Aa


def kl(Y, P: CSR):
    """(KL(P||Q), Z) for general stored values P."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    out = np.zeros(1)
    Z = np.zeros(1)
    _check(lib().oracle_kl(Y, Y.shape[0], P.row_ptr, P.col, P.val, _opt(out), _opt(Z)), "kl")
    return float(out[0]), float(Z[0])


def kl_backward(Y, P: CSR, gC=1.0):
    """(dC/dY float64 [n, 2], dC/dp float64 [nnz]) scaled by gC."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    dY = np.empty_like(Y)
    dP = np.empty(P.nnz)
    _check(lib().oracle_kl_backward(Y, Y.shape[0], P.row_ptr, P.col, P.val, gC, _opt(dY), _opt(dP)),
           "kl_backward")
    return dY, dP


def step(Y, update, gains, grad, lr, momentum, gain_inc=0.2, gain_dec=0.8, min_gain=0.01):
    """In-place gains + momentum step on float64 arrays [n, 2]."""
    for a in (Y, update, gains):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise TypeError("step operates in place on C-contiguous float64 arrays")
    g = np.ascontiguousarray(grad, dtype=np.float64)
    _check(lib().oracle_step(Y, update, gains, g, Y.shape[0], lr, momentum, gain_inc, gain_dec, min_gain), "step")


def tsne_schedule(t, exaggeration=12.0, exaggeration_iters=100, momentum_early=0.5, momentum_late=0.8):
    """(alpha_t, momentum_t): exaggeration and the lower momentum while t < exaggeration_iters."""
    early = t < exaggeration_iters
    return (exaggeration if early else 1.0), (momentum_early if early else momentum_late)
