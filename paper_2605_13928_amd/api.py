"""Torch-tensor front end of the C ABI (argument marshalling only).

Each function checks dtype, device and contiguity, pulls raw device
pointers and torch's current HIP stream, sizes the workspace with the
library's query idiom and calls the entry point of the same name.  Every
computation happens in the HIP kernels.  Nothing here synchronises except
`symmetrize`, which reads the entry count back to size its outputs.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check

# Algorithmic flops of the all-pairs evaluation in tsne_kl_grad.  Each
# unordered pair {i, j} is evaluated once and feeds both rows: 2 sub,
# 2 fma (1 + dx^2 + dy^2), 1 reciprocal, 1 add (Z), 1 mul (w^2), 4 fma
# (force on i and on j) = 17 flops, i.e. 8.5 per ordered pair.
KLGRAD_FLOPS_PER_ORDERED_PAIR = 8.5

__all__ = ["knn", "calibrate_P", "symmetrize", "kl_grad", "kl_grad_noalloc", "step", "optimize", "kl_forward", "kl_backward",
           "umap_fit_ab", "umap_weights", "umap_fuzzy_union", "umap_layout", "SparseP", "Workspace",
           "nonfinite_counter", "raise_if_nonfinite"]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _req(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def nonfinite_counter(device) -> torch.Tensor:
    """A device int64 scalar for the `nonfinite` argument of knn, kl_grad,
    kl_grad_fft and optimize (the call zeroes it, its kernels count)."""
    return torch.zeros(1, dtype=torch.int64, device=device)


def raise_if_nonfinite(counter: torch.Tensor | None, what: str):
    """Synchronises on the counter's value and raises TsneError with
    TSNE_ERR_NONFINITE when it is nonzero."""
    if counter is not None and int(counter.item()) != 0:
        raise _lib.TsneError(f"{what} ({int(counter.item())} non-finite coordinates)", _lib.TSNE_ERR_NONFINITE)


class Workspace:
    """Grow-only device scratch buffer reused across calls, plus the sizes the
    library asked for (keyed by entry point and shape) so repeated calls skip
    the size query."""

    def __init__(self, device=None):
        self.device = device
        self.buf = None
        self.sizes = {}

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        return self.buf


def _run_with_workspace(name, fn, args_before, args_after, device, ws: Workspace | None, key=None):
    ws = ws or Workspace()
    need = ws.sizes.get(key) if key is not None else None
    if need is None:
        q = C.c_size_t(0)
        check(name, fn(*args_before, None, C.byref(q), *args_after))
        need = q.value
        if key is not None:
            ws.sizes[key] = need
    buf = ws.get(need, device)
    have = C.c_size_t(buf.numel())
    check(name, fn(*args_before, _ptr(buf), C.byref(have), *args_after))
    return buf


def knn(X: torch.Tensor, k: int, precision: str = "fp32", n_cand: int | None = None, ws: Workspace | None = None,
        nonfinite: torch.Tensor | None = None):
    """Exact kNN of the rows of X [n, d] float32.  Returns (idx int32 [n, k], d2 float32 [n, k]).
    nonfinite: optional int64 [1] device counter of NaN/inf entries of X."""
    _req(X, "X", torch.float32)
    if X.dim() != 2:
        raise ValueError("X must be [n, d]")
    n, d = X.shape
    prec = {"fp32": _lib.TSNE_KNN_FP32, "bf16": _lib.TSNE_KNN_BF16}[precision]
    if n_cand is None:
        n_cand = min(2 * k, n - 1) if precision == "bf16" else 0
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((n, k), dtype=torch.float32, device=X.device)
    L = _lib.load()
    if nonfinite is not None:
        _req(nonfinite, "nonfinite", torch.int64, (1,))
    _run_with_workspace("tsne_knn", L.tsne_knn,
                        (_ptr(X), n, d, k, prec, n_cand, _ptr(idx), _ptr(d2), _ptr(nonfinite)),
                        (_stream(X.device),), X.device, ws)
    return idx, d2


def calibrate_P(nbr_d2: torch.Tensor, perplexity: float, tol: float = 1e-5, max_iter: int = 200):
    """Per-row beta with entropy ln(perplexity).  Returns (P_cond, beta, converged, n_unconverged[1] int32)."""
    _req(nbr_d2, "nbr_d2", torch.float32)
    n, k = nbr_d2.shape
    dev = nbr_d2.device
    P = torch.empty((n, k), dtype=torch.float32, device=dev)
    beta = torch.empty(n, dtype=torch.float32, device=dev)
    conv = torch.empty(n, dtype=torch.uint8, device=dev)
    nun = torch.empty(1, dtype=torch.int32, device=dev)
    L = _lib.load()
    check("tsne_calibrate_P", L.tsne_calibrate_P(_ptr(nbr_d2), n, k, float(perplexity), float(tol), int(max_iter),
                                                 _ptr(P), _ptr(beta), _ptr(conv), _ptr(nun), _stream(dev)))
    return P, beta, conv, nun


@dataclass
class SparseP:
    """Symmetric P as CSR: row_ptr int64 [n+1], col int32 [nnz], val float32 [nnz], tpos int32 [nnz]."""

    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor
    tpos: torch.Tensor | None
    n: int

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def symmetrize(nbr_idx: torch.Tensor, P_cond: torch.Tensor, want_tpos: bool = True,
               ws: Workspace | None = None) -> SparseP:
    """P = (C + C^T) / (2n) on the union pattern (one host sync to read nnz)."""
    _req(nbr_idx, "nbr_idx", torch.int32)
    n, k = nbr_idx.shape
    _req(P_cond, "P_cond", torch.float32, (n, k))
    dev = nbr_idx.device
    cap = 2 * n * k
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(cap, dtype=torch.int32, device=dev)
    val = torch.empty(cap, dtype=torch.float32, device=dev)
    tpos = torch.empty(cap, dtype=torch.int32, device=dev) if want_tpos else None
    nnz = torch.empty(1, dtype=torch.int64, device=dev)
    L = _lib.load()
    _run_with_workspace("tsne_symmetrize", L.tsne_symmetrize,
                        (_ptr(nbr_idx), _ptr(P_cond), n, k, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(tpos),
                         _ptr(nnz)), (_stream(dev),), dev, ws)
    m = int(nnz.item())
    if m < 0:
        raise ValueError("tsne_symmetrize: a neighbour list holds an out-of-range index, self or a repeat")
    return SparseP(row_ptr, col[:m], val[:m], None if tpos is None else tpos[:m], n)


def kl_grad(Y: torch.Tensor, P: SparseP, exaggeration: float = 1.0, grad: torch.Tensor | None = None,
            want_Z: bool = False, want_kl: bool = False, want_Zrow: bool = False, ws: Workspace | None = None,
            nonfinite: torch.Tensor | None = None):
    """Exact t-SNE gradient.  Returns (grad [n, 2] f32, Z f64[1] or None, KL f64[1] or None, Zrow f64[n] or None).
    nonfinite: optional int64 [1] device counter of NaN/inf coordinates of Y."""
    _req(Y, "Y", torch.float32)
    n = Y.shape[0]
    if Y.shape != (n, 2) or P.n != n:
        raise ValueError("Y must be [n, 2] matching P")
    dev = Y.device
    if grad is None:
        grad = torch.empty_like(Y)
    else:
        _req(grad, "grad", torch.float32, (n, 2))
    Z = torch.empty(1, dtype=torch.float64, device=dev) if want_Z else None
    kl = torch.empty(1, dtype=torch.float64, device=dev) if want_kl else None
    Zrow = torch.empty(n, dtype=torch.float64, device=dev) if want_Zrow else None
    if nonfinite is not None:
        _req(nonfinite, "nonfinite", torch.int64, (1,))
    L = _lib.load()
    _run_with_workspace("tsne_kl_grad", L.tsne_kl_grad,
                        (_ptr(Y), n, _ptr(P.row_ptr), _ptr(P.col), _ptr(P.val), float(exaggeration), _ptr(grad),
                         _ptr(Z), _ptr(kl), _ptr(Zrow), _ptr(nonfinite)), (_stream(dev),), dev, ws,
                        key=("kl_grad", n, want_Zrow))
    return grad, Z, kl, Zrow


def kl_grad_noalloc(Y: torch.Tensor, P: SparseP, exaggeration: float = 1.0, grad: torch.Tensor | None = None,
                    Z: torch.Tensor | None = None, kl: torch.Tensor | None = None, Zrow: torch.Tensor | None = None,
                    nonfinite: torch.Tensor | None = None):
    """tsne_kl_grad_noalloc: kl_grad on the library's static device scratch (no
    workspace).  Outputs are the caller's tensors when given (grad [n, 2] f32,
    Z and kl f64 [1], Zrow f64 [n]); a missing grad is allocated here, the
    others are then not computed.  Returns (grad, Z, kl, Zrow)."""
    _req(Y, "Y", torch.float32)
    n = Y.shape[0]
    if Y.shape != (n, 2) or P.n != n:
        raise ValueError("Y must be [n, 2] matching P")
    if grad is None:
        grad = torch.empty_like(Y)
    _req(grad, "grad", torch.float32, (n, 2))
    for t, name, shape in ((Z, "Z", (1,)), (kl, "kl", (1,)), (Zrow, "Zrow", (n,))):
        if t is not None:
            _req(t, name, torch.float64, shape)
    if nonfinite is not None:
        _req(nonfinite, "nonfinite", torch.int64, (1,))
    L = _lib.load()
    check("tsne_kl_grad_noalloc",
          L.tsne_kl_grad_noalloc(_ptr(Y), n, _ptr(P.row_ptr), _ptr(P.col), _ptr(P.val), float(exaggeration),
                                 _ptr(grad), _ptr(Z), _ptr(kl), _ptr(Zrow), _ptr(nonfinite), _stream(Y.device)))
    return grad, Z, kl, Zrow


def kl_grad_fft(Y: torch.Tensor, P: SparseP, exaggeration: float = 1.0, n_interp: int = 3, min_boxes: int = 50,
                max_box_width: float = 1.0, max_fft: int = 2048, grad: torch.Tensor | None = None,
                want_Z: bool = False, want_kl: bool = False, ws: Workspace | None = None,
                nonfinite: torch.Tensor | None = None):
    """t-SNE gradient with the repulsion and Z by FFT-accelerated interpolation
    (tsne_kl_grad_fft).  Returns (grad [n, 2] f32, Z f64[1] or None, KL f64[1] or None)."""
    _req(Y, "Y", torch.float32)
    n = Y.shape[0]
    if Y.shape != (n, 2) or P.n != n:
        raise ValueError("Y must be [n, 2] matching P")
    dev = Y.device
    if grad is None:
        grad = torch.empty_like(Y)
    else:
        _req(grad, "grad", torch.float32, (n, 2))
    Z = torch.empty(1, dtype=torch.float64, device=dev) if want_Z else None
    kl = torch.empty(1, dtype=torch.float64, device=dev) if want_kl else None
    if nonfinite is not None:
        _req(nonfinite, "nonfinite", torch.int64, (1,))
    L = _lib.load()
    _run_with_workspace("tsne_kl_grad_fft", L.tsne_kl_grad_fft,
                        (_ptr(Y), n, _ptr(P.row_ptr), _ptr(P.col), _ptr(P.val), float(exaggeration), int(n_interp),
                         int(min_boxes), float(max_box_width), int(max_fft), _ptr(grad), _ptr(Z), _ptr(kl),
                         _ptr(nonfinite)),
                        (_stream(dev),), dev, ws, key=("kl_grad_fft", n, int(max_fft)))
    return grad, Z, kl


PCA_SUBSPACE = 64


def pca(X: torch.Tensor, k: int, omega: torch.Tensor, q: int = 2, ws: Workspace | None = None):
    """Randomized PCA (tsne_pca).  X [n, g] f32, omega [g, 64] f32.
    Returns (scores [n, k] f32, components [k, g] f32, singular values [k] f64, mean [g] f32)."""
    _req(X, "X", torch.float32)
    n, g = X.shape
    _req(omega, "omega", torch.float32, (g, PCA_SUBSPACE))
    dev = X.device
    scores = torch.empty((n, k), dtype=torch.float32, device=dev)
    comps = torch.empty((k, g), dtype=torch.float32, device=dev)
    sv = torch.empty(k, dtype=torch.float64, device=dev)
    mean = torch.empty(g, dtype=torch.float32, device=dev)
    L = _lib.load()
    _run_with_workspace("tsne_pca", L.tsne_pca,
                        (_ptr(X), n, g, int(k), int(q), _ptr(omega), _ptr(scores), _ptr(comps), _ptr(sv), _ptr(mean)),
                        (_stream(dev),), dev, ws, key=("pca", n, g))
    return scores, comps, sv, mean


def step(Y, update, gains, grad, lr: float, momentum: float, gain_inc: float = 0.2, gain_dec: float = 0.8,
         min_gain: float = 0.01):
    """In-place momentum + gains step on [n, 2] float32 tensors."""
    n = Y.shape[0]
    for t, name in ((Y, "Y"), (update, "update"), (gains, "gains"), (grad, "grad")):
        _req(t, name, torch.float32, (n, 2))
    L = _lib.load()
    check("tsne_step", L.tsne_step(_ptr(Y), _ptr(update), _ptr(gains), _ptr(grad), n, float(lr), float(momentum),
                                   float(gain_inc), float(gain_dec), float(min_gain), _stream(Y.device)))


def optimize(Y, update, gains, P: SparseP, t_begin: int, t_end: int, lr: float = 200.0, exaggeration: float = 12.0,
             exaggeration_iters: int = 100, momentum_early: float = 0.5, momentum_late: float = 0.8,
             gain_inc: float = 0.2, gain_dec: float = 0.8, min_gain: float = 0.01, log_every: int = 0,
             kl_log: torch.Tensor | None = None, events=None, ws: Workspace | None = None,
             nonfinite: torch.Tensor | None = None):
    """Iterations t_begin .. t_end-1 (gradient + step each) enqueued by the library.

    kl_log: float64 device tensor of t_end - t_begin entries (KL written at
    iterations with (t + 1) % log_every == 0).  events: optional list of
    2 (t_end - t_begin) torch.cuda.Event or None (recorded around each launch
    of the all-pairs repulsion kernel; None entries are skipped).
    nonfinite: optional int64 [1] device counter of NaN/inf coordinates of
    the positions the iterations produce (summed over the iterations).
    """
    n = Y.shape[0]
    for t, name in ((Y, "Y"), (update, "update"), (gains, "gains")):
        _req(t, name, torch.float32, (n, 2))
    if P.n != n:
        raise ValueError("P does not match Y")
    iters = t_end - t_begin
    if kl_log is not None:
        _req(kl_log, "kl_log", torch.float64, (iters,))
    ev_arr = None
    if events is not None:
        if len(events) != 2 * iters:
            raise ValueError("need two events per iteration")
        handles = [0 if e is None else int(e.cuda_event) for e in events]
        if not all(h for h, e in zip(handles, events) if e is not None):
            raise ValueError("events must have been created (record each once) before use")
        ev_arr = C.cast((C.c_void_p * (2 * iters))(*handles), C.c_void_p)
    sc = _lib.Schedule(lr, exaggeration, exaggeration_iters, momentum_early, momentum_late, gain_inc, gain_dec,
                       min_gain)
    if nonfinite is not None:
        _req(nonfinite, "nonfinite", torch.int64, (1,))
    dev = Y.device
    L = _lib.load()
    _run_with_workspace("tsne_optimize", L.tsne_optimize,
                        (_ptr(Y), _ptr(update), _ptr(gains), n, _ptr(P.row_ptr), _ptr(P.col), _ptr(P.val),
                         int(P.nnz), int(t_begin), int(t_end), C.byref(sc), int(log_every), _ptr(kl_log), ev_arr,
                         _ptr(nonfinite)),
                        (_stream(dev),), dev, ws, key=("optimize", n, int(P.nnz)))


def _dtype_code(t):
    if t.dtype == torch.float32:
        return _lib.TSNE_F32
    if t.dtype == torch.float64:
        return _lib.TSNE_F64
    raise TypeError("only float32 and float64 are supported")


def kl_forward(Y: torch.Tensor, val: torch.Tensor, P: SparseP, ws: Workspace | None = None):
    """C = KL(P||Q) for stored values `val` on P's pattern.  Returns (C 0-d tensor, Z f64[1])."""
    dt = _dtype_code(Y)
    n = Y.shape[0]
    _req(Y, "Y", Y.dtype, (n, 2))
    _req(val, "val", Y.dtype, (P.nnz,))
    dev = Y.device
    Cout = torch.empty((), dtype=Y.dtype, device=dev)
    Z = torch.empty(1, dtype=torch.float64, device=dev)
    L = _lib.load()
    _run_with_workspace("tsne_kl_forward", L.tsne_kl_forward,
                        (dt, _ptr(Y), n, _ptr(P.row_ptr), _ptr(P.col), _ptr(val), _ptr(Cout), _ptr(Z)),
                        (_stream(dev),), dev, ws)
    return Cout, Z


def kl_backward(Y: torch.Tensor, val: torch.Tensor, P: SparseP, gC: torch.Tensor, want_dP: bool = True,
                ws: Workspace | None = None):
    """(dC/dY * gC [n, 2], dC/dp * gC [nnz] or None)."""
    dt = _dtype_code(Y)
    n = Y.shape[0]
    _req(Y, "Y", Y.dtype, (n, 2))
    _req(val, "val", Y.dtype, (P.nnz,))
    if P.tpos is None:
        raise ValueError("kl_backward needs P.tpos")
    gC = gC.reshape(()).to(dtype=Y.dtype).contiguous()
    dev = Y.device
    dY = torch.empty_like(Y)
    dP = torch.empty_like(val) if want_dP else None
    L = _lib.load()
    _run_with_workspace("tsne_kl_backward", L.tsne_kl_backward,
                        (dt, _ptr(Y), n, _ptr(P.row_ptr), _ptr(P.col), _ptr(val), _ptr(P.tpos), _ptr(gC), _ptr(dY),
                         _ptr(dP)), (_stream(dev),), dev, ws)
    return dY, dP


# --- UMAP on the kNN graph -------------------------------------------------------

def umap_fit_ab(min_dist: float = 0.5):
    """(a, b) of Phi(d) = 1 / (1 + a d^2b) fitted to the min_dist curve (host computation in the library)."""
    a, b = C.c_double(0.0), C.c_double(0.0)
    check("tsne_umap_fit_ab", _lib.load().tsne_umap_fit_ab(float(min_dist), C.byref(a), C.byref(b)))
    return a.value, b.value


def umap_weights(nbr_d2: torch.Tensor):
    """Smoothed kNN weights of every row.  Returns (rho [n], sigma [n], w [n, k]) float32."""
    _req(nbr_d2, "nbr_d2", torch.float32)
    n, k = nbr_d2.shape
    dev = nbr_d2.device
    rho = torch.empty(n, dtype=torch.float32, device=dev)
    sigma = torch.empty(n, dtype=torch.float32, device=dev)
    w = torch.empty((n, k), dtype=torch.float32, device=dev)
    check("tsne_umap_weights", _lib.load().tsne_umap_weights(_ptr(nbr_d2), n, k, _ptr(rho), _ptr(sigma), _ptr(w),
                                                             _stream(dev)))
    return rho, sigma, w


def umap_fuzzy_union(nbr_idx: torch.Tensor, w: torch.Tensor, ws: Workspace | None = None) -> SparseP:
    """B = A + A^T - A o A^T on the union pattern as CSR (one host sync to read nnz; no tpos)."""
    _req(nbr_idx, "nbr_idx", torch.int32)
    n, k = nbr_idx.shape
    _req(w, "w", torch.float32, (n, k))
    dev = nbr_idx.device
    cap = 2 * n * k
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(cap, dtype=torch.int32, device=dev)
    val = torch.empty(cap, dtype=torch.float32, device=dev)
    nnz = torch.empty(1, dtype=torch.int64, device=dev)
    L = _lib.load()
    _run_with_workspace("tsne_umap_fuzzy_union", L.tsne_umap_fuzzy_union,
                        (_ptr(nbr_idx), _ptr(w), n, k, _ptr(row_ptr), _ptr(col), _ptr(val), None, _ptr(nnz)),
                        (_stream(dev),), dev, ws)
    m = int(nnz.item())
    if m < 0:
        raise ValueError("tsne_umap_fuzzy_union: a neighbour list holds an out-of-range index, self or a repeat")
    return SparseP(row_ptr, col[:m], val[:m], None, n)


def umap_layout(Y: torch.Tensor, G: SparseP, a: float, b: float, n_epochs: int, alpha0: float = 1.0,
                neg_rate: int = 5, seed: int = 0, epochs: tuple[int, int] | None = None, symmetric: bool = True,
                ws: Workspace | None = None) -> torch.Tensor:
    """Epochs [t0, t1) of the layout (all n_epochs by default), in place on Y [n, 2] float32.
    symmetric=True asserts a symmetric graph with equal values in (i, j) and (j, i), as
    umap_fuzzy_union returns; False handles any graph."""
    _req(Y, "Y", torch.float32)
    n = Y.shape[0]
    if Y.shape != (n, 2) or G.n != n:
        raise ValueError("Y must be [n, 2] matching the graph")
    t0, t1 = (0, n_epochs) if epochs is None else epochs
    dev = Y.device
    L = _lib.load()
    _run_with_workspace("tsne_umap_layout", L.tsne_umap_layout,
                        (_ptr(Y), n, _ptr(G.row_ptr), _ptr(G.col), _ptr(G.val), G.nnz, int(bool(symmetric)), float(a),
                         float(b),
                         float(alpha0), int(neg_rate), int(n_epochs), int(t0), int(t1), C.c_uint64(seed)),
                        (_stream(dev),), dev, ws, key=("umap_layout", n))
    return Y
