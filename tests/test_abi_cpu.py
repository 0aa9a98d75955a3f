"""Host-side checks of the C ABI: the library loads without a GPU, exports
every entry point the header declares, answers workspace queries and
rejects invalid arguments before making any HIP call."""
import ctypes as C
import os
import re

import pytest

from paper_2605_13928_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsne_mi355x.h")


@pytest.fixture(scope="module")
def L():
    return _lib.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tsne_[a-zA-Z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"
    assert L.tsne_abi_version() == 3 == _lib.TSNE_ABI_VERSION
    assert L.tsne_status_string(3).decode() == "workspace too small"


NULL = None


def ws_query(fn, *before, after=(NULL,)):
    need = C.c_size_t(0)
    rc = fn(*before, NULL, C.byref(need), *after)
    return rc, need.value


def test_workspace_queries_need_no_device(L):
    fake = C.c_void_p(0x1000)
    rc, need = ws_query(L.tsne_knn, fake, 20000, 50, 90, _lib.TSNE_KNN_FP32, 0, fake, fake, NULL)
    assert rc == 0 and need >= 20000 * 256 * 8
    rc, need_b = ws_query(L.tsne_knn, fake, 20000, 50, 90, _lib.TSNE_KNN_BF16, 180, fake, fake, NULL)
    assert rc == 0 and need_b > need
    rc, need = ws_query(L.tsne_symmetrize, fake, fake, 1000, 90, fake, fake, fake, fake, fake)
    assert rc == 0 and need > 1000 * 90 * 4 * 6
    rc, need = ws_query(L.tsne_kl_grad, fake, 1000, fake, fake, fake, C.c_float(12.0), fake, NULL, NULL, NULL, NULL)
    assert rc == 0 and need > 0
    for dt in (_lib.TSNE_F32, _lib.TSNE_F64):
        rc, need = ws_query(L.tsne_kl_forward, dt, fake, 64, fake, fake, fake, fake, NULL)
        assert rc == 0 and need > 0
        rc, need = ws_query(L.tsne_kl_backward, dt, fake, 64, fake, fake, fake, fake, fake, fake, NULL)
        assert rc == 0 and need > 0


def test_noalloc_rejects_oversized_problems_before_any_hip_call(L):
    fake = C.c_void_p(0x1000)
    nz = None
    g = L.tsne_kl_grad_noalloc
    assert g(fake, 92_161, fake, fake, fake, C.c_float(1.0), fake, nz, nz, nz, nz, nz) == _lib.TSNE_ERR_SCRATCH
    assert g(fake, 53_249, fake, fake, fake, C.c_float(1.0), fake, nz, nz, fake, nz, nz) == _lib.TSNE_ERR_SCRATCH
    assert g(fake, 1, fake, fake, fake, C.c_float(1.0), fake, nz, nz, nz, nz, nz) == _lib.TSNE_ERR_INVALID_ARG
    assert g(fake, 10, fake, fake, fake, C.c_float(0.0), fake, nz, nz, nz, nz, nz) == _lib.TSNE_ERR_INVALID_ARG
    assert g(fake, 10, fake, fake, fake, C.c_float(1.0), nz, nz, nz, nz, nz, nz) == _lib.TSNE_ERR_INVALID_ARG
    assert L.tsne_status_string(_lib.TSNE_ERR_SCRATCH).decode().startswith("problem too large")


def test_too_small_workspace_is_rejected_before_launch(L):
    fake = C.c_void_p(0x1000)
    have = C.c_size_t(16)
    rc = L.tsne_kl_grad(fake, 1000, fake, fake, fake, C.c_float(1.0), fake, NULL, NULL, NULL, NULL,
                        C.c_void_p(0x100000), C.byref(have), NULL)
    assert rc == _lib.TSNE_ERR_WORKSPACE


def test_invalid_arguments_rejected(L):
    fake = C.c_void_p(0x1000)
    IA, UN = _lib.TSNE_ERR_INVALID_ARG, _lib.TSNE_ERR_UNSUPPORTED
    # kNN
    assert ws_query(L.tsne_knn, NULL, 100, 50, 10, 0, 0, fake, fake, NULL)[0] == IA
    assert ws_query(L.tsne_knn, fake, 100, 50, 100, 0, 0, fake, fake, NULL)[0] == IA  # k >= n
    assert ws_query(L.tsne_knn, fake, 1, 50, 1, 0, 0, fake, fake, NULL)[0] == IA  # n < 2
    assert ws_query(L.tsne_knn, fake, 1000, 50, 300, 0, 0, fake, fake, NULL)[0] == UN  # k > 256
    assert ws_query(L.tsne_knn, fake, 1000, 300, 10, 0, 0, fake, fake, NULL)[0] == UN  # d > 256
    assert ws_query(L.tsne_knn, fake, 1000, 64, 10, 1, 20, fake, fake, NULL)[0] == UN  # bf16 needs d <= 58
    assert ws_query(L.tsne_knn, fake, 1000, 50, 90, 1, 80, fake, fake, NULL)[0] == IA  # n_cand < k
    assert ws_query(L.tsne_knn, fake, 1000, 50, 90, 7, 0, fake, fake, NULL)[0] == IA  # unknown precision
    # calibration
    cal = L.tsne_calibrate_P
    assert cal(fake, 10, 30, C.c_float(30.0), C.c_float(1e-5), 200, fake, NULL, NULL, NULL, NULL) == IA  # perp >= k
    assert cal(fake, 10, 30, C.c_float(10.0), C.c_float(0.0), 200, fake, NULL, NULL, NULL, NULL) == IA  # tol
    assert cal(fake, 10, 30, C.c_float(10.0), C.c_float(1e-5), 0, fake, NULL, NULL, NULL, NULL) == IA  # max_iter
    assert cal(NULL, 10, 30, C.c_float(10.0), C.c_float(1e-5), 9, fake, NULL, NULL, NULL, NULL) == IA
    assert cal(fake, 10, 300, C.c_float(10.0), C.c_float(1e-5), 9, fake, NULL, NULL, NULL, NULL) == UN
    # symmetrisation
    assert ws_query(L.tsne_symmetrize, fake, fake, 100, 100, fake, fake, fake, fake, fake)[0] == IA
    assert ws_query(L.tsne_symmetrize, fake, fake, 100, 10, fake, fake, fake, fake, NULL)[0] == IA  # nnz NULL
    # gradient / step
    assert ws_query(L.tsne_kl_grad, fake, 1, fake, fake, fake, C.c_float(1.0), fake, NULL, NULL, NULL, NULL)[0] == IA
    assert ws_query(L.tsne_kl_grad, fake, 10, fake, fake, fake, C.c_float(0.0), fake, NULL, NULL, NULL, NULL)[0] == IA
    assert ws_query(L.tsne_kl_grad, fake, 10, fake, fake, fake, C.c_float(1.0), NULL, NULL, NULL, NULL, NULL)[0] == IA
    # interpolated gradient: n_interp 2..5, min_boxes >= 1, box width > 0,
    # max_fft a power of two in [64, 4096] with 2 p min_boxes <= max_fft
    fg = L.tsne_kl_grad_fft

    def fq(n=10, p=3, mb=50, w=1.0, mf=2048, g=fake):
        return ws_query(fg, fake, n, fake, fake, fake, C.c_float(1.0), p, mb, C.c_float(w), mf, g, NULL, NULL, NULL)

    rc, need = fq()
    plane = 2048 * 2048
    assert rc == 0 and need >= 3 * 16 * plane + 3 * 8 * 1024 * 1024
    assert fq(mf=4096)[1] > 3 * need
    assert fq(n=1)[0] == IA and fq(g=NULL)[0] == IA
    assert fq(p=1)[0] == IA and fq(p=6)[0] == IA and fq(mb=0)[0] == IA
    assert fq(w=0.0)[0] == IA and fq(w=float("inf"))[0] == IA
    assert fq(mf=32)[0] == IA and fq(mf=8192)[0] == IA and fq(mf=1000)[0] == IA
    assert fq(p=5, mb=50, mf=256)[0] == IA  # 2 p min_boxes > max_fft
    assert fq(p=2, mb=16, mf=64)[0] == 0
    # randomized PCA: 64 <= n, 64 <= g, 1 <= k <= 64, 0 <= q <= 16
    pc = L.tsne_pca

    def pq(n=1000, g=300, k=50, q=2, om=fake):
        return ws_query(pc, fake, n, g, k, q, om, fake, fake, fake, fake)

    rc, need = pq()
    assert rc == 0 and need >= 2 * 1000 * 64 * 4 + 300 * 64 * 4
    assert pq(n=63)[0] == IA and pq(g=63)[0] == IA and pq(k=0)[0] == IA and pq(k=65)[0] == IA
    assert pq(q=-1)[0] == IA and pq(q=17)[0] == IA and pq(om=NULL)[0] == IA
    assert pq(n=65535 * 2048 + 1)[0] == UN
    st = L.tsne_step
    assert st(NULL, fake, fake, fake, 10, C.c_float(200), C.c_float(0.5), C.c_float(0.2), C.c_float(0.8),
              C.c_float(0.01), NULL) == IA
    assert st(fake, fake, fake, fake, 0, C.c_float(200), C.c_float(0.5), C.c_float(0.2), C.c_float(0.8),
              C.c_float(0.01), NULL) == IA
    # native optimiser loop
    sc = _lib.Schedule(200.0, 12.0, 100, 0.5, 0.8, 0.2, 0.8, 0.01)
    bad_sc = _lib.Schedule(200.0, 0.0, 100, 0.5, 0.8, 0.2, 0.8, 0.01)
    opt = L.tsne_optimize
    assert ws_query(opt, fake, fake, fake, 100, fake, fake, fake, 900, 0, 10, C.byref(sc), 0, NULL, NULL, NULL)[0] == 0
    assert ws_query(opt, fake, fake, fake, 100, fake, fake, fake, 900, 0, 10, None, 0, NULL, NULL, NULL)[0] == IA
    assert ws_query(opt, fake, fake, fake, 100, fake, fake, fake, 900, 5, 4, C.byref(sc), 0, NULL, NULL, NULL)[0] == IA
    assert ws_query(opt, fake, fake, fake, 100, fake, fake, fake, 900, 0, 10, C.byref(bad_sc), 0, NULL, NULL, NULL)[0] == IA
    assert ws_query(opt, NULL, fake, fake, 100, fake, fake, fake, 900, 0, 10, C.byref(sc), 0, NULL, NULL, NULL)[0] == IA
    assert ws_query(opt, fake, fake, fake, 100, fake, fake, fake, -1, 0, 10, C.byref(sc), 0, NULL, NULL, NULL)[0] == IA
    # the workspace grows with nnz (the job-grouped attraction list)
    small = ws_query(opt, fake, fake, fake, 100, fake, fake, fake, 900, 0, 10, C.byref(sc), 0, NULL, NULL, NULL)[1]
    big = ws_query(opt, fake, fake, fake, 100, fake, fake, fake, 90000, 0, 10, C.byref(sc), 0, NULL, NULL, NULL)[1]
    assert big - small >= 8 * (90000 - 900) - 512
    # differentiation form
    assert ws_query(L.tsne_kl_forward, 5, fake, 64, fake, fake, fake, fake, NULL)[0] == IA  # dtype
    assert ws_query(L.tsne_kl_backward, 0, fake, 64, fake, fake, fake, NULL, fake, fake, NULL)[0] == IA  # tpos


def test_umap_arguments_and_workspace(L):
    fake = C.c_void_p(0x1000)
    IA, UN = _lib.TSNE_ERR_INVALID_ARG, _lib.TSNE_ERR_UNSUPPORTED
    wt = L.tsne_umap_weights
    assert wt(NULL, 10, 15, fake, fake, fake, NULL) == IA
    assert wt(fake, 0, 15, fake, fake, fake, NULL) == IA and wt(fake, 10, 0, fake, fake, fake, NULL) == IA
    assert wt(fake, 10, 300, fake, fake, fake, NULL) == UN
    assert wt(fake, 10, 15, fake, NULL, fake, NULL) == IA
    fu = L.tsne_umap_fuzzy_union
    rc, need = ws_query(fu, fake, fake, 1000, 15, fake, fake, fake, NULL, fake)
    rc_s, need_s = ws_query(L.tsne_symmetrize, fake, fake, 1000, 15, fake, fake, fake, NULL, fake)
    assert rc == 0 and need == need_s
    assert ws_query(fu, fake, fake, 100, 100, fake, fake, fake, NULL, fake)[0] == IA
    lay = L.tsne_umap_layout

    def lq(Y=fake, n=1000, nnz=20000, sym=1, a=1.5, b=0.9, alpha=1.0, neg=5, ne=200, t0=0, t1=200):
        return ws_query(lay, Y, n, fake, fake, fake, nnz, sym, C.c_double(a), C.c_double(b), C.c_double(alpha), neg,
                        ne, t0, t1, C.c_uint64(7))

    rc, need = lq()
    assert rc == 0 and 24 * 1000 <= need <= 24 * 1000 + 4096
    assert lq(sym=0)[0] == 0 and lq(sym=2)[0] == IA
    assert lq(Y=NULL)[0] == IA and lq(n=1)[0] == IA and lq(nnz=0)[0] == IA
    assert lq(a=0.0)[0] == IA and lq(b=-1.0)[0] == IA and lq(alpha=-0.1)[0] == IA
    assert lq(neg=-1)[0] == IA and lq(neg=65)[0] == IA and lq(ne=0)[0] == IA
    assert lq(t0=5, t1=4)[0] == IA and lq(t1=201)[0] == IA and lq(t0=-1)[0] == IA
    assert lq(t0=200, t1=200)[0] == 0
    assert lq(n=1 << 31)[0] == UN
    a, b = C.c_double(0), C.c_double(0)
    assert L.tsne_umap_fit_ab(C.c_double(-0.1), C.byref(a), C.byref(b)) == IA
    assert L.tsne_umap_fit_ab(C.c_double(3.0), C.byref(a), C.byref(b)) == IA
    assert L.tsne_umap_fit_ab(C.c_double(0.1), NULL, C.byref(b)) == IA


@pytest.mark.parametrize("min_dist", [0.0, 0.1, 0.5, 1.0])
def test_umap_fit_ab_matches_oracle(L, min_dist):
    # host-only entry point: the library's Levenberg-Marquardt fit against
    # the oracle's (scipy curve_fit) on the same least-squares problem
    from oracle import umap as U

    a, b = C.c_double(0), C.c_double(0)
    assert L.tsne_umap_fit_ab(C.c_double(min_dist), C.byref(a), C.byref(b)) == 0
    oa, ob = U.fit_ab(min_dist)
    assert abs(a.value - oa) <= 1e-7 * oa and abs(b.value - ob) <= 1e-7 * ob, (a.value, b.value, oa, ob)
    assert U.fit_objective(a.value, b.value, min_dist) <= U.fit_objective(oa, ob, min_dist) * (1 + 1e-12)


def test_no_gfx950_device_is_unsupported(L):
    # valid arguments and a large enough (aligned, never touched) workspace:
    # with no gfx950 device current every entry point that does device work
    # returns TSNE_ERR_UNSUPPORTED before its first launch
    if _gpu_present():
        pytest.skip("a HIP device is present")
    fake = C.c_void_p(0x1000)
    ws = C.c_void_p(1 << 20)
    UN = _lib.TSNE_ERR_UNSUPPORTED
    big = C.c_size_t(1 << 62)

    def full(fn, *before, after=(NULL,)):
        return fn(*before, ws, C.byref(big), *after)

    sc = _lib.Schedule(200.0, 12.0, 100, 0.5, 0.8, 0.2, 0.8, 0.01)
    assert full(L.tsne_knn, fake, 1000, 50, 90, _lib.TSNE_KNN_FP32, 0, fake, fake, fake) == UN
    assert full(L.tsne_knn, fake, 1000, 50, 90, _lib.TSNE_KNN_BF16, 180, fake, fake, NULL) == UN
    assert L.tsne_calibrate_P(fake, 1000, 90, C.c_float(30.0), C.c_float(1e-5), 200, fake, NULL, NULL, fake,
                              NULL) == UN
    assert full(L.tsne_symmetrize, fake, fake, 1000, 90, fake, fake, fake, fake, fake) == UN
    assert full(L.tsne_kl_grad, fake, 1000, fake, fake, fake, C.c_float(12.0), fake, fake, fake, NULL, fake) == UN
    assert full(L.tsne_kl_grad_fft, fake, 1000, fake, fake, fake, C.c_float(1.0), 3, 50, C.c_float(1.0), 2048, fake,
                NULL, NULL, fake) == UN
    assert full(L.tsne_optimize, fake, fake, fake, 1000, fake, fake, fake, 90000, 0, 10, C.byref(sc), 0, NULL, NULL,
                fake) == UN
    assert L.tsne_step(fake, fake, fake, fake, 1000, C.c_float(200), C.c_float(0.5), C.c_float(0.2), C.c_float(0.8),
                       C.c_float(0.01), NULL) == UN
    for dt in (_lib.TSNE_F32, _lib.TSNE_F64):
        assert full(L.tsne_kl_forward, dt, fake, 64, fake, fake, fake, fake, NULL) == UN
        assert full(L.tsne_kl_backward, dt, fake, 64, fake, fake, fake, fake, fake, fake, NULL) == UN
    assert full(L.tsne_pca, fake, 1000, 300, 50, 2, fake, fake, fake, fake, fake) == UN
    assert L.tsne_umap_weights(fake, 1000, 15, fake, fake, fake, NULL) == UN
    assert full(L.tsne_umap_fuzzy_union, fake, fake, 1000, 15, fake, fake, fake, NULL, fake) == UN
    assert full(L.tsne_umap_layout, fake, 1000, fake, fake, fake, 20000, 1, C.c_double(1.5), C.c_double(0.9),
                C.c_double(1.0), 5, 200, 0, 200, C.c_uint64(7)) == UN
    assert L.tsne_last_hip_error() == 0
    assert "gfx950" in L.tsne_status_string(UN).decode()
    assert L.tsne_status_string(_lib.TSNE_ERR_NONFINITE).decode().startswith("non-finite")


def _gpu_present():
    try:
        import torch

        return torch.cuda.device_count() > 0
    except Exception:
        return False
