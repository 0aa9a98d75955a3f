// tsne_pca: principal components of X (n x g, row-major FP32) by randomized
// truncated SVD of the column-centred matrix: randomized subspace iteration
// with re-orthonormalisation and the direct SVD of the projected matrix
// (Halko, Martinsson & Tropp 2011, SIAM Review 53, Algorithm 4.4 and
// Algorithm 5.1), with a subspace of l = 64 columns:
//   Q = orth((X - 1 mu^T) Omega);  q times: Q~ = orth(Xc^T Q), Q = orth(Xc Q~)
//   Z = Xc^T Q (= B^T),  Z^T Z = U diag(s^2) U^T,
//   components V = Z U diag(1/s),  scores = Q U diag(s).
// The two products with X -- Xc W (n x 64) and Xc^T Q (g x 64) -- run on the
// FP32 matrix cores (v_mfma_f32_16x16x4_f32), X centred on the fly as it is
// staged in LDS (no cancellation against the mean).  orth() is CholeskyQR2
// (Gram matrix in FP64, Cholesky + triangular inverse in one FP64 block,
// the first pass shifted), the 64 x 64 symmetric eigenproblem a cyclic
// Jacobi method in FP64 (tournament ordering, 32 disjoint rotations per
// step).  Sums over rows are per-chunk partials added in a fixed order:
// the result is bitwise reproducible.
#include <math.h>

#include "common.hpp"

namespace tsne {

constexpr int PCA_L = 64;       // subspace width = one 64-column MFMA tile row
constexpr int PCA_RC = 2048;    // rows per partial of the column sums and X^T Q
constexpr int PCA_GRC = 512;    // rows per partial of a Gram matrix (the least, where m allows)
constexpr int PCA_GMAX = 1024;  // partials of a Gram matrix (at most)

typedef float floatx4_t __attribute__((ext_vector_type(4)));

// --- column means ---------------------------------------------------------

// part[r][j] = sum of X[i][j] over the rows i of chunk r = blockIdx.y (FP64,
// eight independent partial sums per thread, added in a fixed order).
__global__ __launch_bounds__(256) void pca_colsum_kernel(const float* __restrict__ X, int64_t n, int g,
                                                         double* __restrict__ part) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= g) return;
  const int64_t r0 = int64_t(blockIdx.y) * PCA_RC;
  const int64_t r1 = r0 + PCA_RC < n ? r0 + PCA_RC : n;
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t i = r0;
  for (; i + 8 <= r1; i += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += double(X[(i + u) * g + j]);
  for (; i < r1; ++i) s[0] += double(X[i * g + j]);
  part[int64_t(blockIdx.y) * g + j] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

__global__ __launch_bounds__(256) void pca_colmean_kernel(const double* __restrict__ part, int64_t nchunk, int g,
                                                          int64_t n, float* __restrict__ mean) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= g) return;
  double s = 0.0;
  for (int64_t r = 0; r < nchunk; ++r) s += part[r * g + j];
  mean[j] = float(s / double(n));
}

// --- C = (A - 1 mu^T) W  (M x K times K x 64; the first ncols columns stored) --

// Block: 128 rows of A, 4 waves x 32 rows; K in chunks of 64 staged in LDS,
// the next chunk loaded into registers while the current one is used (VEC:
// 16-byte loads, K a multiple of 4).  The loads are unconditional, their
// addresses clamped into the matrices, so that none waits inside a branch:
// rows past M and columns past K are zeroed, and the mean subtracted, when
// the registers are written to LDS.  MFMA 16x16x4 operands: lane l holds
// A[l % 16][l / 16] and W[l / 16][l % 16]; the result tile
// D[4 (l / 16) + r][l % 16] in register r.
template <bool CENTER, bool VEC>
__global__ __launch_bounds__(256) void pca_gemm_tall_kernel(const float* __restrict__ A, int64_t M, int K,
                                                            const float* __restrict__ mu,
                                                            const float* __restrict__ W, float* __restrict__ C,
                                                            int ldc, int ncols) {
  constexpr int BM = 128, KC = 64, SA = KC + 4, SW = PCA_L + 16;
  constexpr int AE = VEC ? (BM * KC) / (4 * 256) : (BM * KC) / 256;  // loads per thread
  constexpr int RSTEP = VEC ? 16 : 4;                                // rows between a thread's loads
  __shared__ __attribute__((aligned(16))) float As[BM * SA];
  __shared__ __attribute__((aligned(16))) float Ws[KC * SW];
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t m0 = int64_t(blockIdx.x) * BM;
  // this thread's A column offset within a chunk and first row within the block
  const int ac = VEC ? 4 * (tid & 15) : (tid & 63);
  const int ar = VEC ? (tid >> 4) : (tid >> 6);
  floatx4_t acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
  float4 ra[VEC ? AE : 1];
  float rs[VEC ? 1 : AE];
  float4 rm = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float4 rw[4];
  auto load = [&](int k0) {
    const int c = k0 + ac < K ? k0 + ac : 0;
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int64_t row = m0 + ar + RSTEP * e;
      const float* src = A + (row < M ? row : M - 1) * K + c;
      if (VEC) ra[VEC ? e : 0] = *reinterpret_cast<const float4*>(src);
      else rs[VEC ? 0 : e] = *src;
    }
    if (CENTER) {
      if (VEC) rm = *reinterpret_cast<const float4*>(mu + c);
      else rm.x = mu[c];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = k0 + (tid >> 4) + 16 * e;
      rw[e] = *reinterpret_cast<const float4*>(W + int64_t(r < K ? r : K - 1) * PCA_L + 4 * (tid & 15));
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    const bool cok = k0 + ac < K;
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const bool ok = cok && m0 + ar + RSTEP * e < M;
      float* dst = As + (ar + RSTEP * e) * SA + ac;
      if (VEC) {
        float4 v = ra[VEC ? e : 0];
        if (CENTER) {
          v.x -= rm.x;
          v.y -= rm.y;
          v.z -= rm.z;
          v.w -= rm.w;
        }
        *reinterpret_cast<float4*>(dst) = ok ? v : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      } else {
        const float v = CENTER ? rs[VEC ? 0 : e] - rm.x : rs[VEC ? 0 : e];
        *dst = ok ? v : 0.0f;
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = (tid >> 4) + 16 * e;
      *reinterpret_cast<float4*>(Ws + r * SW + 4 * (tid & 15)) =
          k0 + r < K ? rw[e] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);  // in flight during the products below
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      float av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[(w * 32 + 16 * a + li) * SA + kk + lk];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Ws[(kk + lk) * SW + 16 * b + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + w * 32 + 16 * a + 4 * lk + r;
        const int col = 16 * b + li;
        if (row < M && col < ncols) C[row * ldc + col] = acc[a][b][r];
      }
}

// --- part[r] = (A - 1 mu^T)^T Bm over the rows of chunk r  (K x 64 each) -----

// Block (256 columns of A from c0 = 256 blockIdx.x, row chunk r = blockIdx.y
// of PCA_RC rows); wave w owns columns c0 + 64 w .. + 63 (4 tiles of 16)
// against all 64 columns of Bm (4 tiles); rows staged 32 at a time, the
// next stage loaded into registers while the current one is used.  As in
// the tall product, the loads are unconditional (clamped addresses) and the
// zeroing and centring happen on the way to LDS.
template <bool CENTER, bool VEC>
__global__ __launch_bounds__(256) void pca_gemm_red_kernel(const float* __restrict__ A, int64_t M, int K,
                                                           const float* __restrict__ mu,
                                                           const float* __restrict__ Bm, float* __restrict__ part) {
  constexpr int MS = 32, NB = 256, SA = NB + 16, SB = PCA_L + 16;
  constexpr int AE = VEC ? (MS * NB) / (4 * 256) : (MS * NB) / 256;
  constexpr int RSTEP = VEC ? 4 : 1;  // rows between a thread's loads
  __shared__ __attribute__((aligned(16))) float At[MS * SA];
  __shared__ __attribute__((aligned(16))) float Bt[MS * SB];
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int c0 = blockIdx.x * NB;
  const int64_t r0 = int64_t(blockIdx.y) * PCA_RC;
  const int64_t r1 = r0 + PCA_RC < M ? r0 + PCA_RC : M;
  // this thread's column of A (fixed for the block) and first row of a stage
  const int ac = VEC ? 4 * (tid & 63) : tid;
  const int ar = VEC ? (tid >> 6) : 0;
  const bool cok = c0 + ac < K;
  const int c = cok ? c0 + ac : 0;
  float4 rm = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (CENTER) {
    if (VEC) rm = *reinterpret_cast<const float4*>(mu + c);
    else rm.x = mu[c];
  }
  floatx4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
  float4 ra[VEC ? AE : 1];
  float rs[VEC ? 1 : AE];
  float4 rb[2];
  auto load = [&](int64_t ms) {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int64_t row = ms + ar + RSTEP * e;
      const float* src = A + (row < r1 ? row : r1 - 1) * K + c;
      if (VEC) ra[VEC ? e : 0] = *reinterpret_cast<const float4*>(src);
      else rs[VEC ? 0 : e] = *src;
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int64_t row = ms + (tid >> 4) + 16 * e;
      rb[e] = *reinterpret_cast<const float4*>(Bm + (row < r1 ? row : r1 - 1) * PCA_L + 4 * (tid & 15));
    }
  };
  load(r0);
  for (int64_t ms = r0; ms < r1; ms += MS) {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const bool ok = cok && ms + ar + RSTEP * e < r1;
      float* dst = At + (ar + RSTEP * e) * SA + ac;
      if (VEC) {
        float4 v = ra[VEC ? e : 0];
        if (CENTER) {
          v.x -= rm.x;
          v.y -= rm.y;
          v.z -= rm.z;
          v.w -= rm.w;
        }
        *reinterpret_cast<float4*>(dst) = ok ? v : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      } else {
        const float v = CENTER ? rs[VEC ? 0 : e] - rm.x : rs[VEC ? 0 : e];
        *dst = ok ? v : 0.0f;
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int r = (tid >> 4) + 16 * e;
      *reinterpret_cast<float4*>(Bt + r * SB + 4 * (tid & 15)) =
          ms + r < r1 ? rb[e] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    __syncthreads();
    if (ms + MS < r1) load(ms + MS);
#pragma unroll
    for (int kk = 0; kk < MS; kk += 4) {
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = At[(kk + lk) * SA + 64 * w + 16 * a + li];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bt[(kk + lk) * SB + 16 * b + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  float* out = part + int64_t(blockIdx.y) * K * PCA_L;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = c0 + 64 * w + 16 * a + 4 * lk + r;
        if (col < K) out[int64_t(col) * PCA_L + 16 * b + li] = acc[a][b][r];
      }
}

// out[i][c] = sum over chunks r (in order) of part[r][i][c], as float.
__global__ __launch_bounds__(256) void pca_reduce_kernel(const float* __restrict__ part, int64_t nchunk,
                                                         int64_t count, float* __restrict__ out) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= count) return;
  double s = 0.0;
  for (int64_t r = 0; r < nchunk; ++r) s += double(part[r * count + t]);
  out[t] = float(s);
}

// --- Gram matrix Y^T Y of an m x 64 factor, FP64 -------------------------

// Block r sums rows [r rpb, (r + 1) rpb) of Y (rpb a multiple of 32).  Rows
// are staged 32 at a time in LDS as doubles, the next stage loaded into
// registers (clamped addresses, rows past the end zeroed on the way to LDS)
// while the current one is used; wave w takes rows w, w + 4, ... of a stage
// and lane l accumulates the 8 x 8 entries (8 (l / 8) + i, 8 (l % 8) + j).
// The four waves' sums are added in wave order.
__global__ __launch_bounds__(256) void pca_gram_kernel(const float* __restrict__ Y, int64_t m, int64_t rpb,
                                                       double* __restrict__ part) {
  constexpr int RS = 32;
  __shared__ __attribute__((aligned(16))) double ys[RS * PCA_L];
  __shared__ double sum[PCA_L * PCA_L];
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  const int ia = 8 * (lane >> 3), ib = 8 * (lane & 7);
  const int64_t r0 = int64_t(blockIdx.x) * rpb;
  const int64_t r1 = r0 + rpb < m ? r0 + rpb : m;
  double acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
  float4 rv[2];
  auto load = [&](int64_t s) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int64_t row = s + (tid >> 4) + 16 * e;
      rv[e] = *reinterpret_cast<const float4*>(Y + (row < r1 ? row : r1 - 1) * PCA_L + 4 * (tid & 15));
    }
  };
  load(r0);
  for (int64_t s = r0; s < r1; s += RS) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int r = (tid >> 4) + 16 * e;
      const bool ok = s + r < r1;
      double* d = ys + r * PCA_L + 4 * (tid & 15);
      d[0] = ok ? double(rv[e].x) : 0.0;
      d[1] = ok ? double(rv[e].y) : 0.0;
      d[2] = ok ? double(rv[e].z) : 0.0;
      d[3] = ok ? double(rv[e].w) : 0.0;
    }
    __syncthreads();
    if (s + RS < r1) load(s + RS);
#pragma unroll 2
    for (int t = 0; t < RS / 4; ++t) {
      const double* yr = ys + (w + 4 * t) * PCA_L;
      double av[8], bv[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        av[i] = yr[ia + i];
        bv[i] = yr[ib + i];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  for (int v = 0; v < 4; ++v) {
    if (w == v) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          double& o = sum[(ia + i) * PCA_L + ib + j];
          o = v == 0 ? acc[i][j] : o + acc[i][j];
        }
    }
    __syncthreads();
  }
  double* out = part + int64_t(blockIdx.x) * PCA_L * PCA_L;
  for (int e = tid; e < PCA_L * PCA_L; e += 256) out[e] = sum[e];
}

// G[e] = sum over the nchunk partials (eight running sums, added in a fixed
// order), e < 64 x 64; 64 threads per block.
__global__ __launch_bounds__(64) void pca_gram_reduce_kernel(const double* __restrict__ part, int64_t nchunk,
                                                             double* __restrict__ G) {
  const int e = blockIdx.x * 64 + threadIdx.x;
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t r = 0;
  for (; r + 8 <= nchunk; r += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += part[(r + u) * PCA_L * PCA_L + e];
  for (; r < nchunk; ++r) s[0] += part[r * PCA_L * PCA_L + e];
  G[e] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// --- Cholesky G = R^T R (upper R) and R^-1, one block, FP64 ------------------

// shift > 0 adds shift * trace / 64 to the diagonal (the first, shifted pass
// of CholeskyQR2).  Right-looking: per column j the pivot, row j of R, then
// the trailing update of the upper triangle.  Thread t owns the entries
// (t / 64 + 4 u, t % 64), u < 16, of every update; it loads all of them
// before it stores any, so one LDS round trip serves a whole step.  The
// inverse comes from the same pass: the row operations that take G to R
// (row i minus R[j][i] times the scaled row j, row j divided by R[j][j])
// form the matrix E with E G = R, i.e. E = R^-T; applied to X = I alongside,
// they leave X = R^-T (lower triangular).  Rinv = X^T (float, 64 x 64
// row-major) is the W of the next product Q = Y Rinv.
__global__ __launch_bounds__(256) void pca_cholinv_kernel(const double* __restrict__ Gin, double shift,
                                                          float* __restrict__ Rinv) {
  constexpr int NU = PCA_L * PCA_L / 256;
  __shared__ double A[PCA_L][PCA_L + 1];
  __shared__ double X[PCA_L][PCA_L + 1];
  __shared__ double red[4];
  const int tid = threadIdx.x, r0 = tid >> 6, c = tid & 63;
  for (int e = tid; e < PCA_L * PCA_L; e += 256) {
    A[e / PCA_L][e % PCA_L] = Gin[e];
    X[e / PCA_L][e % PCA_L] = (e / PCA_L == e % PCA_L) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (shift > 0.0) {
    const double tr = block_sum_d(tid < PCA_L ? A[tid][tid] : 0.0, red);
    if (tid < PCA_L) A[tid][tid] += shift * tr / PCA_L;
    __syncthreads();
  }
  for (int j = 0; j < PCA_L; ++j) {
    // row j of R and row j of X divided by the pivot: every thread of the
    // first wave takes the pivot itself (lane c: R[j][c] for c >= j, X[j][c]
    // for c <= j, the only nonzeros of that row of X)
    if (tid < PCA_L) {
      const double d = A[j][j];
      const double rjj = sqrt(d > 1e-300 ? d : 1e-300);
      const double v = tid == j ? rjj : A[j][tid] / rjj;
      const double x = X[j][tid] / rjj;
      __builtin_amdgcn_wave_barrier();  // every lane has read A[j][j] before lane j replaces it
      if (tid >= j) A[j][tid] = v;
      if (tid <= j) X[j][tid] = x;
    }
    __syncthreads();
    double rji[NU], aic[NU], xic[NU];
    const double rjc = A[j][c], xjc = X[j][c];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      rji[u] = A[j][r0 + 4 * u];
      aic[u] = A[r0 + 4 * u][c];
      xic[u] = X[r0 + 4 * u][c];
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int i = r0 + 4 * u;
      if (i > j && c >= i) A[i][c] = aic[u] - rji[u] * rjc;
      if (i > j && c <= j) X[i][c] = xic[u] - rji[u] * xjc;
    }
    __syncthreads();
  }
  for (int e = tid; e < PCA_L * PCA_L; e += 256) Rinv[e] = float(X[e % PCA_L][e / PCA_L]);
}

// --- symmetric eigenproblem of the 64 x 64 Gram matrix, one block, FP64 -------

// Cyclic Jacobi, tournament ordering: in step s of a sweep, player 0 stays
// and players 1..63 rotate; pair i of the step is (arr[i], arr[63 - i]).
// Outputs the eigenvalues in descending order (lam) and the matching
// eigenvectors as the columns of U (row-major 64 x 64, FP64).
__global__ __launch_bounds__(256) void pca_jacobi_kernel(const double* __restrict__ Gin, double* __restrict__ lam,
                                                         double* __restrict__ U) {
  __shared__ double A[PCA_L][PCA_L + 1];
  __shared__ double V[PCA_L][PCA_L + 1];
  __shared__ double cs[32], sn[32];
  __shared__ int pp[32], qq[32];
  __shared__ double red[4];
  __shared__ int order[PCA_L];
  const int tid = threadIdx.x;
  for (int e = tid; e < PCA_L * PCA_L; e += 256) {
    A[e / PCA_L][e % PCA_L] = Gin[e];
    V[e / PCA_L][e % PCA_L] = (e / PCA_L == e % PCA_L) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int e = tid; e < PCA_L * PCA_L; e += 256) {
      const double v = A[e / PCA_L][e % PCA_L];
      if (e / PCA_L == e % PCA_L) dg += v * v;
      else off += v * v;
    }
    off = block_sum_d(off, red);  // same bits in every thread: a uniform exit
    dg = block_sum_d(dg, red);
    if (!(off > 1e-30 * dg)) break;
    for (int step = 0; step < PCA_L - 1; ++step) {
      if (tid < 32) {
        auto player = [&](int j) { return j == 0 ? 0 : 1 + (j - 1 + step) % (PCA_L - 1); };
        int p = player(tid), q = player(PCA_L - 1 - tid);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        const double apq = A[p][q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-300) {
          const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = q;
      }
      __syncthreads();
      // A <- J^T A J on the 2 x 2 blocks (rows of pair I, columns of pair J):
      // the rows rotated first, then the columns, as in the two-pass order;
      // V <- V J on the columns of every pair.  The blocks and the pairs are
      // disjoint, so each thread loads all of its entries before it stores.
      {
        constexpr int NBK = 32 * 32 / 256, NV = 32 * PCA_L / 256;
        double blk[NBK][4], vv[NV][2];
#pragma unroll
        for (int u = 0; u < NBK; ++u) {
          const int e = tid + 256 * u, I = e >> 5, J = e & 31;
          const int p1 = pp[I], q1 = qq[I], p2 = pp[J], q2 = qq[J];
          blk[u][0] = A[p1][p2];
          blk[u][1] = A[p1][q2];
          blk[u][2] = A[q1][p2];
          blk[u][3] = A[q1][q2];
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          const int e = tid + 256 * u, i = e / PCA_L, j = e % PCA_L;
          vv[u][0] = V[j][pp[i]];
          vv[u][1] = V[j][qq[i]];
        }
#pragma unroll
        for (int u = 0; u < NBK; ++u) {
          const int e = tid + 256 * u, I = e >> 5, J = e & 31;
          const int p1 = pp[I], q1 = qq[I], p2 = pp[J], q2 = qq[J];
          const double c1 = cs[I], s1 = sn[I], c2 = cs[J], s2 = sn[J];
          const double rpp = c1 * blk[u][0] - s1 * blk[u][2], rpq = c1 * blk[u][1] - s1 * blk[u][3];
          const double rqp = s1 * blk[u][0] + c1 * blk[u][2], rqq = s1 * blk[u][1] + c1 * blk[u][3];
          A[p1][p2] = c2 * rpp - s2 * rpq;
          A[p1][q2] = s2 * rpp + c2 * rpq;
          A[q1][p2] = c2 * rqp - s2 * rqq;
          A[q1][q2] = s2 * rqp + c2 * rqq;
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          const int e = tid + 256 * u, i = e / PCA_L, j = e % PCA_L;
          const double c = cs[i], s = sn[i];
          V[j][pp[i]] = c * vv[u][0] - s * vv[u][1];
          V[j][qq[i]] = s * vv[u][0] + c * vv[u][1];
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    for (int i = 0; i < PCA_L; ++i) order[i] = i;
    for (int i = 1; i < PCA_L; ++i) {  // insertion sort, descending, stable
      const int o = order[i];
      int j = i - 1;
      while (j >= 0 && A[order[j]][order[j]] < A[o][o]) {
        order[j + 1] = order[j];
        --j;
      }
      order[j + 1] = o;
    }
  }
  __syncthreads();
  if (tid < PCA_L) lam[tid] = A[order[tid]][order[tid]];
  for (int e = tid; e < PCA_L * PCA_L; e += 256) U[e] = V[e / PCA_L][order[e % PCA_L]];
}

// W1 = U diag(1/s) (float), s = sqrt(max(lam, 0)).
__global__ __launch_bounds__(256) void pca_post_eig_kernel(const double* __restrict__ lam,
                                                           const double* __restrict__ U, float* __restrict__ W1) {
  for (int e = threadIdx.x; e < PCA_L * PCA_L; e += 256) {
    const double s = sqrt(fmax(lam[e % PCA_L], 0.0));
    W1[e] = float(s > 0.0 ? U[e] / s : 0.0);
  }
}

// Sign of each of the first k components (the entry of largest magnitude
// positive, the first on ties), the components out (k x g, signed), the
// singular values, and W2 = U diag(s sign) for the scores.  One block per
// component c < k (blockIdx.x), V = g x 64.
__global__ __launch_bounds__(256) void pca_sign_kernel(const float* __restrict__ V, int g, int k,
                                                       const double* __restrict__ lam, const double* __restrict__ U,
                                                       float* __restrict__ comps, double* __restrict__ sv,
                                                       float* __restrict__ W2) {
  __shared__ float bv[256];
  __shared__ int bi[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  float best = -1.0f;
  int bidx = 0x7fffffff;
  for (int j = tid; j < g; j += 256) {
    const float a = fabsf(V[int64_t(j) * PCA_L + c]);
    if (a > best) {  // j increases per thread: keeps the first maximum
      best = a;
      bidx = j;
    }
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      const float o = bv[tid + h];
      const int oi = bi[tid + h];
      if (o > bv[tid] || (o == bv[tid] && oi < bi[tid])) {
        bv[tid] = o;
        bi[tid] = oi;
      }
    }
    __syncthreads();
  }
  const float sign = V[int64_t(bi[0]) * PCA_L + c] < 0.0f ? -1.0f : 1.0f;
  for (int j = tid; j < g; j += 256) comps[int64_t(c) * g + j] = sign * V[int64_t(j) * PCA_L + c];
  const double s = sqrt(fmax(lam[c], 0.0));
  if (tid == 0) sv[c] = s;
  if (tid < PCA_L) W2[tid * PCA_L + c] = float(U[tid * PCA_L + c] * s * double(sign));
}

struct PcaPlan {
  size_t o_mpart, o_Ya, o_Yb, o_Za, o_Zb, o_part, o_gpart, o_G, o_Rinv, o_lam, o_U, o_W1, o_W2, bytes;
  int64_t nchunk_n, nchunk_g, gchunk_max;
};

// Row blocks of a Gram matrix over m rows: at most PCA_GMAX blocks, each a
// multiple of 32 rows and at least PCA_GRC rows where m allows.
struct GramSplit {
  int64_t nblk, rpb;
};
GramSplit gram_split(int64_t m) {
  int64_t nblk = ceil_div(m, PCA_GRC);
  if (nblk > PCA_GMAX) nblk = PCA_GMAX;
  const int64_t rpb = ceil_div(ceil_div(m, nblk), 32) * 32;
  return {ceil_div(m, rpb), rpb};
}

PcaPlan pca_plan(int64_t n, int g) {
  PcaPlan L;
  Carve c;
  L.nchunk_n = ceil_div(n, PCA_RC);
  L.nchunk_g = ceil_div(g, PCA_RC);
  const int64_t gn = gram_split(n).nblk, gg = gram_split(g).nblk;
  L.gchunk_max = gn > gg ? gn : gg;
  L.o_mpart = c.take(sizeof(double) * size_t(L.nchunk_n) * size_t(g));
  L.o_Ya = c.take(sizeof(float) * size_t(n) * PCA_L);
  L.o_Yb = c.take(sizeof(float) * size_t(n) * PCA_L);
  L.o_Za = c.take(sizeof(float) * size_t(g) * PCA_L);
  L.o_Zb = c.take(sizeof(float) * size_t(g) * PCA_L);
  L.o_part = c.take(sizeof(float) * size_t(L.nchunk_n) * size_t(g) * PCA_L);
  L.o_gpart = c.take(sizeof(double) * size_t(L.gchunk_max) * PCA_L * PCA_L);
  L.o_G = c.take(sizeof(double) * PCA_L * PCA_L);
  L.o_Rinv = c.take(sizeof(float) * PCA_L * PCA_L);
  L.o_lam = c.take(sizeof(double) * PCA_L);
  L.o_U = c.take(sizeof(double) * PCA_L * PCA_L);
  L.o_W1 = c.take(sizeof(float) * PCA_L * PCA_L);
  L.o_W2 = c.take(sizeof(float) * PCA_L * PCA_L);
  L.bytes = c.off;
  return L;
}

struct PcaCtx {
  const PcaPlan& L;
  char* ws;
  hipStream_t s;
  template <typename T>
  T* at(size_t o) const {
    return reinterpret_cast<T*>(ws + o);
  }
};

// C (M x ncols, ldc) = (A - mu) W, A is M x K (mu nullable: no centring)
int pca_tall(const PcaCtx& x, const float* A, int64_t M, int K, const float* mu, const float* W, float* C, int ldc,
             int ncols) {
  const dim3 grid(unsigned(ceil_div(M, 128)));
  const bool vec = K % 4 == 0;
  if (mu && vec)
    hipLaunchKernelGGL((pca_gemm_tall_kernel<true, true>), grid, dim3(256), 0, x.s, A, M, K, mu, W, C, ldc, ncols);
  else if (mu)
    hipLaunchKernelGGL((pca_gemm_tall_kernel<true, false>), grid, dim3(256), 0, x.s, A, M, K, mu, W, C, ldc, ncols);
  else if (vec)
    hipLaunchKernelGGL((pca_gemm_tall_kernel<false, true>), grid, dim3(256), 0, x.s, A, M, K, mu, W, C, ldc, ncols);
  else
    hipLaunchKernelGGL((pca_gemm_tall_kernel<false, false>), grid, dim3(256), 0, x.s, A, M, K, mu, W, C, ldc, ncols);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

// out (K x 64) = (A - mu)^T Bm, A is M x K
int pca_red(const PcaCtx& x, const float* A, int64_t M, int K, const float* mu, const float* Bm, float* out) {
  float* part = x.at<float>(x.L.o_part);
  const int64_t nchunk = ceil_div(M, PCA_RC);
  const dim3 grid(unsigned(ceil_div(K, 256)), unsigned(nchunk));
  if (K % 4 == 0) hipLaunchKernelGGL((pca_gemm_red_kernel<true, true>), grid, dim3(256), 0, x.s, A, M, K, mu, Bm, part);
  else hipLaunchKernelGGL((pca_gemm_red_kernel<true, false>), grid, dim3(256), 0, x.s, A, M, K, mu, Bm, part);
  TSNE_CHECK_LAUNCH();
  const int64_t count = int64_t(K) * PCA_L;
  hipLaunchKernelGGL(pca_reduce_kernel, dim3(unsigned(ceil_div(count, 256))), dim3(256), 0, x.s, part, nchunk, count,
                     out);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

// G (64 x 64, FP64, in the workspace) = Y^T Y
int pca_gram(const PcaCtx& x, const float* Y, int64_t m) {
  const GramSplit sp = gram_split(m);
  hipLaunchKernelGGL(pca_gram_kernel, dim3(unsigned(sp.nblk)), dim3(256), 0, x.s, Y, m, sp.rpb,
                     x.at<double>(x.L.o_gpart));
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(pca_gram_reduce_kernel, dim3(PCA_L * PCA_L / 64), dim3(64), 0, x.s, x.at<double>(x.L.o_gpart),
                     sp.nblk, x.at<double>(x.L.o_G));
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

// CholeskyQR2 of the m x 64 factor in `a` (result in `a`, `b` scratch)
int pca_orth(const PcaCtx& x, float* a, float* b, int64_t m) {
  int rc;
  float* Rinv = x.at<float>(x.L.o_Rinv);
  if ((rc = pca_gram(x, a, m))) return rc;
  hipLaunchKernelGGL(pca_cholinv_kernel, dim3(1), dim3(256), 0, x.s, x.at<double>(x.L.o_G), 1e-12, Rinv);
  TSNE_CHECK_LAUNCH();
  if ((rc = pca_tall(x, a, m, PCA_L, nullptr, Rinv, b, PCA_L, PCA_L))) return rc;
  if ((rc = pca_gram(x, b, m))) return rc;
  hipLaunchKernelGGL(pca_cholinv_kernel, dim3(1), dim3(256), 0, x.s, x.at<double>(x.L.o_G), 0.0, Rinv);
  TSNE_CHECK_LAUNCH();
  return pca_tall(x, b, m, PCA_L, nullptr, Rinv, a, PCA_L, PCA_L);
}

}  // namespace tsne

extern "C" int tsne_pca(const float* X, int64_t n, int32_t g, int32_t k, int32_t q, const float* omega,
                        float* scores, float* components, double* singular_values, float* mean, void* workspace,
                        size_t* workspace_bytes, void* stream) {
  using namespace tsne;
  if (!X || !omega || !scores || !components || !singular_values || !mean) return TSNE_ERR_INVALID_ARG;
  if (n < PCA_L || g < PCA_L || k < 1 || k > PCA_L || q < 0 || q > 16) return TSNE_ERR_INVALID_ARG;
  if (n > int64_t(65535) * PCA_RC || g > (1 << 20)) return TSNE_ERR_UNSUPPORTED;  // row chunks index grid.y
  const PcaPlan L = pca_plan(n, g);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  const PcaCtx x{L, static_cast<char*>(workspace), as_stream(stream)};
  float* Ya = x.at<float>(L.o_Ya);
  float* Yb = x.at<float>(L.o_Yb);
  float* Za = x.at<float>(L.o_Za);
  float* Zb = x.at<float>(L.o_Zb);
  // column means
  hipLaunchKernelGGL(pca_colsum_kernel, dim3(unsigned(ceil_div(g, 256)), unsigned(L.nchunk_n)), dim3(256), 0, x.s,
                     X, n, g, x.at<double>(L.o_mpart));
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(pca_colmean_kernel, dim3(unsigned(ceil_div(g, 256))), dim3(256), 0, x.s,
                     x.at<double>(L.o_mpart), L.nchunk_n, g, n, mean);
  TSNE_CHECK_LAUNCH();
  // range finder with power iterations
  if ((rc = pca_tall(x, X, n, g, mean, omega, Ya, PCA_L, PCA_L))) return rc;
  if ((rc = pca_orth(x, Ya, Yb, n))) return rc;
  for (int it = 0; it < q; ++it) {
    if ((rc = pca_red(x, X, n, g, mean, Ya, Za))) return rc;
    if ((rc = pca_orth(x, Za, Zb, g))) return rc;
    if ((rc = pca_tall(x, X, n, g, mean, Za, Ya, PCA_L, PCA_L))) return rc;
    if ((rc = pca_orth(x, Ya, Yb, n))) return rc;
  }
  // Z = Xc^T Q = B^T; Z^T Z = U diag(s^2) U^T
  if ((rc = pca_red(x, X, n, g, mean, Ya, Za))) return rc;
  if ((rc = pca_gram(x, Za, g))) return rc;
  double* lam = x.at<double>(L.o_lam);
  double* U = x.at<double>(L.o_U);
  hipLaunchKernelGGL(pca_jacobi_kernel, dim3(1), dim3(256), 0, x.s, x.at<double>(L.o_G), lam, U);
  TSNE_CHECK_LAUNCH();
  float* W1 = x.at<float>(L.o_W1);
  float* W2 = x.at<float>(L.o_W2);
  hipLaunchKernelGGL(pca_post_eig_kernel, dim3(1), dim3(256), 0, x.s, lam, U, W1);
  TSNE_CHECK_LAUNCH();
  // components V = Z U diag(1/s) (g x 64, in Zb), signs, outputs
  if ((rc = pca_tall(x, Za, g, PCA_L, nullptr, W1, Zb, PCA_L, PCA_L))) return rc;
  if ((rc = launch_fill<float>(W2, PCA_L * PCA_L, 0.0f, x.s))) return rc;
  hipLaunchKernelGGL(pca_sign_kernel, dim3(unsigned(k)), dim3(256), 0, x.s, Zb, g, k, lam, U, components,
                     singular_values, W2);
  TSNE_CHECK_LAUNCH();
  // scores = Q U diag(s sign): the first k columns, straight into the output
  return pca_tall(x, Ya, n, PCA_L, nullptr, W2, scores, k, k);
}
