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
constexpr int PCA_GRC = 1024;   // rows per partial of the Gram matrices

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
// 16-byte loads, K a multiple of 4).  MFMA 16x16x4 operands: lane l holds
// A[l % 16][l / 16] and W[l / 16][l % 16]; the result tile
// D[4 (l / 16) + r][l % 16] in register r.
template <bool CENTER, bool VEC>
__global__ __launch_bounds__(256) void pca_gemm_tall_kernel(const float* __restrict__ A, int64_t M, int K,
                                                            const float* __restrict__ mu,
                                                            const float* __restrict__ W, float* __restrict__ C,
                                                            int ldc, int ncols) {
  constexpr int BM = 128, KC = 64, SA = KC + 4, SW = PCA_L + 16;
  constexpr int AE = VEC ? (BM * KC) / (4 * 256) : (BM * KC) / 256;  // loads per thread
  __shared__ __attribute__((aligned(16))) float As[BM * SA];
  __shared__ __attribute__((aligned(16))) float Ws[KC * SW];
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t m0 = int64_t(blockIdx.x) * BM;
  floatx4_t acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
  float4 ra[VEC ? AE : 1];
  float rs[VEC ? 1 : AE];
  float4 rw[4];
  auto load = [&](int k0) {
    if (VEC) {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        const int r = idx >> 4, c = k0 + 4 * (idx & 15);
        const int64_t row = m0 + r;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (row < M && c < K) {
          v = *reinterpret_cast<const float4*>(A + row * K + c);
          if (CENTER) {
            const float4 m = *reinterpret_cast<const float4*>(mu + c);
            v.x -= m.x;
            v.y -= m.y;
            v.z -= m.z;
            v.w -= m.w;
          }
        }
        ra[VEC ? e : 0] = v;
      }
    } else {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        const int r = idx >> 6, c = k0 + (idx & 63);
        const int64_t row = m0 + r;
        float v = 0.0f;
        if (row < M && c < K) {
          v = A[row * K + c];
          if (CENTER) v -= mu[c];
        }
        rs[VEC ? 0 : e] = v;
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 256 * e;
      const int r = k0 + (idx >> 4);
      rw[e] = r < K ? *reinterpret_cast<const float4*>(W + int64_t(r) * PCA_L + 4 * (idx & 15))
                    : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    if (VEC) {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        *reinterpret_cast<float4*>(As + (idx >> 4) * SA + 4 * (idx & 15)) = ra[VEC ? e : 0];
      }
    } else {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        As[(idx >> 6) * SA + (idx & 63)] = rs[VEC ? 0 : e];
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 256 * e;
      *reinterpret_cast<float4*>(Ws + (idx >> 4) * SW + 4 * (idx & 15)) = rw[e];
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
// next stage loaded into registers while the current one is used.
template <bool CENTER, bool VEC>
__global__ __launch_bounds__(256) void pca_gemm_red_kernel(const float* __restrict__ A, int64_t M, int K,
                                                           const float* __restrict__ mu,
                                                           const float* __restrict__ Bm, float* __restrict__ part) {
  constexpr int MS = 32, NB = 256, SA = NB + 16, SB = PCA_L + 16;
  constexpr int AE = VEC ? (MS * NB) / (4 * 256) : (MS * NB) / 256;
  __shared__ __attribute__((aligned(16))) float At[MS * SA];
  __shared__ __attribute__((aligned(16))) float Bt[MS * SB];
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int c0 = blockIdx.x * NB;
  const int64_t r0 = int64_t(blockIdx.y) * PCA_RC;
  const int64_t r1 = r0 + PCA_RC < M ? r0 + PCA_RC : M;
  floatx4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
  float4 ra[VEC ? AE : 1];
  float rs[VEC ? 1 : AE];
  float4 rb[2];
  auto load = [&](int64_t ms) {
    if (VEC) {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        const int64_t row = ms + (idx >> 6);
        const int c = c0 + 4 * (idx & 63);
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (row < r1 && c < K) {
          v = *reinterpret_cast<const float4*>(A + row * K + c);
          if (CENTER) {
            const float4 m = *reinterpret_cast<const float4*>(mu + c);
            v.x -= m.x;
            v.y -= m.y;
            v.z -= m.z;
            v.w -= m.w;
          }
        }
        ra[VEC ? e : 0] = v;
      }
    } else {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        const int64_t row = ms + (idx >> 8);
        const int c = c0 + (idx & 255);
        float v = 0.0f;
        if (row < r1 && c < K) {
          v = A[row * K + c];
          if (CENTER) v -= mu[c];
        }
        rs[VEC ? 0 : e] = v;
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = tid + 256 * e;
      const int64_t row = ms + (idx >> 4);
      rb[e] = row < r1 ? *reinterpret_cast<const float4*>(Bm + row * PCA_L + 4 * (idx & 15))
                       : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  };
  load(r0);
  for (int64_t ms = r0; ms < r1; ms += MS) {
    if (VEC) {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        *reinterpret_cast<float4*>(At + (idx >> 6) * SA + 4 * (idx & 63)) = ra[VEC ? e : 0];
      }
    } else {
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + 256 * e;
        At[(idx >> 8) * SA + (idx & 255)] = rs[VEC ? 0 : e];
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int idx = tid + 256 * e;
      *reinterpret_cast<float4*>(Bt + (idx >> 4) * SB + 4 * (idx & 15)) = rb[e];
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

// Block r sums rows [r PCA_GRC, ...): thread t owns entries (t / 4, 16 (t % 4) + e).
__global__ __launch_bounds__(256) void pca_gram_kernel(const float* __restrict__ Y, int64_t m,
                                                       double* __restrict__ part) {
  constexpr int RS = 32;
  __shared__ float ys[RS * PCA_L];
  const int tid = threadIdx.x;
  const int a = tid >> 2, b0 = 16 * (tid & 3);
  const int64_t r0 = int64_t(blockIdx.x) * PCA_GRC;
  const int64_t r1 = r0 + PCA_GRC < m ? r0 + PCA_GRC : m;
  double acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;
  for (int64_t s = r0; s < r1; s += RS) {
#pragma unroll
    for (int e = 0; e < (RS * PCA_L) / 256; ++e) {
      const int idx = tid + 256 * e;
      const int64_t row = s + idx / PCA_L;
      ys[idx] = row < r1 ? Y[row * PCA_L + idx % PCA_L] : 0.0f;
    }
    __syncthreads();
    for (int r = 0; r < RS; ++r) {
      const double ya = double(ys[r * PCA_L + a]);
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e] = fma(ya, double(ys[r * PCA_L + b0 + e]), acc[e]);
    }
    __syncthreads();
  }
  double* out = part + int64_t(blockIdx.x) * PCA_L * PCA_L;
#pragma unroll
  for (int e = 0; e < 16; ++e) out[a * PCA_L + b0 + e] = acc[e];
}

// G[e] = sum over the nchunk partials (in order), e < 64 x 64.
__global__ __launch_bounds__(256) void pca_gram_reduce_kernel(const double* __restrict__ part, int64_t nchunk,
                                                              double* __restrict__ G) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= PCA_L * PCA_L) return;
  double s = 0.0;
  for (int64_t r = 0; r < nchunk; ++r) s += part[r * PCA_L * PCA_L + e];
  G[e] = s;
}

// --- Cholesky G = R^T R (upper R) and R^-1, one block, FP64 ------------------

// shift > 0 adds shift * trace / 64 to the diagonal (the first, shifted pass
// of CholeskyQR2).  Right-looking: per column, the pivot, the row of R, then
// the trailing update of the upper triangle in parallel.  Rinv (float,
// 64 x 64 row-major) is the W of the next product Q = Y Rinv.
__global__ __launch_bounds__(256) void pca_cholinv_kernel(const double* __restrict__ Gin, double shift,
                                                          float* __restrict__ Rinv) {
  __shared__ double A[PCA_L][PCA_L + 1];
  __shared__ double X[PCA_L][PCA_L + 1];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  for (int e = tid; e < PCA_L * PCA_L; e += 256) A[e / PCA_L][e % PCA_L] = Gin[e];
  __syncthreads();
  if (shift > 0.0) {
    const double tr = block_sum_d(tid < PCA_L ? A[tid][tid] : 0.0, red);
    if (tid < PCA_L) A[tid][tid] += shift * tr / PCA_L;
    __syncthreads();
  }
  for (int j = 0; j < PCA_L; ++j) {
    if (tid == 0) {
      const double d = A[j][j];
      A[j][j] = sqrt(d > 1e-300 ? d : 1e-300);
    }
    __syncthreads();
    if (tid > j && tid < PCA_L) A[j][tid] /= A[j][j];
    __syncthreads();
    for (int e = tid; e < PCA_L * PCA_L; e += 256) {
      const int i = e / PCA_L, c = e % PCA_L;
      if (i > j && c >= i) A[i][c] -= A[j][i] * A[j][c];
    }
    __syncthreads();
  }
  // R X = I with R the upper triangle of A: row i of X from rows i+1 ..,
  // one thread per column
  for (int i = PCA_L - 1; i >= 0; --i) {
    if (tid < PCA_L) {
      const int c = tid;
      double v = (i == c) ? 1.0 : 0.0;
      for (int p = i + 1; p <= c; ++p) v -= A[i][p] * X[p][c];
      X[i][c] = i <= c ? v / A[i][i] : 0.0;
    }
    __syncthreads();
  }
  for (int e = tid; e < PCA_L * PCA_L; e += 256) Rinv[e] = float(X[e / PCA_L][e % PCA_L]);
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
      // rows p, q of A (A <- J^T A)
      for (int e = tid; e < 32 * PCA_L; e += 256) {
        const int i = e / PCA_L, j = e % PCA_L;
        const int p = pp[i], q = qq[i];
        const double c = cs[i], s = sn[i];
        const double ap = A[p][j], aq = A[q][j];
        A[p][j] = c * ap - s * aq;
        A[q][j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of A and of V (A <- A J, V <- V J)
      for (int e = tid; e < 32 * PCA_L; e += 256) {
        const int i = e / PCA_L, j = e % PCA_L;
        const int p = pp[i], q = qq[i];
        const double c = cs[i], s = sn[i];
        const double ap = A[j][p], aq = A[j][q];
        A[j][p] = c * ap - s * aq;
        A[j][q] = s * ap + c * aq;
        const double vp = V[j][p], vq = V[j][q];
        V[j][p] = c * vp - s * vq;
        V[j][q] = s * vp + c * vq;
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

PcaPlan pca_plan(int64_t n, int g) {
  PcaPlan L;
  Carve c;
  L.nchunk_n = ceil_div(n, PCA_RC);
  L.nchunk_g = ceil_div(g, PCA_RC);
  const int64_t gn = ceil_div(n, PCA_GRC), gg = ceil_div(g, PCA_GRC);
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
  const int64_t nch = ceil_div(m, PCA_GRC);
  hipLaunchKernelGGL(pca_gram_kernel, dim3(unsigned(nch)), dim3(256), 0, x.s, Y, m, x.at<double>(x.L.o_gpart));
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(pca_gram_reduce_kernel, dim3(PCA_L * PCA_L / 256), dim3(256), 0, x.s, x.at<double>(x.L.o_gpart),
                     nch, x.at<double>(x.L.o_G));
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
