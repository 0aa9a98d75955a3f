// All-pairs Student-t repulsion, the O(n^2) part of the exact t-SNE
// gradient (van der Maaten & Hinton 2008, eq. 4-5): for every ordered pair
// i != j, w_ij = 1 / (1 + ||y_i - y_j||^2); per row R_i = sum_j w_ij^2
// (y_i - y_j) and Z_i = sum_j w_ij.  Q is never materialised.
//
// Layout: a block of 256 threads owns IREG*256 consecutive rows i, each
// thread IREG of them in registers; blockIdx.y selects a chunk of columns
// j.  Column points are staged through LDS in tiles of REP_TJ (coalesced
// float2 loads) and read back as wave-wide broadcasts.  Pair terms use T
// arithmetic (FP32: one v_rcp_f32 per pair); each thread folds its per-tile
// partial sums into FP64, and writes one FP64 partial per row and chunk;
// consumers add the chunks in index order.  Tail columns are padded with a
// point so far away that its weight is exactly 0; the self pair is masked
// in the tiles that can contain it.
#pragma once

#include "common.hpp"

namespace tsne {

template <typename T>
struct PairOps;
template <>
struct PairOps<float> {
  static __device__ __forceinline__ float recip(float q) { return __builtin_amdgcn_rcpf(q); }
  static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
  static constexpr float far = 1e30f;  // far^2 overflows to +inf, so w = 0
};
template <>
struct PairOps<double> {
  static __device__ __forceinline__ double recip(double q) { return 1.0 / q; }
  static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
  static constexpr double far = 1e200;
};

constexpr int REP_TJ = 512;
constexpr int REP_IREG = 4;

// One LDS tile of columns against the thread's IREG rows.  With MASK, row
// r of this thread is column (self0 + 256 r) of the tile and its own pair
// gets weight 0.
template <typename T, int IREG, bool WANT_R, bool MASK>
__device__ __forceinline__ void rep_tile(const T* __restrict__ sy, int jn, const T (&xi)[IREG], const T (&yi)[IREG],
                                         T (&rx)[IREG], T (&ry)[IREG], T (&z)[IREG], int self0) {
  for (int jj = 0; jj < jn; jj += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T xj = sy[2 * (jj + u)], yj = sy[2 * (jj + u) + 1];
#pragma unroll
      for (int r = 0; r < IREG; ++r) {
        const T dx = xi[r] - xj, dy = yi[r] - yj;
        const T q = PairOps<T>::fma(dx, dx, PairOps<T>::fma(dy, dy, T(1)));
        T w = PairOps<T>::recip(q);
        if (MASK && jj + u == self0 + 256 * r) w = T(0);
        z[r] += w;
        if (WANT_R) {
          const T w2 = w * w;
          rx[r] = PairOps<T>::fma(w2, dx, rx[r]);
          ry[r] = PairOps<T>::fma(w2, dy, ry[r]);
        }
      }
    }
  }
}

template <typename T, int IREG, bool WANT_R>
__global__ __launch_bounds__(256) void rep_kernel(const T* __restrict__ Y, int64_t n, int64_t jchunk,
                                                  double* __restrict__ Rpart, double* __restrict__ Zrowpart,
                                                  double* __restrict__ Zblock) {
  __shared__ T sy[2 * REP_TJ];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t ibase = int64_t(blockIdx.x) * 256 * IREG;
  const int64_t j0 = int64_t(blockIdx.y) * jchunk;
  const int64_t j1 = (j0 + jchunk < n) ? j0 + jchunk : n;

  T xi[IREG], yi[IREG];
  bool vi[IREG];
#pragma unroll
  for (int r = 0; r < IREG; ++r) {
    const int64_t i = ibase + r * 256 + tid;
    vi[r] = i < n;
    xi[r] = vi[r] ? Y[2 * i] : T(0);
    yi[r] = vi[r] ? Y[2 * i + 1] : T(0);
  }
  double Rx[IREG], Ry[IREG], Zr[IREG];
#pragma unroll
  for (int r = 0; r < IREG; ++r) Rx[r] = Ry[r] = Zr[r] = 0.0;

  for (int64_t t0 = j0; t0 < j1; t0 += REP_TJ) {
    const int cnt = int((j1 - t0) < REP_TJ ? (j1 - t0) : REP_TJ);
    __syncthreads();
    for (int u = tid; u < REP_TJ; u += 256) {
      T a = PairOps<T>::far, b = PairOps<T>::far;
      if (u < cnt) {
        a = Y[2 * (t0 + u)];
        b = Y[2 * (t0 + u) + 1];
      }
      sy[2 * u] = a;
      sy[2 * u + 1] = b;
    }
    __syncthreads();
    T rx[IREG], ry[IREG], z[IREG];
#pragma unroll
    for (int r = 0; r < IREG; ++r) rx[r] = ry[r] = z[r] = T(0);
    const int jn = (cnt + 3) & ~3;
    // Tiles that hold one of this block's own rows take the masked loop,
    // which gives the self pair weight 0; all other tiles run unmasked.
    const bool diag = t0 < ibase + 256 * IREG && ibase < t0 + cnt;
    if (diag)
      rep_tile<T, IREG, WANT_R, true>(sy, jn, xi, yi, rx, ry, z, int(ibase + tid - t0));
    else
      rep_tile<T, IREG, WANT_R, false>(sy, jn, xi, yi, rx, ry, z, 0);
#pragma unroll
    for (int r = 0; r < IREG; ++r) {
      Rx[r] += double(rx[r]);
      Ry[r] += double(ry[r]);
      Zr[r] += double(z[r]);
    }
  }

  double zsum = 0.0;
#pragma unroll
  for (int r = 0; r < IREG; ++r) {
    const int64_t i = ibase + r * 256 + tid;
    if (!vi[r]) continue;
    zsum += Zr[r];
    if (WANT_R) {
      Rpart[2 * (int64_t(blockIdx.y) * n + i)] = Rx[r];
      Rpart[2 * (int64_t(blockIdx.y) * n + i) + 1] = Ry[r];
    }
    if (Zrowpart) Zrowpart[int64_t(blockIdx.y) * n + i] = Zr[r];
  }
  const double bz = block_sum_d(zsum, red);
  if (tid == 0) Zblock[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = bz;
}

// Grid of the repulsion pass for n points: (row blocks, column chunks).
struct RepGrid {
  int64_t nib, S, jchunk;
  static RepGrid make(int64_t n, int ireg) {
    RepGrid g;
    g.nib = ceil_div(n, 256 * int64_t(ireg));
    int64_t S = ceil_div(2048, g.nib);
    const int64_t s_cols = ceil_div(n, 128);  // at least 128 columns per chunk
    if (S > s_cols) S = s_cols;
    if (S < 1) S = 1;
    g.jchunk = ceil_div(n, S);
    g.S = ceil_div(n, g.jchunk);
    return g;
  }
  int64_t blocks() const { return nib * S; }
};

}  // namespace tsne
