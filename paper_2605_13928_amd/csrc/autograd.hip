// Differentiation form: KL(P||Q) and its exact derivatives with respect to
// the embedding Y and the stored values of P (the KL of van der Maaten &
// Hinton 2008, eq. 2, written over stored entries; P symmetric in pattern,
// values free).  One templated source serves float and double.
//   forward : Z-only all-pairs pass + per-row sparse sums -> C, Z
//   backward: all-pairs repulsion pass (recomputing w tile by tile, Q never
//             stored) + per-row sparse pass that gathers p_e + p_tpos(e)
//             and writes dC/dp_e.
#include "common.hpp"
#include "rep.hpp"

namespace tsne {

template <typename T>
__device__ __forceinline__ T log_t(T x);
template <>
__device__ __forceinline__ float log_t<float>(float x) { return logf(x); }
template <>
__device__ __forceinline__ double log_t<double>(double x) { return log(x); }

template <typename T>
__device__ __forceinline__ T row16_sum_t(T v);
template <>
__device__ __forceinline__ float row16_sum_t<float>(float v) { return row16_sum(v); }
template <>
__device__ __forceinline__ double row16_sum_t<double>(double v) {
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) v += shfl_xor_d(v, m);
  return v;
}

// Per-row sums (16 lanes per row) of p ln p, p ln q (q = 1/w) and p, folded
// into one FP64 triple per block.
template <typename T>
__global__ __launch_bounds__(256) void sparse_sums_kernel(const T* __restrict__ Y, int64_t n,
                                                          const int64_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col, const T* __restrict__ val,
                                                          double* __restrict__ part) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t row = int64_t(blockIdx.x) * 16 + (tid >> 4);
  const int sl = tid & 15;
  T plp = 0, plq = 0, ps = 0;
  if (row < n) {
    const T xi = Y[2 * row], yi = Y[2 * row + 1];
    for (int64_t e = row_ptr[row] + sl; e < row_ptr[row + 1]; e += 16) {
      const int32_t j = col[e];
      const T p = val[e];
      const T dx = xi - Y[2 * j], dy = yi - Y[2 * j + 1];
      const T q = PairOps<T>::fma(dx, dx, PairOps<T>::fma(dy, dy, T(1)));
      if (p > T(0)) plp += p * log_t<T>(p);
      plq += p * log_t<T>(q);
      ps += p;
    }
  }
  plp = row16_sum_t<T>(plp);
  plq = row16_sum_t<T>(plq);
  ps = row16_sum_t<T>(ps);
  const bool own = row < n && sl == 0;
  const double a = block_sum_d(own ? double(plp) : 0.0, red);
  const double b = block_sum_d(own ? double(plq) : 0.0, red);
  const double c = block_sum_d(own ? double(ps) : 0.0, red);
  if (tid == 0) {
    part[3 * blockIdx.x] = a;
    part[3 * blockIdx.x + 1] = b;
    part[3 * blockIdx.x + 2] = c;
  }
}

// C = sum p ln p + sum p ln q + S ln Z.
template <typename T>
__global__ __launch_bounds__(256) void kl_combine_kernel(const double* __restrict__ part, int64_t nb,
                                                         const double* __restrict__ Zblock, int64_t nZ,
                                                         T* __restrict__ C, double* __restrict__ Z_out) {
  __shared__ double red[256];
  const double Z = sum_zblocks(Zblock, nZ, red);
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t t = threadIdx.x; t < nb; t += 256) {
    a += part[3 * t];
    b += part[3 * t + 1];
    c += part[3 * t + 2];
  }
  a = block_sum_d(a, red);
  b = block_sum_d(b, red);
  c = block_sum_d(c, red);
  if (threadIdx.x == 0) {
    *C = T(a + b + c * log(Z));
    if (Z_out) *Z_out = Z;
  }
}

// dY_i = gC (2 sum_{e in row i} (p_e + p_tpos(e)) w_e (y_i - y_j) - (4 S / Z) R_i)
// dP_e = gC (1 + ln p_e + ln q_e + ln Z)
template <typename T>
__global__ __launch_bounds__(256) void kl_backward_rows_kernel(
    const T* __restrict__ Y, int64_t n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, const int32_t* __restrict__ tpos, const T* __restrict__ gC,
    const double* __restrict__ Rpart, int64_t S_chunks, const double* __restrict__ Zblock, int64_t nZ,
    const double* __restrict__ spart, int64_t nsp, T* __restrict__ dY, T* __restrict__ dP) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const double Z = sum_zblocks(Zblock, nZ, red);
  double st = 0.0;
  for (int64_t t = tid; t < nsp; t += 256) st += spart[3 * t + 2];
  const double S = block_sum_d(st, red);
  const T g = *gC;
  const T lnZ = T(log(Z));
  const int64_t row = int64_t(blockIdx.x) * 16 + (tid >> 4);
  const int sl = tid & 15;
  T ax = 0, ay = 0;
  if (row < n) {
    const T xi = Y[2 * row], yi = Y[2 * row + 1];
    for (int64_t e = row_ptr[row] + sl; e < row_ptr[row + 1]; e += 16) {
      const int32_t j = col[e];
      const T p = val[e];
      const T pt = val[tpos[e]];
      const T dx = xi - Y[2 * j], dy = yi - Y[2 * j + 1];
      const T q = PairOps<T>::fma(dx, dx, PairOps<T>::fma(dy, dy, T(1)));
      const T pw = (p + pt) * PairOps<T>::recip(q);
      ax = PairOps<T>::fma(pw, dx, ax);
      ay = PairOps<T>::fma(pw, dy, ay);
      if (dP) dP[e] = g * (T(1) + log_t<T>(p) + log_t<T>(q) + lnZ);
    }
  }
  ax = row16_sum_t<T>(ax);
  ay = row16_sum_t<T>(ay);
  if (row < n && sl == 0) {
    double rx = 0.0, ry = 0.0;
    for (int64_t s = 0; s < S_chunks; ++s) {
      rx += Rpart[2 * (s * n + row)];
      ry += Rpart[2 * (s * n + row) + 1];
    }
    const double c = 4.0 * S / Z;
    dY[2 * row] = T(double(g) * (2.0 * double(ax) - c * rx));
    dY[2 * row + 1] = T(double(g) * (2.0 * double(ay) - c * ry));
  }
}

struct KlLayout {
  RepGrid g;
  int64_t nrow_blocks;
  size_t o_R, o_Zb, o_sp, bytes;
  static KlLayout make(int64_t n) {
    KlLayout L;
    L.g = RepGrid::make(n, REP_IREG);
    L.nrow_blocks = ceil_div(n, 16);
    Carve c;
    L.o_R = c.take(sizeof(double) * 2 * size_t(L.g.S) * size_t(n));
    L.o_Zb = c.take(sizeof(double) * size_t(L.g.blocks()));
    L.o_sp = c.take(sizeof(double) * 3 * size_t(L.nrow_blocks));
    L.bytes = c.off;
    return L;
  }
};

template <typename T>
int kl_forward_impl(const T* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const T* val, T* C, double* Z,
                    char* ws, const KlLayout& L, hipStream_t s) {
  double* Zblock = reinterpret_cast<double*>(ws + L.o_Zb);
  double* spart = reinterpret_cast<double*>(ws + L.o_sp);
  hipLaunchKernelGGL((rep_kernel<T, REP_IREG, false>), dim3(unsigned(L.g.nib), unsigned(L.g.S)), dim3(256), 0, s, Y, n,
                     L.g.jchunk, nullptr, nullptr, Zblock);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(sparse_sums_kernel<T>, dim3(unsigned(L.nrow_blocks)), dim3(256), 0, s, Y, n, row_ptr, col, val,
                     spart);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(kl_combine_kernel<T>, dim3(1), dim3(256), 0, s, spart, L.nrow_blocks, Zblock, L.g.blocks(), C, Z);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

template <typename T>
int kl_backward_impl(const T* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const T* val,
                     const int32_t* tpos, const T* gC, T* dY, T* dP, char* ws, const KlLayout& L, hipStream_t s) {
  double* Rpart = reinterpret_cast<double*>(ws + L.o_R);
  double* Zblock = reinterpret_cast<double*>(ws + L.o_Zb);
  double* spart = reinterpret_cast<double*>(ws + L.o_sp);
  hipLaunchKernelGGL((rep_kernel<T, REP_IREG, true>), dim3(unsigned(L.g.nib), unsigned(L.g.S)), dim3(256), 0, s, Y, n,
                     L.g.jchunk, Rpart, nullptr, Zblock);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(sparse_sums_kernel<T>, dim3(unsigned(L.nrow_blocks)), dim3(256), 0, s, Y, n, row_ptr, col, val,
                     spart);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(kl_backward_rows_kernel<T>, dim3(unsigned(L.nrow_blocks)), dim3(256), 0, s, Y, n, row_ptr, col,
                     val, tpos, gC, Rpart, L.g.S, Zblock, L.g.blocks(), spart, L.nrow_blocks, dY, dP);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

}  // namespace tsne

extern "C" int tsne_kl_forward(int32_t dtype, const void* Y, int64_t n, const int64_t* row_ptr, const int32_t* col,
                               const void* val, void* C, double* Z, void* workspace, size_t* workspace_bytes,
                               void* stream) {
  using namespace tsne;
  if (!Y || !row_ptr || !col || !val || !C || n < 2) return TSNE_ERR_INVALID_ARG;
  if (dtype != TSNE_F32 && dtype != TSNE_F64) return TSNE_ERR_INVALID_ARG;
  if (n > (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  const KlLayout L = KlLayout::make(n);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = as_stream(stream);
  if (dtype == TSNE_F32)
    return kl_forward_impl<float>(static_cast<const float*>(Y), n, row_ptr, col, static_cast<const float*>(val),
                                  static_cast<float*>(C), Z, ws, L, s);
  return kl_forward_impl<double>(static_cast<const double*>(Y), n, row_ptr, col, static_cast<const double*>(val),
                                 static_cast<double*>(C), Z, ws, L, s);
}

extern "C" int tsne_kl_backward(int32_t dtype, const void* Y, int64_t n, const int64_t* row_ptr, const int32_t* col,
                                const void* val, const int32_t* tpos, const void* gC, void* dY, void* dP,
                                void* workspace, size_t* workspace_bytes, void* stream) {
  using namespace tsne;
  if (!Y || !row_ptr || !col || !val || !tpos || !gC || !dY || n < 2) return TSNE_ERR_INVALID_ARG;
  if (dtype != TSNE_F32 && dtype != TSNE_F64) return TSNE_ERR_INVALID_ARG;
  if (n > (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  const KlLayout L = KlLayout::make(n);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = as_stream(stream);
  if (dtype == TSNE_F32)
    return kl_backward_impl<float>(static_cast<const float*>(Y), n, row_ptr, col, static_cast<const float*>(val), tpos,
                                   static_cast<const float*>(gC), static_cast<float*>(dY), static_cast<float*>(dP), ws,
                                   L, s);
  return kl_backward_impl<double>(static_cast<const double*>(Y), n, row_ptr, col, static_cast<const double*>(val), tpos,
                                  static_cast<const double*>(gC), static_cast<double*>(dY), static_cast<double*>(dP),
                                  ws, L, s);
}
