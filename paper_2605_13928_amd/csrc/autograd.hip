// Differentiation form: KL(P||Q) and its exact derivatives with respect to
// the embedding Y and the stored values of P (the KL of van der Maaten &
// Hinton 2008, eq. 2, written over stored entries; P symmetric in pattern,
// values free).
//   FP32: the symmetric all-pairs passes of tsne_kl_grad (each unordered
//         pair once).  forward: the Z-only pass (zsum_sym_kernel) and the
//         per-row sparse sums give C = sum p ln p + sum p ln q + S ln Z,
//         S = sum p.  backward: the gradient pass with attraction weight 0
//         gives g0 = -4 R / Z per row; a per-row sparse pass gathers
//         p_e + p_tpos(e), adds S g0 and writes dC/dp_e.
//   FP64 (for gradcheck): one templated ordered-pair pass (rep.hpp), a
//         Z-only pass for the forward, the repulsion pass for the backward,
//         and per-row sparse sums.
// In every case w is recomputed tile by tile; Q is never stored.
#include "common.hpp"
#include "klgrad.hpp"
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

// FP32 backward from g0 = -4 R / Z (the gradient pass with attraction
// weight 0) and Z: dY_i = gC (2 sum_{e in row i} (p_e + p_tpos(e)) w_e
// (y_i - y_j) + S g0_i), dP_e = gC (1 + ln p_e + ln q_e + ln Z).
__global__ __launch_bounds__(256) void kl_backward_g0_kernel(
    const float* __restrict__ Y, int64_t n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, const int32_t* __restrict__ tpos, const float* __restrict__ gC,
    const float* __restrict__ g0, const double* __restrict__ Zp, const double* __restrict__ spart, int64_t nsp,
    float* __restrict__ dY, float* __restrict__ dP) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double st = 0.0;
  for (int64_t t = tid; t < nsp; t += 256) st += spart[3 * t + 2];
  const double S = block_sum_d(st, red);
  const float g = *gC;
  const float lnZ = float(log(*Zp));
  const int64_t row = int64_t(blockIdx.x) * 16 + (tid >> 4);
  const int sl = tid & 15;
  float ax = 0.0f, ay = 0.0f;
  if (row < n) {
    const float xi = Y[2 * row], yi = Y[2 * row + 1];
    for (int64_t e = row_ptr[row] + sl; e < row_ptr[row + 1]; e += 16) {
      const int32_t j = col[e];
      const float p = val[e];
      const float pt = val[tpos[e]];
      const float dx = xi - Y[2 * j], dy = yi - Y[2 * j + 1];
      const float q = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1.0f));
      const float pw = (p + pt) * __builtin_amdgcn_rcpf(q);
      ax = __builtin_fmaf(pw, dx, ax);
      ay = __builtin_fmaf(pw, dy, ay);
      // ln p + ln q as one logarithm (p q stays within [p, p q_max])
      if (dP) dP[e] = g * (1.0f + logf(p * q) + lnZ);
    }
  }
  ax = row16_sum(ax);
  ay = row16_sum(ay);
  if (row < n && sl == 0) {
    dY[2 * row] = float(double(g) * (2.0 * double(ax) + S * double(g0[2 * row])));
    dY[2 * row + 1] = float(double(g) * (2.0 * double(ay) + S * double(g0[2 * row + 1])));
  }
}

// Block partials of S = sum of the stored values (FP64; a fixed grid, so the
// order of the sums is fixed), in the layout the backward kernel reads (the
// third of three doubles per block).  The values are row_ptr[0] = 0 ..
// row_ptr[n] - 1.
constexpr int KL32_SBLOCKS = 256;
__global__ __launch_bounds__(256) void val_sums_kernel(const float* __restrict__ val,
                                                       const int64_t* __restrict__ row_ptr, int64_t n,
                                                       double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t nnz = row_ptr[n];
  double a = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < nnz; e += int64_t(gridDim.x) * 256)
    a += double(val[e]);
  a = block_sum_d(a, red);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = 0.0;
    part[3 * blockIdx.x + 1] = 0.0;
    part[3 * blockIdx.x + 2] = a;
  }
}

// Workspace of the FP32 forms: the Z-only pass's workgroup partials and the
// sparse sums (forward); one gradient evaluation, its g0 output and Z
// (backward).
struct KlLayout32 {
  KlGradPlan kg;
  int64_t nrow_blocks;
  size_t o_kg, o_g0, o_Z, o_Zb, o_sp, bytes;
  static KlLayout32 make(int64_t n) {
    KlLayout32 L;
    L.kg = klgrad_plan(n, false, false);
    L.nrow_blocks = ceil_div(n, 16);
    Carve c;
    L.o_kg = c.take(L.kg.bytes);
    L.o_g0 = c.take(sizeof(float) * 2 * size_t(n));
    L.o_Z = c.take(sizeof(double));
    L.o_Zb = c.take(sizeof(double) * size_t(L.kg.g.nwg));
    const int64_t nsp = L.nrow_blocks > KL32_SBLOCKS ? L.nrow_blocks : KL32_SBLOCKS;
    L.o_sp = c.take(sizeof(double) * 3 * size_t(nsp));
    L.bytes = c.off;
    return L;
  }
};

int kl_forward_f32(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val, float* C,
                   double* Z, char* ws, const KlLayout32& L, hipStream_t s) {
  const SymGrid& g = L.kg.g;
  double* Zblock = reinterpret_cast<double*>(ws + L.o_Zb);
  double* spart = reinterpret_cast<double*>(ws + L.o_sp);
  const float2* Y2 = reinterpret_cast<const float2*>(Y);
  const dim3 grid(unsigned(g.nwg)), block(256);
  if (g.S == 256) hipLaunchKernelGGL(zsum_sym_kernel<1>, grid, block, 0, s, Y2, n, g.ns, Zblock);
  else if (g.S == 512) hipLaunchKernelGGL(zsum_sym_kernel<2>, grid, block, 0, s, Y2, n, g.ns, Zblock);
  else hipLaunchKernelGGL(zsum_sym_kernel<4>, grid, block, 0, s, Y2, n, g.ns, Zblock);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(sparse_sums_kernel<float>, dim3(unsigned(L.nrow_blocks)), dim3(256), 0, s, Y, n, row_ptr, col,
                     val, spart);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(kl_combine_kernel<float>, dim3(1), dim3(256), 0, s, spart, L.nrow_blocks, Zblock, g.nwg, C, Z);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

int kl_backward_f32(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                    const int32_t* tpos, const float* gC, float* dY, float* dP, char* ws, const KlLayout32& L,
                    hipStream_t s) {
  float* g0 = reinterpret_cast<float*>(ws + L.o_g0);
  double* Zs = reinterpret_cast<double*>(ws + L.o_Z);
  double* spart = reinterpret_cast<double*>(ws + L.o_sp);
  int rc = klgrad_launch(L.kg, ws + L.o_kg, Y, n, row_ptr, col, val, 0.0f, g0, Zs, nullptr, nullptr, s);
  if (rc) return rc;
  // S in 256 block partials (the stored values are contiguous: row_ptr[0] = 0)
  hipLaunchKernelGGL(val_sums_kernel, dim3(unsigned(KL32_SBLOCKS)), dim3(256), 0, s, val, row_ptr, n, spart);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(kl_backward_g0_kernel, dim3(unsigned(L.nrow_blocks)), dim3(256), 0, s, Y, n, row_ptr, col, val,
                     tpos, gC, g0, Zs, spart, int64_t(KL32_SBLOCKS), dY, dP);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
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
  if (dtype == TSNE_F32) {
    const KlLayout32 L = KlLayout32::make(n);
    int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
    if (rc >= 0) return rc;
    TSNE_REQUIRE_GFX950();
    return kl_forward_f32(static_cast<const float*>(Y), n, row_ptr, col, static_cast<const float*>(val),
                          static_cast<float*>(C), Z, static_cast<char*>(workspace), L, as_stream(stream));
  }
  const KlLayout L = KlLayout::make(n);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = as_stream(stream);
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
  if (dtype == TSNE_F32) {
    const KlLayout32 L = KlLayout32::make(n);
    int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
    if (rc >= 0) return rc;
    TSNE_REQUIRE_GFX950();
    return kl_backward_f32(static_cast<const float*>(Y), n, row_ptr, col, static_cast<const float*>(val), tpos,
                           static_cast<const float*>(gC), static_cast<float*>(dY), static_cast<float*>(dP),
                           static_cast<char*>(workspace), L, as_stream(stream));
  }
  const KlLayout L = KlLayout::make(n);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = as_stream(stream);
  return kl_backward_impl<double>(static_cast<const double*>(Y), n, row_ptr, col, static_cast<const double*>(val), tpos,
                                  static_cast<const double*>(gC), static_cast<double*>(dY), static_cast<double*>(dP),
                                  ws, L, s);
}
