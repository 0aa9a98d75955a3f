// tsne_kl_grad: exact t-SNE gradient with early exaggeration
// (van der Maaten & Hinton 2008, eq. 5 and Sec. 3.4) and optional Z / KL.
// Launch sequence: the all-pairs repulsion pass (rep.hpp), then one
// finalize pass that gathers the sparse attraction over the CSR rows
// (16 lanes per row, reduced with DPP row rotations), sums the repulsion
// chunks and Z in a fixed order and writes g_i = 4 (alpha A_i - R_i / Z);
// and, when KL is requested, a one-block reduction of the per-block
// sum p ln p, sum p ln q (q = 1/w) and sum p.
#include "common.hpp"
#include "rep.hpp"

namespace tsne {

__global__ __launch_bounds__(256) void finalize_tsne_kernel(
    const float2* __restrict__ Y, int64_t n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, float alpha, const double* __restrict__ Rpart, const double* __restrict__ Zrowpart,
    int64_t S, const double* __restrict__ Zblock, int64_t nZ, float2* __restrict__ grad, double* __restrict__ Zrow,
    double* __restrict__ Z_out, double* __restrict__ klpart) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const double Z = sum_zblocks(Zblock, nZ, red);
  if (blockIdx.x == 0 && tid == 0 && Z_out) *Z_out = Z;

  const int64_t row = int64_t(blockIdx.x) * 16 + (tid >> 4);
  const int sl = tid & 15;
  float ax = 0.0f, ay = 0.0f, plp = 0.0f, plq = 0.0f, ps = 0.0f;
  if (row < n) {
    const float2 yi = Y[row];
    const int64_t e1 = row_ptr[row + 1];
    for (int64_t e = row_ptr[row] + sl; e < e1; e += 16) {
      const int32_t j = col[e];
      const float p = val[e];
      const float2 yj = Y[j];
      const float dx = yi.x - yj.x, dy = yi.y - yj.y;
      const float q = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1.0f));
      const float pw = p * __builtin_amdgcn_rcpf(q);
      ax = __builtin_fmaf(pw, dx, ax);
      ay = __builtin_fmaf(pw, dy, ay);
      if (klpart) {
        if (p > 0.0f) plp += p * logf(p);
        plq += p * logf(q);
        ps += p;
      }
    }
  }
  ax = row16_sum(ax);
  ay = row16_sum(ay);
  if (row < n && sl == 0) {
    double rx = 0.0, ry = 0.0;
    for (int64_t s = 0; s < S; ++s) {
      rx += Rpart[2 * (s * n + row)];
      ry += Rpart[2 * (s * n + row) + 1];
    }
    const double gx = 4.0 * (double(alpha) * double(ax) - rx / Z);
    const double gy = 4.0 * (double(alpha) * double(ay) - ry / Z);
    grad[row] = make_float2(float(gx), float(gy));
    if (Zrow) {
      double zr = 0.0;
      for (int64_t s = 0; s < S; ++s) zr += Zrowpart[s * n + row];
      Zrow[row] = zr;
    }
  }
  if (klpart) {
    plp = row16_sum(plp);
    plq = row16_sum(plq);
    ps = row16_sum(ps);
    const bool own = row < n && sl == 0;
    const double a = block_sum_d(own ? double(plp) : 0.0, red);
    const double b = block_sum_d(own ? double(plq) : 0.0, red);
    const double c = block_sum_d(own ? double(ps) : 0.0, red);
    if (tid == 0) {
      klpart[3 * blockIdx.x] = a;
      klpart[3 * blockIdx.x + 1] = b;
      klpart[3 * blockIdx.x + 2] = c;
    }
  }
}

// KL = sum p ln p + sum p ln q + S ln Z  (ln w = -ln q).
__global__ __launch_bounds__(256) void kl_reduce_kernel(const double* __restrict__ klpart, int64_t nb,
                                                        const double* __restrict__ Zblock, int64_t nZ,
                                                        double* __restrict__ kl_out) {
  __shared__ double red[256];
  const double Z = sum_zblocks(Zblock, nZ, red);
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t t = threadIdx.x; t < nb; t += 256) {
    a += klpart[3 * t];
    b += klpart[3 * t + 1];
    c += klpart[3 * t + 2];
  }
  a = block_sum_d(a, red);
  b = block_sum_d(b, red);
  c = block_sum_d(c, red);
  if (threadIdx.x == 0) *kl_out = a + b + c * log(Z);
}

}  // namespace tsne

extern "C" int tsne_kl_grad(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                            float exaggeration, float* grad, double* Z, double* kl, double* Zrow, void* workspace,
                            size_t* workspace_bytes, void* stream) {
  using namespace tsne;
  if (!Y || !row_ptr || !col || !val || !grad || n < 2) return TSNE_ERR_INVALID_ARG;
  if (!(exaggeration > 0.0f) || !(exaggeration < INFINITY)) return TSNE_ERR_INVALID_ARG;
  if (n > (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  const RepGrid g = RepGrid::make(n, REP_IREG);
  const int64_t nfin = ceil_div(n, 16);
  Carve c;
  const size_t o_R = c.take(sizeof(double) * 2 * size_t(g.S) * size_t(n));
  const size_t o_Zr = c.take(sizeof(double) * size_t(g.S) * size_t(n));
  const size_t o_Zb = c.take(sizeof(double) * size_t(g.blocks()));
  const size_t o_kl = c.take(sizeof(double) * 3 * size_t(nfin));
  int rc = workspace_protocol(workspace, workspace_bytes, c.off);
  if (rc >= 0) return rc;
  char* ws = static_cast<char*>(workspace);
  double* Rpart = reinterpret_cast<double*>(ws + o_R);
  double* Zrowpart = Zrow ? reinterpret_cast<double*>(ws + o_Zr) : nullptr;
  double* Zblock = reinterpret_cast<double*>(ws + o_Zb);
  double* klpart = kl ? reinterpret_cast<double*>(ws + o_kl) : nullptr;
  hipStream_t s = as_stream(stream);

  hipLaunchKernelGGL((rep_kernel<float, REP_IREG, true>), dim3(unsigned(g.nib), unsigned(g.S)), dim3(256), 0, s, Y, n,
                     g.jchunk, Rpart, Zrowpart, Zblock);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(finalize_tsne_kernel, dim3(unsigned(nfin)), dim3(256), 0, s, reinterpret_cast<const float2*>(Y), n,
                     row_ptr, col, val, exaggeration, Rpart, Zrowpart, g.S, Zblock, g.blocks(),
                     reinterpret_cast<float2*>(grad), Zrow, Z, klpart);
  TSNE_CHECK_LAUNCH();
  if (kl) {
    hipLaunchKernelGGL(kl_reduce_kernel, dim3(1), dim3(256), 0, s, klpart, nfin, Zblock, g.blocks(), kl);
    TSNE_CHECK_LAUNCH();
  }
  return TSNE_OK;
}
