// tsne_calibrate_P: per-row perplexity calibration (van der Maaten &
// Hinton 2008, eq. 1 and eq. 3).  One wave64 per row; the row's k <= 256
// distances live in registers (up to 4 per lane); the two sums of each
// entropy evaluation are wave reductions (DPP rotations within rows of 16,
// then two cross-row exchanges), so every lane sees identical bits and the
// bisection control flow stays uniform.  FP32 throughout.
#include "common.hpp"

namespace tsne {

// Largest beta the bracket expansion reaches (a power of two, so the
// doubling stays exact; far below FLT_MAX).
constexpr float CALIB_BETA_MAX = 0x1p126f;

template <int KPL>
__global__ __launch_bounds__(256) void calibrate_kernel(const float* __restrict__ d2, int64_t n, int k, float Hstar,
                                                        float tol, int max_iter, float* __restrict__ P,
                                                        float* __restrict__ beta_out, uint8_t* __restrict__ conv_out,
                                                        int* __restrict__ n_unconv) {
  const int lane = lane_id();
  const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= n) return;  // wave-uniform
  const float* d = d2 + row * k;
  float s[KPL];
  bool valid[KPL];
  float dmin = INFINITY;
#pragma unroll
  for (int t = 0; t < KPL; ++t) {
    const int j = lane + 64 * t;
    valid[t] = j < k;
    s[t] = valid[t] ? d[j] : INFINITY;
    dmin = fminf(dmin, s[t]);
  }
  dmin = wave_min(dmin);
#pragma unroll
  for (int t = 0; t < KPL; ++t) s[t] = valid[t] ? s[t] - dmin : 0.0f;

  float beta = 1.0f, lo = 0.0f, hi = INFINITY;
  float e[KPL];
  float S = 1.0f;
  bool ok = false;
  for (int it = 0; it < max_iter; ++it) {
    float sl = 0.0f, ml = 0.0f;
#pragma unroll
    for (int t = 0; t < KPL; ++t) {
      e[t] = valid[t] ? expf(-beta * s[t]) : 0.0f;
      sl += e[t];
      ml += e[t] * s[t];
    }
    S = wave_sum(sl);
    const float M = wave_sum(ml);
    const float H = logf(S) + beta * M / S;
    if (fabsf(H - Hstar) < tol) {
      ok = true;
      break;
    }
    if (it == max_iter - 1) break;
    if (H > Hstar) {
      lo = beta;
      if (isinf(hi)) {
        // Not bracketed yet.  A row whose nearest distance is shared by
        // more than `perplexity` neighbours keeps H above the target for
        // every beta (its limit is uniform over those ties): stop at the
        // cap, where every positive s of a normal size already gives
        // e = 0, instead of doubling beta to infinity (-inf * 0 = NaN).
        if (beta >= CALIB_BETA_MAX) break;
        beta *= 2.0f;
      } else {
        beta = 0.5f * (beta + hi);
      }
    } else {
      hi = beta;
      beta = 0.5f * (lo + beta);
    }
  }
  const float invS = 1.0f / S;
  float* p = P + row * k;
#pragma unroll
  for (int t = 0; t < KPL; ++t)
    if (valid[t]) p[lane + 64 * t] = e[t] * invS;
  if (lane == 0) {
    if (beta_out) beta_out[row] = beta;
    if (conv_out) conv_out[row] = ok ? 1 : 0;
    if (n_unconv && !ok) atomicAdd(n_unconv, 1);
  }
}

}  // namespace tsne

extern "C" int tsne_calibrate_P(const float* nbr_d2, int64_t n, int32_t k, float perplexity, float tol,
                                int32_t max_iter, float* P_cond, float* beta, uint8_t* converged,
                                int32_t* n_unconverged, void* stream) {
  using namespace tsne;
  if (!nbr_d2 || !P_cond || n < 1 || k < 1) return TSNE_ERR_INVALID_ARG;
  if (!(perplexity > 0.0f) || !(perplexity < float(k)) || !(tol > 0.0f) || max_iter < 1) return TSNE_ERR_INVALID_ARG;
  if (k > TSNE_MAX_K) return TSNE_ERR_UNSUPPORTED;
  if (n > (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  TSNE_REQUIRE_GFX950();
  hipStream_t s = as_stream(stream);
  if (n_unconverged) {
    int rc = launch_fill<int>(n_unconverged, 1, 0, s);
    if (rc) return rc;
  }
  const float Hstar = logf(perplexity);
  // the search compares an FP32 evaluation of H; stopping that much inside
  // tol keeps the entropy at the returned beta within tol
  const float tol_fp32 = tol - fminf(TSNE_CALIB_H_MARGIN, 0.5f * tol);
  dim3 grid(unsigned(ceil_div(n, 4))), block(256);
  const int kpl = int(ceil_div(k, 64));
  switch (kpl) {
    case 1: hipLaunchKernelGGL(calibrate_kernel<1>, grid, block, 0, s, nbr_d2, n, k, Hstar, tol_fp32, max_iter, P_cond, beta, converged, n_unconverged); break;
    case 2: hipLaunchKernelGGL(calibrate_kernel<2>, grid, block, 0, s, nbr_d2, n, k, Hstar, tol_fp32, max_iter, P_cond, beta, converged, n_unconverged); break;
    case 3: hipLaunchKernelGGL(calibrate_kernel<3>, grid, block, 0, s, nbr_d2, n, k, Hstar, tol_fp32, max_iter, P_cond, beta, converged, n_unconverged); break;
    default: hipLaunchKernelGGL(calibrate_kernel<4>, grid, block, 0, s, nbr_d2, n, k, Hstar, tol_fp32, max_iter, P_cond, beta, converged, n_unconverged); break;
  }
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}
