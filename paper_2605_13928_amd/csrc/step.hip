// tsne_step: momentum + adaptive-gains update of the embedding
// (van der Maaten & Hinton 2008, Algorithm 1; Jacobs 1988 gains).
// HBM-bound elementwise pass: 28 bytes in + 24 bytes out per point.
#include "common.hpp"
#include "klgrad.hpp"

namespace tsne {

__global__ __launch_bounds__(256) void step_kernel(float2* __restrict__ Y, float2* __restrict__ U,
                                                   float2* __restrict__ G, const float2* __restrict__ grad,
                                                   int64_t n, float lr, float mom, float inc, float dec, float mn) {
  const int64_t i = gtid();
  if (i >= n) return;
  float2 y = Y[i], u = U[i], ga = G[i];
  const float2 g = grad[i];
  step_coord(y.x, u.x, ga.x, g.x, lr, mom, inc, dec, mn);
  step_coord(y.y, u.y, ga.y, g.y, lr, mom, inc, dec, mn);
  Y[i] = y;
  U[i] = u;
  G[i] = ga;
}

int step_launch(float* Y, float* update, float* gains, const float* grad, int64_t n, float lr, float momentum,
                float gain_inc, float gain_dec, float min_gain, hipStream_t s) {
  hipLaunchKernelGGL(step_kernel, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, s, reinterpret_cast<float2*>(Y),
                     reinterpret_cast<float2*>(update), reinterpret_cast<float2*>(gains),
                     reinterpret_cast<const float2*>(grad), n, lr, momentum, gain_inc, gain_dec, min_gain);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

}  // namespace tsne

extern "C" int tsne_step(float* Y, float* update, float* gains, const float* grad, int64_t n, float lr,
                         float momentum, float gain_inc, float gain_dec, float min_gain, void* stream) {
  if (!Y || !update || !gains || !grad || n < 1) return TSNE_ERR_INVALID_ARG;
  if (n > (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  TSNE_REQUIRE_GFX950();
  return tsne::step_launch(Y, update, gains, grad, n, lr, momentum, gain_inc, gain_dec, min_gain,
                           tsne::as_stream(stream));
}
