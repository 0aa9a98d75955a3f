// Exclusive prefix sum over n counts (int or int64) into int64 offsets
// (out has n + 1 entries, out[n] = total): chunk sums, one-block scan of the
// chunk sums, then per-chunk application.  Deterministic (integer sums).
#pragma once

#include "common.hpp"

namespace tsne {

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = 256 * SCAN_ITEMS;

template <typename TIn>
__global__ __launch_bounds__(256) void scan_chunk_sums(const TIn* __restrict__ in, int64_t n, int64_t* __restrict__ bsum) {
  __shared__ double red_unused[1];
  __shared__ int64_t part[256];
  (void)red_unused;
  const int64_t base = int64_t(blockIdx.x) * SCAN_CHUNK + threadIdx.x * SCAN_ITEMS;
  int64_t s = 0;
#pragma unroll
  for (int t = 0; t < SCAN_ITEMS; ++t)
    if (base + t < n) s += int64_t(in[base + t]);
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = part[0];
}

// Exclusive scan of nb chunk sums in place by one block; bsum[nb] = total.
static __global__ __launch_bounds__(256) void scan_chunk_prefix(int64_t* __restrict__ bsum, int64_t nb) {
  __shared__ int64_t buf[256];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += 256) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t v = b < nb ? bsum[b] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      int64_t add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (b < nb) bsum[b] = carry + buf[threadIdx.x] - v;
    const int64_t tot = buf[255];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

// out[t] = sum_{u < t} in[u] for t = 0..n (out has n + 1 entries).
template <typename TIn>
__global__ __launch_bounds__(256) void scan_apply(const TIn* __restrict__ in, int64_t n,
                                                  const int64_t* __restrict__ bsum, int64_t nb,
                                                  int64_t* __restrict__ out) {
  __shared__ int64_t buf[256];
  const int64_t base = int64_t(blockIdx.x) * SCAN_CHUNK + threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    v[t] = (base + t < n) ? int64_t(in[base + t]) : 0;
    s += v[t];
  }
  buf[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int64_t add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
    __syncthreads();
    buf[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = bsum[blockIdx.x] + buf[threadIdx.x] - s;
#pragma unroll
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    if (base + t < n) out[base + t] = run;
    run += v[t];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

template <typename TIn>
inline int exclusive_scan(const TIn* in, int64_t n, int64_t* out, int64_t* bsum, hipStream_t s) {
  const int64_t nb = ceil_div(n, SCAN_CHUNK);
  hipLaunchKernelGGL(scan_chunk_sums<TIn>, dim3(unsigned(nb)), dim3(256), 0, s, in, n, bsum);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(scan_chunk_prefix, dim3(1), dim3(256), 0, s, bsum, nb);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(scan_apply<TIn>, dim3(unsigned(nb)), dim3(256), 0, s, in, n, bsum, nb, out);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

}  // namespace tsne
