// Stable least-significant-digit radix sort of (key, value) pairs by the low
// `bits` bits of the keys, 8 bits per pass.  A pass counts the digits of
// each block of 2048 items (LDS integer atomics), takes one exclusive scan
// over the counts laid out digit-major (so every (digit, block) gets its
// global start), and scatters: each block places its items in input order,
// 256 at a time, an item's rank among the equal digits of its wave coming
// from eight ballots and the waves before it adding their counts.  Equal
// keys keep their input order, and nothing depends on timing, so the result
// is deterministic.
#pragma once

#include "common.hpp"
#include "scan.hpp"

namespace tsne {

constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;
constexpr int RS_ROUNDS = 8;
constexpr int RS_ITEMS = 256 * RS_ROUNDS;  // items per block

// cnt[d * nblk + b] = items of block b whose digit is d.
__global__ __launch_bounds__(256) void rs_count_kernel(const uint32_t* __restrict__ key, int64_t n, int shift,
                                                       int64_t nblk, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t h[RS_BINS];
  const int tid = threadIdx.x;
  h[tid] = 0u;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * RS_ITEMS;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + r * 256 + tid;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & (RS_BINS - 1)], 1u);
  }
  __syncthreads();
  cnt[int64_t(tid) * nblk + blockIdx.x] = h[tid];
}

// Items of block b to off[d * nblk + b] + (their rank among the block's
// items of digit d, in input order).
__global__ __launch_bounds__(256) void rs_scatter_kernel(const uint32_t* __restrict__ kin,
                                                         const int32_t* __restrict__ vin, int64_t n, int shift,
                                                         int64_t nblk, const int64_t* __restrict__ off,
                                                         uint32_t* __restrict__ kout, int32_t* __restrict__ vout) {
  __shared__ int64_t run[RS_BINS];    // next free position of each digit
  __shared__ uint32_t wc[4][RS_BINS];  // this round's digit counts per wave
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  run[tid] = off[int64_t(tid) * nblk + blockIdx.x];
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  const int64_t base = int64_t(blockIdx.x) * RS_ITEMS;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + r * 256 + tid;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const int32_t v = valid ? vin[i] : 0;
    const uint32_t d = (k >> shift) & (RS_BINS - 1);
    // lanes of this wave holding a valid item with the same digit
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RS_BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) wc[u][tid] = 0u;
    __syncthreads();  // counts cleared; run[] of the previous round complete
    const uint32_t rank = uint32_t(__popcll(m & lt));
    if (valid && rank == 0) wc[w][d] = uint32_t(__popcll(m));
    __syncthreads();
    if (valid) {
      uint32_t pre = 0;
      for (int u = 0; u < w; ++u) pre += wc[u][d];
      const int64_t pos = run[d] + pre + rank;
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();  // every read of run[] and wc[] of this round done
    run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
  }
}

// Workspace of a sort of n items: digit counts, their offsets and the scan's
// chunk sums.
struct RadixScratch {
  int64_t nblk, ncnt;
  size_t cnt_bytes, off_bytes, bsum_bytes;
  static RadixScratch make(int64_t n) {
    RadixScratch r;
    r.nblk = ceil_div(n, RS_ITEMS);
    r.ncnt = int64_t(RS_BINS) * r.nblk;
    r.cnt_bytes = sizeof(uint32_t) * size_t(r.ncnt);
    r.off_bytes = sizeof(int64_t) * size_t(r.ncnt + 1);
    r.bsum_bytes = sizeof(int64_t) * (size_t(ceil_div(r.ncnt + 1, SCAN_CHUNK)) + 1);
    return r;
  }
};

// Sorts the n >= 1 pairs in (ka, va) by the low `bits` bits of the keys;
// (kb, vb) is the second buffer of each pass, and both pairs are
// overwritten.  The result is in (kb, vb) when `in_b` comes back true (an
// odd number of passes), else in (ka, va).
inline int radix_sort_pairs(uint32_t* ka, int32_t* va, uint32_t* kb, int32_t* vb, int64_t n, int bits,
                            const RadixScratch& R, uint32_t* cnt, int64_t* off, int64_t* bsum, hipStream_t s,
                            bool& in_b) {
  in_b = false;
  for (int shift = 0; shift < bits; shift += RS_BITS) {
    hipLaunchKernelGGL(rs_count_kernel, dim3(unsigned(R.nblk)), dim3(256), 0, s, ka, n, shift, R.nblk, cnt);
    TSNE_CHECK_LAUNCH();
    int rc = exclusive_scan<uint32_t>(cnt, R.ncnt, off, bsum, s);
    if (rc) return rc;
    hipLaunchKernelGGL(rs_scatter_kernel, dim3(unsigned(R.nblk)), dim3(256), 0, s, ka, va, n, shift, R.nblk, off, kb,
                       vb);
    TSNE_CHECK_LAUNCH();
    uint32_t* tk = ka;
    ka = kb;
    kb = tk;
    int32_t* tv = va;
    va = vb;
    vb = tv;
    in_b = !in_b;
  }
  return TSNE_OK;
}

}  // namespace tsne
