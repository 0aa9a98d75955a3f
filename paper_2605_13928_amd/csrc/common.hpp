// Shared helpers of the gfx950 t-SNE library: launch/error plumbing,
// workspace carving, wave64 reductions and a wave-level bitonic sort of
// 64-bit (distance, index) keys.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsne_mi355x.h"

namespace tsne {

void set_last_hip_error(hipError_t e);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// TSNE_OK when the calling thread's current HIP device is a gfx950, the only
// architecture the kernels are built for; TSNE_ERR_UNSUPPORTED for any other
// architecture or when no HIP device is present; TSNE_ERR_HIP when the
// runtime fails otherwise.  The answer is cached per device ordinal, so only
// the first call on a device queries its properties.  Enqueues nothing.
int require_gfx950();

// Returns from the enclosing entry point unless the current device is a
// gfx950 (after argument validation, before the first launch).
#define TSNE_REQUIRE_GFX950()                  \
  do {                                         \
    const int rc_dev_ = ::tsne::require_gfx950(); \
    if (rc_dev_ != TSNE_OK) return rc_dev_;    \
  } while (0)

// Returns TSNE_ERR_HIP from the enclosing entry point if the preceding
// launch failed.
#define TSNE_CHECK_LAUNCH()                         \
  do {                                              \
    hipError_t e_ = hipGetLastError();              \
    if (e_ != hipSuccess) {                         \
      ::tsne::set_last_hip_error(e_);               \
      return TSNE_ERR_HIP;                          \
    }                                               \
  } while (0)

// Workspace carving: every sub-buffer starts on a 256-byte boundary.
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off = (off + bytes + 255) & ~size_t(255);
    return o;
  }
};

// Common tail of the workspace query idiom.  Returns -1 to continue with
// the launch, or the status to return.
inline int workspace_protocol(void* ws, size_t* ws_bytes, size_t need) {
  if (!ws_bytes) return TSNE_ERR_INVALID_ARG;
  if (!ws) {
    *ws_bytes = need;
    return TSNE_OK;
  }
  if (*ws_bytes < need) return TSNE_ERR_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return TSNE_ERR_INVALID_ARG;
  return -1;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------
// Device helpers.

// 2^31-safe linear thread index.
__device__ __forceinline__ int64_t gtid() { return int64_t(blockIdx.x) * blockDim.x + threadIdx.x; }

// Workgroups are dealt to the 8 XCDs of an MI355X round-robin by index.
// xcd_block() renumbers them so that the ones on XCD x get consecutive
// numbers (the x-th eighth of 0 .. gridDim.x - 1, in launch order): work
// items that are near each other in a locality order then share the L2 of
// one XCD.  A bijection of [0, gridDim.x).
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t nb = gridDim.x, b = blockIdx.x, x = b % 8;
  int64_t base = 0;
  for (int64_t u = 0; u < x; ++u) base += (nb - u + 7) / 8;  // blocks on the XCDs before
  return base + b / 8;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// DPP move within a row of 16 lanes (row_ror:n is 0x120 + n).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

// Sum over each row of 16 lanes by rotations 8, 4, 2, 1; every lane of the
// row ends with the same bits (each step adds a commutative pair).
__device__ __forceinline__ float row16_sum(float v) {
  v += dpp_f<0x128>(v);
  v += dpp_f<0x124>(v);
  v += dpp_f<0x122>(v);
  v += dpp_f<0x121>(v);
  return v;
}
__device__ __forceinline__ float row16_min(float v) {
  v = fminf(v, dpp_f<0x128>(v));
  v = fminf(v, dpp_f<0x124>(v));
  v = fminf(v, dpp_f<0x122>(v));
  v = fminf(v, dpp_f<0x121>(v));
  return v;
}

// Value held by lane (lane ^ M), M a power of two below 64, with no trip
// through the LDS unit: DPP quad permutations (M = 1, 2), two DPP row shifts
// and a select (M = 4), a DPP row rotation (M = 8), and gfx950's
// v_permlane16_swap / v_permlane32_swap (M = 16, 32: with both operands v,
// the first result holds the lower row / half in both places, the second
// the upper one).
template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32, "power of two below 64");
  const int x = int(v);
  if constexpr (M == 1) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xf, 0xf, false));  // quad_perm [1, 0, 3, 2]
  } else if constexpr (M == 2) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xf, 0xf, false));  // quad_perm [2, 3, 0, 1]
  } else if constexpr (M == 4) {
    const int up = __builtin_amdgcn_update_dpp(0, x, 0x104, 0xf, 0xf, false);  // row_shl:4, lane i <- i + 4
    const int dn = __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4, lane i <- i - 4
    return uint32_t((lane_id() & 4) ? dn : up);
  } else if constexpr (M == 8) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, x, 0x128, 0xf, 0xf, false));  // row_ror:8
  } else if constexpr (M == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane_id() & 16) ? r[0] : r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane_id() & 32) ? r[0] : r[1];
  }
}
// The same for a mask known only after unrolling.
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int m) {
  switch (m) {
    case 1: return xor_lane<1>(v);
    case 2: return xor_lane<2>(v);
    case 4: return xor_lane<4>(v);
    case 8: return xor_lane<8>(v);
    case 16: return xor_lane<16>(v);
    default: return xor_lane<32>(v);
  }
}
__device__ __forceinline__ float xor_lane_f(float v, int m) { return __uint_as_float(xor_lane(__float_as_uint(v), m)); }
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = xor_lane(uint32_t(v), m);
  const uint32_t hi = xor_lane(uint32_t(v >> 32), m);
  return (uint64_t(hi) << 32) | lo;
}
__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  return __builtin_bit_cast(double, shfl_xor_u64(__builtin_bit_cast(uint64_t, v), m));
}

// Whole-wave reductions; all 64 lanes return the same bits.
__device__ __forceinline__ float wave_sum(float v) {
  v = row16_sum(v);
  v += xor_lane_f(v, 16);
  v += xor_lane_f(v, 32);
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v += int(xor_lane(uint32_t(v), m));
  return v;
}
__device__ __forceinline__ float wave_min(float v) {
  v = row16_min(v);
  v = fminf(v, xor_lane_f(v, 16));
  v = fminf(v, xor_lane_f(v, 32));
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v += shfl_xor_d(v, m);
  return v;
}

// Fixed-order block reduction of one double per thread (blockDim.x = 256):
// butterfly within each wave, then the four wave sums in order.  Result
// valid (same bits) in every thread.  `lds` needs 4 doubles.
__device__ __forceinline__ double block_sum_d(double v, double* lds) {
  v = wave_sum_d(v);
  if (lane_id() == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
  return r;
}

// Fixed-order sum of the per-block partials (Z), computed identically by
// every block that needs it: thread t adds entries t, t + 256, ... (eight
// loads in flight), then the block reduction.
__device__ __forceinline__ double zblock_thread_sum(const double* __restrict__ Zblock, int64_t nz) {
  double t = 0.0;
  int64_t b = threadIdx.x;
  for (; b + 7 * 256 < nz; b += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = Zblock[b + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) t += v[u];
  }
  for (; b < nz; b += 256) t += Zblock[b];
  return t;
}
__device__ __forceinline__ double sum_zblocks(const double* __restrict__ Zblock, int64_t nz, double* red) {
  return block_sum_d(zblock_thread_sum(Zblock, nz), red);
}

// ---------------------------------------------------------------------
// Neighbour keys: (distance bits << 32) | index.  For distances >= 0 the
// unsigned order of the bits is the numeric order, so the unsigned order of
// the key is the lexicographic order (d, j).
__device__ __forceinline__ uint64_t make_key(float d, int32_t j) {
  return (uint64_t(__float_as_uint(d)) << 32) | uint32_t(j);
}
__device__ __forceinline__ float key_dist(uint64_t k) { return __uint_as_float(uint32_t(k >> 32)); }
__device__ __forceinline__ int32_t key_index(uint64_t k) { return int32_t(uint32_t(k)); }
constexpr uint64_t KEY_MAX = ~uint64_t(0);

// Ascending bitonic sort of EPL*64 keys held EPL per lane; element index
// e = r*64 + lane for register r.  Partners 64 or more apart are in the
// same lane (register exchange); closer partners are exchanged across
// lanes.
template <int EPL>
__device__ __forceinline__ void wave_sort(uint64_t (&v)[EPL]) {
  const int lane = lane_id();
  constexpr int N = EPL * 64;
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= 64) {
        const int rs = stride >> 6;
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          const int p = r ^ rs;
          if (p > r) {
            const bool asc = (((r << 6) + lane) & size) == 0;
            uint64_t a = v[r], b = v[p];
            bool sw = asc ? (a > b) : (a < b);
            v[r] = sw ? b : a;
            v[p] = sw ? a : b;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          uint64_t o = shfl_xor_u64(v[r], stride);
          const bool asc = (((r << 6) + lane) & size) == 0;
          const bool lower = (lane & stride) == 0;
          const bool take_min = (lower == asc);
          uint64_t mn = v[r] < o ? v[r] : o;
          uint64_t mx = v[r] < o ? o : v[r];
          v[r] = take_min ? mn : mx;
        }
      }
    }
  }
}

// Read register r of lane `src` (both wave-uniform) as a uniform value.
template <int EPL>
__device__ __forceinline__ uint64_t wave_pick(const uint64_t (&v)[EPL], int e) {
  const int r = e >> 6, src = e & 63;
  uint64_t x = 0;
#pragma unroll
  for (int t = 0; t < EPL; ++t)
    if (t == r) x = v[t];
  uint32_t lo = __builtin_amdgcn_readlane(uint32_t(x), src);
  uint32_t hi = __builtin_amdgcn_readlane(uint32_t(x >> 32), src);
  return (uint64_t(hi) << 32) | lo;
}

// Small fill kernel (used instead of memset so the enqueued work is plain
// kernels only).
template <typename T>
__global__ void fill_kernel(T* __restrict__ p, int64_t count, T value) {
  for (int64_t t = gtid(); t < count; t += int64_t(gridDim.x) * blockDim.x) p[t] = value;
}

template <typename T>
inline int launch_fill(T* p, int64_t count, T value, hipStream_t s) {
  if (count <= 0) return TSNE_OK;
  int64_t blocks = ceil_div(count, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_kernel<T>, dim3(unsigned(blocks)), dim3(256), 0, s, p, count, value);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

}  // namespace tsne
