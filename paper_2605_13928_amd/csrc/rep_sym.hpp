// Symmetric all-pairs repulsion (FP32): every unordered pair {i, j} is
// evaluated once and its Student-t weight w = 1 / (1 + ||y_i - y_j||^2)
// (van der Maaten & Hinton 2008, eq. 4) feeds both rows:
//   R_i += w^2 (y_i - y_j),  R_j -= w^2 (y_i - y_j),  Z += 2 w.
// That halves the reciprocals and differences of the ordered-pair sweep.
//
// Decomposition.  Points are cut into superblocks of S (a multiple of 256);
// a job is one superblock pair (s, t), s <= t, numbered off-diagonal pairs
// first (job_pair).  A persistent grid of P workgroups deals the jobs in
// rounds of P, heaviest first (sym_sched: the full off-diagonal jobs, then
// the diagonal jobs and the jobs against the last, partly filled superblock
// in the order of their cost, the last diagonal job at the end), forward
// over the workgroups in even rounds and backward in odd ones, so that a
// workgroup that got a heavier job in one round gets a lighter one in the
// next.  Each workgroup's job list, and with it every sum, is fixed; while
// it computes one job it already loads the points of its next one into
// registers.  A workgroup has 4 waves; a wave tile is 64
// i-points x 64 j-points on an 8 x 8 lane grid: lane (a, b) = lane (8a + b)
// holds i-points 8a..8a+7 and j-points 8b..8b+7 in registers and evaluates
// their 64 pairs with no data movement.  Each wave sweeps its i-subblocks
// (64 points of s, round robin over the 4 waves) across the j-tiles of t
// (both staged in LDS): i-side sums stay in registers; after every tile the
// j-side sums are reduce-scattered over the 8 lanes that share a j-group
// (gfx950 v_permlane32_swap / v_permlane16_swap, then a DPP row rotation)
// and added to the wave's own LDS accumulator.  In the off-diagonal jobs
// of the launches without per-row Z, a wave takes its PF = S / 256
// subblocks together instead, the j-tiles in the outer loop: the PF tiles
// of one j-tile add into the same j-side registers, so one reduce-scatter
// serves PF tiles (at S = 1024 that takes the per-pair instruction count
// from about 11.9 to 11.3).  At the end of a job the
// workgroup adds the 4 wave accumulators in a fixed order and writes one
// partial per point and opposite superblock: slice t for i in s and slice
// s for j in t (for s == t both sides land in the same slot and are added
// first).  A later pass sums the ns partials of a row in index
// order, and the P per-workgroup Z sums in index order, so the result is
// deterministic.
// In the diagonal superblock each unordered pair of subblocks {u, v} is one
// tile, taken by the wave of the subblock whose cyclic distance to the other
// is the shorter (u takes v = u + 1 ... u + nsub/2 mod nsub, the distance
// nsub/2 only for u < nsub/2), so that its waves carry nearly equal shares;
// the 64 x 64 diagonal tiles take every ordered pair on the i side only,
// with the self pair masked.  Points past n are placed far away,
// each at its own position, so all their weights are exactly 0.
#pragma once

#include "common.hpp"

namespace tsne {

constexpr int SYM_WAVES = 4;

// --- exchange steps of the 8-lane reduce-scatter -------------------------
// Each step halves the values a lane holds: for pairs (x, y) = (v[k], v[k+h])
// the lanes with the step's bit clear end with x summed over the lane pair,
// the others with y summed.

// lanes l and l ^ 32 (v_permlane32_swap: the upper half of x trades places
// with the lower half of y)
__device__ __forceinline__ float xstep32(float x, float y) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// lanes l and l ^ 16 (v_permlane16_swap: odd 16-lane rows of x trade places
// with even rows of y)
__device__ __forceinline__ float xstep16(float x, float y) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// lanes l and l ^ 8 (DPP row rotation by 8 within rows of 16)
__device__ __forceinline__ float xstep8(float x, float y, bool hi) {
  const float send = hi ? x : y;
  const float keep = hi ? y : x;
  return keep + dpp_f<0x128>(send);
}
// lanes l and l ^ m, m in {1, 2, 4} (ds_swizzle bit-mask mode: xor m)
template <int M>
__device__ __forceinline__ float xstep_small(float x, float y, bool hi) {
  const float send = hi ? x : y;
  const float keep = hi ? y : x;
  const float recv = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(send), 0x1F | (M << 10)));
  return keep + recv;
}

// Reduce-scatter of v[0..15] over the 8 lanes sharing (lane & 7): after it,
// the lane holds v[base] and v[base + 1] summed over those lanes, with
// base = 8*bit5 + 4*bit4 + 2*bit3.
__device__ __forceinline__ void rs16_hi(const float (&v)[16], float& o0, float& o1) {
  const int lane = lane_id();
  float u[8], t[4];
#pragma unroll
  for (int k = 0; k < 8; ++k) u[k] = xstep32(v[k], v[k + 8]);
#pragma unroll
  for (int k = 0; k < 4; ++k) t[k] = xstep16(u[k], u[k + 4]);
  const bool h3 = (lane >> 3) & 1;
  o0 = xstep8(t[0], t[2], h3);
  o1 = xstep8(t[1], t[3], h3);
}
// Same for 8 values: the lane ends with v[4*bit5 + 2*bit4 + bit3].
__device__ __forceinline__ float rs8_hi(const float (&v)[8]) {
  const int lane = lane_id();
  float u[4], t[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = xstep32(v[k], v[k + 4]);
#pragma unroll
  for (int k = 0; k < 2; ++k) t[k] = xstep16(u[k], u[k + 2]);
  return xstep8(t[0], t[1], (lane >> 3) & 1);
}
// Reduce-scatter over the 8 lanes sharing (lane >> 3): the lane holds
// v[base], v[base + 1] with base = 8*bit2 + 4*bit1 + 2*bit0.
__device__ __forceinline__ void rs16_lo(const float (&v)[16], float& o0, float& o1) {
  const int lane = lane_id();
  float u[8], t[4];
  const bool b2 = (lane >> 2) & 1, b1 = (lane >> 1) & 1, b0 = lane & 1;
#pragma unroll
  for (int k = 0; k < 8; ++k) u[k] = xstep_small<4>(v[k], v[k + 8], b2);
#pragma unroll
  for (int k = 0; k < 4; ++k) t[k] = xstep_small<2>(u[k], u[k + 4], b1);
  o0 = xstep_small<1>(t[0], t[2], b0);
  o1 = xstep_small<1>(t[1], t[3], b0);
}
__device__ __forceinline__ float rs8_lo(const float (&v)[8]) {
  const int lane = lane_id();
  float u[4], t[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = xstep_small<4>(v[k], v[k + 4], (lane >> 2) & 1);
#pragma unroll
  for (int k = 0; k < 2; ++k) t[k] = xstep_small<2>(u[k], u[k + 2], (lane >> 1) & 1);
  return xstep_small<1>(t[0], t[1], lane & 1);
}

// Position of point p: its coordinates, or for p >= n a far point of its
// own (pairs among such points have dy^2 = inf, so w = 0 as well).
__device__ __forceinline__ float2 load_point(const float2* __restrict__ Y, int64_t p, int64_t n) {
  if (p < n) return Y[p];
  return make_float2(1e30f, 1e25f * float(p - n + 1));
}

// Partial of point p for opposite superblock k.  Grouped layout (small
// superblocks, where the finalize pass dominates): points are grouped by 16
// and each group keeps its ns slices together (16 consecutive points per
// slice), so the finalize pass reads one contiguous run per group of 16
// rows while a job still writes whole 128-byte lines.  Slice-major layout
// (large superblocks, where the partial writes dominate): slice k holds all
// n points, so a job writes S consecutive points per side.  The buffer holds
// ns * round_up(n, 16) entries either way.
__device__ __forceinline__ int64_t part_index(int64_t p, int64_t k, int64_t ns, int64_t n, bool grouped) {
  return grouped ? ((p >> 4) * ns + k) * 16 + (p & 15) : k * n + p;
}
// The layout that goes with superblock size S.
__host__ __device__ constexpr bool part_grouped(int64_t S) { return S <= 256; }

// Persistent grid: two workgroups per CU (the kernel's register use allows
// two waves per SIMD) on the 256 CUs of an MI355X.
constexpr int64_t SYM_GRID = 512;
constexpr int SYM_MAX_S = 1024;

struct SymGrid {
  int64_t S, ns, njobs, nwg;
  static SymGrid make(int64_t n) {
    SymGrid g;
    // largest S in {1024, 512, 256} that still gives each workgroup >= 4 jobs
    int64_t S = SYM_MAX_S;
    while (S > 256) {
      const int64_t ns = ceil_div(n, S);
      if (ns * (ns + 1) / 2 >= 4 * SYM_GRID) break;
      S >>= 1;
    }
    g.S = S;
    g.ns = ceil_div(n, S);
    g.njobs = g.ns * (g.ns + 1) / 2;
    g.nwg = g.njobs < SYM_GRID ? g.njobs : SYM_GRID;
    return g;
  }
};

// Job q -> superblock pair (s, t): the ns (ns - 1) / 2 pairs s < t in
// row-major order over t, then the ns diagonal pairs.
__device__ __forceinline__ void job_pair(int64_t q, int64_t ns, int64_t& s, int64_t& t) {
  const int64_t noff = ns * (ns - 1) / 2;
  if (q >= noff) {
    s = t = q - noff;
    return;
  }
  int64_t tt = int64_t((1.0 + sqrt(1.0 + 8.0 * double(q))) * 0.5);
  while (tt * (tt - 1) / 2 > q) --tt;
  while ((tt + 1) * tt / 2 <= q) ++tt;
  t = tt;
  s = q - tt * (tt - 1) / 2;
}

// Job at position pos of the dealing order: jobs [0, nF) are the full
// off-diagonal pairs (t < ns - 1), then the ns - 1 diagonal jobs s < ns - 1
// (cost per wave about nsub / 2 tiles) and the ns - 1 jobs (s, ns - 1)
// against the last superblock (nj_last tiles per subblock), the costlier
// class first, then the last diagonal job.  In job_pair's numbering the
// last-superblock jobs are [nF, noff) and the diagonal ones [noff, njobs).
__device__ __forceinline__ int64_t sym_sched(int64_t pos, int64_t ns, bool last_first) {
  const int64_t nF = (ns - 1) * (ns - 2) / 2, noff = ns * (ns - 1) / 2;
  if (last_first || pos < nF || pos == noff + ns - 1) return pos;
  return pos < nF + ns - 1 ? noff + (pos - nF) : pos - (ns - 1);
}

// One 64 x 64 wave tile.  DIAG: i and j blocks coincide; all ordered pairs
// go to the i side, self pairs masked, Z weight 1 (else 2, via the caller).
// CLEARJ: start the j-side sums at zero (else add to them).  ROWFENCE:
// keep each row's 8 pairs together in the schedule (bounds the registers
// that hold differences in flight) and spread the row's reciprocals
// evenly over it, one per ten other VALU instructions: left to itself the
// scheduler issues some reciprocals two to four instructions apart, where
// they wait on one another in the transcendental unit (12-16 % of the
// launch time).  Every caller sets it.
template <bool DIAG, bool ZROW, bool CLEARJ = true, bool ROWFENCE = false>
__device__ __forceinline__ void sym_tile(const float (&xi)[8], const float (&yi)[8], const float4 (&pjv)[4],
                                         float (&rix)[8], float (&riy)[8], float (&zi)[8], float (&rj)[16],
                                         float (&zj)[8], float& z, bool same_group) {
  float xj[8], yj[8];
#pragma unroll
  for (int c = 0; c < 8; c += 2) {
    const float4 v = pjv[c / 2];
    xj[c] = v.x;
    yj[c] = v.y;
    xj[c + 1] = v.z;
    yj[c + 1] = v.w;
  }
  if (CLEARJ) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      rj[c] = 0.0f;
      rj[8 + c] = 0.0f;
      if (ZROW) zj[c] = 0.0f;
    }
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float dx = xi[r] - xj[c], dy = yi[r] - yj[c];
      const float q = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1.0f));
      float w = __builtin_amdgcn_rcpf(q);
      if (DIAG && r == c) w = same_group ? 0.0f : w;
      z += w;
      const float w2 = w * w;
      rix[r] = __builtin_fmaf(w2, dx, rix[r]);
      riy[r] = __builtin_fmaf(w2, dy, riy[r]);
      if (ZROW) zi[r] += w;
      if (!DIAG) {
        rj[c] = __builtin_fmaf(w2, dx, rj[c]);
        rj[8 + c] = __builtin_fmaf(w2, dy, rj[8 + c]);
        if (ZROW) zj[c] += w;
      }
    }
    if (ROWFENCE) {
      // the row's 8 reciprocals spread evenly over its 88 instructions:
      // back-to-back reciprocals contend for the half-rate unit.  The
      // first four VALU form the first pair's argument; after each
      // reciprocal, ten VALU: the next pair's argument and this pair's uses
      __builtin_amdgcn_sched_group_barrier(0x0002, 4, 0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        __builtin_amdgcn_sched_group_barrier(0x0400, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x0002, 10, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// LDS layout of a workgroup (floats): ipts[2*S] | jpts[2*S] | iacc[NC*S] |
// jacc[4][NC*S] with NC = 2 (x, y) or 3 (x, y, Z_row), component-major per
// accumulator; with ATT then aacc[4][S] (64-bit).
// PF = S / 256: points per thread and side.
// Attraction entries grouped by job (built once per P): job q owns entries
// [off[q], off[q + 1]); entry e is the unordered pair {i, j}, i < j, with
// local indices packed as (i - s S) | (j - t S) << 16, and its value p_ij.
struct AttList {
  const int64_t* off;
  const uint32_t* ij;
  const float* p;
  int64_t cap;  // entries the list can hold; offsets are clamped to it
};

// Fixed-point scale of the attraction sums (see the ATT phase below).
constexpr float ATT_SCALE = 0x1p56f;

// (256, 2): two workgroups per CU (the LDS allows no more), at most 256
// registers per lane, so that two waves share each SIMD; without the bound
// the compiler lets the largest instantiation grow past 256, and one wave
// per SIMD runs it 15 % slower.
template <bool ZROW, int PF, bool ATT>
__global__ __launch_bounds__(256, 2) void rep_sym_kernel(const float2* __restrict__ Y, int64_t n, int64_t ns,
                                                      float* __restrict__ part, float* __restrict__ zpart,
                                                      double* __restrict__ Zblock, AttList att,
                                                      float2* __restrict__ apart) {
  static_assert(!(ATT && ZROW), "the fused attraction is for the gradient-only launch");
  constexpr int NC = ZROW ? 3 : 2;
  constexpr int S = 256 * PF;
  extern __shared__ __attribute__((aligned(16))) float lds[];
  __shared__ double red[4];
  float2* ipts = reinterpret_cast<float2*>(lds);
  float2* jpts = ipts + S;
  float* iacc = lds + 4 * S;
  float* jacc = iacc + NC * S;
  // subblocks per wave swept together in off-diagonal jobs, and the tiles
  // between two folds of their i-side sums into FP64 (8 j-points per tile)
  constexpr int GS = ZROW ? 1 : PF;
  constexpr int GS_FOLD = 16;
  // attraction sums of the job in 64-bit fixed point: i x, i y, j x, j y.
  // Small superblocks have room for a separate array; the largest reuse the
  // j accumulators before the pair tiles need them (ATT_SEP false).
  constexpr bool ATT_SEP = PF < 4;
  constexpr bool ATT_PRE = ATT && PF < 4;  // registers allow the entry prefetch
  unsigned long long* aacc = reinterpret_cast<unsigned long long*>(ATT_SEP ? jacc + SYM_WAVES * NC * S : jacc);
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  const int a = lane >> 3, b = lane & 7;
  const int nsub = S / 64;
  const int64_t njobs = ns * (ns + 1) / 2;
  const int64_t P = gridDim.x;
  float* myj = jacc + w * NC * S;

  // points of job q into registers (thread tid holds points tid + 256 k),
  // and the job's superblock pair (fs, ft)
  float2 pi[PF], pj[PF];
  int64_t fs = 0, ft = 0;
  auto fetch = [&](int64_t q) {
    job_pair(q, ns, fs, ft);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int u = tid + 256 * k;
      pi[k] = load_point(Y, fs * S + u, n);
      pj[k] = load_point(Y, ft * S + u, n);
    }
  };
  // attraction entries: the next job's range and first two entries per
  // thread are loaded while the current job computes
  int64_t ne0 = 0, ne1 = 0;
  uint32_t npk[2] = {0u, 0u};
  float npv[2] = {0.0f, 0.0f};
  auto fetch_range = [&](int64_t q) {
    ne0 = min(att.off[q], att.cap);
    ne1 = min(att.off[q + 1], att.cap);
  };
  auto fetch_entries = [&]() {
    if (!ATT_PRE) return;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int64_t e = ne0 + tid + 256 * m;
      npk[m] = e < ne1 ? att.ij[e] : 0u;
      npv[m] = e < ne1 ? att.p[e] : 0.0f;
    }
  };

  // attraction partials of job (s, t): the exact fixed-point sums, rounded
  // once; the accumulators are cleared for the next use
  auto write_att = [&](int64_t s, int64_t t, bool diag_sb) {
    const double sc = 1.0 / double(ATT_SCALE);
    for (int u = tid; u < S; u += 256) {
      const double aix = double((long long)aacc[u]), aiy = double((long long)aacc[S + u]);
      const double ajx = double((long long)aacc[2 * S + u]), ajy = double((long long)aacc[3 * S + u]);
#pragma unroll
      for (int c = 0; c < 4; ++c) aacc[c * S + u] = 0ull;
      const int64_t pi_ = s * S + u, pj_ = t * S + u;
      if (diag_sb) {
        if (pi_ < n)
          apart[part_index(pi_, t, ns, n, part_grouped(S))] =
              make_float2(float((aix + ajx) * sc), float((aiy + ajy) * sc));
      } else {
        if (pi_ < n) apart[part_index(pi_, t, ns, n, part_grouped(S))] = make_float2(float(aix * sc), float(aiy * sc));
        if (pj_ < n) apart[part_index(pj_, s, ns, n, part_grouped(S))] = make_float2(float(ajx * sc), float(ajy * sc));
      }
    }
  };

  // this workgroup's job of round r, or -1 past the last
  const int64_t nj_last = min(int64_t(nsub), (n - (ns - 1) * S + 63) / 64);
  const bool last_first = 2 * nj_last > nsub + 1;
  auto job_at = [&](int64_t r) -> int64_t {
    const int64_t pos = r * P + ((r & 1) ? P - 1 - int64_t(blockIdx.x) : int64_t(blockIdx.x));
    return pos < njobs ? sym_sched(pos, ns, last_first) : -1;
  };
  int64_t rnd = 0;
  int64_t q = job_at(0);
  if (q >= 0) {
    fetch(q);
    if (ATT_PRE) {
      fetch_range(q);
      fetch_entries();
    }
  }
  for (int u = tid; u < NC * S; u += 256) iacc[u] = 0.0f;
  for (int u = tid; u < SYM_WAVES * NC * S; u += 256) jacc[u] = 0.0f;
  if (ATT_SEP && ATT)
    for (int u = tid; u < 4 * S; u += 256) aacc[u] = 0ull;
  double zsum = 0.0;
  for (; q >= 0; q = job_at(++rnd)) {
    const int64_t s = fs, t = ft;  // job q, decoded by its fetch
    const int64_t qn = job_at(rnd + 1);
    const bool diag_sb = s == t;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int u = tid + 256 * k;
      ipts[u] = pi[k];
      jpts[u] = pj[k];
    }
    __syncthreads();  // points staged, accumulators zeroed
    if (qn >= 0) fetch(qn);  // lands while this job computes

    if (ATT) {
      // Attraction of the job's P entries, A_i += p w (y_i - y_j) and
      // A_j -= p w (y_i - y_j), from the staged points, before the pair
      // tiles.  The sums are kept in 64-bit fixed point (scale 2^56), so
      // the integer LDS atomics give an exact, order-independent
      // (deterministic) result; |p w (y_i - y_j)| <= p / 2 and a row's p
      // sum to at most 1 keep every sum below 2^55.
      if (!ATT_PRE) fetch_range(q);  // (no prefetch: keep registers free)
      const int64_t ae0 = ne0, ae1 = ne1;
      const uint32_t pk0 = npk[0], pk1 = npk[1];
      const float pv0 = npv[0], pv1 = npv[1];
      if (ATT_PRE && qn >= 0) fetch_range(qn);  // used after the tiles
      auto add_entry = [&](uint32_t pk, float pv) {
        const int il = int(pk & 0xFFFFu), jl = int(pk >> 16);
        const float2 yi = ipts[il], yj = jpts[jl];
        const float dx = yi.x - yj.x, dy = yi.y - yj.y;
        const float c = pv * __builtin_amdgcn_rcpf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1.0f)));
        const long long fx = __float2ll_rn(c * dx * ATT_SCALE), fy = __float2ll_rn(c * dy * ATT_SCALE);
        atomicAdd(&aacc[il], (unsigned long long)fx);
        atomicAdd(&aacc[S + il], (unsigned long long)fy);
        atomicAdd(&aacc[2 * S + jl], (unsigned long long)(-fx));
        atomicAdd(&aacc[3 * S + jl], (unsigned long long)(-fy));
      };
      int64_t e = ae0 + tid;
      if (ATT_PRE) {
        if (e < ae1) add_entry(pk0, pv0);
        if (e + 256 < ae1) add_entry(pk1, pv1);
        e += 512;
      }
      for (; e < ae1; e += 256) add_entry(att.ij[e], att.p[e]);
      if (!ATT_SEP) {
        __syncthreads();
        write_att(s, t, diag_sb);  // and clear: the pair tiles accumulate there next
        __syncthreads();
      }
    }

    // subblocks past the last point are skipped: a padded point sits at
    // 1e30, so every pair with it has weight exactly 0 and adds exact zeros
    // (the result is the same bits as with them)
    const int ni_end = int(min(int64_t(nsub), (n - s * S + 63) / 64));
    const int nj_end = int(min(int64_t(nsub), (n - t * S + 63) / 64));
    if (GS > 1 && !diag_sb) {
      // Off-diagonal job (superblock s is full): the wave's GS subblocks
      // us = w + 4 k are swept together, the j-tiles in the outer loop, so
      // one reduce-scatter carries the j-side sums of GS 64 x 64 tiles.
      float xi[GS][8], yi[GS][8], rix[GS][8], riy[GS][8];
      double di[GS][2];
#pragma unroll
      for (int k = 0; k < GS; ++k) {
        const int us = w + SYM_WAVES * k;
#pragma unroll
        for (int r = 0; r < 8; r += 2) {
          const float4 v = *reinterpret_cast<const float4*>(ipts + 64 * us + 8 * a + r);
          xi[k][r] = v.x;
          yi[k][r] = v.y;
          xi[k][r + 1] = v.z;
          yi[k][r + 1] = v.w;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) rix[k][r] = riy[k][r] = 0.0f;
        di[k][0] = di[k][1] = 0.0;
      }
      auto fold_all = [&]() {
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          float vi[16];
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            vi[r] = rix[k][r];
            vi[8 + r] = riy[k][r];
            rix[k][r] = riy[k][r] = 0.0f;
          }
          float o0, o1;
          rs16_lo(vi, o0, o1);
          di[k][0] += double(o0);
          di[k][1] += double(o1);
        }
      };
      const int comp = lane >> 5;
      const int c0 = 2 * ((lane >> 3) & 1) + 4 * ((lane >> 4) & 1);
      int since_fold = 0;
      for (int v = 0; v < nj_end; ++v) {
        float4 jc[4];
        {
          const float4* p = reinterpret_cast<const float4*>(jpts + 64 * v + 8 * b);
#pragma unroll
          for (int c = 0; c < 4; ++c) jc[c] = p[c];
        }
        float2* dst = reinterpret_cast<float2*>(myj + comp * S + 64 * v + 8 * b + c0);
        float2 cur = *dst;
        float rj[16], zj[8], zi[8];
        float z = 0.0f;
#pragma unroll
        for (int c = 0; c < 16; ++c) rj[c] = 0.0f;
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          sym_tile<false, false, false, true>(xi[k], yi[k], jc, rix[k], riy[k], zi, rj, zj, z, false);
          // keep the scheduler from interleaving the GS tiles (their live
          // differences would not fit the register file)
          __builtin_amdgcn_sched_barrier(0);
        }
        // z complete here: otherwise its chain of adds is sunk below the
        // fold and every w of the tiles stays live until then
        asm volatile("" : "+v"(z));
        zsum += 2.0 * double(z);
        float o0, o1;
        rs16_hi(rj, o0, o1);
        cur.x += o0;
        cur.y += o1;
        *dst = cur;
        if (++since_fold == GS_FOLD) {
          since_fold = 0;
          fold_all();
        }
      }
      if (since_fold) fold_all();
      {
        const int comp = (lane >> 2) & 1;
        const int c0 = 2 * (lane & 1) + 4 * ((lane >> 1) & 1);
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          float* dst = iacc + comp * S + 64 * (w + SYM_WAVES * k) + 8 * a + c0;
          dst[0] = float(di[k][0]);
          dst[1] = float(di[k][1]);
        }
      }
    } else
    for (int us = w; us < ni_end; us += SYM_WAVES) {
      // this wave's i-subblock us: points s S + 64 us + 8a + r
      float xi[8], yi[8];
#pragma unroll
      for (int r = 0; r < 8; r += 2) {
        const float4 v = *reinterpret_cast<const float4*>(ipts + 64 * us + 8 * a + r);
        xi[r] = v.x;
        yi[r] = v.y;
        xi[r + 1] = v.z;
        yi[r + 1] = v.w;
      }
      float rix[8], riy[8], zi[8];
      // after each fold this lane owns component bit2 of points 8a + c0 and
      // 8a + c0 + 1 (c0 = 4 bit1 + 2 bit0), and Z_row of point 8a + cz
      double di[2] = {0.0, 0.0}, dz = 0.0;
#pragma unroll
      for (int r = 0; r < 8; ++r) rix[r] = riy[r] = zi[r] = 0.0f;
      // fold the i-side sums into FP64 (after an 8-lane reduce)
      auto fold = [&]() {
        float vi[16];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          vi[r] = rix[r];
          vi[8 + r] = riy[r];
          rix[r] = riy[r] = 0.0f;
        }
        float o0, o1;
        rs16_lo(vi, o0, o1);
        di[0] += double(o0);
        di[1] += double(o1);
        if (ZROW) {
          const float oz = rs8_lo(zi);
          dz += double(oz);
#pragma unroll
          for (int r = 0; r < 8; ++r) zi[r] = 0.0f;
        }
      };
      // tiles of this subblock: j-subblocks 0 .. nj_end - 1, or in the
      // diagonal superblock us, us + 1, ... (mod nsub), cyclic distance up
      // to nsub / 2, taken only for us < nsub / 2 (every unordered pair once)
      const int ntile = diag_sb ? (us < nsub / 2 ? nsub / 2 + 1 : nsub / 2) : nj_end;
      int since_fold = 0;
      const int comp = lane >> 5;
      const int c0 = 2 * ((lane >> 3) & 1) + 4 * ((lane >> 4) & 1);
      for (int e = 0; e < ntile; ++e) {
        const int v = diag_sb ? (us + e < nsub ? us + e : us + e - nsub) : e;
        if (v >= nj_end) continue;  // past the last point (partly filled superblock)
        float4 jc[4];
        {
          const float4* p = reinterpret_cast<const float4*>(jpts + 64 * v + 8 * b);
#pragma unroll
          for (int c = 0; c < 4; ++c) jc[c] = p[c];
        }
        float rj[16], zj[8];
        float z = 0.0f;
        if (diag_sb && v == us) {
          sym_tile<true, ZROW, true, true>(xi, yi, jc, rix, riy, zi, rj, zj, z, a == b);
          zsum += double(z);
        } else {
          // this tile's slot of the wave's j accumulator, read early
          float2* dst = reinterpret_cast<float2*>(myj + comp * S + 64 * v + 8 * b + c0);
          float2 cur = *dst;
          sym_tile<false, ZROW, true, true>(xi, yi, jc, rix, riy, zi, rj, zj, z, false);
          zsum += 2.0 * double(z);
          // j side: reduce over the 8 lanes of this j-group, add into LDS
          float o0, o1;
          rs16_hi(rj, o0, o1);
          cur.x += o0;
          cur.y += o1;
          *dst = cur;
          if (ZROW) {
            const float oz = rs8_hi(zj);
            const int cz = 4 * ((lane >> 5) & 1) + 2 * ((lane >> 4) & 1) + ((lane >> 3) & 1);
            myj[2 * S + 64 * v + 8 * b + cz] += oz;
          }
        }
        if (++since_fold == 8) {
          since_fold = 0;
          fold();
        }
      }
      if (since_fold) fold();
      // i side of this subblock -> LDS (each point owned by exactly one wave)
      {
        const int comp = (lane >> 2) & 1;
        const int c0 = 2 * (lane & 1) + 4 * ((lane >> 1) & 1);
        float* dst = iacc + comp * S + 64 * us + 8 * a + c0;
        dst[0] = float(di[0]);
        dst[1] = float(di[1]);
        if (ZROW) {
          const int cz = 4 * ((lane >> 2) & 1) + 2 * ((lane >> 1) & 1) + (lane & 1);
          iacc[2 * S + 64 * us + 8 * a + cz] = float(dz);
        }
      }
    }
    // the next job's first attraction entries (its range arrived meanwhile)
    if (ATT_PRE && qn >= 0) fetch_entries();
    __syncthreads();  // job's accumulators complete; staged points free

    // write the partials part[t][i in s] and part[s][j in t]; each thread
    // clears the accumulator entries it read, for the next job
    const int64_t i0 = s * S, j0 = t * S;
    for (int u = tid; u < S; u += 256) {
      float jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
      for (int ww = 0; ww < SYM_WAVES; ++ww) {
        jx += jacc[ww * NC * S + u];
        jy += jacc[ww * NC * S + S + u];
        if (ZROW) jz += jacc[ww * NC * S + 2 * S + u];
        jacc[ww * NC * S + u] = 0.0f;
        jacc[ww * NC * S + S + u] = 0.0f;
        if (ZROW) jacc[ww * NC * S + 2 * S + u] = 0.0f;
      }
      const float ix = iacc[u], iy = iacc[S + u], iz = ZROW ? iacc[2 * S + u] : 0.0f;
      iacc[u] = 0.0f;
      iacc[S + u] = 0.0f;
      if (ZROW) iacc[2 * S + u] = 0.0f;
      const int64_t pi_ = i0 + u, pj_ = j0 + u;
      if (diag_sb) {
        if (pi_ < n) {
          reinterpret_cast<float2*>(part)[part_index(pi_, t, ns, n, part_grouped(S))] = make_float2(ix - jx, iy - jy);
          if (ZROW) zpart[part_index(pi_, t, ns, n, part_grouped(S))] = iz + jz;
        }
      } else {
        if (pi_ < n) {
          reinterpret_cast<float2*>(part)[part_index(pi_, t, ns, n, part_grouped(S))] = make_float2(ix, iy);
          if (ZROW) zpart[part_index(pi_, t, ns, n, part_grouped(S))] = iz;
        }
        if (pj_ < n) {
          reinterpret_cast<float2*>(part)[part_index(pj_, s, ns, n, part_grouped(S))] = make_float2(-jx, -jy);
          if (ZROW) zpart[part_index(pj_, s, ns, n, part_grouped(S))] = jz;
        }
      }
    }
    if (ATT_SEP && ATT) write_att(s, t, diag_sb);  // its atomics finished before the barrier above
  }
  const double bz = block_sum_d(zsum, red);
  if (tid == 0) Zblock[blockIdx.x] = bz;
}

// Z alone (the KL's forward): the sum of w over all ordered pairs i != j
// with the decomposition, job dealing and diagonal tiles of rep_sym_kernel
// but no per-point sums, so a pair costs the two differences, the two FMAs
// of q, the reciprocal and one add.  Per workgroup one FP64 partial (each
// tile's FP32 sum folded into FP64), in Zblock[blockIdx.x].
template <bool DIAG>
__device__ __forceinline__ void sym_tile_z(const float (&xi)[8], const float (&yi)[8], const float4 (&pjv)[4],
                                           float& z, bool same_group) {
  float xj[8], yj[8];
#pragma unroll
  for (int c = 0; c < 8; c += 2) {
    const float4 v = pjv[c / 2];
    xj[c] = v.x;
    yj[c] = v.y;
    xj[c + 1] = v.z;
    yj[c + 1] = v.w;
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float dx = xi[r] - xj[c], dy = yi[r] - yj[c];
      float w = __builtin_amdgcn_rcpf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1.0f)));
      if (DIAG && r == c) w = same_group ? 0.0f : w;
      z += w;
    }
    // one reciprocal per five other VALU, as in sym_tile
    __builtin_amdgcn_sched_group_barrier(0x0002, 4, 0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      __builtin_amdgcn_sched_group_barrier(0x0400, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x0002, 5, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int PF>
__global__ __launch_bounds__(256) void zsum_sym_kernel(const float2* __restrict__ Y, int64_t n, int64_t ns,
                                                       double* __restrict__ Zblock) {
  constexpr int S = 256 * PF;
  __shared__ __attribute__((aligned(16))) float2 ipts[S];
  __shared__ __attribute__((aligned(16))) float2 jpts[S];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  const int a = lane >> 3, b = lane & 7;
  const int nsub = S / 64;
  const int64_t njobs = ns * (ns + 1) / 2;
  const int64_t P = gridDim.x;
  const int64_t nj_last = min(int64_t(nsub), (n - (ns - 1) * S + 63) / 64);
  const bool last_first = 2 * nj_last > nsub + 1;
  double zsum = 0.0;
  for (int64_t rnd = 0;; ++rnd) {
    const int64_t pos = rnd * P + ((rnd & 1) ? P - 1 - int64_t(blockIdx.x) : int64_t(blockIdx.x));
    if (pos >= njobs) break;
    int64_t s, t;
    job_pair(sym_sched(pos, ns, last_first), ns, s, t);
    const bool diag_sb = s == t;
    __syncthreads();  // the previous job's points are no longer read
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int u = tid + 256 * k;
      ipts[u] = load_point(Y, s * S + u, n);
      jpts[u] = load_point(Y, t * S + u, n);
    }
    __syncthreads();
    const int ni_end = int(min(int64_t(nsub), (n - s * S + 63) / 64));
    const int nj_end = int(min(int64_t(nsub), (n - t * S + 63) / 64));
    for (int us = w; us < ni_end; us += SYM_WAVES) {
      float xi[8], yi[8];
#pragma unroll
      for (int r = 0; r < 8; r += 2) {
        const float4 v = *reinterpret_cast<const float4*>(ipts + 64 * us + 8 * a + r);
        xi[r] = v.x;
        yi[r] = v.y;
        xi[r + 1] = v.z;
        yi[r + 1] = v.w;
      }
      const int ntile = diag_sb ? (us < nsub / 2 ? nsub / 2 + 1 : nsub / 2) : nj_end;
      for (int e = 0; e < ntile; ++e) {
        const int v = diag_sb ? (us + e < nsub ? us + e : us + e - nsub) : e;
        if (v >= nj_end) continue;
        float4 jc[4];
        const float4* p = reinterpret_cast<const float4*>(jpts + 64 * v + 8 * b);
#pragma unroll
        for (int c = 0; c < 4; ++c) jc[c] = p[c];
        float z = 0.0f;
        if (diag_sb && v == us) {
          sym_tile_z<true>(xi, yi, jc, z, a == b);
          zsum += double(z);
        } else {
          sym_tile_z<false>(xi, yi, jc, z, false);
          zsum += 2.0 * double(z);
        }
      }
    }
  }
  const double bz = block_sum_d(zsum, red);
  if (tid == 0) Zblock[blockIdx.x] = bz;
}

inline size_t rep_sym_lds_bytes(int64_t S, bool zrow, bool att) {
  const int nc = zrow ? 3 : 2;
  const bool sep = att && S < 1024;  // ATT_SEP of the kernel
  return sizeof(float) * size_t(S) * size_t(4 + nc + SYM_WAVES * nc) + (sep ? 4 * sizeof(uint64_t) * size_t(S) : 0);
}

}  // namespace tsne
