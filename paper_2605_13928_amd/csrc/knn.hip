// tsne_knn: exact k nearest neighbours by squared Euclidean distance
// (the kNN input of tree-accelerated t-SNE, van der Maaten 2014, Sec. 4.1),
// in two precisions:
//   FP32  -- distances as FP32 direct differences on the VALU;
//   BF16  -- distances between bf16-rounded points from MFMA tiles
//            (v_mfma_f32_16x16x32_bf16, FP32 accumulation; the norms ride
//            in spare K slots, so the tile output IS the distance), the
//            n_cand best per row kept, then re-ranked by FP32 direct
//            differences on the original points.
// Selection (both paths): every row owns a candidate buffer in global
// memory, a count in LDS and a threshold tau in registers of the wave that
// owns the row.  A candidate with d <= tau is appended; a lane reserves the
// slots of all its candidates of one row and step with one LDS atomic.  Before a
// buffer could overflow, the owning wave finds the k-th smallest distance
// tau by a radix select, keeps the keys with d <= tau and makes tau the
// new threshold.  The true k best always satisfy d <= tau, so nothing is
// lost; ties at tau are kept and resolved by index in the final sort (a
// wave-wide bitonic sort of the (d, j) keys).  Since the kept keys are the
// best ones whatever order the candidates arrive in, both paths sweep them
// in a locality order (points sorted by a Morton key of their leading
// coordinates, each query block starting next to its own queries), so that
// tau is tight after a few tiles and few candidates are appended, and skip
// the candidate tiles whose bounding box lies beyond every threshold of
// the block (a bound that leaves the results those of the full sweep).
#include <cfloat>
#include <type_traits>

#include "common.hpp"
#include "scan.hpp"

namespace tsne {

// ---------------------------------------------------------------------
// Candidate buffers.

// A row's buffer is only ever written and read by the wave that owns the
// row, so workgroup scope suffices: wait for this wave's stores, no cache
// write-back or invalidation beyond the CU.
__device__ __forceinline__ void wg_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// Inclusive prefix sum over the 64 lanes of a wave, in DPP: shifts by 1, 2,
// 4 and 8 within each row of 16 (lanes shifted in from outside the row add
// 0), then row 0's total into row 1 and row 2's into row 3 (row_bcast:15),
// then lane 31's running total into rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1 and 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Shrink a row's buffer of c keys to the keys whose distance is at most the
// keep-th smallest distance tau_d (all of the best `keep` by (d, j), plus
// any further keys tied at tau_d), and set tau = tau_d.  tau_d is found by
// a radix select on the distance bits (8 bits per pass, histograms in the
// wave's 256-entry LDS array `hist`), so no sort is needed; the kept keys
// are written in lane order.  If ties would leave more than `limit` keys,
// the buffer is sorted instead and exactly `keep` are kept.  Returns the new
// count.  Called by the whole wave with uniform arguments, c > keep.
template <int EPL>
__device__ int compact_row(uint64_t* __restrict__ buf, int c, int keep, int limit, float& tau,
                           uint32_t* __restrict__ hist) {
  const int lane = lane_id();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  wg_fence();  // earlier appends of this wave visible to the loads below
  uint64_t v[EPL];
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int e = t * 64 + lane;
    v[t] = e < c ? buf[e] : KEY_MAX;
  }
  uint32_t prefix = 0, pmask = 0;
  int k = keep, eq = 0;
#pragma unroll
  for (int shift = 24; shift >= 0; shift -= 8) {
#pragma unroll
    for (int u = 0; u < 4; ++u) hist[lane * 4 + u] = 0;
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      const uint32_t d = uint32_t(v[t] >> 32);
      if (t * 64 + lane < c && (d & pmask) == prefix) atomicAdd(&hist[(d >> shift) & 255u], 1u);
    }
    uint32_t h[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) h[u] = hist[lane * 4 + u];
    const int local = int(h[0] + h[1] + h[2] + h[3]);
    const int incl = wave_incl_scan(local);
    const int excl = incl - local;
    const uint64_t owner = __ballot(excl < k && k <= incl);  // exactly one lane
    const int L = __ffsll((unsigned long long)owner) - 1;
    int run = excl, bin = lane * 4, hb = 0;
    {
      // first bin of this lane whose cumulative count reaches k
      int acc = excl;
      bool found = false;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!found && acc + int(h[u]) >= k) {
          found = true;
          bin = lane * 4 + u;
          hb = int(h[u]);
          run = acc;
        }
        acc += int(h[u]);
      }
    }
    bin = __builtin_amdgcn_readlane(bin, L);
    run = __builtin_amdgcn_readlane(run, L);
    hb = __builtin_amdgcn_readlane(hb, L);
    prefix |= uint32_t(bin) << shift;
    pmask |= 0xFFu << shift;
    k -= run;
    eq = hb;
  }
  const int kept = (keep - k) + eq;  // keys with d < tau_d, plus those equal
  if (kept <= limit) {
    int base = 0;
#pragma unroll
    for (int t = 0; t < EPL; ++t) {
      const bool take = t * 64 + lane < c && uint32_t(v[t] >> 32) <= prefix;
      const uint64_t m = __ballot(take);
      if (take) buf[base + __popcll(m & lt)] = v[t];
      base += __popcll(m);
    }
    tau = __uint_as_float(prefix);
    wg_fence();
    return kept;
  }
  // many keys tied at tau_d: sort and keep exactly `keep`
  wave_sort<EPL>(v);
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int e = t * 64 + lane;
    if (e < keep) buf[e] = v[t];
  }
  tau = key_dist(wave_pick<EPL>(v, keep - 1));
  wg_fence();
  return keep;
}

// Sort a row's buffer and write its first `keep` keys out.
template <int EPL>
__device__ void emit_row(const uint64_t* __restrict__ buf, int c, int keep, int32_t* __restrict__ oidx,
                         float* __restrict__ od2) {
  const int lane = lane_id();
  wg_fence();
  uint64_t v[EPL];
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int e = t * 64 + lane;
    v[t] = e < c ? buf[e] : KEY_MAX;
  }
  wave_sort<EPL>(v);
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int e = t * 64 + lane;
    if (e < keep) {
      oidx[e] = key_index(v[t]);
      if (od2) od2[e] = key_dist(v[t]);
    }
  }
}

// ---------------------------------------------------------------------
// Tile skipping (both paths).  The points are put in a locality order
// (below), so that a tile of consecutive positions is narrow in the leading
// coordinates; a tile whose box is farther from the box of a wave's
// queries than every threshold of the wave can hold no candidate for it,
// so the wave skips it, and the block fetches only the tiles some wave
// needs.  Boxes span the leading BOX_D coordinates.
constexpr int BOX_D = 16;

// ---------------------------------------------------------------------
// FP32 exact path.  Block = 4 waves x RW rows (RW = 16, or 8 where that
// gives the busiest CU fewer rows: fknn_small_blocks); each step covers 128
// columns, 2 per lane; the rows' coordinates are LDS broadcasts, the
// columns' are per-lane LDS reads, dimension chunks of 56.  Rows and
// columns are positions of the locality order (Xs = X in that order; perm
// maps a position to its point, which keys and outputs name); a block
// sweeps the column tiles cyclically from the one before its own rows and
// skips those the box tests of its waves rule out.

constexpr int F_COLS = 128;
constexpr int F_DC = 56;
constexpr int XJ_S = F_COLS + 4;  // LDS row strides: multiples of 4 floats keep the
                                  // 16-byte reads aligned and spread the stores' banks
// Three blocks of either size are resident per CU (LDS and registers), on
// 256 CUs.  32-row blocks are taken when all of them are resident at once
// and the CU with the most blocks then holds fewer rows than with 64-row
// blocks (20 k points: 3 x 32 = 96 rows against 2 x 64 = 128).
constexpr int64_t F_CUS = 256, F_RESIDENT = 3;
inline bool fknn_small_blocks(int64_t n) {
  const int64_t b8 = ceil_div(n, 32), b16 = ceil_div(n, 64);
  return b8 <= F_CUS * F_RESIDENT && ceil_div(b8, F_CUS) * 32 < ceil_div(b16, F_CUS) * 64;
}

// Stage rows [r0, r0 + nrows) x dims [dc, dc + dl) of X transposed into
// dst[c * stride + r]: one row per wave instruction (coalesced), rows past
// n as zeros.
__device__ __forceinline__ void stage_rows_t(float* __restrict__ dst, int stride, const float* __restrict__ X,
                                             int64_t r0, int nrows, int64_t n, int d, int dc, int dl) {
  const int lane = lane_id(), w = threadIdx.x >> 6;
  for (int r = w; r < nrows; r += 16) {
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int rr = r + 4 * u;
      const int64_t g = r0 + rr;
      v[u] = (rr < nrows && g < n && lane < dl) ? X[g * d + dc + lane] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int rr = r + 4 * u;
      if (rr < nrows && lane < dl) dst[lane * stride + rr] = v[u];
    }
  }
}

// Boxes of the FP32 column tiles: tile u holds positions F_COLS u ..
// F_COLS u + F_COLS - 1 of Xs (those below n); box[u][c] = (min, max) of
// coordinate c < BOX_D ((0, 0) past d; NaN left out).  Lane 16 g + c scans
// coordinate c of rows g, g + 4, ...; the four groups merge by lane
// exchange.
__global__ __launch_bounds__(256) void f32_box_kernel(const float* __restrict__ Xs, int64_t n, int d, int64_t ntiles,
                                                      float2* __restrict__ box) {
  const int lane = lane_id(), c = lane & 15, g = lane >> 4;
  const int64_t u = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (u >= ntiles) return;
  const int64_t r0 = u * F_COLS;
  const int rows = int(n - r0 < F_COLS ? n - r0 : F_COLS);
  float lo = INFINITY, hi = -INFINITY;
  if (c < d) {
    for (int r = g; r < rows; r += 4) {
      const float v = Xs[(r0 + r) * d + c];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
  }
  lo = fminf(lo, xor_lane_f(lo, 16));
  lo = fminf(lo, xor_lane_f(lo, 32));
  hi = fmaxf(hi, xor_lane_f(hi, 16));
  hi = fmaxf(hi, xor_lane_f(hi, 32));
  if (lane < BOX_D) box[u * BOX_D + lane] = lane < d ? make_float2(lo, hi) : make_float2(0.0f, 0.0f);
}

// Xs[p] = X[perm[p]]: the rows in the locality order, one wave per row.
__global__ __launch_bounds__(256) void gather_rows_kernel(const float* __restrict__ X, int64_t n, int d,
                                                          const int32_t* __restrict__ perm, float* __restrict__ Xs) {
  const int64_t p = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (p >= n) return;
  const int64_t src = perm[p];
  for (int c = lane_id(); c < d; c += 64) Xs[p * d + c] = X[src * d + c];
}

// Skipping test of the FP32 path.  Its distance sums d non-negative terms
// (a rounded difference, squared and added by one FMA each), so it is at
// least (1 - (d + 2) u) >= 1 - 2^-15 of the exact one for d <= 256; the
// box bound LB (16 terms) is within 2^-19 of exact.  With the box of a
// wave's 16 rows, LB (1 - 2^-12) > tau_max (the wave's largest threshold)
// therefore means every distance of the tile exceeds every threshold of
// the wave: it would append nothing for it, and skipping it leaves the
// buffers, and the outputs, as the full sweep makes them.  The block
// stages the tiles that some wave evaluates (the OR of the waves' window
// masks, exchanged through LDS).
template <int EPL, int F_RW>
__global__ __launch_bounds__(256, 3) void knn_fp32_kernel(const float* __restrict__ Xs, const int32_t* __restrict__ perm,
                                                       const float4* __restrict__ cbox4, int64_t n, int d, int k,
                                                       uint64_t* __restrict__ bufs, int32_t* __restrict__ out_idx,
                                                       float* __restrict__ out_d2) {
  static_assert(F_RW == 8 || F_RW == 16, "rows per wave");
  constexpr int F_ROWS = 4 * F_RW;
  constexpr int XI_S = F_ROWS + 4;
  constexpr int CAP = 64 * EPL;
  __shared__ __attribute__((aligned(16))) float xi_s[F_DC * XI_S];
  __shared__ __attribute__((aligned(16))) float xj_s[F_DC * XJ_S];
  __shared__ uint32_t hist_s[4][256];  // per-wave radix-select histograms
  __shared__ int32_t pj_s[F_COLS];     // the points of the staged columns
  __shared__ float4 qbox[4][BOX_D / 2];  // box of each wave's rows: (lo, hi) of two coordinates each
  __shared__ uint64_t wmask_s[2][4];     // each wave's live positions, by window parity
  const int tid = threadIdx.x, lane = lane_id(), w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t row0 = int64_t(blockIdx.x) * F_ROWS;
  __shared__ int cnt_s[F_ROWS];  // buffer counts (appended by LDS atomics)
  if (tid < F_ROWS) cnt_s[tid] = 0;  // published by the first barrier
  // per row of this wave (uniform): threshold
  float tau[F_RW];
#pragma unroll
  for (int r = 0; r < F_RW; ++r) tau[r] = row0 + w * F_RW + r < n ? INFINITY : -INFINITY;  // rows past n never accept
  const int64_t wrow0 = row0 + w * F_RW;  // this wave's rows
  const bool has_rows = wrow0 < n;
  {
    // this wave's box (rows past n left out)
    const int c = lane & 15, g = lane >> 4;
    float lo = INFINITY, hi = -INFINITY;
    if (c < d) {
      for (int r = g; r < F_RW && wrow0 + r < n; r += 4) {
        const float v = Xs[(wrow0 + r) * d + c];
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
      }
    }
    lo = fminf(lo, xor_lane_f(lo, 16));
    lo = fminf(lo, xor_lane_f(lo, 32));
    hi = fmaxf(hi, xor_lane_f(hi, 16));
    hi = fmaxf(hi, xor_lane_f(hi, 32));
    if (lane < BOX_D)
      reinterpret_cast<float2*>(qbox[w])[lane] = lane < d ? make_float2(lo, hi) : make_float2(0.0f, 0.0f);
  }
  const bool one_chunk = d <= F_DC;
  if (one_chunk) stage_rows_t(xi_s, XI_S, Xs, row0, F_ROWS, n, d, 0, d);
  const int ntc = int((n + F_COLS - 1) / F_COLS);
  int tstart = int(row0 / F_COLS) - 1;
  if (tstart < 0) tstart += ntc;
  auto tile_of = [&](int it) -> int {
    const int ti = tstart + it;
    return ti < ntc ? ti : ti - ntc;
  };
  // live positions of the window [p0, p0 + 64): this wave's (returned) and
  // the block's (any wave's, in `blk`); called by all waves together
  int wpar = 0;
  auto window = [&](int p0, uint64_t& blk) -> uint64_t {
    // this wave's largest threshold now (uniform per row; rows past n hold -inf)
    float tm = tau[0];
#pragma unroll
    for (int r = 1; r < F_RW; ++r) tm = fmaxf(tm, tau[r]);
    const int p = p0 + lane;
    bool live = has_rows && p < ntc;
    if (tm < INFINITY) {
      const float4* tb = cbox4 + tile_of(live ? p : 0) * (BOX_D / 2);
      float lb = 0.0f;
#pragma unroll 2
      for (int h = 0; h < BOX_D / 2; ++h) {
        const float4 v = tb[h], q = qbox[w][h];  // (lo, hi) of coordinates 2h and 2h + 1
        const float g0 = fmaxf(fmaxf(v.x - q.y, q.x - v.y), 0.0f);
        const float g1 = fmaxf(fmaxf(v.z - q.w, q.z - v.w), 0.0f);
        lb = fmaf(g0, g0, lb);
        lb = fmaf(g1, g1, lb);
      }
      live = live && !(lb * (1.0f - 1.0f / 4096.0f) > tm);
    }
    const uint64_t mine = __ballot(live);
    // two buffers: a wave may write the next window's mask while another
    // still reads this one's
    if (lane == 0) wmask_s[wpar][w] = mine;
    __syncthreads();
    blk = wmask_s[wpar][0] | wmask_s[wpar][1] | wmask_s[wpar][2] | wmask_s[wpar][3];
    wpar ^= 1;
    return mine;
  };
  int wb = -64;  // first position of the current window (none yet)
  uint64_t win = 0, mine = 0;
  int from = 0;
  for (;;) {
    __syncthreads();  // every wave is done with the previous tile
    // the next position some wave evaluates
    int pos = from;
    bool pos_mine = false;
    while (pos < ntc) {
      if (pos >= wb + 64) {
        wb = pos;
        mine = window(wb, win);
      }
      const uint64_t m = win >> (pos - wb);
      if (m) {
        pos += __builtin_ctzll(m);
        pos_mine = (mine >> (pos - wb)) & 1;
        break;
      }
      pos = wb + 64;
    }
    if (pos >= ntc) break;
    const int64_t c0 = int64_t(tile_of(pos)) * F_COLS;
    float acc[F_RW][2];
#pragma unroll
    for (int r = 0; r < F_RW; ++r) acc[r][0] = acc[r][1] = 0.0f;
    for (int dc = 0; dc < d; dc += F_DC) {
      const int dl = (d - dc) < F_DC ? (d - dc) : F_DC;
      if (dc > 0) __syncthreads();
      if (!one_chunk) stage_rows_t(xi_s, XI_S, Xs, row0, F_ROWS, n, d, dc, dl);
      stage_rows_t(xj_s, XJ_S, Xs, c0, F_COLS, n, d, dc, dl);
      if (dc == 0 && tid < F_COLS) pj_s[tid] = c0 + tid < n ? perm[c0 + tid] : -1;
      __syncthreads();
      if (!pos_mine) continue;  // no distance of this tile can pass a threshold of this wave
      for (int c = 0; c < dl; ++c) {
        const float4* ap = reinterpret_cast<const float4*>(&xi_s[c * XI_S + w * F_RW]);
        float a[F_RW];
#pragma unroll
        for (int q4 = 0; q4 < F_RW / 4; ++q4) {
          const float4 v = ap[q4];
          a[4 * q4] = v.x;
          a[4 * q4 + 1] = v.y;
          a[4 * q4 + 2] = v.z;
          a[4 * q4 + 3] = v.w;
        }
        const float2 b = *reinterpret_cast<const float2*>(&xj_s[c * XJ_S + lane * 2]);
#pragma unroll
        for (int r = 0; r < F_RW; ++r) {
          const float t0 = a[r] - b.x, t1 = a[r] - b.y;
          acc[r][0] = __builtin_fmaf(t0, t0, acc[r][0]);
          acc[r][1] = __builtin_fmaf(t1, t1, acc[r][1]);
        }
      }
    }
    // filter: one compare per candidate; the append path (and, only in the
    // tail step and the step holding the block's own rows, the index checks)
    // runs when some lane has a candidate at or below its row's threshold
    bool any = false;
#pragma unroll
    for (int r = 0; r < F_RW; ++r) any |= (acc[r][0] <= tau[r]) | (acc[r][1] <= tau[r]);
    if (pos_mine && __ballot(any)) {
      const bool edge = (c0 + F_COLS > n) || (c0 < row0 + F_ROWS && row0 < c0 + F_COLS);
      const int64_t j0 = c0 + lane * 2;
      const int32_t pj0 = pj_s[lane * 2], pj1 = pj_s[lane * 2 + 1];
#pragma unroll
      for (int r = 0; r < F_RW; ++r) {
        const int64_t gi = row0 + w * F_RW + r;
        const bool p0 = acc[r][0] <= tau[r] && (!edge || (j0 < n && j0 != gi));
        const bool p1 = acc[r][1] <= tau[r] && (!edge || (j0 + 1 < n && j0 + 1 != gi));
        const int c = int(p0) + int(p1);
        if (c) {
          int slot = atomicAdd(&cnt_s[w * F_RW + r], c);
          uint64_t* buf = bufs + gi * CAP;
          if (p0) buf[slot++] = make_key(acc[r][0], pj0);
          if (p1) buf[slot] = make_key(acc[r][1], pj1);
        }
      }
      // compaction of rows that could overflow in the next step
      const int cl = cnt_s[w * F_RW + (lane & (F_RW - 1))];
      uint64_t need = __ballot(lane < F_RW && cl > CAP - F_COLS);
      while (need) {
        const int r = __ffsll((unsigned long long)need) - 1;
        need &= need - 1;
        float nt;
        const int nc = compact_row<EPL>(bufs + (row0 + w * F_RW + r) * CAP, __builtin_amdgcn_readlane(cl, r), k,
                                        CAP - F_COLS, nt, hist_s[w]);
        if (lane == 0) cnt_s[w * F_RW + r] = nc;
#pragma unroll
        for (int rr = 0; rr < F_RW; ++rr)
          if (rr == r) tau[rr] = nt;
      }
    }
    from = pos + 1;
  }
  for (int r = 0; r < F_RW; ++r) {
    const int64_t gi = row0 + w * F_RW + r;
    if (gi >= n) break;
    const int64_t pt = perm[gi];
    emit_row<EPL>(bufs + gi * CAP, cnt_s[w * F_RW + r], k, out_idx + pt * k, out_d2 + pt * k);
  }
}

// ---------------------------------------------------------------------
// BF16 path.

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return uint16_t((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

constexpr uint16_t BF16_ONE = 0x3F80;
constexpr uint16_t BF16_INF = 0x7F80;

// Locality order (both paths).  Points are counting-sorted by a 16-bit
// Morton key of their first three coordinates (6, 5 and 5 bits over each
// coordinate's range; fewer coordinates when d < 3): position p of the
// sorted order holds point perm[p].  Within a key the order is that of the
// scatter's atomics; nothing downstream depends on it (the selection keeps
// the best keys (d, original index) whatever order they arrive in).
constexpr int LOC_BINS = 1 << 16;
constexpr int LOC_DIMS = 3;
constexpr int LOC_BITS[LOC_DIMS] = {6, 5, 5};

// float <-> unsigned int with the same order, for integer atomic min / max
__device__ __forceinline__ uint32_t f_ord(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_f(uint32_t u) { return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u); }

// rng[c] = min and rng[LOC_DIMS + c] = max (order-encoded) of the finite
// values of coordinate c < min(d, 3); rng starts at {~0 x 3, 0 x 3}.
__global__ __launch_bounds__(256) void loc_range_kernel(const float* __restrict__ X, int64_t n, int d,
                                                        uint32_t* __restrict__ rng) {
  const int nd = d < LOC_DIMS ? d : LOC_DIMS;
  float mn[LOC_DIMS], mx[LOC_DIMS];
#pragma unroll
  for (int c = 0; c < LOC_DIMS; ++c) {
    mn[c] = INFINITY;
    mx[c] = -INFINITY;
  }
  for (int64_t i = gtid(); i < n; i += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int c = 0; c < LOC_DIMS; ++c) {
      if (c < nd) {
        const float v = X[i * d + c];
        if (isfinite(v)) {
          mn[c] = fminf(mn[c], v);
          mx[c] = fmaxf(mx[c], v);
        }
      }
    }
  }
  // the block's extremes (waves, then wave 0 over the four), one atomic per
  // block and bound: the grid is small, so few atomics meet at one address
  __shared__ float part[4][2 * LOC_DIMS];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < LOC_DIMS; ++c) {
    const float a = wave_min(mn[c]), b = -wave_min(-mx[c]);
    if (lane_id() == 0) {
      part[w][c] = a;
      part[w][LOC_DIMS + c] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < nd) {
    const int c = threadIdx.x;
    const float a = fminf(fminf(part[0][c], part[1][c]), fminf(part[2][c], part[3][c]));
    const float b = fmaxf(fmaxf(part[0][LOC_DIMS + c], part[1][LOC_DIMS + c]),
                          fmaxf(part[2][LOC_DIMS + c], part[3][LOC_DIMS + c]));
    if (a <= b) {
      atomicMin(&rng[c], f_ord(a));
      atomicMax(&rng[LOC_DIMS + c], f_ord(b));
    }
  }
}

// key[i] = the Morton key of point i (0 for non-finite coordinates), and its
// count in hist.
__global__ __launch_bounds__(256) void loc_key_kernel(const float* __restrict__ X, int64_t n, int d,
                                                      const uint32_t* __restrict__ rng, uint16_t* __restrict__ key,
                                                      int* __restrict__ hist) {
  const int nd = d < LOC_DIMS ? d : LOC_DIMS;
  for (int64_t i = gtid(); i < n; i += int64_t(gridDim.x) * blockDim.x) {
    uint32_t q[LOC_DIMS] = {0u, 0u, 0u};
#pragma unroll
    for (int c = 0; c < LOC_DIMS; ++c) {
      if (c >= nd || rng[c] > rng[LOC_DIMS + c]) continue;  // no finite value at all
      const float lo = ord_f(rng[c]), hi = ord_f(rng[LOC_DIMS + c]);
      const float v = X[i * d + c];
      const float cells = float(1u << LOC_BITS[c]);
      const float t = hi > lo ? (v - lo) / (hi - lo) * cells : 0.0f;
      q[c] = (isfinite(t) && t > 0.0f) ? (t < cells ? uint32_t(t) : (1u << LOC_BITS[c]) - 1u) : 0u;
    }
    // interleave from the top: q0 bit 5, then (q0, q1, q2) bits 4 .. 0
    uint32_t k = (q[0] >> 5) & 1u;
#pragma unroll
    for (int b = 4; b >= 0; --b) k = (k << 3) | (((q[0] >> b) & 1u) << 2) | (((q[1] >> b) & 1u) << 1) | ((q[2] >> b) & 1u);
    key[i] = uint16_t(k);
    atomicAdd(&hist[k], 1);
  }
}

// perm[off[key] + rank among the points of that key] = i.
__global__ __launch_bounds__(256) void loc_scatter_kernel(const uint16_t* __restrict__ key, int64_t n,
                                                          const int64_t* __restrict__ off, int* __restrict__ cur,
                                                          int32_t* __restrict__ perm) {
  for (int64_t i = gtid(); i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const uint32_t k = key[i];
    perm[off[k] + atomicAdd(&cur[k], 1)] = int32_t(i);
  }
}

// One wave per position p of the locality order, for point perm[p].
// Query row:      [x~ (d), nh, nm, nl, 1, 1, 1, 0 ...]
// candidate row:  [-2 x~ (d), 1, 1, 1, nh, nm, nl, 0 ...]
// so that <query_i, candidate_j> = |x~_i|^2 + |x~_j|^2 - 2 <x~_i, x~_j>, the
// squared distance of the rounded points; |x~|^2 (FP32) is carried as the
// sum nh + nm + nl of three bf16 parts.  Candidate rows n .. nrows - 1
// (nrows = n + 1 rounded up to a whole tile) are points at infinite
// distance from every query ([0 ..., inf at d + 3, 0 ...]): the last tile
// is filled with them, so the tile loads need no bounds test.
__global__ __launch_bounds__(256) void bf16_prep_kernel(const float* __restrict__ X, int64_t n, int64_t nrows, int d,
                                                        const int32_t* __restrict__ perm, uint16_t* __restrict__ Xq,
                                                        uint16_t* __restrict__ Xc) {
  const int lane = lane_id();
  const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= nrows) return;
  if (row >= n) {
    Xc[row * 64 + lane] = lane == d + 3 ? BF16_INF : uint16_t(0);
    return;
  }
  const int64_t src = perm[row];
  const bool has = lane < d;
  const uint16_t h = has ? bf16_rne(X[src * d + lane]) : uint16_t(0);
  const float xr = bf16_to_f(h);
  const float nrm = wave_sum(xr * xr);
  const uint16_t nh = bf16_rne(nrm);
  const float r1 = nrm - bf16_to_f(nh);
  const uint16_t nm = bf16_rne(r1);
  const float r2 = r1 - bf16_to_f(nm);
  const uint16_t nl = bf16_rne(r2);
  uint16_t q = 0, c = 0;
  if (has) {
    q = h;
    c = bf16_rne(-2.0f * xr);  // exact: scaling by -2 keeps the 8-bit significand
  } else if (lane < d + 3) {
    const int t = lane - d;
    q = t == 0 ? nh : (t == 1 ? nm : nl);
    c = BF16_ONE;
  } else if (lane < d + 6) {
    const int t = lane - d - 3;
    q = BF16_ONE;
    c = t == 0 ? nh : (t == 1 ? nm : nl);
  }
  Xq[row * 64 + lane] = q;
  Xc[row * 64 + lane] = c;
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

constexpr int B_TJ = 64;  // candidates per LDS tile

// candidate rows: the n points and at least one infinite row, up to a
// whole number of tiles
__host__ __device__ constexpr int64_t bf16_rows(int64_t n) { return (n + B_TJ) / B_TJ * B_TJ; }

// Tile boxes for skipping candidate tiles.  Tile u holds rows
// 64 u .. 64 u + 63 of the locality order (those below n); box[u][c] is
// the (min, max) of the rounded coordinate c over them for c < BOX_D
// ((0, 0) past d), and tnrm[u] bounds their squared norms from above: the
// leading bf16 part nh of a row's FP32 norm is within 2^-9 of it
// (round to nearest), so max nh (1 + 2^-7) bounds the norm.  NaN values
// are left out of the box and of the bound; such a row's distances are
// NaN and never pass a threshold.
__global__ __launch_bounds__(256) void bf16_box_kernel(const uint16_t* __restrict__ Xq, int64_t n, int d,
                                                       int64_t ntiles, float2* __restrict__ box,
                                                       float* __restrict__ tnrm) {
  const int lane = lane_id();
  const int64_t u = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (u >= ntiles) return;
  const int64_t r0 = u * B_TJ;
  const int rows = int(n - r0 < B_TJ ? n - r0 : B_TJ);
  float lo = INFINITY, hi = -INFINITY;
  for (int r = 0; r < rows; ++r) {
    const float v = bf16_to_f(Xq[(r0 + r) * 64 + lane]);
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  }
  if (lane < BOX_D) box[u * BOX_D + lane] = lane < d ? make_float2(lo, hi) : make_float2(0.0f, 0.0f);
  if (lane == d) tnrm[u] = hi * (1.0f + 1.0f / 128.0f);
}

// LDS tile of B_TJ candidate rows, 8 chunks of 16 bytes each; chunk c of
// row r is stored at r * 8 + (c ^ (r & 7)) so that 16 lanes reading chunk c
// of 16 consecutive rows hit distinct banks.
__device__ __forceinline__ int tile_slot(int r, int c) { return r * 8 + (c ^ (r & 7)); }

// Block = 4 waves x 64 queries, positions of the locality order (Xq, Xc and
// the buffers are in that order; perm maps a position to its point, which
// is what keys and outputs name).  The candidate tiles are swept cyclically
// from two tiles before the block's first query, so the block's own
// neighbourhood comes first.  Lane l works on queries 16 t + (l % 16),
// t = 0..3, of its wave and, per 16-candidate subtile, on candidates
// 4 (l / 16) .. + 3 (the MFMA C layout).  A query's threshold and buffer
// count are held (identically) by its four lanes.  Four blocks fit a CU
// (at most 128 VGPRs, which the kernel fits without VGPR spills; the
// selection is bound by memory instructions, so resident waves count more
// than registers), and 1024 resident blocks cover 262144 queries in one
// round.
// Tile skipping.  A wave does not evaluate a tile in which no distance can
// pass the threshold of any of its 64 queries, and the block does not
// fetch a tile that none of its waves evaluates.  With B the box of the
// wave's queries (they are one tile of the order, so B is that tile's box)
// and T the candidate tile's (leading BOX_D coordinates), LB = sum_c
// gap_c(B, T)^2 is at most the squared distance of any of the queries to
// any candidate of the tile, and the MFMA's distance differs from the
// exact one of the rounded points by less than 2^-15 (N_q + N_c) (64
// products of exact bf16 pairs, FP32 accumulation; N the squared norms, a
// sum of absolute terms of at most 2 (N_q + N_c); the norm's bf16 parts
// add 2^-20 of it), so LB > tau_max + 2^-12 (N_q + N_c), with tau_max the
// wave's largest threshold, means every distance of the tile exceeds every
// threshold of the wave: the tile would append nothing for it, and
// skipping it changes no buffer.  The outputs are those of the full sweep,
// bit for bit.  The test is taken for windows of 64 sweep positions at a
// time (one position per lane, a ballot per wave, the four masks OR-ed
// through LDS), with the thresholds of that moment; they only decrease, so
// a window's stale value skips less, never wrongly.
template <int EPL>
__global__ __launch_bounds__(256, 4) void knn_bf16_kernel(const uint4* __restrict__ Xq, const uint4* __restrict__ Xc,
                                                       const int32_t* __restrict__ perm, const float4* __restrict__ box4,
                                                       const float* __restrict__ tnrm, int64_t n, int ncand,
                                                       uint64_t* __restrict__ bufs, int32_t* __restrict__ cand) {
  constexpr int CAP = 64 * EPL;
  __shared__ uint4 tile[2][B_TJ * 8];  // double-buffered: 64 rows x 128 bytes each
  __shared__ int32_t ptile[2][B_TJ];    // the original indices of those rows
  __shared__ uint32_t hist_s[4][256];   // per-wave radix-select histograms
  __shared__ float4 qbox[4][BOX_D / 2];  // box of each wave's queries: (lo, hi) of two coordinates each
  __shared__ float qnrm_s[4];            // bound on the squared norms of each wave's queries
  __shared__ uint64_t wmask_s[2][4];     // each wave's live positions, by window parity
  const int tid = threadIdx.x, lane = lane_id(), w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q16 = lane & 15, g4 = lane >> 4;
  // indices are 32-bit (n < 2^31 is checked by the caller); products that
  // address memory are taken in 64 bits
  const int n32 = int(n);
  const int qblock = int(blockIdx.x) * 256;
  const int qbase = qblock + w * 64;
  int cnt[4] = {0, 0, 0, 0};  // buffer count of query (t, q16), the same in its four lanes
  // query fragments: tile t, k-step s; lane holds query qbase + 16 t + q16,
  // k elements 32 s + 8 g4 ... + 7
  bf16x8_t bq[4][2];
  float tau[4];
  // the subtile filter compares raw bit patterns as signed integers: for a
  // non-negative threshold, d <= tau implies bits(d) <= bits(tau) (a
  // negative d has a negative pattern), so no candidate that passes is
  // filtered out; a negative threshold (the padding queries, or a row whose
  // best distances round below 0) lets every subtile through to the exact
  // per-candidate test
  int tau_key[4];
  auto key_of = [](float t) { return t >= 0.0f ? __float_as_int(t) : INT_MAX; };
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int qi = qbase + t * 16 + q16;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      uint4 v = make_uint4(0, 0, 0, 0);
      if (qi < n32) v = Xq[int64_t(qi) * 8 + s * 4 + g4];
      bq[t][s] = __builtin_bit_cast(bf16x8_t, v);
    }
    // queries past n never accept; the others accept any finite distance
    // until their buffer is first compacted (the padding rows are infinite)
    tau[t] = qi < n32 ? FLT_MAX : -INFINITY;
    tau_key[t] = key_of(tau[t]);
  }
  // Tiles go from global memory straight to LDS (global_load_lds_dwordx4:
  // lane l of a wave writes the 16 bytes at the wave's LDS base + 16 l), so
  // the swizzle is applied on the global side: LDS slot u holds chunk
  // (u % 8) ^ (row % 8) of row u / 8.  Rows past n are the infinite rows.
  // Thread tid loads slots u = tid and tid + 256: a per-thread source
  // offset fixed for the whole sweep, and a wave-uniform LDS base.
  uint32_t soff[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int u = tid + 256 * h;
    const int r = u >> 3;
    soff[h] = uint32_t(r * 8 + ((u & 7) ^ (r & 7)));
  }
  // Wave 0 also brings the tile's 64 entries of perm (padded to whole
  // tiles), so an append reads its candidate's index from LDS.
  auto load_tile = [&](int c0, int b) {
    const uint4* base = Xc + int64_t(c0) * 8;
#pragma unroll
    for (int h = 0; h < 2; ++h) __builtin_amdgcn_global_load_lds(base + soff[h], tile[b] + 64 * w + 256 * h, 16, 0, 0);
    // (the LDS operand as an explicit element pointer: an array operand is
    // taken by value by this builtin)
    if (w == 0) __builtin_amdgcn_global_load_lds(perm + c0 + lane, &ptile[b][0], 4, 0, 0);
  };
  const int ntiles = (n32 + B_TJ - 1) / B_TJ;
  int t0 = (qblock / B_TJ - 2) % ntiles;
  if (t0 < 0) t0 += ntiles;
  auto tile_of = [&](int it) -> int {
    const int ti = t0 + it;
    return ti < ntiles ? ti : ti - ntiles;
  };
  auto tile_c0 = [&](int it) -> int { return tile_of(it) * B_TJ; };
  // each wave's query box: its 64 queries are candidate tile qblock / 64 + w
  const int qt = qblock / B_TJ + w;
  const bool has_q = qt < ntiles;  // else the wave holds only padding queries
  if (has_q) {
    if (lane < BOX_D / 2) qbox[w][lane] = box4[qt * (BOX_D / 2) + lane];
    if (lane == 0) qnrm_s[w] = tnrm[qt];
  }
  __syncthreads();
  // live positions of the window [p0, p0 + 64): this wave's (returned) and
  // the block's (any wave's, in `blk`); called by all waves together
  int wpar = 0;
  auto window = [&](int p0, uint64_t& blk) -> uint64_t {
    // this wave's largest threshold now (padding queries hold -inf)
    const float m4 = fmaxf(fmaxf(tau[0], tau[1]), fmaxf(tau[2], tau[3]));
    const float tm = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(-wave_min(-m4))));
    const int p = p0 + lane;
    bool live = has_q && p < ntiles;
    if (tm < FLT_MAX) {
      const int t = tile_of(live ? p : 0);
      const float4* tb = box4 + t * (BOX_D / 2);
      float lb = 0.0f;
#pragma unroll 2
      for (int h = 0; h < BOX_D / 2; ++h) {
        const float4 v = tb[h], q = qbox[w][h];  // (lo, hi) of coordinates 2h and 2h + 1
        const float g0 = fmaxf(fmaxf(v.x - q.y, q.x - v.y), 0.0f);
        const float g1 = fmaxf(fmaxf(v.z - q.w, q.z - v.w), 0.0f);
        lb = fmaf(g0, g0, lb);
        lb = fmaf(g1, g1, lb);
      }
      const float margin = (qnrm_s[w] + tnrm[t]) * (1.0f / 4096.0f);
      live = live && !(lb > tm + margin);
    }
    const uint64_t mine = __ballot(live);
    // two buffers: a wave may write the next window's mask while another
    // still reads this one's
    if (lane == 0) wmask_s[wpar][w] = mine;
    __syncthreads();
    blk = wmask_s[wpar][0] | wmask_s[wpar][1] | wmask_s[wpar][2] | wmask_s[wpar][3];
    wpar ^= 1;
    return mine;
  };
  int wb = 0;  // first position of the current window
  uint64_t win = 0;
  uint64_t mine = window(0, win);
  int pos = 0, buf = 0;
  bool cur_mine = mine & 1;  // position 0 is live for every wave with queries
  load_tile(tile_c0(0), 0);
  while (pos < ntiles) {
    const int c0 = tile_c0(pos);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's part of the tile has landed
    __syncthreads();                // ... and every wave's; the other buffer is free
    // the next position some wave evaluates
    int nxt = pos + 1;
    bool nxt_mine = false;
    while (nxt < ntiles) {
      if (nxt >= wb + 64) {
        wb = nxt;
        mine = window(wb, win);
      }
      const uint64_t m = win >> (nxt - wb);
      if (m) {
        nxt += __builtin_ctzll(m);
        nxt_mine = (mine >> (nxt - wb)) & 1;
        break;
      }
      nxt = wb + 64;
    }
    // fetch the next tile while this one is consumed
    if (nxt < ntiles) load_tile(tile_c0(nxt), buf ^ 1);
    const uint4* tl = tile[buf];
    const int32_t* pt = ptile[buf];
    // tiles that hold some of this block's queries exclude the self pairs;
    // the others need only the threshold test
    auto sweep = [&](auto edge_c) {
      constexpr bool EDGE = decltype(edge_c)::value;
#pragma unroll
      for (int sub = 0; sub < B_TJ / 16; ++sub) {
        const int rloc = sub * 16 + q16;
        const bf16x8_t a0 = __builtin_bit_cast(bf16x8_t, tl[tile_slot(rloc, g4)]);
        const bf16x8_t a1 = __builtin_bit_cast(bf16x8_t, tl[tile_slot(rloc, 4 + g4)]);
        floatx4_t acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc[t] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bq[t][0], acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bq[t][1], acc[t], 0, 0, 0);
        }
        // acc[t][r] = distance(query qbase + 16 t + q16, candidate c0 + 16 sub + 4 g4 + r)
        bool any = false;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          any |= min(min(__float_as_int(acc[t][0]), __float_as_int(acc[t][1])),
                     min(__float_as_int(acc[t][2]), __float_as_int(acc[t][3]))) <= tau_key[t];
        if (__ballot(any)) {
          const int jb = c0 + sub * 16 + 4 * g4;
          const int4 pj = *reinterpret_cast<const int4*>(pt + sub * 16 + 4 * g4);  // perm[jb .. jb + 3]
          const int pjr[4] = {pj.x, pj.y, pj.z, pj.w};
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int qi = qbase + t * 16 + q16;
            bool p[4];
            int c = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              p[r] = acc[t][r] <= tau[t] && (!EDGE || jb + r != qi);
              c += int(p[r]);
            }
            if (__ballot(c != 0) == 0) continue;
            // slots of query qi over its four lanes (rows g4 of 16 lanes):
            // exclusive prefix and total of c across the rows, by a 16-lane
            // and a 32-lane permute (no atomics, no memory)
            const auto r16 = __builtin_amdgcn_permlane16_swap(uint32_t(c), uint32_t(c), false, false);
            const int lo = int(r16[0]), hi = int(r16[1]);  // c of rows g4 & ~1 and g4 | 1
            const auto r32 = __builtin_amdgcn_permlane32_swap(uint32_t(lo + hi), uint32_t(lo + hi), false, false);
            const int s01 = int(r32[0]), s23 = int(r32[1]);  // c of rows 0 + 1 and 2 + 3
            int pos = cnt[t] + ((g4 & 1) ? lo : 0) + ((g4 & 2) ? s01 : 0);
            cnt[t] += s01 + s23;
            // the buffers of queries qbase + 16 t ..: a wave-uniform base and
            // a small per-lane offset (no 64-bit pointer per query and t)
            uint64_t* tbuf = bufs + int64_t(qbase + t * 16) * CAP;
            const uint32_t lo_off = uint32_t(q16 * CAP);
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (p[r]) tbuf[lo_off + uint32_t(pos++)] = make_key(fmaxf(acc[t][r], 0.0f), pjr[r]);
          }
        }
      }
    };
    if (cur_mine) {
      if (c0 < qblock + 256 && qblock < c0 + B_TJ) sweep(std::true_type{});
      else sweep(std::false_type{});
    }
    // compaction of queries that could overflow in the next tile; lanes
    // 0..15 speak for queries 16 t + lane
    uint64_t need = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) need |= (__ballot(cnt[t] > CAP - B_TJ) & 0xFFFFull) << (16 * t);
    while (need) {
      const int r = __ffsll((unsigned long long)need) - 1;
      need &= need - 1;
      const int t = r >> 4, q = r & 15;
      const int c = __builtin_amdgcn_readlane(t == 0 ? cnt[0] : t == 1 ? cnt[1] : t == 2 ? cnt[2] : cnt[3], q);
      float nt;
      const int nc = compact_row<EPL>(bufs + int64_t(qbase + r) * CAP, c, ncand, CAP - B_TJ, nt, hist_s[w]);
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
        if (tt == t && q16 == q) {
          cnt[tt] = nc;
          tau[tt] = nt;
          tau_key[tt] = key_of(nt);
        }
    }
    buf ^= 1;
    pos = nxt;
    cur_mine = nxt_mine;
  }
  for (int r = 0; r < 64; ++r) {
    const int qi = qbase + r;
    if (qi >= n32) break;
    const int t = r >> 4;
    const int c = __builtin_amdgcn_readlane(t == 0 ? cnt[0] : t == 1 ? cnt[1] : t == 2 ? cnt[2] : cnt[3], r & 15);
    emit_row<EPL>(bufs + int64_t(qi) * CAP, c, ncand, cand + int64_t(perm[qi]) * ncand, nullptr);
  }
}

// Rows of X padded to dp = d rounded up to 4 (zeros past d), 16-byte
// aligned, for the re-rank's gathers: one wave per row.
__global__ __launch_bounds__(256) void pad_rows_kernel(const float* __restrict__ X, int64_t n, int d, int dp,
                                                       float* __restrict__ Xp) {
  const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int c = lane_id();
  if (i >= n || c >= dp) return;
  Xp[i * dp + c] = c < d ? X[i * d + c] : 0.0f;
}

// Re-rank: one wave per row; FP32 direct differences (same arithmetic as the
// FP32 path: squares accumulated in dimension order) of the row's
// candidates, sorted by (d, j); best k written.  Rows are taken in the
// locality order (wave w re-ranks row perm[w]), so the waves resident at one
// time gather overlapping candidate rows from the caches.  The query row is
// read with uniform (scalar) loads; each lane issues all loads of a
// candidate row before the arithmetic, four coordinates per load from the
// padded rows Xp (dp <= DP floats each), which quarters the scattered
// requests the address units must serve; coordinates past dp re-read the
// row's last four (in bounds) and, like the zeros past d, add an exact 0.
template <int DP>
__global__ __launch_bounds__(256) void rerank_kernel(const float* __restrict__ Xp, int64_t n, int d, int dp,
                                                     const int32_t* __restrict__ perm, const int32_t* __restrict__ cand,
                                                     int ncand, int k, int32_t* __restrict__ out_idx,
                                                     float* __restrict__ out_d2) {
  static_assert(DP % 4 == 0, "whole float4 loads");
  const int lane = lane_id();
  const int64_t pos = int64_t(__builtin_amdgcn_readfirstlane(int(blockIdx.x) * 4 + int(threadIdx.x >> 6)));
  if (pos >= n) return;
  const int64_t row = int64_t(__builtin_amdgcn_readfirstlane(perm[pos]));
  float xi[DP];
#pragma unroll
  for (int c = 0; c < DP; ++c) xi[c] = c < d ? Xp[row * dp + c] : 0.0f;
  const int last = dp / 4 - 1;
  uint64_t v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = t * 64 + lane;
    v[t] = KEY_MAX;
    const int32_t j = e < ncand ? cand[row * ncand + e] : -1;
    if (j >= 0 && j < n) {  // a row short of candidates (non-finite input) holds -1
      const float4* xj4 = reinterpret_cast<const float4*>(Xp + int64_t(j) * dp);
      float xv[DP];
#pragma unroll
      for (int c = 0; c < DP; c += 4) {
        const float4 q = xj4[c / 4 < last ? c / 4 : last];
        xv[c] = q.x;
        xv[c + 1] = q.y;
        xv[c + 2] = q.z;
        xv[c + 3] = q.w;
      }
      float s2 = 0.0f;
#pragma unroll
      for (int c = 0; c < DP; ++c) {
        const float u = c < d ? xi[c] - xv[c] : 0.0f;
        s2 = __builtin_fmaf(u, u, s2);
      }
      v[t] = make_key(s2, j);
    }
  }
  wave_sort<4>(v);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = t * 64 + lane;
    if (e < k) {
      out_idx[row * k + e] = key_index(v[t]);
      out_d2[row * k + e] = key_dist(v[t]);
    }
  }
}

// Adds to *out the number of non-finite values among a[0, count): each wave
// sums its lanes' counts and, if any, adds them with one integer atomic.
__global__ __launch_bounds__(256) void count_nonfinite_kernel(const float* __restrict__ a, int64_t count,
                                                              unsigned long long* __restrict__ out) {
  int c = 0;
  for (int64_t i = gtid(); i < count; i += int64_t(gridDim.x) * blockDim.x) c += !isfinite(a[i]);
  c = wave_sum_i(c);
  if (__lane_id() == 0 && c) atomicAdd(out, static_cast<unsigned long long>(c));
}

struct KnnLayout {
  int epl;
  size_t o_buf, o_xq, o_xc, o_xs, o_xp, o_cand, o_perm, o_key, o_rng, o_hist, o_cur, o_off, o_bsum, o_box, o_tnrm,
      bytes;
  static KnnLayout make(int64_t n, int d, int precision, int ncand) {
    KnnLayout L;
    Carve c;
    L.epl = 8;  // capacity 512: room for 384 (FP32) or 448 (BF16) appends between compactions
    L.o_buf = c.take(sizeof(uint64_t) * size_t(n) * size_t(64 * L.epl));
    // the locality order (both paths)
    L.o_perm = c.take(sizeof(int32_t) * size_t(bf16_rows(n)));  // padded like the BF16 candidate rows
    L.o_key = c.take(sizeof(uint16_t) * size_t(n));
    L.o_rng = c.take(sizeof(uint32_t) * 2 * LOC_DIMS);
    L.o_hist = c.take(sizeof(int) * LOC_BINS);
    L.o_cur = c.take(sizeof(int) * LOC_BINS);
    L.o_off = c.take(sizeof(int64_t) * (LOC_BINS + 1));
    L.o_bsum = c.take(sizeof(int64_t) * (size_t(ceil_div(LOC_BINS + 1, SCAN_CHUNK)) + 1));
    if (precision == TSNE_KNN_FP32) {
      L.o_xs = c.take(sizeof(float) * size_t(n) * size_t(d));  // X in the locality order
      L.o_xq = L.o_xc = L.o_cand = L.o_tnrm = L.o_xp = 0;
      L.o_box = c.take(sizeof(float2) * BOX_D * size_t(ceil_div(n, F_COLS)));
    } else {
      L.o_xs = 0;
      L.o_xp = c.take(sizeof(float) * size_t(n) * size_t((d + 3) / 4 * 4));  // X padded, for the re-rank
      L.o_xq = c.take(sizeof(uint16_t) * size_t(n) * 64);
      L.o_xc = c.take(sizeof(uint16_t) * size_t(bf16_rows(n)) * 64);  // + the infinite rows
      L.o_cand = c.take(sizeof(int32_t) * size_t(n) * size_t(ncand));
      L.o_box = c.take(sizeof(float2) * BOX_D * size_t(ceil_div(n, B_TJ)));
      L.o_tnrm = c.take(sizeof(float) * size_t(ceil_div(n, B_TJ)));
    }
    L.bytes = c.off;
    return L;
  }
};

}  // namespace tsne

extern "C" int tsne_knn(const float* X, int64_t n, int32_t d, int32_t k, int32_t precision, int32_t n_cand,
                        int32_t* nbr_idx, float* nbr_d2, int64_t* nonfinite, void* workspace, size_t* workspace_bytes,
                        void* stream) {
  using namespace tsne;
  if (!X || !nbr_idx || !nbr_d2 || n < 2 || d < 1 || k < 1 || k >= n) return TSNE_ERR_INVALID_ARG;
  if (precision != TSNE_KNN_FP32 && precision != TSNE_KNN_BF16) return TSNE_ERR_INVALID_ARG;
  if (precision == TSNE_KNN_BF16 && (n_cand < k || n_cand >= n)) return TSNE_ERR_INVALID_ARG;
  if (k > TSNE_MAX_K || d > TSNE_MAX_D) return TSNE_ERR_UNSUPPORTED;
  if (precision == TSNE_KNN_BF16 && (n_cand > TSNE_MAX_K || d > TSNE_MAX_D_BF16)) return TSNE_ERR_UNSUPPORTED;
  if (n > (int64_t(1) << 31) - 1) return TSNE_ERR_UNSUPPORTED;
  const KnnLayout L = KnnLayout::make(n, d, precision, n_cand);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  char* ws = static_cast<char*>(workspace);
  uint64_t* bufs = reinterpret_cast<uint64_t*>(ws + L.o_buf);
  hipStream_t s = as_stream(stream);
  if (nonfinite) {
    unsigned long long* nf = reinterpret_cast<unsigned long long*>(nonfinite);
    if ((rc = launch_fill<unsigned long long>(nf, 1, 0ull, s))) return rc;
    const int64_t cnt = n * int64_t(d);
    const int64_t blocks = ceil_div(cnt, 256) < 2048 ? ceil_div(cnt, 256) : 2048;
    hipLaunchKernelGGL(count_nonfinite_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, X, cnt, nf);
    TSNE_CHECK_LAUNCH();
  }
  // locality order (both paths): key range, keys and their counts,
  // offsets, scatter
  uint32_t* rng = reinterpret_cast<uint32_t*>(ws + L.o_rng);
  uint16_t* key = reinterpret_cast<uint16_t*>(ws + L.o_key);
  int* hist = reinterpret_cast<int*>(ws + L.o_hist);
  int* cur = reinterpret_cast<int*>(ws + L.o_cur);
  int64_t* off = reinterpret_cast<int64_t*>(ws + L.o_off);
  int64_t* bsum = reinterpret_cast<int64_t*>(ws + L.o_bsum);
  int32_t* perm = reinterpret_cast<int32_t*>(ws + L.o_perm);
  if ((rc = launch_fill<uint32_t>(rng, LOC_DIMS, ~0u, s))) return rc;
  if ((rc = launch_fill<uint32_t>(rng + LOC_DIMS, LOC_DIMS, 0u, s))) return rc;
  if ((rc = launch_fill<int>(hist, LOC_BINS, 0, s))) return rc;
  if ((rc = launch_fill<int>(cur, LOC_BINS, 0, s))) return rc;
  const dim3 lgrid(unsigned(ceil_div(n, 256) < 2048 ? ceil_div(n, 256) : 2048));
  hipLaunchKernelGGL(loc_range_kernel, dim3(unsigned(ceil_div(n, 256) < 256 ? ceil_div(n, 256) : 256)), dim3(256), 0,
                     s, X, n, d, rng);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(loc_key_kernel, lgrid, dim3(256), 0, s, X, n, d, rng, key, hist);
  TSNE_CHECK_LAUNCH();
  if ((rc = exclusive_scan<int>(hist, LOC_BINS, off, bsum, s))) return rc;
  hipLaunchKernelGGL(loc_scatter_kernel, lgrid, dim3(256), 0, s, key, n, off, cur, perm);
  TSNE_CHECK_LAUNCH();
  if (precision == TSNE_KNN_FP32) {
    float* Xs = reinterpret_cast<float*>(ws + L.o_xs);
    float2* box = reinterpret_cast<float2*>(ws + L.o_box);
    const int64_t ntc = ceil_div(n, F_COLS);
    hipLaunchKernelGGL(gather_rows_kernel, dim3(unsigned(ceil_div(n, 4))), dim3(256), 0, s, X, n, d, perm, Xs);
    TSNE_CHECK_LAUNCH();
    hipLaunchKernelGGL(f32_box_kernel, dim3(unsigned(ceil_div(ntc, 4))), dim3(256), 0, s, Xs, n, d, ntc, box);
    TSNE_CHECK_LAUNCH();
    const float4* box4 = reinterpret_cast<const float4*>(box);
    if (fknn_small_blocks(n))
      hipLaunchKernelGGL((knn_fp32_kernel<8, 8>), dim3(unsigned(ceil_div(n, 32))), dim3(256), 0, s, Xs, perm, box4, n,
                         d, k, bufs, nbr_idx, nbr_d2);
    else
      hipLaunchKernelGGL((knn_fp32_kernel<8, 16>), dim3(unsigned(ceil_div(n, 64))), dim3(256), 0, s, Xs, perm, box4,
                         n, d, k, bufs, nbr_idx, nbr_d2);
    TSNE_CHECK_LAUNCH();
    return TSNE_OK;
  }
  uint16_t* Xq = reinterpret_cast<uint16_t*>(ws + L.o_xq);
  uint16_t* Xc = reinterpret_cast<uint16_t*>(ws + L.o_xc);
  int32_t* cand = reinterpret_cast<int32_t*>(ws + L.o_cand);
  // the padding of perm (the infinite candidate rows) names point 0; such a
  // candidate never passes a threshold, so the value is never used
  if ((rc = launch_fill<int32_t>(perm + n, bf16_rows(n) - n, 0, s))) return rc;
  hipLaunchKernelGGL(bf16_prep_kernel, dim3(unsigned(ceil_div(bf16_rows(n), 4))), dim3(256), 0, s, X, n, bf16_rows(n),
                     d, perm, Xq, Xc);
  TSNE_CHECK_LAUNCH();
  const int64_t ntiles = ceil_div(n, B_TJ);
  float2* box = reinterpret_cast<float2*>(ws + L.o_box);
  float* tnrm = reinterpret_cast<float*>(ws + L.o_tnrm);
  hipLaunchKernelGGL(bf16_box_kernel, dim3(unsigned(ceil_div(ntiles, 4))), dim3(256), 0, s, Xq, n, d, ntiles, box, tnrm);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(knn_bf16_kernel<8>, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, s,
                     reinterpret_cast<const uint4*>(Xq), reinterpret_cast<const uint4*>(Xc), perm,
                     reinterpret_cast<const float4*>(box), tnrm, n, n_cand, bufs, cand);
  TSNE_CHECK_LAUNCH();
  const int dp = (d + 3) / 4 * 4;
  float* Xp = reinterpret_cast<float*>(ws + L.o_xp);
  hipLaunchKernelGGL(pad_rows_kernel, dim3(unsigned(ceil_div(n, 4))), dim3(256), 0, s, X, n, d, dp, Xp);
  TSNE_CHECK_LAUNCH();
  // the exact width for the common 50-coordinate input, else the largest
  if (dp == 52)
    hipLaunchKernelGGL((rerank_kernel<52>), dim3(unsigned(ceil_div(n, 4))), dim3(256), 0, s, Xp, n, d, dp, perm, cand,
                       n_cand, k, nbr_idx, nbr_d2);
  else
    hipLaunchKernelGGL((rerank_kernel<(TSNE_MAX_D_BF16 + 3) / 4 * 4>), dim3(unsigned(ceil_div(n, 4))), dim3(256), 0, s,
                       Xp, n, d, dp, perm, cand, n_cand, k, nbr_idx, nbr_d2);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}
