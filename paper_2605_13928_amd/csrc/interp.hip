// tsne_kl_grad_fft: t-SNE gradient (van der Maaten & Hinton 2008, eq. 5)
// with the repulsive sums and Z approximated by FFT-accelerated polynomial
// interpolation (Linderman, Rachh, Hoskins, Steinerberger & Kluger 2019,
// Nat. Methods 16, 243-245); the attraction stays exact over the CSR rows.
//
// Per call, all on the stream, no host synchronisation:
//   bbox_kernel / params_kernel  the square domain [lo, lo + B h]^2, B boxes
//                                of side h per axis, p x p nodes per box at
//                                local positions (k + 1/2) / p, so N = p B
//                                equispaced nodes (spacing h / p) per axis;
//                                FFT size F = smallest power of two >= 2 N.
//   count / scan / scatter       the points sorted by box (counting sort).
//   accum_kernel                 one thread per box sums its points' charges
//                                1, z_x, z_y (z = y - centre) times the
//                                tensor Lagrange weights into the box's
//                                p x p nodes, in 64-bit fixed point (exact,
//                                so independent of the order the scatter
//                                leaves: deterministic), and writes them;
//                                every node belongs to exactly one box.
//   load_kernel                  three complex F x F grids, zero-padded /
//                                wrapped (circular convolution = linear for
//                                F >= 2N): W0, W1 + i W2, and K1 + i K2 with
//                                K1 = 1 / (1 + r^2), K2 = K1^2 at the node
//                                offsets.
//   2-D FFT (FP64)               row FFTs in LDS, an in-place transpose, row
//                                FFTs again.  The kernels are even, so their
//                                spectra are real: FFT(W0) (K1^ + i K2^)
//                                transforms back to phi1 + i phi2 and
//                                (W1^ + i W2^) K2^ to phi3x + i phi3y -- three
//                                forward and two inverse transforms.
//   gather_kernel                each point interpolates the four node
//                                potentials: R_i = z_i phi2 - (phi3x, phi3y),
//                                Z = sum_i phi1_i - n (the j = i terms).
//   finalize (klgrad.hip)        CSR attraction, g = 4 (alpha A - R / Z), KL.
// Every size is read from the parameters on the device; the launches and
// the workspace are sized for the largest FFT the caller allows.
#include <math.h>

#include "common.hpp"
#include "klgrad.hpp"
#include "scan.hpp"

namespace tsne {

constexpr int FI_GRID = 512;    // blocks of the point passes (and Z partials)
constexpr int FI_MAX_P = 5;     // interpolation nodes per box and axis
constexpr int FI_MIN_FFT = 64;  // FFT sizes: powers of two in [64, 4096]
constexpr int FI_MAX_FFT = 4096;
constexpr int FI_TILE = 32;     // transpose tile

struct FiParams {
  double lo, h, c, scale;  // domain origin, box side, centre, fixed-point scale
  int B, N, F, logF;
};

// --- domain ------------------------------------------------------------

__global__ __launch_bounds__(256) void fi_bbox_kernel(const float2* __restrict__ Y, int64_t n,
                                                      float* __restrict__ part) {
  float mn = INFINITY, mx = -INFINITY;
  for (int64_t i = gtid(); i < n; i += int64_t(gridDim.x) * 256) {
    const float2 y = Y[i];
    mn = fminf(mn, fminf(y.x, y.y));
    mx = fmaxf(mx, fmaxf(y.x, y.y));
  }
  __shared__ float smn[4], smx[4];
  mn = wave_min(mn);
  mx = -wave_min(-mx);
  if (lane_id() == 0) {
    smn[threadIdx.x >> 6] = mn;
    smx[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = fminf(fminf(smn[0], smn[1]), fminf(smn[2], smn[3]));
    part[2 * blockIdx.x + 1] = fmaxf(fmaxf(smx[0], smx[1]), fmaxf(smx[2], smx[3]));
  }
}

// One block: reduce the bounding box and fix the grid.  min and max are
// exact in any order; range and h are FP64 operations on those floats.
__global__ __launch_bounds__(256) void fi_params_kernel(const float* __restrict__ part, int nb, int64_t n, int p,
                                                        int min_boxes, float max_box_width, int max_fft,
                                                        FiParams* __restrict__ out) {
  float mn = INFINITY, mx = -INFINITY;
  for (int b = threadIdx.x; b < nb; b += 256) {
    mn = fminf(mn, part[2 * b]);
    mx = fmaxf(mx, part[2 * b + 1]);
  }
  __shared__ float smn[4], smx[4];
  mn = wave_min(mn);
  mx = -wave_min(-mx);
  if (lane_id() == 0) {
    smn[threadIdx.x >> 6] = mn;
    smx[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double lo = double(fminf(fminf(smn[0], smn[1]), fminf(smn[2], smn[3])));
  const double hi = double(fmaxf(fmaxf(smx[0], smx[1]), fmaxf(smx[2], smx[3])));
  double rng = hi - lo;
  if (!isfinite(lo) || !isfinite(rng)) {  // non-finite input: any valid grid (results are not finite)
    lo = 0.0;
    rng = 1e-3;
  }
  if (!(rng > 0.0)) rng = 1e-3;
  double Bd = ceil(rng / double(max_box_width));
  Bd = fmax(Bd, double(min_boxes));
  Bd = fmin(Bd, double(max_fft / (2 * p)));
  const int B = int(Bd);
  const int N = p * B;
  int F = FI_MIN_FFT, logF = 6;
  while (F < 2 * N) {
    F <<= 1;
    ++logF;
  }
  FiParams P;
  P.lo = lo;
  P.h = rng / double(B);
  P.c = lo + 0.5 * rng;
  // fixed point: every node sum is at most n (|z| + 1) times the square of
  // the largest Lagrange weight on [0, 1] (1.5, 1.88, 2.19, 3.28 for
  // p = 2 .. 5: squared < 16); keep it below 2^62
  const double bound = double(n) * (0.5 * rng + 1.0) * 16.0;
  P.scale = exp2(floor(log2(4.611686018427388e18 / bound)));
  P.B = B;
  P.N = N;
  P.F = F;
  P.logF = logF;
  *out = P;
}

// Box index and Lagrange weights of one coordinate (the same FP64
// operations as the definition: t = (y - lo) / h, b = floor(t) clamped).
template <int P>
__device__ __forceinline__ int fi_weights(float y, const FiParams& g, double (&L)[P]) {
  const double t = (double(y) - g.lo) / g.h;
  const double bd = fmin(fmax(floor(t), 0.0), double(g.B - 1));
  const double u = t - bd;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    double v = 1.0;
    const double tk = (double(k) + 0.5) / double(P);
#pragma unroll
    for (int m = 0; m < P; ++m) {
      if (m == k) continue;
      const double tm = (double(m) + 0.5) / double(P);
      v *= (u - tm) / (tk - tm);
    }
    L[k] = v;
  }
  return int(bd);
}

// --- spread ------------------------------------------------------------

// Box of a point (the same clamped FP64 floor as fi_weights).
__device__ __forceinline__ int fi_box(float y, const FiParams& g) {
  const double t = (double(y) - g.lo) / g.h;
  return int(fmin(fmax(floor(t), 0.0), double(g.B - 1)));
}

// Counting sort of the points by box, with the counts gathered per block:
// a block counts its points in an LDS table (open addressing, at most
// FI_PROBE probes; a key that finds no slot is counted in global memory
// directly) and adds each distinct box once.  When most points fall in a
// few boxes (a compact or clustered embedding) this replaces the
// contended global atomics on those boxes' counters by one per block.
constexpr int FI_TBL = 4096;      // LDS slots per block
constexpr int FI_PROBE = 8;
constexpr int FI_CBLOCKS = 1024;  // blocks of the counting kernels

__device__ __forceinline__ int fi_tbl_find(int* tkey, int key, bool insert) {
  const uint32_t h = uint32_t(key) * 2654435761u;
  for (int q = 0; q < FI_PROBE; ++q) {
    const int slot = int((h + uint32_t(q)) & (FI_TBL - 1));
    const int prev = insert ? atomicCAS(&tkey[slot], -1, key) : tkey[slot];
    if (prev == key || (insert && prev == -1)) return slot;
    if (!insert && prev == -1) return -1;
  }
  return -1;
}

__global__ __launch_bounds__(256) void fi_count_kernel(const float2* __restrict__ Y, int64_t n,
                                                       const FiParams* __restrict__ gp, int* __restrict__ cnt) {
  __shared__ int tkey[FI_TBL], tcnt[FI_TBL];
  const FiParams g = *gp;
  for (int q = threadIdx.x; q < FI_TBL; q += 256) {
    tkey[q] = -1;
    tcnt[q] = 0;
  }
  __syncthreads();
  for (int64_t i = gtid(); i < n; i += int64_t(gridDim.x) * 256) {
    const float2 y = Y[i];
    const int b = fi_box(y.x, g) * g.B + fi_box(y.y, g);
    const int slot = fi_tbl_find(tkey, b, true);
    if (slot >= 0) atomicAdd(&tcnt[slot], 1);
    else atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < FI_TBL; q += 256)
    if (tcnt[q]) atomicAdd(&cnt[tkey[q]], tcnt[q]);
}

// The same table, twice over the block's points: first the counts, then one
// global reservation per box (the block's range within the box), then each
// point's position (the range's start plus its rank).  A key without a slot
// takes its position from the global cursor directly, in both passes alike.
__global__ __launch_bounds__(256) void fi_scatter_kernel(const float2* __restrict__ Y, int64_t n,
                                                         const FiParams* __restrict__ gp,
                                                         const int64_t* __restrict__ off, int* __restrict__ cur,
                                                         int32_t* __restrict__ order) {
  __shared__ int tkey[FI_TBL], tcnt[FI_TBL], tbase[FI_TBL];
  const FiParams g = *gp;
  for (int q = threadIdx.x; q < FI_TBL; q += 256) {
    tkey[q] = -1;
    tcnt[q] = 0;
  }
  __syncthreads();
  for (int64_t i = gtid(); i < n; i += int64_t(gridDim.x) * 256) {
    const float2 y = Y[i];
    const int b = fi_box(y.x, g) * g.B + fi_box(y.y, g);
    const int slot = fi_tbl_find(tkey, b, true);
    if (slot >= 0) atomicAdd(&tcnt[slot], 1);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < FI_TBL; q += 256) {
    tbase[q] = tcnt[q] ? atomicAdd(&cur[tkey[q]], tcnt[q]) : 0;
    tcnt[q] = 0;
  }
  __syncthreads();
  for (int64_t i = gtid(); i < n; i += int64_t(gridDim.x) * 256) {
    const float2 y = Y[i];
    const int b = fi_box(y.x, g) * g.B + fi_box(y.y, g);
    const int slot = fi_tbl_find(tkey, b, false);
    const int pos = slot >= 0 ? tbase[slot] + atomicAdd(&tcnt[slot], 1) : atomicAdd(&cur[b], 1);
    order[off[b] + pos] = int32_t(i);
  }
}

// Points per thread of the node sums.  A box holding more (a compact or
// clustered embedding can put most points in a few boxes) is split into
// chunks of this many points, one thread each, so no thread walks a long
// box alone.
constexpr int FI_HEAVY = 64;

// Adds the charges 1, z_x, z_y of the sorted points [e0, e1) (one box)
// times the tensor Lagrange weights to acc, in fixed point.  The point
// indices and positions are loaded eight at a time, so the loads of a batch
// are in flight together (the sums keep their order).
template <int P>
__device__ __forceinline__ void fi_accum_point(float2 y, const FiParams& g, long long (&acc)[3][P][P]) {
  double Lx[P], Ly[P];
  fi_weights<P>(y.x, g, Lx);
  fi_weights<P>(y.y, g, Ly);
  const double zx = double(y.x) - g.c, zy = double(y.y) - g.c;
#pragma unroll
  for (int kx = 0; kx < P; ++kx) {
#pragma unroll
    for (int ky = 0; ky < P; ++ky) {
      const double w = Lx[kx] * Ly[ky] * g.scale;
      acc[0][kx][ky] += __double2ll_rn(w);
      acc[1][kx][ky] += __double2ll_rn(w * zx);
      acc[2][kx][ky] += __double2ll_rn(w * zy);
    }
  }
}

template <int P>
__device__ __forceinline__ void fi_accum_range(const float2* __restrict__ Y, const FiParams& g,
                                               const int32_t* __restrict__ order, int64_t e0, int64_t e1,
                                               long long (&acc)[3][P][P]) {
  constexpr int BT = 8;
  int64_t e = e0;
  for (; e + BT <= e1; e += BT) {
    int32_t ix[BT];
    float2 yv[BT];
#pragma unroll
    for (int u = 0; u < BT; ++u) ix[u] = order[e + u];
#pragma unroll
    for (int u = 0; u < BT; ++u) yv[u] = Y[ix[u]];
#pragma unroll
    for (int u = 0; u < BT; ++u) fi_accum_point<P>(yv[u], g, acc);
  }
  for (; e < e1; ++e) fi_accum_point<P>(Y[order[e]], g, acc);
}

// Node sums of box b (thread b < B^2): channel c at G + c N^2, node
// (gx, gy) at gx N + gy.  A box of more than FI_HEAVY points gets zeros
// here; its chunks are added by fi_accum_heavy_kernel.
template <int P>
__global__ __launch_bounds__(256) void fi_accum_kernel(const float2* __restrict__ Y,
                                                       const FiParams* __restrict__ gp,
                                                       const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ order,
                                                       unsigned long long* __restrict__ G) {
  const FiParams g = *gp;
  const int64_t nb = int64_t(g.B) * g.B;
  const int64_t NN = int64_t(g.N) * g.N;
  for (int64_t b = gtid(); b < nb; b += int64_t(gridDim.x) * 256) {
    long long acc[3][P][P];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int kx = 0; kx < P; ++kx)
#pragma unroll
        for (int ky = 0; ky < P; ++ky) acc[c][kx][ky] = 0;
    const int64_t e0 = off[b], e1 = off[b + 1];
    if (e1 - e0 <= FI_HEAVY) fi_accum_range<P>(Y, g, order, e0, e1, acc);
    const int bx = int(b / g.B), by = int(b % g.B);
#pragma unroll
    for (int kx = 0; kx < P; ++kx) {
#pragma unroll
      for (int ky = 0; ky < P; ++ky) {
        const int64_t node = int64_t(P * bx + kx) * g.N + (P * by + ky);
#pragma unroll
        for (int c = 0; c < 3; ++c) G[c * NN + node] = (unsigned long long)acc[c][kx][ky];
      }
    }
  }
}

// nch[b] = FI_HEAVY-point chunks of box b when it holds more than FI_HEAVY
// points, else 0 (b < nbox, the workspace's box count).
__global__ __launch_bounds__(256) void fi_chunks_kernel(const FiParams* __restrict__ gp,
                                                        const int* __restrict__ cnt, int64_t nbox,
                                                        int* __restrict__ nch) {
  const FiParams g = *gp;
  const int64_t nb = int64_t(g.B) * g.B;
  for (int64_t b = gtid(); b < nbox; b += int64_t(gridDim.x) * 256)
    nch[b] = (b < nb && cnt[b] > FI_HEAVY) ? (cnt[b] + FI_HEAVY - 1) / FI_HEAVY : 0;
}

// The chunks of the heavy boxes, one thread each: chunk c belongs to the box
// b with choff[b] <= c < choff[b + 1] (binary search) and covers its sorted
// points off[b] + FI_HEAVY (c - choff[b]) onwards.  Chunks of one box are
// consecutive, so a wave's chunks usually share a box: then its sums are
// added across the wave (integer shuffles, exact) and one lane adds them
// to the box's nodes; otherwise every lane adds its own.  The nodes were
// zeroed by fi_accum_kernel; the integer sums are exact in any order.
template <int P>
__global__ __launch_bounds__(256) void fi_accum_heavy_kernel(const float2* __restrict__ Y,
                                                             const FiParams* __restrict__ gp,
                                                             const int64_t* __restrict__ off,
                                                             const int32_t* __restrict__ order,
                                                             const int64_t* __restrict__ choff, int64_t nbox,
                                                             unsigned long long* __restrict__ G) {
  const FiParams g = *gp;
  const int64_t H = choff[nbox];
  const int64_t NN = int64_t(g.N) * g.N;
  for (int64_t base = int64_t(blockIdx.x) * 256; base < H; base += int64_t(gridDim.x) * 256) {
    const int64_t c = base + threadIdx.x;
    const bool act = c < H;
    int64_t b = -1;
    long long acc[3][P][P];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int kx = 0; kx < P; ++kx)
#pragma unroll
        for (int ky = 0; ky < P; ++ky) acc[q][kx][ky] = 0;
    if (act) {
      int64_t lo = 0, hi = nbox;  // last b with choff[b] <= c
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (choff[mid] <= c) lo = mid;
        else hi = mid;
      }
      b = lo;
      const int64_t e0 = off[b] + FI_HEAVY * (c - choff[b]);
      const int64_t e1 = e0 + FI_HEAVY < off[b + 1] ? e0 + FI_HEAVY : off[b + 1];
      fi_accum_range<P>(Y, g, order, e0, e1, acc);
    }
    // one box across the wave's active lanes?
    int64_t bmin = act ? b : INT64_MAX, bmax = act ? b : -1;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      const int64_t o1 = int64_t(shfl_xor_u64(uint64_t(bmin), m)), o2 = int64_t(shfl_xor_u64(uint64_t(bmax), m));
      bmin = o1 < bmin ? o1 : bmin;
      bmax = o2 > bmax ? o2 : bmax;
    }
    const bool one = bmin == bmax;
    const int64_t bb = one ? bmin : b;
    const int bx = int(bb / g.B), by = int(bb % g.B);
#pragma unroll
    for (int kx = 0; kx < P; ++kx) {
#pragma unroll
      for (int ky = 0; ky < P; ++ky) {
        const int64_t node = int64_t(P * bx + kx) * g.N + (P * by + ky);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          uint64_t v = uint64_t(acc[q][kx][ky]);
          if (one) {
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) v += shfl_xor_u64(v, m);
            if (lane_id() == 0) atomicAdd(&G[q * NN + node], (unsigned long long)v);
          } else if (act) {
            atomicAdd(&G[q * NN + node], (unsigned long long)v);
          }
        }
      }
    }
  }
}

// The three F x F complex grids: W0, W1 + i W2 (zero-padded) and K1 + i K2
// at the wrapped node offsets.  Plane ch at Cg + ch * plane, row-major with
// row stride F.
__global__ __launch_bounds__(256) void fi_load_kernel(const unsigned long long* __restrict__ G,
                                                      const FiParams* __restrict__ gp, int p,
                                                      double2* __restrict__ Cg, int64_t plane) {
  const FiParams g = *gp;
  const int F = g.F, N = g.N;
  const int64_t NN = int64_t(N) * N;
  const double inv = 1.0 / g.scale;
  const double delta = g.h / double(p);
  for (int64_t t = gtid(); t < int64_t(F) * F; t += int64_t(gridDim.x) * 256) {
    const int ix = int(t / F), iy = int(t % F);
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;
    if (ix < N && iy < N) {
      const int64_t node = int64_t(ix) * N + iy;
      w0 = double((long long)G[node]) * inv;
      w1 = double((long long)G[NN + node]) * inv;
      w2 = double((long long)G[2 * NN + node]) * inv;
    }
    const bool vx = ix < N || ix > F - N, vy = iy < N || iy > F - N;
    double k1 = 0.0;
    if (vx && vy) {
      const double dx = delta * double(ix < N ? ix : ix - F), dy = delta * double(iy < N ? iy : iy - F);
      k1 = 1.0 / (1.0 + dx * dx + dy * dy);
    }
    Cg[t] = make_double2(w0, 0.0);
    Cg[plane + t] = make_double2(w1, w2);
    Cg[2 * plane + t] = make_double2(k1, k1 * k1);
  }
}

// --- FFT ---------------------------------------------------------------

// Length-F complex DFT of every row of nch planes (sign -1 forward, +1
// inverse, unnormalised): radix-2 decimation in time in LDS, the input
// loaded in bit-reversed order; twiddles exp(sign 2 pi i k / len) from
// sincospi.  Rows are dealt to the blocks round robin.
__global__ __launch_bounds__(256) void fi_fft_rows_kernel(double2* __restrict__ Cg, int64_t plane, int nch,
                                                          const FiParams* __restrict__ gp, double sign) {
  extern __shared__ double2 sbuf[];
  const int F = gp->F, logF = gp->logF;
  const int64_t rows = int64_t(nch) * F;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    double2* row = Cg + (r / F) * plane + (r % F) * int64_t(F);
    for (int i = threadIdx.x; i < F; i += 256) sbuf[__brev(unsigned(i)) >> (32 - logF)] = row[i];
    __syncthreads();
    for (int half = 1; half < F; half <<= 1) {
      for (int j = threadIdx.x; j < F / 2; j += 256) {
        const int k = j & (half - 1);
        const int i0 = ((j - k) << 1) + k, i1 = i0 + half;
        double sn, cs;
        sincospi(sign * double(k) / double(half), &sn, &cs);
        const double2 a = sbuf[i0], b = sbuf[i1];
        const double2 bw = make_double2(b.x * cs - b.y * sn, b.x * sn + b.y * cs);
        sbuf[i0] = make_double2(a.x + bw.x, a.y + bw.y);
        sbuf[i1] = make_double2(a.x - bw.x, a.y - bw.y);
      }
      __syncthreads();
    }
    for (int i = threadIdx.x; i < F; i += 256) row[i] = sbuf[i];
    __syncthreads();
  }
}

// In-place transpose of nch F x F planes: a block swaps tile (a, b) with
// tile (b, a), a <= b, through LDS.
__global__ __launch_bounds__(256) void fi_transpose_kernel(double2* __restrict__ Cg, int64_t plane, int nch,
                                                           const FiParams* __restrict__ gp) {
  __shared__ double2 ta[FI_TILE][FI_TILE + 1], tb[FI_TILE][FI_TILE + 1];
  const int F = gp->F;
  const int T = F / FI_TILE;
  const int64_t pairs = int64_t(T) * (T + 1) / 2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int64_t w = blockIdx.x; w < pairs * nch; w += gridDim.x) {
    const int ch = int(w / pairs);
    int64_t q = w % pairs;
    int a = 0;  // q -> (a, b), a <= b, row-major over a
    while (q >= T - a) {
      q -= T - a;
      ++a;
    }
    const int b = a + int(q);
    double2* base = Cg + ch * plane;
    for (int y = ty; y < FI_TILE; y += 8) {
      ta[y][tx] = base[int64_t(a * FI_TILE + y) * F + b * FI_TILE + tx];
      tb[y][tx] = base[int64_t(b * FI_TILE + y) * F + a * FI_TILE + tx];
    }
    __syncthreads();
    for (int y = ty; y < FI_TILE; y += 8) {
      base[int64_t(b * FI_TILE + y) * F + a * FI_TILE + tx] = ta[tx][y];
      base[int64_t(a * FI_TILE + y) * F + b * FI_TILE + tx] = tb[tx][y];
    }
    __syncthreads();
  }
}

// Spectra: plane 0 <- W0^ (K1^ + i K2^), plane 1 <- (W1^ + i W2^) K2^, with
// K2^ = Im of plane 2 (K1^, K2^ real).
__global__ __launch_bounds__(256) void fi_mult_kernel(double2* __restrict__ Cg, int64_t plane,
                                                      const FiParams* __restrict__ gp) {
  const int64_t FF = int64_t(gp->F) * gp->F;
  for (int64_t t = gtid(); t < FF; t += int64_t(gridDim.x) * 256) {
    const double2 w0 = Cg[t], w12 = Cg[plane + t], k = Cg[2 * plane + t];
    Cg[t] = make_double2(w0.x * k.x - w0.y * k.y, w0.x * k.y + w0.y * k.x);
    Cg[plane + t] = make_double2(w12.x * k.y, w12.y * k.y);
  }
}

// --- gather ------------------------------------------------------------

// Point values of the potentials (divided by F^2): phi1 + i phi2 from
// plane 0, phi3x + i phi3y from plane 1.  R_i = z_i phi2 - phi3;
// Z partials per block in FP64 (block 0 also subtracts the n self terms).
template <int P>
__global__ __launch_bounds__(256) void fi_gather_kernel(const float2* __restrict__ Y, int64_t n,
                                                        const FiParams* __restrict__ gp,
                                                        const double2* __restrict__ Cg, int64_t plane,
                                                        float2* __restrict__ R, double* __restrict__ Zblock) {
  __shared__ double red[4];
  const FiParams g = *gp;
  const double norm = 1.0 / (double(g.F) * double(g.F));
  double zacc = 0.0;
  for (int64_t i = gtid(); i < n; i += int64_t(gridDim.x) * 256) {
    const float2 y = Y[i];
    double Lx[P], Ly[P];
    const int bx = fi_weights<P>(y.x, g, Lx);
    const int by = fi_weights<P>(y.y, g, Ly);
    double f1 = 0.0, f2 = 0.0, f3x = 0.0, f3y = 0.0;
#pragma unroll
    for (int kx = 0; kx < P; ++kx) {
#pragma unroll
      for (int ky = 0; ky < P; ++ky) {
        const double w = Lx[kx] * Ly[ky];
        const int64_t t = int64_t(P * bx + kx) * g.F + (P * by + ky);
        const double2 a = Cg[t], b = Cg[plane + t];
        f1 += w * a.x;
        f2 += w * a.y;
        f3x += w * b.x;
        f3y += w * b.y;
      }
    }
    f1 *= norm;
    f2 *= norm;
    f3x *= norm;
    f3y *= norm;
    const double zx = double(y.x) - g.c, zy = double(y.y) - g.c;
    R[i] = make_float2(float(zx * f2 - f3x), float(zy * f2 - f3y));
    zacc += f1;
  }
  const double bz = block_sum_d(zacc, red);
  if (threadIdx.x == 0) Zblock[blockIdx.x] = bz - (blockIdx.x == 0 ? double(n) : 0.0);
}

struct FiPlan {
  size_t o_part, o_par, o_G, o_C, o_R, o_Zb, o_kl, o_cnt, o_cur, o_off, o_bsum, o_ord, o_nch, o_choff, bytes;
  int64_t plane, nbox;  // nbox: boxes of the largest grid (B <= max_fft / 4)
};

FiPlan fi_plan(int64_t n, int max_fft) {
  FiPlan L;
  Carve c;
  const int64_t Nmax = max_fft / 2;
  const int64_t Bmax = max_fft / 4;  // p >= 2
  L.plane = int64_t(max_fft) * max_fft;
  L.nbox = Bmax * Bmax;
  L.o_part = c.take(sizeof(float) * 2 * FI_GRID);
  L.o_par = c.take(sizeof(FiParams));
  L.o_cnt = c.take(sizeof(int) * size_t(L.nbox));
  L.o_cur = c.take(sizeof(int) * size_t(L.nbox));
  L.o_off = c.take(sizeof(int64_t) * size_t(L.nbox + 1));
  L.o_bsum = c.take(sizeof(int64_t) * (size_t(ceil_div(L.nbox + 1, SCAN_CHUNK)) + 1));
  L.o_ord = c.take(sizeof(int32_t) * size_t(n));
  L.o_nch = c.take(sizeof(int) * size_t(L.nbox));
  L.o_choff = c.take(sizeof(int64_t) * size_t(L.nbox + 1));
  L.o_G = c.take(sizeof(unsigned long long) * 3 * size_t(Nmax) * size_t(Nmax));
  L.o_C = c.take(sizeof(double2) * 3 * size_t(L.plane));
  L.o_R = c.take(sizeof(float2) * size_t(n));
  L.o_Zb = c.take(sizeof(double) * FI_GRID);
  L.o_kl = c.take(finalize_kl_bytes(n));
  L.bytes = c.off;
  return L;
}

template <int P>
int fi_launch_points(bool spread, const float2* Y, int64_t n, const FiParams* par, const int64_t* off,
                     const int32_t* order, const int64_t* choff, int64_t nbox, unsigned long long* G,
                     const double2* Cg, int64_t plane, float2* R, double* Zb, hipStream_t s) {
  if (spread) {
    hipLaunchKernelGGL(fi_accum_kernel<P>, dim3(unsigned(ceil_div(nbox, 256))), dim3(256), 0, s, Y, par, off, order,
                       G);
    TSNE_CHECK_LAUNCH();
    // at most n / FI_HEAVY + (heavy boxes <= n / FI_HEAVY) chunks
    const int64_t blocks = ceil_div(2 * ceil_div(n, FI_HEAVY), 256);
    hipLaunchKernelGGL(fi_accum_heavy_kernel<P>, dim3(unsigned(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, Y,
                       par, off, order, choff, nbox, G);
  } else {
    hipLaunchKernelGGL(fi_gather_kernel<P>, dim3(FI_GRID), dim3(256), 0, s, Y, n, par, Cg, plane, R, Zb);
  }
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

int fi_points(int p, bool spread, const float2* Y, int64_t n, const FiParams* par, const int64_t* off,
              const int32_t* order, const int64_t* choff, int64_t nbox, unsigned long long* G, const double2* Cg,
              int64_t plane, float2* R,
              double* Zb, hipStream_t s) {
  switch (p) {
    case 2: return fi_launch_points<2>(spread, Y, n, par, off, order, choff, nbox, G, Cg, plane, R, Zb, s);
    case 3: return fi_launch_points<3>(spread, Y, n, par, off, order, choff, nbox, G, Cg, plane, R, Zb, s);
    case 4: return fi_launch_points<4>(spread, Y, n, par, off, order, choff, nbox, G, Cg, plane, R, Zb, s);
    default: return fi_launch_points<5>(spread, Y, n, par, off, order, choff, nbox, G, Cg, plane, R, Zb, s);
  }
}

int fi_fft2(double2* Cg, int64_t plane, int nch, const FiParams* par, int max_fft, double sign, hipStream_t s) {
  const size_t lds = sizeof(double2) * size_t(max_fft);
  const unsigned rgrid = unsigned(max_fft < 2048 ? 2048 : max_fft);
  hipLaunchKernelGGL(fi_fft_rows_kernel, dim3(rgrid), dim3(256), lds, s, Cg, plane, nch, par, sign);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(fi_transpose_kernel, dim3(4096), dim3(256), 0, s, Cg, plane, nch, par);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(fi_fft_rows_kernel, dim3(rgrid), dim3(256), lds, s, Cg, plane, nch, par, sign);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

}  // namespace tsne

extern "C" int tsne_kl_grad_fft(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col,
                                const float* val, float exaggeration, int32_t n_interp, int32_t min_boxes,
                                float max_box_width, int32_t max_fft, float* grad, double* Z, double* kl,
                                int64_t* nonfinite, void* workspace, size_t* workspace_bytes, void* stream) {
  using namespace tsne;
  if (!Y || !row_ptr || !col || !val || !grad || n < 2) return TSNE_ERR_INVALID_ARG;
  if (!(exaggeration > 0.0f) || !(exaggeration < INFINITY)) return TSNE_ERR_INVALID_ARG;
  if (n_interp < 2 || n_interp > FI_MAX_P || min_boxes < 1) return TSNE_ERR_INVALID_ARG;
  if (!(max_box_width > 0.0f) || !(max_box_width < INFINITY)) return TSNE_ERR_INVALID_ARG;
  if (max_fft < FI_MIN_FFT || max_fft > FI_MAX_FFT || (max_fft & (max_fft - 1))) return TSNE_ERR_INVALID_ARG;
  if (2 * int64_t(n_interp) * min_boxes > max_fft) return TSNE_ERR_INVALID_ARG;
  if (n > (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  const FiPlan L = fi_plan(n, max_fft);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = as_stream(stream);
  unsigned long long* nf = reinterpret_cast<unsigned long long*>(nonfinite);
  if (nf && (rc = launch_fill<unsigned long long>(nf, 1, 0ull, s))) return rc;
  const float2* Y2 = reinterpret_cast<const float2*>(Y);
  float* part = reinterpret_cast<float*>(ws + L.o_part);
  FiParams* par = reinterpret_cast<FiParams*>(ws + L.o_par);
  unsigned long long* G = reinterpret_cast<unsigned long long*>(ws + L.o_G);
  double2* Cg = reinterpret_cast<double2*>(ws + L.o_C);
  float2* R = reinterpret_cast<float2*>(ws + L.o_R);
  double* Zb = reinterpret_cast<double*>(ws + L.o_Zb);
  double* klp = reinterpret_cast<double*>(ws + L.o_kl);
  int* cnt = reinterpret_cast<int*>(ws + L.o_cnt);
  int* cur = reinterpret_cast<int*>(ws + L.o_cur);
  int64_t* off = reinterpret_cast<int64_t*>(ws + L.o_off);
  int64_t* bsum = reinterpret_cast<int64_t*>(ws + L.o_bsum);
  int32_t* order = reinterpret_cast<int32_t*>(ws + L.o_ord);
  int* nch = reinterpret_cast<int*>(ws + L.o_nch);
  int64_t* choff = reinterpret_cast<int64_t*>(ws + L.o_choff);

  hipLaunchKernelGGL(fi_bbox_kernel, dim3(FI_GRID), dim3(256), 0, s, Y2, n, part);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(fi_params_kernel, dim3(1), dim3(256), 0, s, part, FI_GRID, n, n_interp, min_boxes,
                     max_box_width, max_fft, par);
  TSNE_CHECK_LAUNCH();
  // counting sort of the points by box, then the per-box node sums
  if ((rc = launch_fill<int>(cnt, L.nbox, 0, s))) return rc;
  if ((rc = launch_fill<int>(cur, L.nbox, 0, s))) return rc;
  const dim3 pgrid(unsigned(ceil_div(n, 256) < FI_CBLOCKS ? ceil_div(n, 256) : FI_CBLOCKS));
  hipLaunchKernelGGL(fi_count_kernel, pgrid, dim3(256), 0, s, Y2, n, par, cnt);
  TSNE_CHECK_LAUNCH();
  if ((rc = exclusive_scan<int>(cnt, L.nbox, off, bsum, s))) return rc;
  hipLaunchKernelGGL(fi_scatter_kernel, pgrid, dim3(256), 0, s, Y2, n, par, off, cur, order);
  TSNE_CHECK_LAUNCH();
  // the chunks of the heavy boxes (more than FI_HEAVY points), listed by a scan
  const int64_t bgrid = ceil_div(L.nbox, 256) < 4096 ? ceil_div(L.nbox, 256) : 4096;
  hipLaunchKernelGGL(fi_chunks_kernel, dim3(unsigned(bgrid)), dim3(256), 0, s, par, cnt, L.nbox, nch);
  TSNE_CHECK_LAUNCH();
  if ((rc = exclusive_scan<int>(nch, L.nbox, choff, bsum, s))) return rc;
  if ((rc = fi_points(n_interp, true, Y2, n, par, off, order, choff, L.nbox, G, Cg, L.plane, R, Zb, s))) return rc;
  hipLaunchKernelGGL(fi_load_kernel, dim3(4096), dim3(256), 0, s, G, par, n_interp, Cg, L.plane);
  TSNE_CHECK_LAUNCH();
  if ((rc = fi_fft2(Cg, L.plane, 3, par, max_fft, -1.0, s))) return rc;
  hipLaunchKernelGGL(fi_mult_kernel, dim3(4096), dim3(256), 0, s, Cg, L.plane, par);
  TSNE_CHECK_LAUNCH();
  if ((rc = fi_fft2(Cg, L.plane, 2, par, max_fft, 1.0, s))) return rc;
  if ((rc = fi_points(n_interp, false, Y2, n, par, off, order, choff, L.nbox, G, Cg, L.plane, R, Zb, s))) return rc;
  // the attraction takes the rows in box order (a spatial order of Y: rows
  // that share P-neighbours run together, so their y_j gathers hit L2); the
  // order within a box follows the scatter's atomics, so a requested KL, whose
  // per-block sums would follow it, takes the rows in index order instead
  return finalize_csr_launch(Y, n, row_ptr, col, val, exaggeration, reinterpret_cast<const float*>(R), Zb, FI_GRID,
                             grad, Z, kl, klp, nf, s, kl ? nullptr : order);
}
