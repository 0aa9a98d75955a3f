// tsne_kl_grad: exact t-SNE gradient with early exaggeration
// (van der Maaten & Hinton 2008, eq. 5 and Sec. 3.4) and optional Z / KL.
// Launch sequence: the symmetric all-pairs repulsion pass (rep_sym.hpp),
// then a finalize pass that gathers the sparse attraction over the CSR rows,
// sums the repulsion partials and Z in a fixed order and writes
// g_i = 4 (alpha A_i - R_i / Z); and, when KL is requested, a one-block
// reduction of the per-block sums p ln p, p ln q (q = 1/w) and p.
#include "common.hpp"
#include "klgrad.hpp"
#include "rep_sym.hpp"
#include "scan.hpp"

#include <mutex>

namespace tsne {

// Finalize, 16 rows per block: rows 16 b .. 16 b + 15, or with `rows` the
// rows rows[16 c .. 16 c + 15] (a permutation of 0 .. n - 1: a spatial order
// makes the y_j gathers of the rows resident together overlap in L2), with c
// the block's place in the eighth of the blocks on its XCD.
// Attraction A_i = sum_{e in row i} p_e w_e (y_i - y_j), entry-parallel: the
// block's CSR entries, numbered flat over its rows, are dealt to all 256
// threads in chunks of FIN_CHUNK (thread t takes flat entries c0 + t + 256 m,
// m < FIN_EPT), so a hub row with thousands of entries costs the block no
// more dependent trips than a short one: every thread issues its
// column/value loads, then its y_j gathers, then writes p w (y_i - y_j) to
// LDS, and lane l of the 16 of group g adds row g's entries l, l + 16, ...
// (counted from the row's first entry, so a row's sum does not depend on
// which rows share its block), then a DPP reduction.
// Optional per-block sums of p ln p, p ln q (q = 1/w) and p for the KL.
// Repulsion partials: thread (g, sl) adds slices g, g + 16, ... of row
// r0 + sl in FP64; the 16 slice sums are combined in a fixed order.  The
// loads that depend on nothing (CSR bounds, the first partial slices, the Z
// partials) are issued first.  Then
// g_i = 4 (alpha A_i - R_i / Z); STEP: instead of storing g, apply the
// optimiser step to the row (FusedStep).  Column indices outside [0, n)
// contribute nothing.  ATTP: the attraction was summed per job by the
// all-pairs kernel (AttList); it is read from its partial slices, exactly
// like the repulsion, and the CSR is not touched.  nonfinite (nullable):
// the block adds the number of non-finite coordinates of its rows of Y (with
// STEP: of its stepped rows, the positions the pass writes).
constexpr int FIN_ROWS = 16;
constexpr int FIN_EPT = 8;
constexpr int FIN_CHUNK = 256 * FIN_EPT;
constexpr int FIN_PRE = 5;  // partial slices per thread loaded up front (all of them for ns <= 80)

template <bool STEP, bool ATTP>
__global__ __launch_bounds__(256) void finalize_tsne_kernel(
    const float2* __restrict__ Y, int64_t n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, float alpha, const float2* __restrict__ Rpart, const float* __restrict__ Zrowpart,
    const float2* __restrict__ Apart, int64_t ns, bool grouped, const double* __restrict__ Zblock, int64_t nZ,
    float2* __restrict__ grad, double* __restrict__ Zrow, double* __restrict__ Z_out, double* __restrict__ klpart,
    FusedStep st, unsigned long long* __restrict__ nonfinite, const int32_t* __restrict__ rows) {
  constexpr int NPR = ATTP ? 5 : 3;  // per-thread sums: R x, R y, Z_row (, A x, A y)
  __shared__ float2 contrib[ATTP ? 1 : FIN_CHUNK];
  __shared__ int64_t rp0[FIN_ROWS];      // first CSR entry of each row of the block
  __shared__ int64_t cum[FIN_ROWS + 1];  // flat offsets of the rows' entries
  __shared__ float2 yrow[FIN_ROWS];
  __shared__ double red[4];
  __shared__ double pr[16][FIN_ROWS][NPR];
  __shared__ float2 att[FIN_ROWS];
  const int tid = threadIdx.x;
  const int g = tid >> 4, sl = tid & 15;
  // With a row order, workgroups (dealt round-robin over the 8 XCDs) take
  // their group of 16 from the contiguous eighth of the order that belongs
  // to their XCD, so each XCD's L2 holds the y_j of one compact region.
  const int64_t r0 = (rows ? xcd_block() : int64_t(blockIdx.x)) * FIN_ROWS;
  // the block's row of local index q (n past the last one)
  auto row_of = [&](int q) -> int64_t {
    const int64_t p = r0 + q;
    return p < n ? (rows ? int64_t(rows[p]) : p) : n;
  };
  const int64_t prow = row_of(sl);  // partial-sum row of this thread
  const int64_t myrow = tid < FIN_ROWS ? row_of(tid) : n;

  // --- loads with no dependences -----------------------------------------
  int64_t len = 0;
  if (tid < FIN_ROWS) {
    const int64_t a = myrow < n ? row_ptr[myrow] : 0, b = myrow < n ? row_ptr[myrow + 1] : 0;
    rp0[tid] = a;
    len = b - a;
    yrow[tid] = myrow < n ? Y[myrow] : make_float2(0.0f, 0.0f);
  }
  float2 rpv[FIN_PRE], apv[FIN_PRE];
#pragma unroll
  for (int u = 0; u < FIN_PRE; ++u) {
    const int64_t k = g + 16 * u;
    const bool ok = prow < n && k < ns;
    rpv[u] = ok ? Rpart[part_index(prow, k, ns, n, grouped)] : make_float2(0.0f, 0.0f);
    apv[u] = (ATTP && ok) ? Apart[part_index(prow, k, ns, n, grouped)] : make_float2(0.0f, 0.0f);
  }
  // the stepped rows' state (in flight while the partials are summed)
  float2 sy = make_float2(0.0f, 0.0f), su = sy, sg = sy;
  if (STEP && myrow < n) {
    sy = Y[myrow];
    su = st.U[myrow];
    sg = st.G[myrow];
  }
  const double zt = zblock_thread_sum(Zblock, nZ);
  if (!STEP && nonfinite && tid < 64) {  // wave 0 covers the block's rows
    const float2 y = myrow < n ? Y[myrow] : make_float2(0.0f, 0.0f);
    const int bad = __popcll(__ballot(!isfinite(y.x))) + __popcll(__ballot(!isfinite(y.y)));
    if (tid == 0 && bad) atomicAdd(nonfinite, static_cast<unsigned long long>(bad));
  }
  if (tid < 64) {  // flat offsets: inclusive sum of the 16 lengths in DPP row 0
    int64_t c = len;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const int64_t u = int64_t(__shfl_up(uint64_t(c), o, 16));
      if ((tid & 15) >= o) c += u;
    }
    if (tid < FIN_ROWS) cum[tid + 1] = c;
    if (tid == 0) cum[0] = 0;
  }
  __syncthreads();

  // --- attraction, entry-parallel -----------------------------------------
  const int64_t F = cum[FIN_ROWS];
  const int64_t ga = cum[g], gb = cum[g + 1];
  float ax = 0.0f, ay = 0.0f, plp = 0.0f, plq = 0.0f, ps = 0.0f;
  for (int64_t c0 = 0; !ATTP && c0 < F; c0 += FIN_CHUNK) {
    int32_t jj[FIN_EPT];
    float pp[FIN_EPT];
    int rr[FIN_EPT];
    int r = 0;  // row of the flat entry (a thread's entries are increasing)
#pragma unroll
    for (int m = 0; m < FIN_EPT; ++m) {
      const int64_t f = c0 + tid + 256 * m;
      const bool ok = f < F;
      while (r < FIN_ROWS - 1 && cum[r + 1] <= f) ++r;
      rr[m] = r;
      const int64_t e = rp0[r] + (f - cum[r]);
      // read once: non-temporal, so the stream of entries does not evict the
      // gathered rows of Y from L2
      jj[m] = ok ? __builtin_nontemporal_load(col + e) : 0;
      pp[m] = ok ? __builtin_nontemporal_load(val + e) : 0.0f;
    }
#pragma unroll
    for (int m = 0; m < FIN_EPT; ++m) {
      if (jj[m] < 0 || jj[m] >= n) {
        jj[m] = 0;
        pp[m] = 0.0f;
      }
    }
    float2 yj[FIN_EPT];
#pragma unroll
    for (int m = 0; m < FIN_EPT; ++m) yj[m] = Y[jj[m]];
#pragma unroll
    for (int m = 0; m < FIN_EPT; ++m) {
      const float2 yi = yrow[rr[m]];
      const float dx = yi.x - yj[m].x, dy = yi.y - yj[m].y;
      const float q = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1.0f));
      const float pw = pp[m] * __builtin_amdgcn_rcpf(q);
      contrib[tid + 256 * m] = make_float2(pw * dx, pw * dy);
      if (klpart) {
        if (pp[m] > 0.0f) plp += pp[m] * logf(pp[m]);
        plq += pp[m] * logf(q);
        ps += pp[m];
      }
    }
    __syncthreads();
    const int64_t lo = ga > c0 ? ga : c0;
    const int64_t hi = gb < c0 + FIN_CHUNK ? gb : c0 + FIN_CHUNK;
    int64_t f = ga + sl;  // this lane's entries of row g: ga + sl + 16 m
    if (f < lo) f += (lo - f + 15) / 16 * 16;
    for (; f < hi; f += 16) {
      const float2 c = contrib[f - c0];
      ax += c.x;
      ay += c.y;
    }
    __syncthreads();
  }

  // --- repulsion partials: slices g, g + 16, ... in order ------------------
  {
    double rx = 0.0, ry = 0.0, zr = 0.0, axd = 0.0, ayd = 0.0;
#pragma unroll
    for (int u = 0; u < FIN_PRE; ++u) {
      rx += double(rpv[u].x);
      ry += double(rpv[u].y);
      if (ATTP) {
        axd += double(apv[u].x);
        ayd += double(apv[u].y);
      }
    }
    if (prow < n) {
      int64_t k = g + 16 * FIN_PRE;
      for (; k + 48 < ns; k += 64) {
        float2 rr[4], aa[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          rr[u] = Rpart[part_index(prow, k + 16 * u, ns, n, grouped)];
          if (ATTP) aa[u] = Apart[part_index(prow, k + 16 * u, ns, n, grouped)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          rx += double(rr[u].x);
          ry += double(rr[u].y);
          if (ATTP) {
            axd += double(aa[u].x);
            ayd += double(aa[u].y);
          }
        }
      }
      for (; k < ns; k += 16) {
        const float2 rr = Rpart[part_index(prow, k, ns, n, grouped)];
        rx += double(rr.x);
        ry += double(rr.y);
        if (ATTP) {
          const float2 aa = Apart[part_index(prow, k, ns, n, grouped)];
          axd += double(aa.x);
          ayd += double(aa.y);
        }
      }
      if (Zrow)
        for (int64_t kk = g; kk < ns; kk += 16) zr += double(Zrowpart[part_index(prow, kk, ns, n, grouped)]);
    }
    pr[g][sl][0] = rx;
    pr[g][sl][1] = ry;
    pr[g][sl][2] = zr;
    if (ATTP) {
      pr[g][sl][3 % NPR] = axd;
      pr[g][sl][4 % NPR] = ayd;
    }
  }
  ax = row16_sum(ax);
  ay = row16_sum(ay);
  if (sl == 0) att[g] = make_float2(ax, ay);
  const double Z = block_sum_d(zt, red);  // its barriers also publish pr and att
  if (blockIdx.x == 0 && tid == 0 && Z_out) *Z_out = Z;
  if (myrow < n) {
    double Rx = 0.0, Ry = 0.0, Zr = 0.0, Ax = 0.0, Ay = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      Rx += pr[k][tid][0];
      Ry += pr[k][tid][1];
      Zr += pr[k][tid][2];
      if (ATTP) {
        Ax += pr[k][tid][3 % NPR];
        Ay += pr[k][tid][4 % NPR];
      }
    }
    if (!ATTP) {
      Ax = double(att[tid].x);
      Ay = double(att[tid].y);
    }
    const float2 gi = make_float2(float(4.0 * (double(alpha) * Ax - Rx / Z)),
                                  float(4.0 * (double(alpha) * Ay - Ry / Z)));
    const int64_t i = myrow;
    if (STEP) {
      step_coord(sy.x, su.x, sg.x, gi.x, st.lr, st.mom, st.inc, st.dec, st.mn);
      step_coord(sy.y, su.y, sg.y, gi.y, st.lr, st.mom, st.inc, st.dec, st.mn);
      st.Yout[i] = sy;
      st.U[i] = su;
      st.G[i] = sg;
    } else {
      grad[i] = gi;
    }
    if (Zrow) Zrow[i] = Zr;
  }
  if (STEP && nonfinite && tid < 64) {  // the stepped rows (sy is 0 outside them)
    const int bad = __popcll(__ballot(!isfinite(sy.x))) + __popcll(__ballot(!isfinite(sy.y)));
    if (tid == 0 && bad) atomicAdd(nonfinite, static_cast<unsigned long long>(bad));
  }
  if (klpart) {
    const double a = block_sum_d(double(plp), red);
    const double b = block_sum_d(double(plq), red);
    const double c = block_sum_d(double(ps), red);
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
  __shared__ double red[4];
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

size_t finalize_kl_bytes(int64_t n) { return sizeof(double) * 3 * size_t(ceil_div(n, FIN_ROWS)); }

int finalize_csr_launch(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                        float alpha, const float* R, const double* Zblock, int64_t nZ, float* grad, double* Z,
                        double* kl, double* klpart, unsigned long long* nonfinite, hipStream_t s,
                        const int32_t* rows) {
  const int64_t nfin = ceil_div(n, FIN_ROWS);
  double* kp = kl ? klpart : nullptr;
  hipLaunchKernelGGL((finalize_tsne_kernel<false, false>), dim3(unsigned(nfin)), dim3(256), 0, s,
                     reinterpret_cast<const float2*>(Y), n, row_ptr, col, val, alpha,
                     reinterpret_cast<const float2*>(R), static_cast<const float*>(nullptr),
                     static_cast<const float2*>(nullptr), int64_t(1), false, Zblock, nZ,
                     reinterpret_cast<float2*>(grad), static_cast<double*>(nullptr), Z, kp, FusedStep{}, nonfinite,
                     rows);
  TSNE_CHECK_LAUNCH();
  if (kl) {
    hipLaunchKernelGGL(kl_reduce_kernel, dim3(1), dim3(256), 0, s, kp, nfin, Zblock, nZ, kl);
    TSNE_CHECK_LAUNCH();
  }
  return TSNE_OK;
}

KlGradPlan klgrad_plan(int64_t n, bool with_att, bool with_zrow) {
  KlGradPlan L;
  L.g = SymGrid::make(n);
  L.nfin = ceil_div(n, FIN_ROWS);
  L.zrow = with_zrow;
  Carve c;
  const size_t n16 = size_t(ceil_div(n, 16)) * 16;
  L.o_R = c.take(sizeof(float2) * size_t(L.g.ns) * n16);
  L.o_Zr = with_zrow ? c.take(sizeof(float) * size_t(L.g.ns) * n16) : 0;
  L.o_Zb = c.take(sizeof(double) * size_t(L.g.nwg));
  L.o_kl = c.take(sizeof(double) * 3 * size_t(L.nfin));
  L.o_A = with_att ? c.take(sizeof(float2) * size_t(L.g.ns) * n16) : 0;
  L.o_g = with_att ? c.take(sizeof(float2) * size_t(n)) : 0;
  L.bytes = c.off;
  return L;
}

// --- job-grouped attraction list ------------------------------------------

__device__ __forceinline__ int64_t job_of(int64_t s, int64_t t, int64_t ns) {
  return s == t ? ns * (ns - 1) / 2 + s : t * (t - 1) / 2 + s;  // inverse of job_pair
}

// Blocks of ATT_ROWS consecutive rows; S is a multiple of ATT_ROWS, so a
// block's rows lie in one superblock s and an entry (i, j), j > i, belongs
// to job (s, j / S).  The block histograms its entries over the opposite
// superblock t in LDS, ATT_BINS superblocks per pass, and touches each job's
// global counter once per pass: at most ns global atomics per block instead
// of one per entry.  ROWS is 256 where that still gives 1024 blocks or
// more (at 10^6 points the 3907 blocks make 4 M such atomics, where 16-row
// blocks made 56 M and took five times as long), else 16, so that small
// problems keep enough blocks.  The order of the entries inside a job's
// range follows the
// LDS atomics; the all-pairs kernel sums them in exact fixed point, so the
// order does not reach any result.
constexpr int ATT_BINS = 1024;
inline bool att_big_blocks(int64_t n) { return ceil_div(n, 256) >= 1024; }

// row of entry e among the block's rows (rp[0..ROWS]); e is increasing per
// thread, so the search resumes from the previous row
template <int ROWS>
__device__ __forceinline__ int att_row(const int64_t* rp, int64_t e, int r) {
  while (r < ROWS - 1 && rp[r + 1] <= e) ++r;
  return r;
}

template <bool SCATTER, int ROWS>
__global__ __launch_bounds__(256) void att_bucket_kernel(int64_t n, int64_t S, int64_t ns,
                                                         const int64_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col,
                                                         const float* __restrict__ val, int* __restrict__ cnt,
                                                         const int64_t* __restrict__ off, int* __restrict__ cur,
                                                         uint32_t* __restrict__ ij, float* __restrict__ p, int64_t cap) {
  __shared__ int h[ATT_BINS];
  __shared__ int64_t base[SCATTER ? ATT_BINS : 1];
  __shared__ int64_t rp[ROWS + 1];
  const int tid = threadIdx.x;
  const int lgS = __builtin_ctzll(uint64_t(S));  // S is a power of two: shifts, not 64-bit divisions
  const int64_t r0 = int64_t(blockIdx.x) * ROWS;
  const int64_t s = r0 >> lgS;
  for (int q = tid; q <= ROWS; q += 256) rp[q] = row_ptr[r0 + q < n ? r0 + q : n];
  __syncthreads();
  const int64_t E0 = rp[0], E1 = rp[ROWS];
  for (int64_t w0 = s; w0 < ns; w0 += ATT_BINS) {  // opposite superblocks t >= s
    const int64_t w1 = w0 + ATT_BINS < ns ? w0 + ATT_BINS : ns;
    for (int b = tid; b < ATT_BINS; b += 256) h[b] = 0;
    __syncthreads();
    int r = 0;
    for (int64_t e = E0 + tid; e < E1; e += 256) {
      r = att_row<ROWS>(rp, e, r);
      const int64_t i = r0 + r;
      const int32_t j = col[e];
      const int64_t t = j >> lgS;
      if (j > i && j < n && t >= w0 && t < w1) atomicAdd(&h[t - w0], 1);
    }
    __syncthreads();
    for (int64_t t = w0 + tid; t < w1; t += 256) {
      const int c = h[t - w0];
      if (!c) continue;
      const int64_t q = job_of(s, t, ns);
      if (SCATTER) {
        base[t - w0] = off[q] + atomicAdd(&cur[q], c);
        h[t - w0] = 0;  // becomes the block's cursor in the range
      } else {
        atomicAdd(&cnt[q], c);
      }
    }
    if (SCATTER) {
      __syncthreads();
      r = 0;
      for (int64_t e = E0 + tid; e < E1; e += 256) {
        r = att_row<ROWS>(rp, e, r);
        const int64_t i = r0 + r;
        const int32_t j = col[e];
        const int64_t t = j >> lgS;
        if (j > i && j < n && t >= w0 && t < w1) {
          const int64_t pos = base[t - w0] + atomicAdd(&h[t - w0], 1);
          if (pos < cap) {  // cap < entries only if the caller's nnz is wrong
            ij[pos] = uint32_t(i - s * S) | (uint32_t(j - t * S) << 16);
            p[pos] = val[e];
          }
        }
      }
    }
    __syncthreads();  // h and base are reused by the next pass
  }
}

AttPlan att_plan(const SymGrid& g, int64_t nnz) {
  AttPlan A;
  Carve c;
  const size_t nb = size_t(ceil_div(g.njobs + 1, SCAN_CHUNK)) + 1;
  A.o_cnt = c.take(sizeof(int) * size_t(g.njobs));
  A.o_cur = c.take(sizeof(int) * size_t(g.njobs));
  A.o_off = c.take(sizeof(int64_t) * (size_t(g.njobs) + 1));
  A.o_bsum = c.take(sizeof(int64_t) * nb);
  A.o_ij = c.take(sizeof(uint32_t) * size_t(nnz > 0 ? nnz : 1));
  A.o_p = c.take(sizeof(float) * size_t(nnz > 0 ? nnz : 1));
  A.bytes = c.off;
  return A;
}

int att_build(const AttPlan& A, const SymGrid& g, char* ws, int64_t n, const int64_t* row_ptr, const int32_t* col,
              const float* val, AttList* out, hipStream_t s) {
  int* cnt = reinterpret_cast<int*>(ws + A.o_cnt);
  int* cur = reinterpret_cast<int*>(ws + A.o_cur);
  int64_t* off = reinterpret_cast<int64_t*>(ws + A.o_off);
  int64_t* bsum = reinterpret_cast<int64_t*>(ws + A.o_bsum);
  uint32_t* ij = reinterpret_cast<uint32_t*>(ws + A.o_ij);
  float* p = reinterpret_cast<float*>(ws + A.o_p);
  int rc;
  if ((rc = launch_fill<int>(cnt, g.njobs, 0, s))) return rc;
  if ((rc = launch_fill<int>(cur, g.njobs, 0, s))) return rc;
  const bool big = att_big_blocks(n);
  const dim3 grid(unsigned(ceil_div(n, big ? 256 : 16))), block(256);
  auto count = big ? att_bucket_kernel<false, 256> : att_bucket_kernel<false, 16>;
  hipLaunchKernelGGL(count, grid, block, 0, s, n, g.S, g.ns, row_ptr, col, val, cnt,
                     static_cast<const int64_t*>(nullptr), static_cast<int*>(nullptr),
                     static_cast<uint32_t*>(nullptr), static_cast<float*>(nullptr), int64_t(0));
  TSNE_CHECK_LAUNCH();
  if ((rc = exclusive_scan<int>(cnt, g.njobs, off, bsum, s))) return rc;
  const int64_t cap = int64_t((A.o_p - A.o_ij) / sizeof(uint32_t));
  auto scatter = big ? att_bucket_kernel<true, 256> : att_bucket_kernel<true, 16>;
  hipLaunchKernelGGL(scatter, grid, block, 0, s, n, g.S, g.ns, row_ptr, col, val, static_cast<int*>(nullptr), off,
                     cur, ij, p, cap);
  TSNE_CHECK_LAUNCH();
  *out = AttList{off, ij, p, cap};
  return TSNE_OK;
}

int klgrad_launch(const KlGradPlan& L, char* ws, const float* Y, int64_t n, const int64_t* row_ptr,
                  const int32_t* col, const float* val, float alpha, float* grad, double* Z, double* kl, double* Zrow,
                  hipStream_t s, const FusedStep* step, hipEvent_t after_repulsion, const AttList* att,
                  unsigned long long* nonfinite) {
  const SymGrid& g = L.g;
  if (Zrow && !L.zrow) return TSNE_ERR_INVALID_ARG;  // plan without room for the per-row Z partials
  const bool fused = att && !Zrow && L.o_A;
  float* Rpart = reinterpret_cast<float*>(ws + L.o_R);
  float* Zrowpart = Zrow ? reinterpret_cast<float*>(ws + L.o_Zr) : nullptr;
  double* Zblock = reinterpret_cast<double*>(ws + L.o_Zb);
  double* klpart = kl ? reinterpret_cast<double*>(ws + L.o_kl) : nullptr;
  float2* Apart = fused ? reinterpret_cast<float2*>(ws + L.o_A) : nullptr;
  const AttList al = fused ? *att : AttList{nullptr, nullptr, nullptr, 0};
  const float2* Y2 = reinterpret_cast<const float2*>(Y);
  const size_t lds = rep_sym_lds_bytes(g.S, Zrow != nullptr, fused);
  const dim3 grid(unsigned(g.nwg)), block(256);
#define TSNE_REP_SYM(Z, PF, A) \
  hipLaunchKernelGGL((rep_sym_kernel<Z, PF, A>), grid, block, lds, s, Y2, n, g.ns, Rpart, Zrowpart, Zblock, al, Apart)
  if (Zrow) {
    if (g.S == 256) TSNE_REP_SYM(true, 1, false);
    else if (g.S == 512) TSNE_REP_SYM(true, 2, false);
    else TSNE_REP_SYM(true, 4, false);
  } else if (fused) {
    if (g.S == 256) TSNE_REP_SYM(false, 1, true);
    else if (g.S == 512) TSNE_REP_SYM(false, 2, true);
    else TSNE_REP_SYM(false, 4, true);
  } else {
    if (g.S == 256) TSNE_REP_SYM(false, 1, false);
    else if (g.S == 512) TSNE_REP_SYM(false, 2, false);
    else TSNE_REP_SYM(false, 4, false);
  }
#undef TSNE_REP_SYM
  TSNE_CHECK_LAUNCH();
  if (after_repulsion) {
    const hipError_t e = hipEventRecord(after_repulsion, s);
    if (e != hipSuccess) {
      set_last_hip_error(e);
      return TSNE_ERR_HIP;
    }
  }
  const dim3 fgrid(unsigned(L.nfin));
  const float2* R2 = reinterpret_cast<const float2*>(Rpart);
  const bool grp = part_grouped(g.S);
  float2* gr = reinterpret_cast<float2*>(grad);
  const FusedStep st = step ? *step : FusedStep{};
#define TSNE_FIN(STEP, A, GR, KLP, NF)                                                                      \
  hipLaunchKernelGGL((finalize_tsne_kernel<STEP, A>), fgrid, block, 0, s, Y2, n, row_ptr, col, val, alpha, R2, \
                     Zrowpart, Apart, g.ns, grp, Zblock, g.nwg, GR, Zrow, Z, KLP, st, NF,                    \
                     static_cast<const int32_t*>(nullptr))
  if (fused) {
    if (step) TSNE_FIN(true, true, nullptr, nullptr, nonfinite);
    else TSNE_FIN(false, true, gr, nullptr, nonfinite);
    if (kl) {
      // the KL sums come from the CSR pass, at the same Y; its gradient
      // output goes to scratch, so logging does not change the trajectory
      TSNE_CHECK_LAUNCH();
      TSNE_FIN(false, false, reinterpret_cast<float2*>(ws + L.o_g), klpart, nullptr);
    }
  } else {
    if (step) TSNE_FIN(true, false, nullptr, klpart, nonfinite);
    else TSNE_FIN(false, false, gr, klpart, nonfinite);
  }
#undef TSNE_FIN
  TSNE_CHECK_LAUNCH();
  if (kl) {
    hipLaunchKernelGGL(kl_reduce_kernel, dim3(1), dim3(256), 0, s, klpart, L.nfin, Zblock, g.nwg, kl);
    TSNE_CHECK_LAUNCH();
  }
  return TSNE_OK;
}

}  // namespace tsne

namespace tsne {

// Argument checks shared by tsne_kl_grad and tsne_kl_grad_noalloc.
static int kl_grad_args(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                        float exaggeration, float* grad) {
  if (!Y || !row_ptr || !col || !val || !grad || n < 2) return TSNE_ERR_INVALID_ARG;
  if (!(exaggeration > 0.0f) || !(exaggeration < INFINITY)) return TSNE_ERR_INVALID_ARG;
  if (n > (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  return TSNE_OK;
}

// The launches of one gradient evaluation on workspace `ws` (plan L).
static int kl_grad_enqueue(const KlGradPlan& L, char* ws, const float* Y, int64_t n, const int64_t* row_ptr,
                           const int32_t* col, const float* val, float exaggeration, float* grad, double* Z,
                           double* kl, double* Zrow, int64_t* nonfinite, hipStream_t s) {
  unsigned long long* nf = reinterpret_cast<unsigned long long*>(nonfinite);
  int rc;
  if (nf && (rc = launch_fill<unsigned long long>(nf, 1, 0ull, s))) return rc;
  return klgrad_launch(L, ws, Y, n, row_ptr, col, val, exaggeration, grad, Z, kl, Zrow, s, nullptr, nullptr, nullptr,
                       nf);
}

// Scratch of tsne_kl_grad_noalloc, for callers that cannot allocate.  Each
// device holds its own copy for the life of the process.  In host code the
// name `scratch` is only a host-side handle, not a device address: the
// address the kernels get is the one hipGetSymbolAddress returns on each
// device, looked up once per device (with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[TSNE_NOALLOC_SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_addr[SCRATCH_MAX_DEVICES];

// Device address of `scratch` on the current device.
static int scratch_address(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_last_hip_error(e);
    return TSNE_ERR_HIP;
  }
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return TSNE_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_last_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return TSNE_ERR_HIP;
    }
    g_scratch_addr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_addr[dev];
  return TSNE_OK;
}

}  // namespace tsne

extern "C" int tsne_kl_grad(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                            float exaggeration, float* grad, double* Z, double* kl, double* Zrow, int64_t* nonfinite,
                            void* workspace, size_t* workspace_bytes, void* stream) {
  using namespace tsne;
  int rc = kl_grad_args(Y, n, row_ptr, col, val, exaggeration, grad);
  if (rc != TSNE_OK) return rc;
  const KlGradPlan L = klgrad_plan(n);
  rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  return kl_grad_enqueue(L, static_cast<char*>(workspace), Y, n, row_ptr, col, val, exaggeration, grad, Z, kl, Zrow,
                         nonfinite, as_stream(stream));
}

extern "C" int tsne_kl_grad_noalloc(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col,
                                    const float* val, float exaggeration, float* grad, double* Z, double* kl,
                                    double* Zrow, int64_t* nonfinite, void* stream) {
  using namespace tsne;
  int rc = kl_grad_args(Y, n, row_ptr, col, val, exaggeration, grad);
  if (rc != TSNE_OK) return rc;
  const KlGradPlan L = klgrad_plan(n, false, Zrow != nullptr);
  if (L.bytes > TSNE_NOALLOC_SCRATCH_BYTES) return TSNE_ERR_SCRATCH;
  TSNE_REQUIRE_GFX950();
  char* ws = nullptr;
  if ((rc = scratch_address(&ws)) != TSNE_OK) return rc;
  return kl_grad_enqueue(L, ws, Y, n, row_ptr, col, val, exaggeration, grad, Z, kl, Zrow, nonfinite,
                         as_stream(stream));
}
