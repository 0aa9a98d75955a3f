// UMAP on a kNN graph (McInnes, Healy & Melville 2018, arXiv:1802.03426):
// the smoothed kNN weights of the local fuzzy simplicial sets (Sec. 3.1),
// the a, b fit of the low-dimensional similarity (Sec. 3.2) and the layout
// epochs (Sec. 3.2, SGD with negative sampling).  The fuzzy union itself is
// tsne_umap_fuzzy_union in symmetrize.hip.
//
// Data-parallel epoch: every step of epoch t is evaluated at the positions
// Y_t and the steps are summed, Y_{t+1} = Y_t + sum.  Each step is rounded
// to 64-bit fixed point (2^-32) before it is added, so the sums are exact
// whatever order the atomics take and an epoch is bitwise reproducible.
// The integer decisions are the same on every implementation of this
// reading: the schedule in FP32 (entry e sampled in epoch t when
// floor((t + 1) r_e) > floor(t r_e), r_e = w_e / w_max), the negatives from
// SplitMix64 (Steele, Lea & Flood 2014) on the counter
// (t nnz + e) neg_rate + p, vertex ((z >> 32) n) >> 32.
#include <math.h>

#include "common.hpp"

namespace tsne {

constexpr float UMAP_CLIP = 4.0f;
constexpr float UMAP_EPS = 1e-3f;        // added to the squared distance of a repulsive step
constexpr float UMAP_FX = 4294967296.0f;  // 2^32: fixed-point scale of the summed steps
constexpr int UMAP_MAX_NEG = 64;
constexpr int UMAP_RED_BLOCKS = 256;

// --- smoothed kNN weights ------------------------------------------------------

// One thread per row: d_j = sqrt(d2_j) (FP64 from the FP32 squared
// distances), rho = the smallest positive d_j (0 if none), sigma by FP64
// bisection of sum_j exp(-max(0, d_j - rho) / sigma) = log2(k) on
// [floor, hi] with floor = 1e-3 mean(d) (1e-3 when all d are 0; sigma stays
// there when the floor already meets the target), w_j = exp(-max(0, d_j -
// rho) / sigma).  The sum is monotone in sigma, so the bisection keeps the
// root bracketed; it stops when the midpoint no longer moves.
__device__ double umap_row_sum(const float* __restrict__ d2, int k, double rho, double s) {
  double acc = 0.0;
  for (int j = 0; j < k; ++j) {
    const double x = sqrt(double(d2[j])) - rho;
    acc += exp(-(x > 0.0 ? x : 0.0) / s);
  }
  return acc;
}

__global__ __launch_bounds__(256) void umap_weights_kernel(const float* __restrict__ d2, int64_t n, int k,
                                                           float* __restrict__ rho_out, float* __restrict__ sigma_out,
                                                           float* __restrict__ w) {
  const int64_t i = gtid();
  if (i >= n) return;
  const float* r = d2 + i * k;
  const double target = log2(double(k));
  double rho = 0.0, sum = 0.0, xmax = 0.0;
  bool any = false;
  for (int j = 0; j < k; ++j) {
    const double d = sqrt(double(r[j]));
    sum += d;
    if (d > 0.0 && (!any || d < rho)) {
      rho = d;
      any = true;
    }
  }
  for (int j = 0; j < k; ++j) {
    const double x = sqrt(double(r[j])) - rho;
    xmax = x > xmax ? x : xmax;
  }
  const double mean = sum / k;
  const double floor_s = mean > 0.0 ? 1e-3 * mean : 1e-3;
  double s = floor_s;
  if (umap_row_sum(r, k, rho, floor_s) < target) {
    double lo = floor_s, hi = fmax(2.0 * floor_s, xmax > 0.0 ? xmax : 1.0);
    for (int it = 0; it < 2100 && umap_row_sum(r, k, rho, hi) < target; ++it) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (umap_row_sum(r, k, rho, mid) < target) lo = mid;
      else hi = mid;
    }
    s = 0.5 * (lo + hi);
  }
  rho_out[i] = float(rho);
  sigma_out[i] = float(s);
  for (int j = 0; j < k; ++j) {
    const double x = sqrt(double(r[j])) - rho;
    w[i * k + j] = float(exp(-(x > 0.0 ? x : 0.0) / s));
  }
}

// --- layout ----------------------------------------------------------------------

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float umap_clip(float v) { return fminf(fmaxf(v, -UMAP_CLIP), UMAP_CLIP); }

__device__ __forceinline__ long long umap_fx(float v) { return __float2ll_rn(v * UMAP_FX); }

// Largest stored weight: block maxima, then one block over them (max is
// exact in any order).
__global__ __launch_bounds__(256) void umap_wmax_kernel(const float* __restrict__ val, int64_t nnz,
                                                        float* __restrict__ part) {
  __shared__ float red[256];
  float m = 0.0f;
  for (int64_t e = gtid(); e < nnz; e += int64_t(gridDim.x) * 256) m = fmaxf(m, val[e]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void umap_wmax_final_kernel(float* __restrict__ part, int nb,
                                                              float* __restrict__ wmax) {
  __shared__ float red[256];
  red[threadIdx.x] = int(threadIdx.x) < nb ? part[threadIdx.x] : 0.0f;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *wmax = red[0];
}

// Memory-level parallelism of the epoch kernels: a thread's loads are
// issued in batches (the values and columns of UMAP_EB entries, the y_j of
// the sampled ones, the y_c of up to UMAP_NB negatives) before any of them
// is used, instead of one dependent round trip per load.  The steps are
// summed in 64-bit fixed point, so the order in which a batch is consumed
// does not change a bit of the result.
constexpr int UMAP_EB = 8;  // entries per batch
constexpr int UMAP_NB = 8;  // negatives per batch

// The neg_rate repulsive steps of sampled entry e of row i (counter base
// (t nnz + e) neg_rate), added to (ax, ay).
__device__ __forceinline__ void umap_negatives(const float2* __restrict__ Y, int64_t n, int64_t i, float2 yi,
                                               uint64_t seed, uint64_t base, int neg_rate, float a, float b,
                                               float alpha, long long& ax, long long& ay) {
  const float c2b = 2.0f * b;
  for (int p0 = 0; p0 < neg_rate; p0 += UMAP_NB) {
    int64_t c[UMAP_NB];
    float2 yc[UMAP_NB];
#pragma unroll
    for (int u = 0; u < UMAP_NB; ++u) {
      const int p = p0 + u;
      const uint64_t z = splitmix64(seed, base + uint64_t(p));
      // slots past neg_rate stand on i itself and are skipped like a draw of i
      c[u] = p < neg_rate ? int64_t(((z >> 32) * uint64_t(n)) >> 32) : i;
    }
#pragma unroll
    for (int u = 0; u < UMAP_NB; ++u) yc[u] = Y[c[u]];
#pragma unroll
    for (int u = 0; u < UMAP_NB; ++u) {
      if (c[u] == i) continue;
      const float ex = yi.x - yc[u].x, ey = yi.y - yc[u].y;
      const float q2 = ex * ex + ey * ey;
      if (q2 > 0.0f) {
        const float cr = c2b / ((UMAP_EPS + q2) * (1.0f + a * powf(q2, b)));
        ax += umap_fx(alpha * umap_clip(cr * ex));
        ay += umap_fx(alpha * umap_clip(cr * ey));
      }
    }
  }
}

// Epoch t, one thread per row i of the CSR graph: for every entry (i, j)
// sampled in this epoch, the attractive step alpha clip(c_a (y_i - y_j))
// added to y_i and, with SCATTER, subtracted from y_j (64-bit integer
// atomics into D), else added to y_i a second time (a symmetric graph, see
// umap_epoch_sym_kernel); then neg_rate repulsive steps alpha clip(c_r (y_i
// - y_c)) added to y_i; c_a = -2ab d2^(b-1) / (1 + a d2^b), c_r = 2b / ((eps
// + d2)(1 + a d2^b)), no step at d2 = 0 or for a draw c = i.  Steps into y_i
// are summed in registers (fixed point): returned in (ax, ay).
template <bool SCATTER>
__device__ __forceinline__ void umap_row_epoch(const float2* __restrict__ Y, int64_t n, int64_t i, float2 yi,
                                               const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                               const float* __restrict__ val, int64_t nnz, float rmax, float a,
                                               float b, float alpha, int neg_rate, uint64_t seed, int t,
                                               unsigned long long* __restrict__ D, long long& ax, long long& ay) {
  const float t0 = float(t), t1 = float(t + 1);
  const float cab = -2.0f * a * b;
  const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
  for (int64_t eb = e0; eb < e1; eb += UMAP_EB) {
    float v[UMAP_EB];
    int32_t cj[UMAP_EB];
#pragma unroll
    for (int u = 0; u < UMAP_EB; ++u) {
      const int64_t e = eb + u;
      v[u] = e < e1 ? val[e] : 0.0f;  // (0: never sampled)
      cj[u] = e < e1 ? col[e] : int32_t(i);
    }
    bool smp[UMAP_EB];
    float2 yj[UMAP_EB];
#pragma unroll
    for (int u = 0; u < UMAP_EB; ++u) {
      const float r = __fdiv_rn(v[u], rmax);  // correctly rounded, as the schedule requires
      smp[u] = eb + u < e1 && floorf(t1 * r) > floorf(t0 * r);
      yj[u] = Y[smp[u] ? int64_t(cj[u]) : i];
    }
    // all eight gathers in flight before the first is used (else the
    // compiler sinks each into its sampled branch, one round trip each)
#pragma unroll
    for (int u = 0; u < UMAP_EB; ++u) asm volatile("" : "+v"(yj[u].x), "+v"(yj[u].y));
#pragma unroll
    for (int u = 0; u < UMAP_EB; ++u) {
      if (!smp[u]) continue;
      const float dx = yi.x - yj[u].x, dy = yi.y - yj[u].y;
      const float d2 = dx * dx + dy * dy;
      if (d2 > 0.0f) {
        const float pb = powf(d2, b);
        const float c = cab * (pb / d2) / (1.0f + a * pb);
        const long long fx = umap_fx(alpha * umap_clip(c * dx)), fy = umap_fx(alpha * umap_clip(c * dy));
        if (SCATTER) {
          ax += fx;
          ay += fy;
          atomicAdd(&D[2 * int64_t(cj[u])], static_cast<unsigned long long>(-fx));
          atomicAdd(&D[2 * int64_t(cj[u]) + 1], static_cast<unsigned long long>(-fy));
        } else {
          ax += 2 * fx;
          ay += 2 * fy;
        }
      }
      const uint64_t base = (uint64_t(t) * uint64_t(nnz) + uint64_t(eb + u)) * uint64_t(neg_rate);
      umap_negatives(Y, n, i, yi, seed, base, neg_rate, a, b, alpha, ax, ay);
    }
  }
}

// Epoch t on any graph: steps into y_j go straight to D with 64-bit
// integer atomics, y_i's own sum is added once.
__global__ __launch_bounds__(256) void umap_epoch_kernel(const float2* __restrict__ Y, int64_t n,
                                                         const int64_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col,
                                                         const float* __restrict__ val, int64_t nnz,
                                                         const float* __restrict__ wmax, float a, float b,
                                                         float alpha, int neg_rate, uint64_t seed, int t,
                                                         unsigned long long* __restrict__ D) {
  const int64_t i = gtid();
  if (i >= n) return;
  long long ax = 0, ay = 0;
  umap_row_epoch<true>(Y, n, i, Y[i], row_ptr, col, val, nnz, *wmax, a, b, alpha, neg_rate, seed, t, D, ax, ay);
  if (ax) atomicAdd(&D[2 * i], static_cast<unsigned long long>(ax));
  if (ay) atomicAdd(&D[2 * i + 1], static_cast<unsigned long long>(ay));
}

// Y_{t+1} = Y_t + D 2^-32 (FP32), D cleared for the next epoch.
__global__ __launch_bounds__(256) void umap_apply_kernel(float2* __restrict__ Y, int64_t n,
                                                         unsigned long long* __restrict__ D) {
  const int64_t i = gtid();
  if (i >= n) return;
  const long long dx = static_cast<long long>(D[2 * i]), dy = static_cast<long long>(D[2 * i + 1]);
  float2 y = Y[i];
  y.x += float(double(dx) * (1.0 / 4294967296.0));
  y.y += float(double(dy) * (1.0 / 4294967296.0));
  Y[i] = y;
  D[2 * i] = 0ull;
  D[2 * i + 1] = 0ull;
}

// Epoch t on a symmetric graph (pattern and values, as the fuzzy union
// writes them): entries (i, j) and (j, i) hold the same FP32 value, so they
// are sampled in the same epochs, and the step that entry (j, i) applies to
// y_i is bitwise equal to y_i's own step for (i, j) (the squared distance
// is the same, c_a is symmetric, and clip is odd).  Each vertex therefore
// takes twice its own attractive steps plus its negatives, and nothing is
// scattered: one thread per row reads Y_in and writes Y_out, with the same
// fixed-point sums -- the result equals the scattering path's bit for bit.
__global__ __launch_bounds__(256) void umap_epoch_sym_kernel(const float2* __restrict__ Yin,
                                                             float2* __restrict__ Yout, int64_t n,
                                                             const int64_t* __restrict__ row_ptr,
                                                             const int32_t* __restrict__ col,
                                                             const float* __restrict__ val, int64_t nnz,
                                                             const float* __restrict__ wmax, float a, float b,
                                                             float alpha, int neg_rate, uint64_t seed, int t) {
  const int64_t i = gtid();
  if (i >= n) return;
  const float2 yi = Yin[i];
  long long ax = 0, ay = 0;
  umap_row_epoch<false>(Yin, n, i, yi, row_ptr, col, val, nnz, *wmax, a, b, alpha, neg_rate, seed, t, nullptr, ax,
                        ay);
  float2 y = yi;
  y.x += float(double(ax) * (1.0 / 4294967296.0));
  y.y += float(double(ay) * (1.0 / 4294967296.0));
  Yout[i] = y;
}

__global__ __launch_bounds__(256) void umap_copy_kernel(const float2* __restrict__ src, float2* __restrict__ dst,
                                                        int64_t n) {
  const int64_t i = gtid();
  if (i < n) dst[i] = src[i];
}

struct UmapLayout {
  size_t o_part, o_wmax, o_D, o_Y, bytes;
  static UmapLayout make(int64_t n) {
    UmapLayout L;
    Carve c;
    L.o_part = c.take(sizeof(float) * UMAP_RED_BLOCKS);
    L.o_wmax = c.take(sizeof(float));
    L.o_D = c.take(sizeof(unsigned long long) * 2 * size_t(n));
    L.o_Y = c.take(sizeof(float2) * size_t(n));
    L.bytes = c.off;
    return L;
  }
};

// --- a, b of Phi(d) = 1 / (1 + a d^2b): least squares against Psi ------------------

// Levenberg-Marquardt (Marquardt's diagonal scaling) from (1, 1) over the 300
// points d = 3 m / 299; a step is taken only if it lowers the sum of squares
// and keeps a > 0.
struct FitAB {
  double x[300], y[300];
  explicit FitAB(double min_dist) {
    for (int m = 0; m < 300; ++m) {
      x[m] = 3.0 * m / 299.0;
      y[m] = x[m] <= min_dist ? 1.0 : exp(-(x[m] - min_dist));
    }
  }
  double cost(double a, double b) const {
    double s = 0.0;
    for (int m = 0; m < 300; ++m) {
      const double r = 1.0 / (1.0 + a * pow(x[m], 2.0 * b)) - y[m];
      s += r * r;
    }
    return s;
  }
};

}  // namespace tsne

extern "C" int tsne_umap_fit_ab(double min_dist, double* a_out, double* b_out) {
  using namespace tsne;
  if (!a_out || !b_out || !(min_dist >= 0.0) || !(min_dist < 3.0)) return TSNE_ERR_INVALID_ARG;
  const FitAB F(min_dist);
  double a = 1.0, b = 1.0, lam = 1e-3, c0 = F.cost(a, b);
  for (int it = 0; it < 2000 && lam < 1e20; ++it) {
    double h00 = 0.0, h01 = 0.0, h11 = 0.0, g0 = 0.0, g1 = 0.0;
    for (int m = 0; m < 300; ++m) {
      const double xm = F.x[m];
      const double p = xm > 0.0 ? pow(xm, 2.0 * b) : 0.0;
      const double phi = 1.0 / (1.0 + a * p);
      const double r = phi - F.y[m];
      const double ja = -p * phi * phi;
      const double jb = xm > 0.0 ? -a * p * 2.0 * log(xm) * phi * phi : 0.0;
      h00 += ja * ja;
      h01 += ja * jb;
      h11 += jb * jb;
      g0 += ja * r;
      g1 += jb * r;
    }
    const double m00 = h00 * (1.0 + lam), m11 = h11 * (1.0 + lam);
    const double det = m00 * m11 - h01 * h01;
    if (!(det > 0.0)) {
      lam *= 10.0;
      continue;
    }
    const double da = -(m11 * g0 - h01 * g1) / det, db = -(m00 * g1 - h01 * g0) / det;
    const double an = a + da, bn = b + db;
    const double c1 = an > 0.0 ? F.cost(an, bn) : INFINITY;
    if (c1 < c0) {
      const bool tiny = fabs(da) <= 1e-15 * fabs(a) && fabs(db) <= 1e-15 * fabs(b);
      a = an;
      b = bn;
      c0 = c1;
      lam = fmax(lam * 0.1, 1e-12);
      if (tiny) break;
    } else {
      lam *= 10.0;
    }
  }
  *a_out = a;
  *b_out = b;
  return TSNE_OK;
}

extern "C" int tsne_umap_weights(const float* nbr_d2, int64_t n, int32_t k, float* rho, float* sigma, float* w,
                                 void* stream) {
  using namespace tsne;
  if (!nbr_d2 || !rho || !sigma || !w || n < 1 || k < 1) return TSNE_ERR_INVALID_ARG;
  if (k > TSNE_MAX_K) return TSNE_ERR_UNSUPPORTED;
  TSNE_REQUIRE_GFX950();
  hipLaunchKernelGGL(umap_weights_kernel, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, as_stream(stream), nbr_d2,
                     n, k, rho, sigma, w);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

extern "C" int tsne_umap_layout(float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                                int64_t nnz, int32_t symmetric, double a, double b, double alpha0, int32_t neg_rate,
                                int32_t n_epochs, int32_t epoch_begin, int32_t epoch_end, uint64_t seed,
                                void* workspace, size_t* workspace_bytes, void* stream) {
  using namespace tsne;
  if (!Y || !row_ptr || !col || !val || n < 2 || nnz < 1) return TSNE_ERR_INVALID_ARG;
  if (!(a > 0.0) || !(b > 0.0) || !(alpha0 >= 0.0) || neg_rate < 0 || neg_rate > UMAP_MAX_NEG) return TSNE_ERR_INVALID_ARG;
  if (n_epochs < 1 || epoch_begin < 0 || epoch_begin > epoch_end || epoch_end > n_epochs) return TSNE_ERR_INVALID_ARG;
  if (symmetric != 0 && symmetric != 1) return TSNE_ERR_INVALID_ARG;
  if (n >= (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  const UmapLayout L = UmapLayout::make(n);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  char* ws = static_cast<char*>(workspace);
  float* part = reinterpret_cast<float*>(ws + L.o_part);
  float* wmax = reinterpret_cast<float*>(ws + L.o_wmax);
  unsigned long long* D = reinterpret_cast<unsigned long long*>(ws + L.o_D);
  float2* Yb = reinterpret_cast<float2*>(ws + L.o_Y);
  hipStream_t s = as_stream(stream);
  if (!symmetric && (rc = launch_fill<unsigned long long>(D, 2 * n, 0ull, s))) return rc;
  const int64_t nbk = ceil_div(nnz, 256);
  const int nb = int(nbk < UMAP_RED_BLOCKS ? nbk : UMAP_RED_BLOCKS);
  hipLaunchKernelGGL(umap_wmax_kernel, dim3(unsigned(nb)), dim3(256), 0, s, val, nnz, part);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(umap_wmax_final_kernel, dim3(1), dim3(256), 0, s, part, nb, wmax);
  TSNE_CHECK_LAUNCH();
  const dim3 grid(unsigned(ceil_div(n, 256)));
  float2* Y2 = reinterpret_cast<float2*>(Y);
  float2* cur = Y2;
  float2* nxt = Yb;
  for (int t = epoch_begin; t < epoch_end; ++t) {
    const float alpha = float(alpha0 * (1.0 - double(t) / double(n_epochs)));
    if (symmetric) {
      hipLaunchKernelGGL(umap_epoch_sym_kernel, grid, dim3(256), 0, s, cur, nxt, n, row_ptr, col, val, nnz, wmax,
                         float(a), float(b), alpha, int(neg_rate), seed, int(t));
      TSNE_CHECK_LAUNCH();
      float2* tmp = cur;
      cur = nxt;
      nxt = tmp;
    } else {
      hipLaunchKernelGGL(umap_epoch_kernel, grid, dim3(256), 0, s, Y2, n, row_ptr, col, val, nnz, wmax, float(a),
                         float(b), alpha, int(neg_rate), seed, int(t), D);
      TSNE_CHECK_LAUNCH();
      hipLaunchKernelGGL(umap_apply_kernel, grid, dim3(256), 0, s, Y2, n, D);
      TSNE_CHECK_LAUNCH();
    }
  }
  if (cur != Y2) {
    hipLaunchKernelGGL(umap_copy_kernel, grid, dim3(256), 0, s, cur, Y2, n);
    TSNE_CHECK_LAUNCH();
  }
  return TSNE_OK;
}
