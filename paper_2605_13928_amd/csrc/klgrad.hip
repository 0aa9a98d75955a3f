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

namespace tsne {

// Finalize, 16 rows per block.  All loads that depend on nothing are
// issued first (CSR bounds, the first repulsion partials, the Z partials,
// the stepped rows' state), so the block's critical path is the three
// dependent trips of the attraction gather (row_ptr -> col, val -> y_j).
// Repulsion partials: thread (g, sl) adds slices g, g + 16, ... of row
// r0 + sl in FP64; the 16 slice sums are combined in a fixed order.
// Attraction A_i = sum_{e in row i} p_e w_e (y_i - y_j): lane group g owns
// row r0 + g, 16 lanes, eight entries per lane in flight, reduced by DPP
// row rotations; optional per-block sums of p ln p, p ln q (q = 1/w) and p
// for the KL.  Then g_i = 4 (alpha A_i - R_i / Z).  STEP: instead of
// storing g, apply the optimiser step to the row (FusedStep).
constexpr int FIN_ROWS = 16;
constexpr int FIN_PRE = 8;  // partial slices per thread loaded up front

template <bool STEP>
__global__ __launch_bounds__(256) void finalize_tsne_kernel(
    const float2* __restrict__ Y, int64_t n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const float* __restrict__ val, float alpha, const float2* __restrict__ Rpart, const float* __restrict__ Zrowpart,
    int64_t ns, const double* __restrict__ Zblock, int64_t nZ, float2* __restrict__ grad, double* __restrict__ Zrow,
    double* __restrict__ Z_out, double* __restrict__ klpart, FusedStep st) {
  __shared__ double red[4];
  __shared__ double pr[16][FIN_ROWS][3];
  __shared__ float2 att[FIN_ROWS];
  const int tid = threadIdx.x;
  const int g = tid >> 4, sl = tid & 15;
  const int64_t r0 = int64_t(blockIdx.x) * FIN_ROWS;
  const int64_t row = r0 + g;    // attraction row of lane group g
  const int64_t prow = r0 + sl;  // partial-sum row of this thread

  // --- loads with no dependences -----------------------------------------
  int64_t e0 = 0, e1 = 0;
  float2 yi = make_float2(0.0f, 0.0f);
  if (row < n) {
    e0 = row_ptr[row];
    e1 = row_ptr[row + 1];
    yi = Y[row];
  }
  float2 rp[FIN_PRE];
#pragma unroll
  for (int u = 0; u < FIN_PRE; ++u) {
    const int64_t k = g + 16 * u;
    rp[u] = (prow < n && k < ns) ? Rpart[k * n + prow] : make_float2(0.0f, 0.0f);
  }
  const double zt = zblock_thread_sum(Zblock, nZ);
  float2 sy = make_float2(0.0f, 0.0f), su = sy, sg = sy;
  if (STEP && tid < FIN_ROWS && r0 + tid < n) {
    sy = Y[r0 + tid];
    su = st.U[r0 + tid];
    sg = st.G[r0 + tid];
  }

  // --- attraction --------------------------------------------------------
  float ax = 0.0f, ay = 0.0f, plp = 0.0f, plq = 0.0f, ps = 0.0f;
  for (int64_t e = e0 + sl; e < e1; e += 128) {
    int32_t jj[8];
    float pp[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t ee = e + 16 * u;
      const bool ok = ee < e1;
      jj[u] = ok ? col[ee] : int32_t(row);
      pp[u] = ok ? val[ee] : 0.0f;
    }
    float2 yj[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) yj[u] = Y[jj[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float dx = yi.x - yj[u].x, dy = yi.y - yj[u].y;
      const float q = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1.0f));
      const float pw = pp[u] * __builtin_amdgcn_rcpf(q);
      ax = __builtin_fmaf(pw, dx, ax);
      ay = __builtin_fmaf(pw, dy, ay);
      if (klpart) {
        if (pp[u] > 0.0f) plp += pp[u] * logf(pp[u]);
        plq += pp[u] * logf(q);
        ps += pp[u];
      }
    }
  }

  // --- repulsion partials: slices g, g + 16, ... in order ------------------
  {
    double rx = 0.0, ry = 0.0, zr = 0.0;
#pragma unroll
    for (int u = 0; u < FIN_PRE; ++u) {
      rx += double(rp[u].x);
      ry += double(rp[u].y);
    }
    if (prow < n) {
      int64_t k = g + 16 * FIN_PRE;
      for (; k + 48 < ns; k += 64) {
        float2 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = Rpart[(k + 16 * u) * n + prow];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          rx += double(r[u].x);
          ry += double(r[u].y);
        }
      }
      for (; k < ns; k += 16) {
        const float2 r = Rpart[k * n + prow];
        rx += double(r.x);
        ry += double(r.y);
      }
      if (Zrow)
        for (int64_t kk = g; kk < ns; kk += 16) zr += double(Zrowpart[kk * n + prow]);
    }
    pr[g][sl][0] = rx;
    pr[g][sl][1] = ry;
    pr[g][sl][2] = zr;
  }
  ax = row16_sum(ax);
  ay = row16_sum(ay);
  if (sl == 0) att[g] = make_float2(ax, ay);
  const double Z = block_sum_d(zt, red);  // its barriers also publish pr and att
  if (blockIdx.x == 0 && tid == 0 && Z_out) *Z_out = Z;
  if (tid < FIN_ROWS && r0 + tid < n) {
    double Rx = 0.0, Ry = 0.0, Zr = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      Rx += pr[k][tid][0];
      Ry += pr[k][tid][1];
      Zr += pr[k][tid][2];
    }
    const float2 a = att[tid];
    const float2 gi = make_float2(float(4.0 * (double(alpha) * double(a.x) - Rx / Z)),
                                  float(4.0 * (double(alpha) * double(a.y) - Ry / Z)));
    const int64_t i = r0 + tid;
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
  if (klpart) {
    plp = row16_sum(plp);
    plq = row16_sum(plq);
    ps = row16_sum(ps);
    const bool own = row < n && sl == 0;
    const double a = block_sum_d(own ? double(plp) : 0.0, red);
    const double b = block_sum_d(own ? double(plq) : 0.0, red);
    const double c = block_sum_d(own ? double(ps) : 0.0, red);
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

KlGradPlan klgrad_plan(int64_t n) {
  KlGradPlan L;
  L.g = SymGrid::make(n);
  L.nfin = ceil_div(n, FIN_ROWS);
  Carve c;
  L.o_R = c.take(sizeof(float2) * size_t(L.g.ns) * size_t(n));
  L.o_Zr = c.take(sizeof(float) * size_t(L.g.ns) * size_t(n));
  L.o_Zb = c.take(sizeof(double) * size_t(L.g.nwg));
  L.o_kl = c.take(sizeof(double) * 3 * size_t(L.nfin));
  L.bytes = c.off;
  return L;
}

int klgrad_launch(const KlGradPlan& L, char* ws, const float* Y, int64_t n, const int64_t* row_ptr,
                  const int32_t* col, const float* val, float alpha, float* grad, double* Z, double* kl, double* Zrow,
                  hipStream_t s, const FusedStep* step, hipEvent_t after_repulsion) {
  const SymGrid& g = L.g;
  float* Rpart = reinterpret_cast<float*>(ws + L.o_R);
  float* Zrowpart = Zrow ? reinterpret_cast<float*>(ws + L.o_Zr) : nullptr;
  double* Zblock = reinterpret_cast<double*>(ws + L.o_Zb);
  double* klpart = kl ? reinterpret_cast<double*>(ws + L.o_kl) : nullptr;
  const float2* Y2 = reinterpret_cast<const float2*>(Y);
  const size_t lds = rep_sym_lds_bytes(g.S, Zrow != nullptr);
  const dim3 grid(unsigned(g.nwg)), block(256);
#define TSNE_REP_SYM(Z, PF) \
  hipLaunchKernelGGL((rep_sym_kernel<Z, PF>), grid, block, lds, s, Y2, n, g.ns, Rpart, Zrowpart, Zblock)
  if (Zrow) {
    if (g.S == 256) TSNE_REP_SYM(true, 1);
    else if (g.S == 512) TSNE_REP_SYM(true, 2);
    else TSNE_REP_SYM(true, 4);
  } else {
    if (g.S == 256) TSNE_REP_SYM(false, 1);
    else if (g.S == 512) TSNE_REP_SYM(false, 2);
    else TSNE_REP_SYM(false, 4);
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
  if (step)
    hipLaunchKernelGGL(finalize_tsne_kernel<true>, dim3(unsigned(L.nfin)), dim3(256), 0, s, Y2, n, row_ptr, col, val,
                       alpha, reinterpret_cast<const float2*>(Rpart), Zrowpart, g.ns, Zblock, g.nwg, nullptr, Zrow, Z,
                       klpart, *step);
  else
    hipLaunchKernelGGL(finalize_tsne_kernel<false>, dim3(unsigned(L.nfin)), dim3(256), 0, s, Y2, n, row_ptr, col,
                       val, alpha, reinterpret_cast<const float2*>(Rpart), Zrowpart, g.ns, Zblock, g.nwg,
                       reinterpret_cast<float2*>(grad), Zrow, Z, klpart, FusedStep{});
  TSNE_CHECK_LAUNCH();
  if (kl) {
    hipLaunchKernelGGL(kl_reduce_kernel, dim3(1), dim3(256), 0, s, klpart, L.nfin, Zblock, g.nwg, kl);
    TSNE_CHECK_LAUNCH();
  }
  return TSNE_OK;
}

}  // namespace tsne

extern "C" int tsne_kl_grad(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                            float exaggeration, float* grad, double* Z, double* kl, double* Zrow, void* workspace,
                            size_t* workspace_bytes, void* stream) {
  using namespace tsne;
  if (!Y || !row_ptr || !col || !val || !grad || n < 2) return TSNE_ERR_INVALID_ARG;
  if (!(exaggeration > 0.0f) || !(exaggeration < INFINITY)) return TSNE_ERR_INVALID_ARG;
  if (n > (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  const KlGradPlan L = klgrad_plan(n);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  return klgrad_launch(L, static_cast<char*>(workspace), Y, n, row_ptr, col, val, exaggeration, grad, Z, kl, Zrow,
                       as_stream(stream));
}
