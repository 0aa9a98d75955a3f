// Internal launch helpers shared by tsne_kl_grad and tsne_optimize.
#pragma once

#include "common.hpp"
#include "rep_sym.hpp"

namespace tsne {

// Momentum + adaptive-gains update of one coordinate (van der Maaten &
// Hinton 2008, Algorithm 1; Jacobs 1988 gains): the gain grows by `inc` when
// the gradient and the previous update have opposite signs, else shrinks by
// the factor `dec`, floored at `mn`.
__device__ __forceinline__ void step_coord(float& y, float& u, float& gain, float g, float lr, float mom, float inc,
                                           float dec, float mn) {
  float ng = (g * u < 0.0f) ? gain + inc : gain * dec;
  ng = fmaxf(ng, mn);
  u = mom * u - lr * ng * g;
  y = y + u;
  gain = ng;
}

// Optimiser step applied by the gradient's finalize pass: reads y_i from the
// gradient's input Y and writes the stepped point to Yout (a different
// buffer, since other rows still gather y_i in the same pass).
struct FusedStep {
  float2* Yout;
  float2* U;
  float2* G;
  float lr, mom, inc, dec, mn;
};

struct KlGradPlan {
  SymGrid g;
  int64_t nfin;
  bool zrow;  // o_Zr is valid (the per-row Z partials have room)
  size_t o_R, o_Zr, o_Zb, o_kl, o_A, o_g, bytes;  // o_A, o_g: attraction partials, scratch gradient (with_att)
};

// Workspace layout of one gradient evaluation for n points; with_att adds
// the attraction partials of the fused path (AttList), with_zrow the
// per-row Z partials (needed only when Zrow is requested).
KlGradPlan klgrad_plan(int64_t n, bool with_att = false, bool with_zrow = true);

// Workspace layout and build of the job-grouped attraction list of a CSR P
// with nnz stored entries (unordered pairs i < j; see AttList).
struct AttPlan {
  size_t o_cnt, o_cur, o_off, o_bsum, o_ij, o_p, bytes;
};
AttPlan att_plan(const SymGrid& g, int64_t nnz);
int att_build(const AttPlan& A, const SymGrid& g, char* ws, int64_t n, const int64_t* row_ptr, const int32_t* col,
              const float* val, AttList* out, hipStream_t s);

// Enqueue one gradient evaluation (arguments as tsne_kl_grad, validated).
// With `step`, the finalize pass applies the optimiser step to every row
// instead of writing the gradient (grad may then be null).  after_repulsion
// (nullable) is recorded on s between the all-pairs pass and the finalize.
// Zrow needs a plan made with_zrow.  With `att` (plan made with_att; Zrow
// not requested) the attraction is
// summed inside the all-pairs kernel from the job-grouped list; a requested
// KL then comes from an extra CSR pass at the same Y.
// nonfinite (nullable): device counter that receives += the number of
// non-finite coordinates of Y (with `step`: of the stepped positions).
int klgrad_launch(const KlGradPlan& L, char* ws, const float* Y, int64_t n, const int64_t* row_ptr,
                  const int32_t* col, const float* val, float alpha, float* grad, double* Z, double* kl, double* Zrow,
                  hipStream_t s, const FusedStep* step = nullptr, hipEvent_t after_repulsion = nullptr,
                  const AttList* att = nullptr, unsigned long long* nonfinite = nullptr);

// Finalize of a gradient whose repulsion R (one float2 per point) and Z
// block partials (Z = their sum, in index order) were computed elsewhere:
// attraction over the CSR rows, g = 4 (alpha A - R / Z), optional Z and KL
// outputs.  klpart: finalize_kl_bytes(n) of workspace (used when kl).
// rows (nullable): a permutation of the rows, the order the blocks take them
// in (a row's result does not depend on it; the KL's per-block sums do, so
// pass none when kl is requested and the order is not reproducible).
size_t finalize_kl_bytes(int64_t n);
int finalize_csr_launch(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                        float alpha, const float* R, const double* Zblock, int64_t nZ, float* grad, double* Z,
                        double* kl, double* klpart, unsigned long long* nonfinite, hipStream_t s,
                        const int32_t* rows = nullptr);

// Enqueue one optimiser step (arguments as tsne_step, validated).
int step_launch(float* Y, float* update, float* gains, const float* grad, int64_t n, float lr, float momentum,
                float gain_inc, float gain_dec, float min_gain, hipStream_t s);

}  // namespace tsne
