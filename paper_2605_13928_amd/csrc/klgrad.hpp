// Internal launch helpers shared by tsne_kl_grad and tsne_optimize.
#pragma once

#include "common.hpp"
#include "rep_sym.hpp"

namespace tsne {

struct KlGradPlan {
  SymGrid g;
  int64_t nfin;
  size_t o_R, o_Zr, o_Zb, o_kl, bytes;
};

// Workspace layout of one gradient evaluation for n points.
KlGradPlan klgrad_plan(int64_t n);

// Enqueue one gradient evaluation (arguments as tsne_kl_grad, validated).
int klgrad_launch(const KlGradPlan& L, char* ws, const float* Y, int64_t n, const int64_t* row_ptr,
                  const int32_t* col, const float* val, float alpha, float* grad, double* Z, double* kl, double* Zrow,
                  hipStream_t s);

// Enqueue one optimiser step (arguments as tsne_step, validated).
int step_launch(float* Y, float* update, float* gains, const float* grad, int64_t n, float lr, float momentum,
                float gain_inc, float gain_dec, float min_gain, hipStream_t s);

}  // namespace tsne
