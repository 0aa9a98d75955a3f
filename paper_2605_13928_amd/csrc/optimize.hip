// tsne_optimize: a run of optimiser iterations enqueued from native code --
// per iteration one gradient evaluation (tsne_kl_grad's kernels) and one
// step (tsne_step's kernel), with the schedule of van der Maaten & Hinton
// 2008 (Sec. 3.4, Algorithm 1): early exaggeration and the lower momentum
// while t < exaggeration_iters.  The step is applied by the gradient's
// finalize pass (one launch fewer per iteration); the embedding ping-pongs
// between Y and a workspace copy, because that pass still reads the old
// positions of other rows while it writes new ones.  The attraction is
// summed inside the all-pairs kernel from a job-grouped copy of P's upper
// triangle, built once per call (no per-iteration gathers of y_j); on the
// iterations that log the KL an extra CSR pass at the same Y adds the KL
// sums without changing the trajectory.
#include "common.hpp"
#include "klgrad.hpp"

extern "C" int tsne_optimize(float* Y, float* update, float* gains, int64_t n, const int64_t* row_ptr,
                             const int32_t* col, const float* val, int64_t nnz, int32_t t_begin, int32_t t_end,
                             const tsne_schedule* schedule, int32_t log_every, double* kl_log, void* const* events,
                             int64_t* nonfinite, void* workspace, size_t* workspace_bytes, void* stream) {
  using namespace tsne;
  if (!Y || !update || !gains || !row_ptr || !col || !val || !schedule || n < 2 || nnz < 0) return TSNE_ERR_INVALID_ARG;
  if (t_begin < 0 || t_end < t_begin || log_every < 0) return TSNE_ERR_INVALID_ARG;
  const tsne_schedule sc = *schedule;
  if (!(sc.exaggeration > 0.0f) || !(sc.exaggeration < INFINITY) || !(sc.lr > 0.0f)) return TSNE_ERR_INVALID_ARG;
  if (n > (int64_t(1) << 31)) return TSNE_ERR_UNSUPPORTED;
  const KlGradPlan L = klgrad_plan(n, true, false);  // Zrow is never requested here
  const AttPlan A = att_plan(L.g, nnz);
  Carve c;
  const size_t o_kg = c.take(L.bytes);
  const size_t o_y = c.take(sizeof(float) * 2 * size_t(n));
  const size_t o_att = c.take(A.bytes);
  int rc = workspace_protocol(workspace, workspace_bytes, c.off);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  char* ws = static_cast<char*>(workspace);
  float* ycur = Y;
  float* ynext = reinterpret_cast<float*>(ws + o_y);
  hipStream_t s = as_stream(stream);
  unsigned long long* nf = reinterpret_cast<unsigned long long*>(nonfinite);
  if (nf && (rc = launch_fill<unsigned long long>(nf, 1, 0ull, s))) return rc;
  AttList att;
  if (t_end > t_begin && (rc = att_build(A, L.g, ws + o_att, n, row_ptr, col, val, &att, s))) return rc;
  for (int32_t t = t_begin; t < t_end; ++t) {
    const bool early = t < sc.exaggeration_iters;
    const float alpha = early ? sc.exaggeration : 1.0f;
    const float mom = early ? sc.momentum_early : sc.momentum_late;
    const bool log = kl_log && log_every > 0 && (t + 1) % log_every == 0;
    const int64_t slot = int64_t(t - t_begin);
    if (events && events[2 * slot]) {
      const hipError_t e = hipEventRecord(static_cast<hipEvent_t>(events[2 * slot]), s);
      if (e != hipSuccess) { set_last_hip_error(e); return TSNE_ERR_HIP; }
    }
    const FusedStep st{reinterpret_cast<float2*>(ynext), reinterpret_cast<float2*>(update),
                       reinterpret_cast<float2*>(gains), sc.lr, mom, sc.gain_inc, sc.gain_dec, sc.min_gain};
    rc = klgrad_launch(L, ws + o_kg, ycur, n, row_ptr, col, val, alpha, nullptr, nullptr,
                       log ? kl_log + slot : nullptr, nullptr, s, &st,
                       events ? static_cast<hipEvent_t>(events[2 * slot + 1]) : nullptr, &att, nf);
    if (rc) return rc;
    float* tmp = ycur;
    ycur = ynext;
    ynext = tmp;
  }
  if (ycur != Y) {
    const hipError_t e = hipMemcpyAsync(Y, ycur, sizeof(float) * 2 * size_t(n), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) { set_last_hip_error(e); return TSNE_ERR_HIP; }
  }
  return TSNE_OK;
}
