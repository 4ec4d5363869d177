// Launch-shape table and its autotuner.  The table holds only launch
// shapes (tile rows, block sizes, grid caps, PCG replay lengths): every
// kernel computes the same values, and lists pairs in the same order, for
// any entry, so tuning changes times, never results.
#include <chrono>
#include <cmath>
#include <initializer_list>
#include <vector>

#include "abd_internal.h"

namespace {

bool one_of(int v, std::initializer_list<int> set) {
  for (int s : set)
    if (v == s) return true;
  return false;
}

bool tune_valid(const abd_tune &t) {
  return one_of(t.tile_rows, {8, 16, 32, 64}) && one_of(t.barrier_waves, {1, 2, 4}) &&
         one_of(t.ccd_block, {64, 128, 256}) && t.ccd_max_blocks >= 64 && t.ccd_max_blocks <= 16384 &&
         one_of(t.energy_block, {64, 128, 256, 512, 1024}) && t.pcg_short >= 2 && t.pcg_short % 2 == 0 &&
         t.pcg_long >= t.pcg_short && t.pcg_long % 2 == 0 && t.pcg_long <= 256 && one_of(t.cull_levels, {1, 3});
}

}  // namespace

extern "C" int abd_tune_get(const abd_ctx *ctx, abd_tune *out) {
  if (!ctx || !out) return ABD_E_INVALID;
  *out = ctx->tune;
  return ABD_OK;
}

extern "C" int abd_tune_set(abd_ctx *ctx, const abd_tune *in) {
  if (!ctx || !in) return abd_fail(ctx, ABD_E_INVALID, "abd_tune_set: null");
  if (!tune_valid(*in)) return abd_fail(ctx, ABD_E_INVALID, "abd_tune_set: a value outside its set");
  ctx->tune = *in;
  return ABD_OK;
}

extern "C" int abd_autotune(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, double *q, double *qdot,
                            int n_steps, int reps, abd_tune *out, double *best_ms_per_step, hipStream_t s) {
  if (!ctx || !sc || !prm || !q || !qdot || !out || n_steps < 1 || reps < 1)
    return abd_fail(ctx, ABD_E_INVALID, "abd_autotune: null or non-positive count");
  const size_t n12 = 12 * (size_t)sc->n_bodies;
  double *q_keep, *qd_keep;
  ABD_TRY(ws(ctx, "tune_q", n12, &q_keep, s));
  ABD_TRY(ws(ctx, "tune_qd", n12, &qd_keep, s));
  HIP_TRY(ctx, hipMemcpyAsync(q_keep, q, n12 * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(qd_keep, qdot, n12 * sizeof(double), hipMemcpyDeviceToDevice, s));
  auto restore = [&]() -> int {
    HIP_TRY(ctx, hipMemcpyAsync(q, q_keep, n12 * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(qdot, qd_keep, n12 * sizeof(double), hipMemcpyDeviceToDevice, s));
    return ABD_OK;
  };
  // wall time per step of n_steps steps from the start state, best of reps
  auto measure = [&](double *ms) -> int {
    double best = INFINITY;
    for (int r = 0; r < reps; ++r) {
      ABD_TRY(restore());
      HIP_TRY(ctx, hipStreamSynchronize(s));
      const auto t0 = std::chrono::steady_clock::now();
      for (int i = 0; i < n_steps; ++i) ABD_TRY(abd_time_step(ctx, sc, prm, q, qdot, nullptr, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      best = t < best ? t : best;
    }
    *ms = best / n_steps;
    return ABD_OK;
  };
  // candidate values per entry (the struct's order)
  const std::vector<std::vector<int>> cand = {
      {8, 16, 32, 64}, {1, 2, 4}, {64, 128, 256}, {256, 512, 1024, 2048, 4096}, {128, 256, 512}, {2, 4, 8, 16, 32},
      {1, 3}};
  abd_tune cur = ctx->tune;
  double best = 0.0;
  int rc = measure(&best);
  for (size_t e = 0; rc == ABD_OK && e < cand.size(); ++e) {
    for (int v : cand[e]) {
      abd_tune t = cur;
      int32_t *f[7] = {&t.tile_rows, &t.barrier_waves, &t.ccd_block, &t.ccd_max_blocks, &t.energy_block,
                       &t.pcg_short, &t.cull_levels};
      if (*f[e] == v) continue;
      *f[e] = v;
      if (e == 5) t.pcg_long = 4 * v < 64 ? 64 : 4 * v;  // (the longest replay: at least 64)
      if (!tune_valid(t)) continue;
      ctx->tune = t;
      double ms = 0.0;
      rc = measure(&ms);
      if (rc != ABD_OK) break;
      if (ms < 0.99 * best) {
        best = ms;
        cur = t;
      }
    }
  }
  ctx->tune = cur;
  const int rc2 = restore();
  if (rc == ABD_OK) HIP_TRY(ctx, hipStreamSynchronize(s));
  if (rc != ABD_OK) return rc;
  if (rc2 != ABD_OK) return rc2;
  *out = cur;
  if (best_ms_per_step) *best_ms_per_step = best;
  return ABD_OK;
}
