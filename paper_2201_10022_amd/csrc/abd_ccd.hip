// Continuous collision detection (ABD sec. 4.1): along the step every vertex
// moves on a straight line x + t dx, so each PT / EE pair is bounded with
// additive CCD: remove the pair's mean displacement, bound the closing speed
// l_p by the largest displacement on each side, and advance t by safe
// increments (1-s) d0 / l_p, then 0.9 d / l_p, until the distance drops
// below s d0 (return the last safe t) or t exceeds tmax.
//
// The number of advances per pair ranges from 1 (pairs far apart or
// separating) to ~l_p / d0 (pairs sliding at a small distance), so a lane
// per pair would leave most of a wave idle behind its slowest lane.  The
// kernel is persistent instead: each lane runs a small state machine; its
// first pair is its global thread index, and whenever it finishes a pair
// it takes the next one beyond the grid from a global work counter (one
// atomic per wave and refill, none when the grid covers every pair), so a
// wave's lanes stay busy until the queue is empty.  Every lane performs at
// most one distance evaluation per loop trip; the sequence of operations
// per pair is the same as the one-pair-per-lane form.
#include <cstdlib>

#include "abd_internal.h"

namespace {

__device__ __forceinline__ double pair_distance(int is_ee, const d3 X[4]) {
#pragma clang fp contract(off)
  const int ty = classify_pair(is_ee, X);
  double num, den;
  case_nd(ty, X, num, den);
  return sqrt(num / den);
}

__device__ __forceinline__ void atomic_min_nonneg(double *addr, double v) {
  // non-negative IEEE doubles order like their bit patterns; a value not
  // below the one already there (read without the atomic: it only ever
  // decreases) would change nothing, so it skips the contended atomic
  if (!(v < *reinterpret_cast<volatile double *>(addr))) return;
  atomicMin(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

template <int BS>
__global__ void __launch_bounds__(BS) k_accd(int64_t n_pt, int64_t n, const int32_t *pt, const int32_t *ee,
                                                    const int32_t *tris, const int32_t *edges,
                                                    const int32_t *vert_body, const int32_t *body_scene,
                                                    const double *x, const double *dx, double s, double tmax,
                                                    int max_iter, unsigned long long *counter, double *t_pt,
                                                    double *t_ee, double *alpha, const double *x1) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  // the first pair of every lane is its global thread index (no atomic);
  // lanes that finish take the next pairs beyond the grid from the counter
  const int64_t nlanes = (int64_t)gridDim.x * blockDim.x;
  int64_t cur = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // pair index, >= n = queue exhausted
  bool fresh = true;  // cur assigned, its state not loaded yet
  int phase = 0;      // 0: distance at start pending, 1: advancing
  int is_ee = 0, it = 0, scene = 0;
  // running minimum of this lane's finished pairs, per sub-scene (pairs come
  // from the queue in index order, so a lane rarely changes scene); flushed
  // with one atomic per wave and scene instead of one per pair
  int mscene = -1;
  double mval = 1.0;
  d3 X[4], U[4];
  double lp = 0.0, gap = 0.0, t = 0.0, tl = 0.0;
  for (;;) {
    // ---- refill idle lanes from the global queue (one atomic per wave)
    const unsigned long long need = __ballot(cur < 0);
    if (need) {
      unsigned long long base = 0;
      const int leader = __ffsll((long long)need) - 1;
      if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(need));
      base = __shfl(base, leader, 64);
      if (cur < 0) {
        cur = nlanes + (int64_t)(base + __popcll(need & ((1ull << lane) - 1ull)));
        fresh = true;
      }
    }
    if (fresh) {
      fresh = false;
      {
        if (cur >= n) {
          cur = n;
        } else {
          is_ee = cur >= n_pt;
          const int32_t *pr = is_ee ? ee + 2 * (cur - n_pt) : pt + 2 * cur;
          int vid[4];
          pair_vids(is_ee, pr, tris, edges, vid);
          scene = body_scene[vert_body[vid[0]]];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            X[k] = ld3(x, vid[k]);
            // (the displacement x1 - x formed here when the end positions
            // are given: the same subtraction as a separate pass)
            U[k] = x1 ? xsub(ld3(x1, vid[k]), ld3(x, vid[k])) : ld3(dx, vid[k]);
          }
          const d3 mean = {((U[0].x + U[1].x) + (U[2].x + U[3].x)) * 0.25,
                           ((U[0].y + U[1].y) + (U[2].y + U[3].y)) * 0.25,
                           ((U[0].z + U[1].z) + (U[2].z + U[3].z)) * 0.25};
          double len[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            U[k] = xsub(U[k], mean);
            len[k] = sqrt(xdot(U[k], U[k]));
          }
          lp = is_ee ? fmax(len[0], len[1]) + fmax(len[2], len[3]) : len[0] + fmax(len[1], fmax(len[2], len[3]));
          phase = 0;
          it = 0;
          t = 0.0;
        }
      }
    }
    if (__all(cur >= n)) {
      // flush the running minima: one wave-wide min and atomic per scene
      if (alpha) {
        for (;;) {
          const unsigned long long has = __ballot(mscene >= 0);
          if (!has) break;
          const int leader = __ffsll((long long)has) - 1;
          const int s0 = __shfl(mscene, leader, 64);
          const double m = wave_min(mscene == s0 ? mval : 1.0);
          if (lane == leader) atomic_min_nonneg(alpha + s0, m);
          if (mscene == s0) mscene = -1;
        }
      }
      break;
    }
    bool finish = false;
    double result = 0.0;
    if (cur >= 0 && cur < n) {
      if (phase == 0 && lp == 0.0) {
        finish = true;
        result = tmax;
      } else {
        const double d = pair_distance(is_ee, X);
        bool advance = false;
        if (phase == 0) {
          if (d == 0.0) {
            finish = true;
            result = 0.0;
          } else {
            gap = s * d;
            tl = (1.0 - s) * d / lp;
            phase = 1;
            advance = true;
          }
        } else if (t > 0.0 && d < gap) {
          finish = true;
          result = t;
        } else {
          t += tl;
          if (t > tmax) {
            finish = true;
            result = tmax;
          } else if (++it >= max_iter) {
            finish = true;
            result = t;
          } else {
            tl = 0.9 * d / lp;
            advance = true;
          }
        }
        if (advance) {
#pragma unroll
          for (int k = 0; k < 4; ++k) X[k] = {X[k].x + tl * U[k].x, X[k].y + tl * U[k].y, X[k].z + tl * U[k].z};
        }
      }
    }
    if (finish) {
      if (is_ee) {
        if (t_ee) t_ee[cur - n_pt] = result;
      } else if (t_pt) {
        t_pt[cur] = result;
      }
      if (alpha) {
        if (mscene != scene) {
          if (mscene >= 0) atomic_min_nonneg(alpha + mscene, mval);
          mscene = scene;
          mval = 1.0;
        }
        mval = fmin(mval, result);
      }
      cur = nlanes >= n ? n : -1;  // (every pair had a lane: nothing to take)
    }
  }
}

__global__ void k_ccd_init(double *alpha, int ns, double v, unsigned long long *counter) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) alpha[i] = v;
  if (i == 0) *counter = 0ull;
}

}  // namespace

int op_ccd(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x0, const double *dx,
           const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, double *t_pt, double *t_ee,
           double *alpha, hipStream_t s, const double *x1) {
  const int ns = sc->n_scenes > 0 ? sc->n_scenes : 1;
  unsigned long long *counter;
  ABD_TRY(ws(ctx, "ccd_counter", 1, &counter, s));
  hipLaunchKernelGGL(k_ccd_init, dim3(grid_for(ns, 256)), dim3(256), 0, s, alpha, alpha ? ns : 0, 1.0, counter);
  const int64_t n = n_pt + n_ee;
  if (n > 0) {
    // persistent grid: enough waves to fill the chip, never more than the
    // work (block size and grid cap from the launch-shape table)
    const int bs = ctx->tune.ccd_block;
    int64_t blocks = (n + bs - 1) / bs;
    if (blocks > ctx->tune.ccd_max_blocks) blocks = ctx->tune.ccd_max_blocks;
    // (environment ABD_CCD_MAX_BLOCKS: a smaller grid, so that tests reach
    // the work counter with few pairs)
    if (const char *mb = getenv("ABD_CCD_MAX_BLOCKS")) {
      const long cap = atol(mb);
      if (cap >= 1 && blocks > cap) blocks = cap;
    }
    hipEvent_t pe = prof_begin(ctx, s);
#define ABD_ACCD_ARGS                                                                                          \
  n_pt, n, pt, ee, sc->tris, sc->edges, sc->vert_body, sc->body_scene, x0, dx, prm->ccd_s, prm->ccd_tmax, \
      prm->ccd_max_iter, counter, t_pt, t_ee, alpha, x1
    if (bs == 64)
      hipLaunchKernelGGL(k_accd<64>, dim3((unsigned)blocks), dim3(64), 0, s, ABD_ACCD_ARGS);
    else if (bs == 128)
      hipLaunchKernelGGL(k_accd<128>, dim3((unsigned)blocks), dim3(128), 0, s, ABD_ACCD_ARGS);
    else
      hipLaunchKernelGGL(k_accd<256>, dim3((unsigned)blocks), dim3(256), 0, s, ABD_ACCD_ARGS);
#undef ABD_ACCD_ARGS
    prof_end(ctx, pe, "accd", n, s);
  }
  return abd_hip_check(ctx, hipGetLastError(), "k_accd");
}

extern "C" int abd_ccd_max_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x0,
                                const double *dx, const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee,
                                double *t_pt, double *t_ee, double *alpha, hipStream_t stream) {
  if (!ctx || !sc || !prm || !x0 || !dx || (n_pt && !pt) || (n_ee && !ee))
    return abd_fail(ctx, ABD_E_INVALID, "abd_ccd_max_step: null");
  return op_ccd(ctx, sc, prm, x0, dx, pt, n_pt, ee, n_ee, t_pt, t_ee, alpha, stream);
}
