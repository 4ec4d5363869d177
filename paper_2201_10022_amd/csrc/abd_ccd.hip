// Continuous collision detection (ABD sec. 4.1): along the step every vertex
// moves on a straight line x + t dx, so each PT / EE pair is bounded with
// additive CCD: remove the pair's mean displacement, bound the closing speed
// l_p by the largest displacement on each side, and advance t by safe
// increments (1-s) d0 / l_p, then 0.9 d / l_p, until the distance drops
// below s d0 (return the last safe t) or t exceeds tmax.
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
  // non-negative IEEE doubles order like their bit patterns
  atomicMin(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

__global__ void __launch_bounds__(128) k_accd(int64_t n_pt, int64_t n, const int32_t *pt, const int32_t *ee,
                                              const int32_t *tris, const int32_t *edges, const int32_t *vert_body,
                                              const int32_t *body_scene, const double *x, const double *dx,
                                              double s, double tmax, int max_iter, double *t_pt, double *t_ee,
                                              double *alpha) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int is_ee = i >= n_pt;
  const int32_t *pr = is_ee ? ee + 2 * (i - n_pt) : pt + 2 * i;
  int vid[4];
  pair_vids(is_ee, pr, tris, edges, vid);
  d3 X[4], U[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    X[k] = ld3(x, vid[k]);
    U[k] = ld3(dx, vid[k]);
  }
  const d3 mean = {((U[0].x + U[1].x) + (U[2].x + U[3].x)) * 0.25, ((U[0].y + U[1].y) + (U[2].y + U[3].y)) * 0.25,
                   ((U[0].z + U[1].z) + (U[2].z + U[3].z)) * 0.25};
  double len[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    U[k] = xsub(U[k], mean);
    len[k] = sqrt(xdot(U[k], U[k]));
  }
  const double lp = is_ee ? fmax(len[0], len[1]) + fmax(len[2], len[3])
                          : len[0] + fmax(len[1], fmax(len[2], len[3]));
  double t;
  if (lp == 0.0) {
    t = tmax;
  } else {
    const double d0 = pair_distance(is_ee, X);
    if (d0 == 0.0) {
      t = 0.0;
    } else {
      const double gap = s * d0;
      double tl = (1.0 - s) * d0 / lp;
      t = 0.0;
      int it = 0;
      for (;;) {
#pragma unroll
        for (int k = 0; k < 4; ++k) X[k] = {X[k].x + tl * U[k].x, X[k].y + tl * U[k].y, X[k].z + tl * U[k].z};
        const double d = pair_distance(is_ee, X);
        if (t > 0.0 && d < gap) break;
        t += tl;
        if (t > tmax) {
          t = tmax;
          break;
        }
        if (++it >= max_iter) break;
        tl = 0.9 * d / lp;
      }
    }
  }
  if (is_ee) {
    if (t_ee) t_ee[i - n_pt] = t;
  } else if (t_pt) {
    t_pt[i] = t;
  }
  if (alpha) atomic_min_nonneg(alpha + body_scene[vert_body[vid[0]]], fmin(t, 1.0));
}

__global__ void k_fill(double *a, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

}  // namespace

int op_ccd(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x0, const double *dx,
           const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, double *t_pt, double *t_ee,
           double *alpha, hipStream_t s) {
  const int ns = sc->n_scenes > 0 ? sc->n_scenes : 1;
  if (alpha) hipLaunchKernelGGL(k_fill, dim3(grid_for(ns, 256)), dim3(256), 0, s, alpha, ns, 1.0);
  const int64_t n = n_pt + n_ee;
  hipEvent_t pe = n > 0 ? prof_begin(ctx, s) : nullptr;
  if (n > 0)
    hipLaunchKernelGGL(k_accd, dim3(grid_for(n, 128)), dim3(128), 0, s, n_pt, n, pt, ee, sc->tris, sc->edges,
                       sc->vert_body, sc->body_scene, x0, dx, prm->ccd_s, prm->ccd_tmax, prm->ccd_max_iter, t_pt,
                       t_ee, alpha);
  prof_end(ctx, pe, "accd", n, s);
  return abd_hip_check(ctx, hipGetLastError(), "k_accd");
}

extern "C" int abd_ccd_max_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x0,
                                const double *dx, const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee,
                                double *t_pt, double *t_ee, double *alpha, hipStream_t stream) {
  if (!ctx || !sc || !prm || !x0 || !dx || (n_pt && !pt) || (n_ee && !ee))
    return abd_fail(ctx, ABD_E_INVALID, "abd_ccd_max_step: null");
  return op_ccd(ctx, sc, prm, x0, dx, pt, n_pt, ee, n_ee, t_pt, t_ee, alpha, stream);
}
