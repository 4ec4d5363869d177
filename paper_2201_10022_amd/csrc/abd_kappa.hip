// Adaptive barrier stiffness.  The paper scales the barrier by a stiffness
// kappa (sec. 4, Eq. barrier) and gives neither a value nor a rule; this is
// IPC's rule, per scene of a batch, per time step:
//  - at q^t, kappa = clamp(-(g_E . g_B) / (g_B . g_B), kappa_b, kappa_max),
//    with g_B the barrier's gradient at kappa = 1 and g_E that of the rest
//    of the incremental potential (inertia, rigidity potential, joints),
//    over the scene's free bodies; kappa_b when g_B = 0;
//  - before every Newton iteration, with d the smallest distance of an
//    active pair at the iterate and d_prev the one before (at q^t for the
//    first iteration), kappa doubles, up to kappa_max, when d < eps_d and
//    d < d_prev.
// Distances are compared as squares (d^2 = num / den of the pair's distance
// case).  The per-scene values live in the context's workspace and every
// barrier kernel reads its scene's value while a time step runs.
#include "abd_barrier_math.h"

#include <utility>

namespace {
using namespace abd_math;

// Smallest squared distance of an active pair per scene: the bit pattern of
// a non-negative double orders like the double, so an integer atomic
// minimum takes it (order-independent, hence deterministic).
__global__ void __launch_bounds__(256) k_scene_min_d2(int64_t n_pt, int64_t n, const int32_t *pt, const int32_t *ee,
                                                      const int32_t *tris, const int32_t *edges, const double *x,
                                                      const int32_t *vert_body, const int32_t *body_scene,
                                                      double dhat2, unsigned long long *d2min) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int is_ee = i >= n_pt;
  const int32_t *pr = is_ee ? ee + 2 * (i - n_pt) : pt + 2 * i;
  int vid[4];
  pair_vids(is_ee, pr, tris, edges, vid);
  d3 X[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) X[k] = ld3(x, vid[k]);
  const int ty = classify_pair(is_ee, X);
  double num, den;
  case_nd(ty, X, num, den);
  if (!(num < dhat2 * den)) return;
  const double d2 = num / den;
  atomicMin(d2min + body_scene[vert_body[vid[0]]], (unsigned long long)__double_as_longlong(d2));
}

__global__ void k_fill_u64(int n, unsigned long long *a, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__device__ __forceinline__ int scene_lo(const int32_t *body_scene, int nb, int j) {
  int lo = 0, hi = nb;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (body_scene[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One block per scene: the two dot products over its free bodies' DOFs in
// a fixed order (strided partial sums, then a tree), then kappa and d_prev.
constexpr int KB = 256;
__global__ void __launch_bounds__(KB) k_kappa_init(int nb, const int32_t *body_scene, const uint8_t *fixed,
                                                   const double *gE, const double *gB,
                                                   const unsigned long long *d2min, double kmin, double kmax,
                                                   double *kappa, double *d2prev) {
  __shared__ double sa[KB], sb[KB];
  const int j = blockIdx.x, t = threadIdx.x;
  const int lo = scene_lo(body_scene, nb, j), hi = scene_lo(body_scene, nb, j + 1);
  double a = 0.0, b = 0.0;
  for (int64_t i = 12 * (int64_t)lo + t; i < 12 * (int64_t)hi; i += KB) {
    if (fixed[i / 12]) continue;
    a = fma(gE[i], gB[i], a);
    b = fma(gB[i], gB[i], b);
  }
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
  for (int w = KB / 2; w > 0; w >>= 1) {
    if (t < w) {
      sa[t] += sa[t + w];
      sb[t] += sb[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    double k = kmin;
    if (sb[0] > 0.0) k = fmin(fmax(-sa[0] / sb[0], kmin), kmax);
    kappa[j] = k;
    d2prev[j] = __longlong_as_double((long long)d2min[j]);
  }
}

__global__ void k_kappa_update(int S, const unsigned long long *d2min, double eps2, double kmax, double *kappa,
                               double *d2prev) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S) return;
  const double d2 = __longlong_as_double((long long)d2min[j]);
  if (d2 < eps2 && d2 < d2prev[j]) kappa[j] = fmin(2.0 * kappa[j], kmax);
  d2prev[j] = d2;
}

__global__ void k_zero_f64(int64_t n, double *a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

constexpr unsigned long long U64_INF = 0x7FF0000000000000ull;  // +inf

int scene_min_d2(abd_ctx *ctx, const abd_scene *sc, double dhat, const double *x, const int32_t *pt, int64_t npt,
                 const int32_t *ee, int64_t nee, unsigned long long *d2min, hipStream_t s) {
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(S, 256)), dim3(256), 0, s, S, d2min, U64_INF);
  const int64_t n = npt + nee;
  if (n > 0)
    hipLaunchKernelGGL(k_scene_min_d2, dim3(grid_for(n, 256)), dim3(256), 0, s, npt, n, pt, ee, sc->tris, sc->edges,
                       x, sc->vert_body, sc->body_scene, dhat * dhat, d2min);
  return abd_hip_check(ctx, hipGetLastError(), "k_scene_min_d2");
}

}  // namespace

int op_kappa_init(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, const double *qt,
                  hipStream_t s) {
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  const int nb = sc->n_bodies;
  const size_t n12 = 12 * (size_t)nb;
  double *kappa, *d2prev, *x, *gE, *gB, *e, *diag;
  unsigned long long *d2min;
  ABD_TRY(ws(ctx, "kappa_sc", S, &kappa, s));
  ABD_TRY(ws(ctx, "kappa_d2prev", S, &d2prev, s));
  ABD_TRY(ws(ctx, "kappa_d2min", S, &d2min, s));
  ABD_TRY(ws(ctx, "kp_x", 3 * (size_t)sc->n_verts, &x, s));
  ABD_TRY(ws(ctx, "kp_gE", n12, &gE, s));
  ABD_TRY(ws(ctx, "kp_gB", n12, &gB, s));
  ABD_TRY(ws(ctx, "kp_e", 2, &e, s));
  ABD_TRY(ws(ctx, "kp_diag", 144 * (size_t)nb, &diag, s));
  ctx->kappa_sc = nullptr;  // (the gradients below take the scalar stiffness)
  ABD_TRY(op_vertex_map(ctx, sc, q, x, s));
  int32_t *pt, *ee, *keys;
  int64_t npt, nee, nk;
  ABD_TRY(op_candidates(ctx, sc, x, nullptr, prm->dhat, &pt, &npt, &ee, &nee, "kp_c", s));
  ABD_TRY(op_offdiag(ctx, sc, pt, npt, ee, nee, &keys, &nk, "kp_c", s));
  double *off;
  ABD_TRY(ws(ctx, "kp_off", 144 * (size_t)(nk + 1), &off, s));
  for (auto zb : {std::make_pair(gE, (int64_t)n12), std::make_pair(gB, (int64_t)n12),
                  std::make_pair(diag, 144 * (int64_t)nb), std::make_pair(e, (int64_t)2)})
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(zb.second, 256)), dim3(256), 0, s, zb.second, zb.first);
  ABD_TRY(op_body_terms(ctx, sc, prm, q, qt, e, gE, diag, 0, s));
  abd_params unit = *prm;
  unit.kappa_b = 1.0;
  ABD_TRY(op_barrier(ctx, sc, &unit, x, pt, npt, ee, nee, keys, nk, e + 1, gB, diag, off, 0, nullptr, nullptr, s));
  ABD_TRY(scene_min_d2(ctx, sc, prm->dhat, x, pt, npt, ee, nee, d2min, s));
  hipLaunchKernelGGL(k_kappa_init, dim3(S), dim3(KB), 0, s, nb, sc->body_scene, sc->body_fixed, gE, gB, d2min,
                     prm->kappa_b, prm->kappa_max, kappa, d2prev);
  return abd_hip_check(ctx, hipGetLastError(), "k_kappa_init");
}

int op_kappa_update(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x, const int32_t *pt,
                    int64_t npt, const int32_t *ee, int64_t nee, hipStream_t s) {
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  double *kappa, *d2prev;
  unsigned long long *d2min;
  ABD_TRY(ws(ctx, "kappa_sc", S, &kappa, s));
  ABD_TRY(ws(ctx, "kappa_d2prev", S, &d2prev, s));
  ABD_TRY(ws(ctx, "kappa_d2min", S, &d2min, s));
  ABD_TRY(scene_min_d2(ctx, sc, prm->dhat, x, pt, npt, ee, nee, d2min, s));
  hipLaunchKernelGGL(k_kappa_update, dim3(grid_for(S, 256)), dim3(256), 0, s, S, d2min,
                     prm->kappa_eps_d * prm->kappa_eps_d, prm->kappa_max, kappa, d2prev);
  return abd_hip_check(ctx, hipGetLastError(), "k_kappa_update");
}

extern "C" int abd_barrier_stiffness(abd_ctx *ctx, const abd_scene *sc, double *kappa_out) {
  if (!ctx || !sc || !kappa_out) return abd_fail(ctx, ABD_E_INVALID, "abd_barrier_stiffness: null");
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  auto it = ctx->bufs.find("kappa_sc");
  if (it == ctx->bufs.end() || !it->second.ptr || it->second.bytes < S * sizeof(double))
    return abd_fail(ctx, ABD_E_INVALID, "abd_barrier_stiffness: no adaptive time step has run on this context");
  HIP_TRY(ctx, hipDeviceSynchronize());
  HIP_TRY(ctx, hipMemcpy(kappa_out, it->second.ptr, S * sizeof(double), hipMemcpyDeviceToHost));
  return ABD_OK;
}
