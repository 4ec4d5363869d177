// Lagged friction (ABD sec. 4, friction potential V_F: the sum over active
// contact pairs of mu lambda f0(|u|); the lagging follows IPC's model).
//
// At the start of a time step every active pair gets, from the vertex
// positions x^t: the normal-force magnitude lambda = kappa m |B'(d)| (m the
// EE mollifier, held fixed), the closest-point weights w (r = sum_k w_k x_k
// is the closest-point difference of the two primitives) and an orthonormal
// tangent basis T (3x2) of the plane normal to r.  During the step the
// sliding displacement of a pair is u = T^T sum_k w_k (x_k - x^t_k) and its
// energy mu lambda f0(|u|), with f0 the C1 smoothing of |u| below
// eps = eps_v dt.  The local Hessian is the Kronecker product
// (w w^T) (x) K with K = mu lambda T M T^T (rank 2, PSD by construction),
// so no eigen-projection is needed; local records go through the same
// fixed-order assembly as the barrier.
#include "abd_barrier_math.h"

namespace {
using namespace abd_math;

__device__ __forceinline__ void load_vids(int64_t idx, int64_t n_pt, const int32_t *pt, const int32_t *ee,
                                          const int32_t *tris, const int32_t *edges, int &is_ee, int vid[4]) {
  is_ee = idx >= n_pt;
  const int32_t *pr = is_ee ? ee + 2 * (idx - n_pt) : pt + 2 * idx;
  pair_vids(is_ee, pr, tris, edges, vid);
}

// closest-point weights per distance case, with compile-time vertex slots
template <int I, int J>
__device__ __forceinline__ void w_pp(double w[4]) {
  w[I] = 1.0;
  w[J] = -1.0;
}
// point I against the edge (J, K): parameter t of the projection on the line
template <int I, int J, int K>
__device__ __forceinline__ void w_pe(const d3 X[4], double w[4]) {
  const d3 e = xsub(X[K], X[J]);
  const double t = xdot(xsub(X[I], X[J]), e) / xdot(e, e);
  w[I] = 1.0;
  w[J] = -(1.0 - t);
  w[K] = -t;
}
// point 0 against the triangle (1, 2, 3): barycentric coordinates of the
// projection from cross products (no normal-equation cancellation)
__device__ __forceinline__ void w_face(const d3 X[4], double w[4]) {
  const d3 e1 = xsub(X[2], X[1]), e2 = xsub(X[3], X[1]), dp = xsub(X[0], X[1]);
  const d3 n = xcross(e1, e2);
  const double nn = xdot(n, n);
  const double u = xdot(xcross(dp, e2), n) / nn, v = xdot(xcross(e1, dp), n) / nn;
  w[0] = 1.0;
  w[1] = -(1.0 - u - v);
  w[2] = -u;
  w[3] = -v;
}
// closest points of the lines (0,1) and (2,3): with n = u x v the
// difference of the closest points is parallel to n, which gives s and t
// from triple products
__device__ __forceinline__ void w_ll(const d3 X[4], double w[4]) {
  const d3 u = xsub(X[1], X[0]), v = xsub(X[3], X[2]), r0 = xsub(X[2], X[0]);
  const d3 n = xcross(u, v);
  const double nn = xdot(n, n);
  const double s = xdot(xcross(r0, v), n) / nn, t = xdot(xcross(r0, u), n) / nn;
  w[0] = 1.0 - s;
  w[1] = s;
  w[2] = -(1.0 - t);
  w[3] = -t;
}

__device__ __forceinline__ void closest_weights(int type, const d3 X[4], double w[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = 0.0;
  switch (type) {
    case PT_PP0: w_pp<0, 1>(w); break;
    case PT_PP1: w_pp<0, 2>(w); break;
    case PT_PP2: w_pp<0, 3>(w); break;
    case PT_PE01: w_pe<0, 1, 2>(X, w); break;
    case PT_PE12: w_pe<0, 2, 3>(X, w); break;
    case PT_PE02: w_pe<0, 1, 3>(X, w); break;
    case PT_FACE: w_face(X, w); break;
    case EE_BASE + 0: w_pp<0, 2>(w); break;
    case EE_BASE + 1: w_pp<0, 3>(w); break;
    case EE_BASE + 2: w_pe<0, 2, 3>(X, w); break;
    case EE_BASE + 3: w_pp<1, 2>(w); break;
    case EE_BASE + 4: w_pp<1, 3>(w); break;
    case EE_BASE + 5: w_pe<1, 2, 3>(X, w); break;
    case EE_BASE + 6: w_pp<2, 0>(w); break;
    case EE_BASE + 7: w_pp<2, 1>(w); break;
    case EE_BASE + 8: w_pe<2, 0, 1>(X, w); break;
    case EE_BASE + 9: w_pp<3, 0>(w); break;
    case EE_BASE + 10: w_pp<3, 1>(w); break;
    case EE_BASE + 11: w_pe<3, 0, 1>(X, w); break;
    default: w_ll(X, w); break;
  }
}

// T columns t1 = n x e_a / |n x e_a| (e_a the axis of the smallest |n_a|,
// the first on ties) and t2 = n x t1, with n = r / |r|
__device__ __forceinline__ void tangent_basis(d3 r, double T[6]) {
  const double inv = 1.0 / sqrt(xdot(r, r));
  const d3 n{r.x * inv, r.y * inv, r.z * inv};
  const double ax = fabs(n.x), ay = fabs(n.y), az = fabs(n.z);
  d3 t1;
  if (ay < ax && ay <= az)
    t1 = {-n.z, 0.0, n.x};  // n x e_y
  else if (az < ax && az < ay)
    t1 = {n.y, -n.x, 0.0};  // n x e_z
  else
    t1 = {0.0, n.z, -n.y};  // n x e_x
  const double l1 = 1.0 / sqrt(xdot(t1, t1));
  t1 = {t1.x * l1, t1.y * l1, t1.z * l1};
  const d3 t2 = xcross(n, t1);
  T[0] = t1.x, T[1] = t1.y, T[2] = t1.z;
  T[3] = t2.x, T[4] = t2.y, T[5] = t2.z;
}

__global__ void __launch_bounds__(256) k_friction_lag(int64_t n, int64_t n_pt, const int32_t *pt, const int32_t *ee,
                                                      const int32_t *tris, const int32_t *edges, const double *xt,
                                                      const double *xbar, double dhat, double kappa, double *lam,
                                                      double *T, double *w, const double *kappa_sc,
                                                      const int32_t *vert_body, const int32_t *body_scene) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int is_ee, vid[4];
  load_vids(i, n_pt, pt, ee, tris, edges, is_ee, vid);
  d3 X[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) X[k] = ld3(xt, vid[k]);
  int ty;
  double num, den;
  bool act;
  {
#pragma clang fp contract(off)
    ty = classify_pair(is_ee, X);
    case_nd(ty, X, num, den);
    act = num < (dhat * dhat) * den && num != 0.0;
  }
  double wl[4] = {0.0, 0.0, 0.0, 0.0}, Tl[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, l = 0.0;
  if (act) {
    const double d = sqrt(num / den);
    const double Bp = -2.0 * (d - dhat) * log(d / dhat) - (d - dhat) * (d - dhat) / d;
    double m = 1.0;
    if (is_ee) {
      const d3 nn = xcross(xsub(X[1], X[0]), xsub(X[3], X[2]));
      const double c = xdot(nn, nn);
      const d3 uu = xsub(ld3(xbar, vid[1]), ld3(xbar, vid[0])), vv = xsub(ld3(xbar, vid[3]), ld3(xbar, vid[2]));
      const double eps = (1e-3 * xdot(uu, uu)) * xdot(vv, vv);
      if (c < eps) m = (2.0 - c / eps) * (c / eps);
    }
    // (per-scene stiffness when it adapts)
    const double kap = kappa_sc ? kappa_sc[body_scene[vert_body[vid[0]]]] : kappa;
    l = -kap * m * Bp;
    closest_weights(ty, X, wl);
    d3 r{0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) r = {r.x + wl[k] * X[k].x, r.y + wl[k] * X[k].y, r.z + wl[k] * X[k].z};
    tangent_basis(r, Tl);
  }
  lam[i] = l;
#pragma unroll
  for (int k = 0; k < 6; ++k) T[6 * i + k] = Tl[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[4 * i + k] = wl[k];
}

// smoothed sliding norm: f0(y) = -y^3/(3 eps^2) + y^2/eps + eps/3 below eps,
// y beyond; f1 = f0'
__device__ __forceinline__ double f0_of(double y, double eps) {
  return y < eps ? -y * y * y / (3.0 * eps * eps) + y * y / eps + eps / 3.0 : y;
}
__device__ __forceinline__ double f1_of(double y, double eps) {
  return y < eps ? -y * y / (eps * eps) + 2.0 * y / eps : 1.0;
}

// one lane per friction pair: energy and (unless ENERGY_ONLY) the 12-vector
// gradient and packed 12x12 Hessian, plus the pair's assembly record.
// HVP: in place of the gradient, the local Hessian times J v for the body
// vector v [nb][12] (so that assembling it gives the friction Hessian times
// v).
template <bool ENERGY_ONLY, bool HVP = false>
__global__ void __launch_bounds__(128) k_friction_local(int64_t n, int64_t n_pt, const int32_t *pt,
                                                        const int32_t *ee, const int32_t *tris,
                                                        const int32_t *edges, const int32_t *vert_body,
                                                        const double *x, const double *xt, const double *lam,
                                                        const double *T, const double *w, double mu, double eps,
                                                        double *e_out, double *g_out, double *H_out,
                                                        PairInfo *info, const int32_t *body_scene,
                                                        int32_t *key_out, const double *v = nullptr,
                                                        const double *xbar = nullptr, int64_t xstride = 0,
                                                        int64_t estride = 0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (ENERGY_ONLY) {  // (grid.y > 1: trial t's positions at x + t xstride, energies at e_out + t estride)
    x += blockIdx.y * xstride;
    e_out += blockIdx.y * (estride > 0 ? estride : n);
  }
  int is_ee, vid[4];
  load_vids(i, n_pt, pt, ee, tris, edges, is_ee, vid);
  if (key_out && blockIdx.y == 0) key_out[i] = body_scene[vert_body[vid[0]]];
  const double ml = mu * lam[i];
  double wk[4], Ti[6];
#pragma unroll
  for (int k = 0; k < 4; ++k) wk[k] = w[4 * i + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) Ti[k] = T[6 * i + k];
  double dl[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) dl[c] += wk[k] * (x[3 * (int64_t)vid[k] + c] - xt[3 * (int64_t)vid[k] + c]);
  const double u0 = Ti[0] * dl[0] + Ti[1] * dl[1] + Ti[2] * dl[2];
  const double u1 = Ti[3] * dl[0] + Ti[4] * dl[1] + Ti[5] * dl[2];
  const double y = sqrt(u0 * u0 + u1 * u1);
  const bool on = ml > 0.0;
  e_out[i] = on ? ml * f0_of(y, eps) : 0.0;
  if (ENERGY_ONLY) return;
  PairInfo pi;
#pragma unroll
  for (int k = 0; k < 4; ++k) pi.vid[k] = vid[k];
  pi.body[0] = vert_body[vid[0]];
  pi.body[1] = vert_body[vid[3]];
  pi.is_ee = is_ee;
  pi.pad = 0;
  info[i] = pi;
  // M = a u u^T + gs I (2x2), gs = f1(y)/y, a = (f1'(y) y - f1(y)) / y^3;
  // both tend to (0, 2/eps) as y -> 0
  double gs, a;
  if (y == 0.0) {
    gs = 2.0 / eps;
    a = 0.0;
  } else {
    const double f1 = f1_of(y, eps);
    const double f1p = y < eps ? -2.0 * y / (eps * eps) + 2.0 / eps : 0.0;
    gs = f1 / y;
    a = (f1p * y - f1) / (y * y * y);
  }
  const double M00 = a * u0 * u0 + gs, M01 = a * u0 * u1, M11 = a * u1 * u1 + gs;
  // force f = ml gs T u and K = ml T M T^T (3x3)
  double f[3], K[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r) f[r] = on ? ml * gs * (Ti[r] * u0 + Ti[3 + r] * u1) : 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = Ti[r] * (M00 * Ti[c] + M01 * Ti[3 + c]) + Ti[3 + r] * (M01 * Ti[c] + M11 * Ti[3 + c]);
      K[r][c] = on ? ml * v : 0.0;
    }
  if (HVP) {
    // J v at the 4 vertices, weighted sum nu = sum_k w_k (J v)_k, then
    // (w w^T (x) K) (J v) = w_k K nu
    double nu[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double *vb = v + 12 * (int64_t)vert_body[vid[k]];
      const double *xb = xbar + 3 * (int64_t)vid[k];
#pragma unroll
      for (int c = 0; c < 3; ++c) nu[c] += wk[k] * (vb[c] + vb[3 + 3 * c] * xb[0] + vb[4 + 3 * c] * xb[1] +
                                                   vb[5 + 3 * c] * xb[2]);
    }
    double Kn[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) Kn[r] = K[r][0] * nu[0] + K[r][1] * nu[1] + K[r][2] * nu[2];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) g_out[12 * i + 3 * k + c] = wk[k] * Kn[c];
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) g_out[12 * i + 3 * k + c] = wk[k] * f[c];
  }
#pragma unroll
  for (int r = 0; r < 12; ++r)
#pragma unroll
    for (int c = r; c < 12; ++c) H_out[78 * i + S12::at(r, c)] = wk[r / 3] * wk[c / 3] * K[r % 3][c % 3];
}

// ------------------------------------------------ lag, differentiated ----
// First-order dual numbers (value, derivative along one seeded coordinate)
// for the adjoint's lag term: the lagged lambda, T and w as functions of the
// step-start positions, one coordinate of the pair's 12 per pass.
struct dl {
  double v, d;
};
__device__ __forceinline__ dl operator+(dl a, dl b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ dl operator-(dl a, dl b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ dl operator*(dl a, dl b) { return {a.v * b.v, a.v * b.d + a.d * b.v}; }
__device__ __forceinline__ dl operator/(dl a, dl b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
__device__ __forceinline__ dl dc(double c) { return {c, 0.0}; }
__device__ __forceinline__ dl dsqrt(dl a) {
  const double s = sqrt(a.v);
  return {s, 0.5 * a.d / s};
}
__device__ __forceinline__ dl dlog(dl a) { return {log(a.v), a.d / a.v}; }
struct dl3 {
  dl x, y, z;
};
__device__ __forceinline__ dl3 dsub(dl3 a, dl3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ dl ddot(dl3 a, dl3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ dl3 dcross(dl3 a, dl3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ dl3 dscale(dl3 a, dl s) { return {a.x * s, a.y * s, a.z * s}; }

template <int I, int J>
__device__ __forceinline__ dl dd2_pp(const dl3 X[4]) {
  const dl3 d = dsub(X[I], X[J]);
  return ddot(d, d);
}
template <int I, int J, int K>
__device__ __forceinline__ dl dd2_pe(const dl3 X[4]) {
  const dl3 e = dsub(X[K], X[J]);
  const dl3 c = dcross(dsub(X[I], X[J]), e);
  return ddot(c, c) / ddot(e, e);
}
__device__ __forceinline__ dl dd2_plane(dl3 p, dl3 o, dl3 n) {
  const dl h = ddot(dsub(p, o), n);
  return h * h / ddot(n, n);
}
// squared distance of the case as a dual
__device__ __forceinline__ dl dd2_case(int ty, const dl3 X[4]) {
  switch (ty) {
    case PT_PP0: return dd2_pp<0, 1>(X);
    case PT_PP1: return dd2_pp<0, 2>(X);
    case PT_PP2: return dd2_pp<0, 3>(X);
    case PT_PE01: return dd2_pe<0, 1, 2>(X);
    case PT_PE12: return dd2_pe<0, 2, 3>(X);
    case PT_PE02: return dd2_pe<0, 1, 3>(X);
    case PT_FACE: return dd2_plane(X[0], X[1], dcross(dsub(X[2], X[1]), dsub(X[3], X[1])));
    case EE_BASE + 0: return dd2_pp<0, 2>(X);
    case EE_BASE + 1: return dd2_pp<0, 3>(X);
    case EE_BASE + 2: return dd2_pe<0, 2, 3>(X);
    case EE_BASE + 3: return dd2_pp<1, 2>(X);
    case EE_BASE + 4: return dd2_pp<1, 3>(X);
    case EE_BASE + 5: return dd2_pe<1, 2, 3>(X);
    case EE_BASE + 6: return dd2_pp<2, 0>(X);
    case EE_BASE + 7: return dd2_pp<2, 1>(X);
    case EE_BASE + 8: return dd2_pe<2, 0, 1>(X);
    case EE_BASE + 9: return dd2_pp<3, 0>(X);
    case EE_BASE + 10: return dd2_pp<3, 1>(X);
    case EE_BASE + 11: return dd2_pe<3, 0, 1>(X);
    default: return dd2_plane(X[2], X[0], dcross(dsub(X[1], X[0]), dsub(X[3], X[2])));
  }
}
template <int I, int J>
__device__ __forceinline__ void dw_pp(dl w[4]) {
  w[I] = dc(1.0);
  w[J] = dc(-1.0);
}
template <int I, int J, int K>
__device__ __forceinline__ void dw_pe(const dl3 X[4], dl w[4]) {
  const dl3 e = dsub(X[K], X[J]);
  const dl t = ddot(dsub(X[I], X[J]), e) / ddot(e, e);
  w[I] = dc(1.0);
  w[J] = t - dc(1.0);
  w[K] = dc(0.0) - t;
}
__device__ __forceinline__ void dclosest_weights(int ty, const dl3 X[4], dl w[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = dc(0.0);
  switch (ty) {
    case PT_PP0: dw_pp<0, 1>(w); break;
    case PT_PP1: dw_pp<0, 2>(w); break;
    case PT_PP2: dw_pp<0, 3>(w); break;
    case PT_PE01: dw_pe<0, 1, 2>(X, w); break;
    case PT_PE12: dw_pe<0, 2, 3>(X, w); break;
    case PT_PE02: dw_pe<0, 1, 3>(X, w); break;
    case PT_FACE: {
      const dl3 e1 = dsub(X[2], X[1]), e2 = dsub(X[3], X[1]), dp = dsub(X[0], X[1]);
      const dl3 n = dcross(e1, e2);
      const dl nn = ddot(n, n);
      const dl u = ddot(dcross(dp, e2), n) / nn, v = ddot(dcross(e1, dp), n) / nn;
      w[0] = dc(1.0);
      w[1] = u + v - dc(1.0);
      w[2] = dc(0.0) - u;
      w[3] = dc(0.0) - v;
      break;
    }
    case EE_BASE + 0: dw_pp<0, 2>(w); break;
    case EE_BASE + 1: dw_pp<0, 3>(w); break;
    case EE_BASE + 2: dw_pe<0, 2, 3>(X, w); break;
    case EE_BASE + 3: dw_pp<1, 2>(w); break;
    case EE_BASE + 4: dw_pp<1, 3>(w); break;
    case EE_BASE + 5: dw_pe<1, 2, 3>(X, w); break;
    case EE_BASE + 6: dw_pp<2, 0>(w); break;
    case EE_BASE + 7: dw_pp<2, 1>(w); break;
    case EE_BASE + 8: dw_pe<2, 0, 1>(X, w); break;
    case EE_BASE + 9: dw_pp<3, 0>(w); break;
    case EE_BASE + 10: dw_pp<3, 1>(w); break;
    case EE_BASE + 11: dw_pe<3, 0, 1>(X, w); break;
    default: {
      const dl3 u = dsub(X[1], X[0]), v = dsub(X[3], X[2]), r0 = dsub(X[2], X[0]);
      const dl3 n = dcross(u, v);
      const dl nn = ddot(n, n);
      const dl s = ddot(dcross(r0, v), n) / nn, t = ddot(dcross(r0, u), n) / nn;
      w[0] = dc(1.0) - s;
      w[1] = s;
      w[2] = t - dc(1.0);
      w[3] = dc(0.0) - t;
      break;
    }
  }
}

// one lane per lagged pair: g_out = grad over the pair's 12 step-start
// coordinates of phi = (J l) . g(x; lambda, T, w), through the lag only
// (the sliding displacement x - x^t is held), for the pair assembly
__global__ void __launch_bounds__(64) k_friction_lag_vjp(int64_t n, int64_t n_pt, const int32_t *pt,
                                                         const int32_t *ee, const int32_t *tris, const int32_t *edges,
                                                         const int32_t *vert_body, const double *x, const double *xt,
                                                         const double *xbar, const double *lam, const double *l,
                                                         double mu, double eps, double dhat, double kappa,
                                                         double *g_out, double *H_out, PairInfo *info) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int is_ee, vid[4];
  load_vids(i, n_pt, pt, ee, tris, edges, is_ee, vid);
  PairInfo pi;
#pragma unroll
  for (int k = 0; k < 4; ++k) pi.vid[k] = vid[k];
  pi.body[0] = vert_body[vid[0]];
  pi.body[1] = vert_body[vid[3]];
  pi.is_ee = is_ee;
  pi.pad = 0;
  info[i] = pi;
  for (int j = 0; j < 78; ++j) H_out[78 * i + j] = 0.0;
  d3 X0[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) X0[k] = ld3(xt, vid[k]);
  int ty;
  {
#pragma clang fp contract(off)
    ty = classify_pair(is_ee, X0);
  }
  // data of the pass: displacements and J l at the 4 vertices
  double dx[4][3], vk[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double *lb = l + 12 * (int64_t)vert_body[vid[k]];
    const double *xb = xbar + 3 * (int64_t)vid[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dx[k][c] = x[3 * (int64_t)vid[k] + c] - xt[3 * (int64_t)vid[k] + c];
      vk[k][c] = lb[c] + lb[3 + 3 * c] * xb[0] + lb[4 + 3 * c] * xb[1] + lb[5 + 3 * c] * xb[2];
    }
  }
  double ep = 0.0;
  if (is_ee) {
    const d3 uu = xsub(ld3(xbar, vid[1]), ld3(xbar, vid[0])), vv = xsub(ld3(xbar, vid[3]), ld3(xbar, vid[2]));
    ep = (1e-3 * xdot(uu, uu)) * xdot(vv, vv);
  }
  const bool on = lam[i] > 0.0;
  for (int s = 0; s < 12; ++s) {
    double gv = 0.0;
    if (on) {
      dl3 X[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        X[k] = {{X0[k].x, s == 3 * k ? 1.0 : 0.0}, {X0[k].y, s == 3 * k + 1 ? 1.0 : 0.0},
                {X0[k].z, s == 3 * k + 2 ? 1.0 : 0.0}};
      const dl d = dsqrt(dd2_case(ty, X));
      const dl dm = d - dc(dhat);
      const dl Bp = dc(0.0) - dc(2.0) * dm * dlog(d / dc(dhat)) - dm * dm / d;
      dl m = dc(1.0);
      if (is_ee) {
        const dl3 nn = dcross(dsub(X[1], X[0]), dsub(X[3], X[2]));
        const dl c = ddot(nn, nn);
        if (c.v < ep) {
          const dl r = c / dc(ep);
          m = (dc(2.0) - r) * r;
        }
      }
      const dl L = dc(-kappa) * m * Bp;
      dl w[4];
      dclosest_weights(ty, X, w);
      dl3 r = {dc(0.0), dc(0.0), dc(0.0)};
#pragma unroll
      for (int k = 0; k < 4; ++k) r = {r.x + w[k] * X[k].x, r.y + w[k] * X[k].y, r.z + w[k] * X[k].z};
      const dl inv = dc(1.0) / dsqrt(ddot(r, r));
      const dl3 nv = dscale(r, inv);
      const double ax = fabs(nv.x.v), ay = fabs(nv.y.v), az = fabs(nv.z.v);
      dl3 t1;
      if (ay < ax && ay <= az)
        t1 = {dc(0.0) - nv.z, dc(0.0), nv.x};
      else if (az < ax && az < ay)
        t1 = {nv.y, dc(0.0) - nv.x, dc(0.0)};
      else
        t1 = {dc(0.0), nv.z, dc(0.0) - nv.y};
      t1 = dscale(t1, dc(1.0) / dsqrt(ddot(t1, t1)));
      const dl3 t2 = dcross(nv, t1);
      dl3 delta = {dc(0.0), dc(0.0), dc(0.0)}, nu = {dc(0.0), dc(0.0), dc(0.0)};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        delta = {delta.x + w[k] * dc(dx[k][0]), delta.y + w[k] * dc(dx[k][1]), delta.z + w[k] * dc(dx[k][2])};
        nu = {nu.x + w[k] * dc(vk[k][0]), nu.y + w[k] * dc(vk[k][1]), nu.z + w[k] * dc(vk[k][2])};
      }
      const dl u0 = ddot(t1, delta), u1 = ddot(t2, delta);
      const dl yy = u0 * u0 + u1 * u1;
      dl gs;
      if (yy.v == 0.0) {
        gs = dc(2.0 / eps);
      } else {
        const dl y = dsqrt(yy);
        gs = y.v < eps ? dc(2.0 / eps) - y / dc(eps * eps) : dc(1.0) / y;
      }
      const dl coef = dc(mu) * L * gs;
      const dl3 f = {coef * (t1.x * u0 + t2.x * u1), coef * (t1.y * u0 + t2.y * u1), coef * (t1.z * u0 + t2.z * u1)};
      gv = ddot(nu, f).d;
    }
    g_out[12 * i + s] = gv;
  }
}

// compaction of the lagged pairs with lambda > 0
__global__ void k_lam_flags(int64_t n, const double *lam, int64_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = lam[i] > 0.0 ? 1 : 0;
}
__global__ void k_lam_compact(int64_t n, int64_t n_pt, const int32_t *pt, const int32_t *ee, const int64_t *flag,
                              const int64_t *pos, const double *lam, const double *T, const double *w,
                              const int64_t *n_keep_pt, int32_t *opt, int32_t *oee, double *olam, double *oT,
                              double *ow) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const int64_t j = pos[i];
  if (i < n_pt) {
    opt[2 * j] = pt[2 * i];
    opt[2 * j + 1] = pt[2 * i + 1];
  } else {
    const int64_t je = j - *n_keep_pt;
    oee[2 * je] = ee[2 * (i - n_pt)];
    oee[2 * je + 1] = ee[2 * (i - n_pt) + 1];
  }
  olam[j] = lam[i];
  for (int k = 0; k < 6; ++k) oT[6 * j + k] = T[6 * i + k];
  for (int k = 0; k < 4; ++k) ow[4 * j + k] = w[4 * i + k];
}

}  // namespace

int op_friction_lag(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *xt, const int32_t *pt,
                    int64_t n_pt, const int32_t *ee, int64_t n_ee, double *lam, double *T, double *w,
                    hipStream_t s) {
  const int64_t n = n_pt + n_ee;
  if (n == 0) return ABD_OK;
  hipLaunchKernelGGL(k_friction_lag, dim3(grid_for(n, 256)), dim3(256), 0, s, n, n_pt, pt, ee, sc->tris, sc->edges,
                     xt, sc->xbar, prm->dhat, prm->kappa_b, lam, T, w, ctx->kappa_sc, sc->vert_body,
                     sc->body_scene);
  return abd_hip_check(ctx, hipGetLastError(), "k_friction_lag");
}

int op_friction_local(abd_ctx *ctx, const abd_scene *sc, const FrictionSet *fr, const double *x, double *e_loc,
                      double *g_loc, double *H_loc, PairInfo *info, hipStream_t s) {
  const int64_t n = fr->n();
  if (n == 0) return ABD_OK;
  hipEvent_t pe = prof_begin(ctx, s);
  hipLaunchKernelGGL(k_friction_local<false>, dim3(grid_for(n, 128)), dim3(128), 0, s, n, fr->n_pt, fr->pt, fr->ee,
                     sc->tris, sc->edges, sc->vert_body, x, fr->xt, fr->lam, fr->T, fr->w, fr->mu, fr->eps, e_loc,
                     g_loc, H_loc, info, sc->body_scene, nullptr);
  prof_end(ctx, pe, "friction_local", n, s);
  return abd_hip_check(ctx, hipGetLastError(), "k_friction_local");
}

int op_friction_hvp(abd_ctx *ctx, const abd_scene *sc, const FrictionSet *fr, const double *x, const double *v,
                    double *out, hipStream_t s) {
  const int64_t n = fr->n();
  if (n == 0) return ABD_OK;
  double *e_loc, *g_loc, *H_loc;
  PairInfo *info;
  ABD_TRY(ws(ctx, "fh_e", n, &e_loc, s));
  ABD_TRY(ws(ctx, "fh_g", 12 * n, &g_loc, s));
  ABD_TRY(ws(ctx, "fh_H", 78 * n, &H_loc, s));
  ABD_TRY(ws(ctx, "fh_info", n, &info, s));
  hipLaunchKernelGGL((k_friction_local<false, true>), dim3(grid_for(n, 128)), dim3(128), 0, s, n, fr->n_pt, fr->pt,
                     fr->ee, sc->tris, sc->edges, sc->vert_body, x, fr->xt, fr->lam, fr->T, fr->w, fr->mu, fr->eps,
                     e_loc, g_loc, H_loc, info, sc->body_scene, nullptr, v, sc->xbar);
  HIP_TRY(ctx, hipGetLastError());
  return op_assemble(ctx, sc, n, info, g_loc, H_loc, nullptr, 0, out, nullptr, nullptr, s);
}

int op_friction_lag_vjp(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const FrictionSet *fr,
                        const double *x, const double *l, double *out, hipStream_t s) {
  const int64_t n = fr->n();
  if (n == 0) return ABD_OK;
  double *g_loc, *H_loc;
  PairInfo *info;
  ABD_TRY(ws(ctx, "fv_g", 12 * n, &g_loc, s));
  ABD_TRY(ws(ctx, "fv_H", 78 * n, &H_loc, s));
  ABD_TRY(ws(ctx, "fv_info", n, &info, s));
  hipLaunchKernelGGL(k_friction_lag_vjp, dim3(grid_for(n, 64)), dim3(64), 0, s, n, fr->n_pt, fr->pt, fr->ee, sc->tris,
                     sc->edges, sc->vert_body, x, fr->xt, sc->xbar, fr->lam, l, fr->mu, fr->eps, prm->dhat,
                     prm->kappa_b, g_loc, H_loc, info);
  HIP_TRY(ctx, hipGetLastError());
  return op_assemble(ctx, sc, n, info, g_loc, H_loc, nullptr, 0, out, nullptr, nullptr, s);
}

int op_friction_energy(abd_ctx *ctx, const abd_scene *sc, const FrictionSet *fr, const double *x, double *energy,
                       hipStream_t s) {
  const int64_t n = fr->n();
  if (n == 0) return ABD_OK;
  double *e;
  ABD_TRY(ws(ctx, "fe_e", n, &e, s));
  hipLaunchKernelGGL(k_friction_local<true>, dim3(grid_for(n, 128)), dim3(128), 0, s, n, fr->n_pt, fr->pt, fr->ee,
                     sc->tris, sc->edges, sc->vert_body, x, fr->xt, fr->lam, fr->T, fr->w, fr->mu, fr->eps, e,
                     nullptr, nullptr, nullptr, sc->body_scene, nullptr);
  HIP_TRY(ctx, hipGetLastError());
  return reduce_sum_f64(ctx, e, n, energy, s);
}


int op_friction_energy_trials(abd_ctx *ctx, const abd_scene *sc, const FrictionSet *fr, const double *x,
                              int n_trials, double *energy, hipStream_t s, double *items, int64_t estride,
                              TrialSums *defer) {
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  const int64_t n = fr->n();
  if (n == 0 || n_trials <= 0) return ABD_OK;
  double *e = items;
  int32_t *key = nullptr;
  if (!e) ABD_TRY(ws(ctx, "fe_e_tr", (size_t)n * n_trials, &e, s));
  if (!items) ABD_TRY(ws(ctx, "fe_key", n, &key, s));
  hipLaunchKernelGGL(k_friction_local<true>, dim3(grid_for(n, 128), n_trials), dim3(128), 0, s, n, fr->n_pt, fr->pt,
                     fr->ee, sc->tris, sc->edges, sc->vert_body, x, fr->xt, fr->lam, fr->T, fr->w, fr->mu, fr->eps, e,
                     nullptr, nullptr, nullptr, sc->body_scene, key, nullptr, nullptr, 3 * (int64_t)sc->n_verts,
                     items ? estride : 0);
  HIP_TRY(ctx, hipGetLastError());
  if (items) return ABD_OK;
  if (defer) {
    if (fr->n_pt) defer->seg[defer->k++] = TrialSeg{e, n, fr->n_pt, key};
    if (fr->n_ee) defer->seg[defer->k++] = TrialSeg{e + fr->n_pt, n, fr->n_ee, key + fr->n_pt};
    return ABD_OK;
  }
  if (fr->n_pt) ABD_TRY(seg_sum_trials(ctx, e, n, fr->n_pt, key, n_trials, S, energy, s));
  if (fr->n_ee) ABD_TRY(seg_sum_trials(ctx, e + fr->n_pt, n, fr->n_ee, key + fr->n_pt, n_trials, S, energy, s));
  return ABD_OK;
}

int op_friction_state(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, FrictionSet *fr, bool *active,
                      hipStream_t s) {
  *active = ctx->fr_set && prm->mu > 0.0;
  if (!*active) return ABD_OK;
  const int64_t n = ctx->fr_n_pt + ctx->fr_n_ee;
  int32_t *fpt, *fee;
  double *lam, *T, *w, *xt;
  ABD_TRY(ws(ctx, "fr_pt", 2 * ctx->fr_n_pt, &fpt, s));
  ABD_TRY(ws(ctx, "fr_ee", 2 * ctx->fr_n_ee, &fee, s));
  ABD_TRY(ws(ctx, "fr_lam", n, &lam, s));
  ABD_TRY(ws(ctx, "fr_T", 6 * n, &T, s));
  ABD_TRY(ws(ctx, "fr_w", 4 * n, &w, s));
  ABD_TRY(ws(ctx, "fr_xt", 3 * (size_t)sc->n_verts, &xt, s));
  fr->pt = fpt;
  fr->ee = fee;
  fr->n_pt = ctx->fr_n_pt;
  fr->n_ee = ctx->fr_n_ee;
  fr->lam = lam;
  fr->T = T;
  fr->w = w;
  fr->xt = xt;
  fr->mu = prm->mu;
  fr->eps = prm->eps_v * prm->dt;
  return ABD_OK;
}

// ------------------------------------------------------------------ ABI ----
static bool fr_args_ok(const abd_scene *sc, const abd_params *prm, const double *x, const int32_t *pt, int64_t n_pt,
                       const int32_t *ee, int64_t n_ee, const double *lam, const double *T, const double *w) {
  if (!sc || !prm || !x || n_pt < 0 || n_ee < 0) return false;
  if ((n_pt && !pt) || (n_ee && !ee)) return false;
  if (n_pt + n_ee > 0 && (!lam || !T || !w)) return false;
  return true;
}

extern "C" int abd_friction_lag(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *xt,
                                const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, double *lam,
                                double *T, double *w, hipStream_t stream) {
  if (!ctx || !fr_args_ok(sc, prm, xt, pt, n_pt, ee, n_ee, lam, T, w))
    return abd_fail(ctx, ABD_E_INVALID, "abd_friction_lag: null or negative size");
  return op_friction_lag(ctx, sc, prm, xt, pt, n_pt, ee, n_ee, lam, T, w, stream);
}

extern "C" int abd_friction_grad_hess(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x,
                                      const double *xt, const int32_t *pt, int64_t n_pt, const int32_t *ee,
                                      int64_t n_ee, const double *lam, const double *T, const double *w,
                                      const int32_t *keys, int64_t n_keys, double *energy, double *grad,
                                      double *diag, double *off, hipStream_t stream) {
  if (!ctx || !fr_args_ok(sc, prm, x, pt, n_pt, ee, n_ee, lam, T, w) || !xt || !grad || (off && n_keys && !keys))
    return abd_fail(ctx, ABD_E_INVALID, "abd_friction_grad_hess: null or negative size");
  FrictionSet fr;
  fr.pt = pt;
  fr.ee = ee;
  fr.n_pt = n_pt;
  fr.n_ee = n_ee;
  fr.lam = lam;
  fr.T = T;
  fr.w = w;
  fr.xt = xt;
  fr.mu = prm->mu;
  fr.eps = prm->eps_v * prm->dt;
  const int64_t n = fr.n();
  if (n == 0) return ABD_OK;
  double *e_loc, *g_loc, *H_loc;
  PairInfo *info;
  ABD_TRY(ws(ctx, "fl_e", n, &e_loc, stream));
  ABD_TRY(ws(ctx, "fl_g", 12 * n, &g_loc, stream));
  ABD_TRY(ws(ctx, "fl_H", 78 * n, &H_loc, stream));
  ABD_TRY(ws(ctx, "fl_info", n, &info, stream));
  ABD_TRY(op_friction_local(ctx, sc, &fr, x, e_loc, g_loc, H_loc, info, stream));
  if (energy) ABD_TRY(reduce_sum_f64(ctx, e_loc, n, energy, stream));
  return op_assemble(ctx, sc, n, info, g_loc, H_loc, keys, n_keys, grad, diag, off, stream);
}

extern "C" int abd_friction_energy(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x,
                                   const double *xt, const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee,
                                   const double *lam, const double *T, const double *w, double *energy,
                                   hipStream_t stream) {
  if (!ctx || !fr_args_ok(sc, prm, x, pt, n_pt, ee, n_ee, lam, T, w) || !xt || !energy)
    return abd_fail(ctx, ABD_E_INVALID, "abd_friction_energy: null or negative size");
  FrictionSet fr;
  fr.pt = pt;
  fr.ee = ee;
  fr.n_pt = n_pt;
  fr.n_ee = n_ee;
  fr.lam = lam;
  fr.T = T;
  fr.w = w;
  fr.xt = xt;
  fr.mu = prm->mu;
  fr.eps = prm->eps_v * prm->dt;
  return op_friction_energy(ctx, sc, &fr, x, energy, stream);
}

static int friction_begin(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, hipStream_t s) {
  ctx->fr_set = false;
  ctx->fr_n_pt = ctx->fr_n_ee = 0;
  double *xt;
  ABD_TRY(ws(ctx, "fr_xt", 3 * (size_t)sc->n_verts, &xt, s));
  ABD_TRY(op_vertex_map(ctx, sc, q, xt, s));
  int32_t *pt, *ee;
  int64_t npt, nee;
  ABD_TRY(op_candidates(ctx, sc, xt, nullptr, prm->dhat, &pt, &npt, &ee, &nee, "fr_c", s));
  const int64_t n = npt + nee;
  if (n > 0) {
    double *lam, *T, *w;
    int64_t *flag, *pos, *tot;
    ABD_TRY(ws(ctx, "frl_lam", n, &lam, s));
    ABD_TRY(ws(ctx, "frl_T", 6 * n, &T, s));
    ABD_TRY(ws(ctx, "frl_w", 4 * n, &w, s));
    ABD_TRY(ws(ctx, "frl_flag", n, &flag, s));
    ABD_TRY(ws(ctx, "frl_pos", n + 1, &pos, s));
    ABD_TRY(ws(ctx, "frl_tot", 2, &tot, s));
    ABD_TRY(op_friction_lag(ctx, sc, prm, xt, pt, npt, ee, nee, lam, T, w, s));
    hipLaunchKernelGGL(k_lam_flags, dim3(grid_for(n, 256)), dim3(256), 0, s, n, lam, flag);
    int64_t *h, *h_d;
    ABD_TRY(mirror_get(ctx, &h, &h_d));
    h += MIR_COMPACT;
    ABD_TRY(scan_exclusive_i64(ctx, flag, pos, n, tot, s, h_d + MIR_COMPACT, npt));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const int64_t keep = h[0], keep_pt = h[1];
    ABD_TRY(mirror_counts_ok(ctx, {keep, keep_pt}, "friction"));
    // the PT count the compaction needs is pos[npt] (or the total)
    const int64_t *n_keep_pt_dev = nee > 0 ? pos + npt : tot;
    int32_t *fpt, *fee;
    double *flam, *fT, *fw;
    ABD_TRY(ws(ctx, "fr_pt", 2 * keep_pt, &fpt, s));
    ABD_TRY(ws(ctx, "fr_ee", 2 * (keep - keep_pt), &fee, s));
    ABD_TRY(ws(ctx, "fr_lam", keep, &flam, s));
    ABD_TRY(ws(ctx, "fr_T", 6 * keep, &fT, s));
    ABD_TRY(ws(ctx, "fr_w", 4 * keep, &fw, s));
    hipLaunchKernelGGL(k_lam_compact, dim3(grid_for(n, 256)), dim3(256), 0, s, n, npt, pt, ee, flag, pos, lam, T, w,
                       n_keep_pt_dev, fpt, fee, flam, fT, fw);
    HIP_TRY(ctx, hipGetLastError());
    ctx->fr_n_pt = keep_pt;
    ctx->fr_n_ee = keep - keep_pt;
  }
  ctx->fr_set = true;
  return ABD_OK;
}

extern "C" int abd_friction_begin_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q,
                                       int64_t *n_pairs, hipStream_t stream) {
  if (!ctx || !sc || !prm || !q) return abd_fail(ctx, ABD_E_INVALID, "abd_friction_begin_step: null");
  ABD_TRY(friction_begin(ctx, sc, prm, q, stream));
  if (n_pairs) *n_pairs = ctx->fr_n_pt + ctx->fr_n_ee;
  return ABD_OK;
}

extern "C" int abd_friction_end_step(abd_ctx *ctx) {
  if (!ctx) return ABD_E_INVALID;
  ctx->fr_set = false;
  ctx->fr_n_pt = ctx->fr_n_ee = 0;
  return ABD_OK;
}
