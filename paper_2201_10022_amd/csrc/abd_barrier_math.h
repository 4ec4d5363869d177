// Pure arithmetic of the barrier pass (host- and device-callable): case
// derivatives of the squared distance, the clamped log barrier with the EE
// mollifier, the local 12x12 Hessian and its PSD projection.
#pragma once
#include "abd_internal.h"
#include "abd_jacobi.h"

namespace abd_math {

// ------------------------------------------------- case derivatives ----
// Distance of a case as the distance between affine hulls:
//   s = |r|^2,  r = sum_k w_k x_k  at the hull minimiser (parameters th).
// Envelope theorem: grad s = 2 w (x) r;  Hessian = 2 (w w^T (x) I3) -
// G_xth G_thth^-1 G_thx, where G = |r(x, th)|^2 with th free.
struct CaseDeriv {
  double w[4];
  double r[3];
  int nc;          // number of hull parameters (0, 1, 2)
  double C[2][12]; // G_x,th columns
  double Gi[3];    // inverse of G_thth (packed 2x2: 00, 01, 11)
};

__host__ __device__ __forceinline__ void set3(double *v, int k, d3 a, double f) {
  v[3 * k] = f * a.x;
  v[3 * k + 1] = f * a.y;
  v[3 * k + 2] = f * a.z;
}

__host__ __device__ __forceinline__ d3 lin(d3 a, double fa, d3 b, double fb) {
  return {fa * a.x + fb * b.x, fa * a.y + fb * b.y, fa * a.z + fb * b.z};
}

__host__ __device__ __forceinline__ void deriv_clear(CaseDeriv &cd) {
#pragma unroll
  for (int k = 0; k < 4; ++k) cd.w[k] = 0.0;
#pragma unroll
  for (int i = 0; i < 12; ++i) cd.C[0][i] = cd.C[1][i] = 0.0;
  cd.Gi[0] = cd.Gi[1] = cd.Gi[2] = 0.0;
}

// point-point (slots I, J): r = x_I - x_J
template <int I, int J>
__host__ __device__ __forceinline__ void deriv_pp(const d3 X[4], CaseDeriv &cd) {
  deriv_clear(cd);
  const d3 r = xsub(X[I], X[J]);
  cd.w[I] = 1.0;
  cd.w[J] = -1.0;
  cd.r[0] = r.x, cd.r[1] = r.y, cd.r[2] = r.z;
  cd.nc = 0;
}

// point-edge (point I, edge J -> K): r = x_I - x_J - t e
template <int I, int J, int K>
__host__ __device__ __forceinline__ void deriv_pe(const d3 X[4], CaseDeriv &cd) {
  deriv_clear(cd);
  const d3 e = xsub(X[K], X[J]);
  const d3 dp = xsub(X[I], X[J]);
  const double ee = e.x * e.x + e.y * e.y + e.z * e.z;
  const double t = (dp.x * e.x + dp.y * e.y + dp.z * e.z) / ee;
  // r = dp - t e written as e x (dp x e) / |e|^2 (no cancellation)
  const d3 rc = xcross(e, xcross(dp, e));
  const d3 r = {rc.x / ee, rc.y / ee, rc.z / ee};
  cd.w[I] = 1.0;
  cd.w[J] = -(1.0 - t);
  cd.w[K] = -t;
  cd.r[0] = r.x, cd.r[1] = r.y, cd.r[2] = r.z;
  cd.nc = 1;
  set3(cd.C[0], I, e, -2.0);
  set3(cd.C[0], J, lin(e, 1.0 - t, r, 1.0), 2.0);
  set3(cd.C[0], K, lin(e, t, r, -1.0), 2.0);
  cd.Gi[0] = 1.0 / (2.0 * ee);
}

// point-face: r = p - t0 - u e1 - v e2
__host__ __device__ __forceinline__ void deriv_face(const d3 X[4], CaseDeriv &cd) {
  deriv_clear(cd);
  const d3 e1 = xsub(X[2], X[1]), e2 = xsub(X[3], X[1]), dp = xsub(X[0], X[1]);
  const double a = e1.x * e1.x + e1.y * e1.y + e1.z * e1.z;
  const double b = e1.x * e2.x + e1.y * e2.y + e1.z * e2.z;
  const double c = e2.x * e2.x + e2.y * e2.y + e2.z * e2.z;
  // barycentric parameters and r from the normal n = e1 x e2 (Cramer's rule
  // written with cross products: better conditioned than the normal
  // equations, and det = |n|^2 exactly in exact arithmetic)
  const d3 n = xcross(e1, e2);
  const double det = xdot(n, n);
  const double u = xdot(xcross(dp, e2), n) / det, v = xdot(xcross(e1, dp), n) / det;
  const double hn = xdot(dp, n) / det;
  const d3 r = {hn * n.x, hn * n.y, hn * n.z};
  const double w0 = 1.0 - u - v;
  cd.w[0] = 1.0;
  cd.w[1] = -w0;
  cd.w[2] = -u;
  cd.w[3] = -v;
  cd.r[0] = r.x, cd.r[1] = r.y, cd.r[2] = r.z;
  cd.nc = 2;
  set3(cd.C[0], 0, e1, -2.0);
  set3(cd.C[0], 1, lin(e1, w0, r, 1.0), 2.0);
  set3(cd.C[0], 2, lin(e1, u, r, -1.0), 2.0);
  set3(cd.C[0], 3, e1, 2.0 * v);
  set3(cd.C[1], 0, e2, -2.0);
  set3(cd.C[1], 1, lin(e2, w0, r, 1.0), 2.0);
  set3(cd.C[1], 2, e2, 2.0 * u);
  set3(cd.C[1], 3, lin(e2, v, r, -1.0), 2.0);
  // G_thth = 2 [[a, b], [b, c]]
  const double id = 1.0 / (2.0 * det);
  cd.Gi[0] = c * id;
  cd.Gi[1] = -b * id;
  cd.Gi[2] = a * id;
}

// line-line: r = (a0 + s u) - (b0 + t v)
__host__ __device__ __forceinline__ void deriv_ll(const d3 X[4], CaseDeriv &cd) {
  deriv_clear(cd);
  const d3 u = xsub(X[1], X[0]), v = xsub(X[3], X[2]), w = xsub(X[0], X[2]);
  const double a = u.x * u.x + u.y * u.y + u.z * u.z;
  const double b = u.x * v.x + u.y * v.y + u.z * v.z;
  const double c = v.x * v.x + v.y * v.y + v.z * v.z;
  // with n = u x v: s = n.(v x w)/|n|^2, t = n.(u x w)/|n|^2 and the
  // closest-point difference r = (w.n/|n|^2) n (Lagrange's identity turns
  // the normal equations into these; they stay accurate for nearly
  // parallel edges, where a c - b^2 cancels)
  const d3 n = xcross(u, v);
  const double D = xdot(n, n);
  const double s = xdot(n, xcross(v, w)) / D, t = xdot(n, xcross(u, w)) / D;
  const double hn = xdot(w, n) / D;
  const d3 r = {hn * n.x, hn * n.y, hn * n.z};
  cd.w[0] = 1.0 - s;
  cd.w[1] = s;
  cd.w[2] = -(1.0 - t);
  cd.w[3] = -t;
  cd.r[0] = r.x, cd.r[1] = r.y, cd.r[2] = r.z;
  cd.nc = 2;
  set3(cd.C[0], 0, lin(u, 1.0 - s, r, -1.0), 2.0);
  set3(cd.C[0], 1, lin(u, s, r, 1.0), 2.0);
  set3(cd.C[0], 2, u, -2.0 * (1.0 - t));
  set3(cd.C[0], 3, u, -2.0 * t);
  set3(cd.C[1], 0, v, -2.0 * (1.0 - s));
  set3(cd.C[1], 1, v, -2.0 * s);
  set3(cd.C[1], 2, lin(v, 1.0 - t, r, 1.0), 2.0);
  set3(cd.C[1], 3, lin(v, t, r, -1.0), 2.0);
  // G_thth = 2 [[a, -b], [-b, c]]
  const double id = 1.0 / (2.0 * D);
  cd.Gi[0] = c * id;
  cd.Gi[1] = b * id;
  cd.Gi[2] = a * id;
}

__host__ __device__ inline void case_deriv(int type, const d3 X[4], CaseDeriv &cd) {
  switch (type) {
    case PT_PP0: deriv_pp<0, 1>(X, cd); break;
    case PT_PP1: deriv_pp<0, 2>(X, cd); break;
    case PT_PP2: deriv_pp<0, 3>(X, cd); break;
    case PT_PE01: deriv_pe<0, 1, 2>(X, cd); break;
    case PT_PE12: deriv_pe<0, 2, 3>(X, cd); break;
    case PT_PE02: deriv_pe<0, 1, 3>(X, cd); break;
    case PT_FACE: deriv_face(X, cd); break;
    case EE_BASE + 0: deriv_pp<0, 2>(X, cd); break;
    case EE_BASE + 1: deriv_pp<0, 3>(X, cd); break;
    case EE_BASE + 2: deriv_pe<0, 2, 3>(X, cd); break;
    case EE_BASE + 3: deriv_pp<1, 2>(X, cd); break;
    case EE_BASE + 4: deriv_pp<1, 3>(X, cd); break;
    case EE_BASE + 5: deriv_pe<1, 2, 3>(X, cd); break;
    case EE_BASE + 6: deriv_pp<2, 0>(X, cd); break;
    case EE_BASE + 7: deriv_pp<2, 1>(X, cd); break;
    case EE_BASE + 8: deriv_pe<2, 0, 1>(X, cd); break;
    case EE_BASE + 9: deriv_pp<3, 0>(X, cd); break;
    case EE_BASE + 10: deriv_pp<3, 1>(X, cd); break;
    case EE_BASE + 11: deriv_pe<3, 0, 1>(X, cd); break;
    default: deriv_ll(X, cd); break;
  }
}

using S12 = SymIdx<12>;
using S9 = SymIdx<9>;

// 4-point Helmert basis (rows orthonormal, orthogonal to (1,1,1,1))
__host__ __device__ __forceinline__ double helm(int m, int k) {
  const double s2 = 0.70710678118654752440, s6 = 0.40824829046386301637, s12 = 0.28867513459481288225;
  if (m == 0) return k == 0 ? s2 : (k == 1 ? -s2 : 0.0);
  if (m == 1) return k < 2 ? s6 : (k == 2 ? -2.0 * s6 : 0.0);
  return k < 3 ? s12 : -3.0 * s12;
}

struct LocalOut {
  double e;
  double g[12];
  double H[78];
};

__host__ __device__ inline void project_translation_invariant(double *H);

// local barrier energy, gradient and (projected) Hessian of one pair
__host__ __device__ inline void barrier_local(int is_ee, int type, const d3 X[4], const double *xb4, double dhat, double kappa,
                              int project, LocalOut &o) {
  double num, den;
  case_nd(type, X, num, den);
  const double s = num / den;
  const double d = sqrt(s);
  const double L = log(d / dhat), t = d - dhat;
  const double B = -t * t * L;
  const double B1 = -2.0 * t * L - t * t / d;
  const double B2 = -2.0 * L - 4.0 * t / d + t * t / (d * d);
  const double b1 = B1 / (2.0 * d);
  const double b2 = (B2 - B1 / d) / (4.0 * s);

  CaseDeriv cd;
  case_deriv(type, X, cd);
  double gs[12];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) gs[3 * k + c] = 2.0 * cd.w[k] * cd.r[c];

  // mollifier (EE): m(c) with c = |u x v|^2
  double m = 1.0, m1 = 0.0, m2 = 0.0;
  double gc[12];
  double uu = 0, vv = 0, uv = 0;
  d3 u = {0, 0, 0}, v = {0, 0, 0};
  bool moll = false;
#pragma unroll
  for (int i = 0; i < 12; ++i) gc[i] = 0.0;
  if (is_ee) {
    u = xsub(X[1], X[0]);
    v = xsub(X[3], X[2]);
    const d3 n = xcross(u, v);
    const double cval = xdot(n, n);
    const double la = (xb4[3] - xb4[0]) * (xb4[3] - xb4[0]) + (xb4[4] - xb4[1]) * (xb4[4] - xb4[1]) +
                      (xb4[5] - xb4[2]) * (xb4[5] - xb4[2]);
    const double lb = (xb4[9] - xb4[6]) * (xb4[9] - xb4[6]) + (xb4[10] - xb4[7]) * (xb4[10] - xb4[7]) +
                      (xb4[11] - xb4[8]) * (xb4[11] - xb4[8]);
    const double eps = (1e-3 * la) * lb;
    if (cval < eps) {
      moll = true;
      const double rr = cval / eps;
      m = (2.0 - rr) * rr;
      m1 = 2.0 * (1.0 - rr) / eps;
      m2 = -2.0 / (eps * eps);
      uu = u.x * u.x + u.y * u.y + u.z * u.z;
      vv = v.x * v.x + v.y * v.y + v.z * v.z;
      uv = u.x * v.x + u.y * v.y + u.z * v.z;
      // dc/du = 2 u (v.v) - 2 (u.v) v ; dc/dv = 2 v (u.u) - 2 (u.v) u
      const d3 cu = lin(u, 2.0 * vv, v, -2.0 * uv), cv = lin(v, 2.0 * uu, u, -2.0 * uv);
      set3(gc, 0, cu, -1.0);
      set3(gc, 1, cu, 1.0);
      set3(gc, 2, cv, -1.0);
      set3(gc, 3, cv, 1.0);
    }
  }
  o.e = kappa * m * B;
#pragma unroll
  for (int i = 0; i < 12; ++i) o.g[i] = kappa * (m * b1 * gs[i] + B * m1 * gc[i]);

  // Hessian (packed upper 12x12)
  const double fss = kappa * m * b2, fs = kappa * m * b1;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int l = k; l < 4; ++l)
#pragma unroll
        for (int c2 = 0; c2 < 3; ++c2) {
          const int i = 3 * k + c, j = 3 * l + c2;
          if (j < i) continue;
          // Hessian of s
          double hs = (c == c2) ? 2.0 * cd.w[k] * cd.w[l] : 0.0;
          if (cd.nc >= 1) hs -= cd.C[0][i] * cd.Gi[0] * cd.C[0][j];
          if (cd.nc == 2)
            hs -= cd.C[0][i] * cd.Gi[1] * cd.C[1][j] + cd.C[1][i] * cd.Gi[1] * cd.C[0][j] +
                  cd.C[1][i] * cd.Gi[2] * cd.C[1][j];
          o.H[S12::at(i, j)] = fss * gs[i] * gs[j] + fs * hs;
        }
  if (moll) {
    const double kb1 = kappa * m1 * b1, kB2 = kappa * B * m2, kB1 = kappa * B * m1;
    // d2c/du2 = 2 (v.v) I - 2 v v^T ; d2c/dv2 = 2 (u.u) I - 2 u u^T ;
    // d2c/du dv^T = 4 u v^T - 2 v u^T - 2 (u.v) I
    const double U[3] = {u.x, u.y, u.z}, V[3] = {v.x, v.y, v.z};
    const int sgn[4] = {-1, 1, -1, 1};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int l = k; l < 4; ++l)
#pragma unroll
          for (int c2 = 0; c2 < 3; ++c2) {
            const int i = 3 * k + c, j = 3 * l + c2;
            if (j < i) continue;
            double hc;
            const bool ku = k < 2, lu = l < 2;
            if (ku && lu)
              hc = 2.0 * vv * (c == c2 ? 1.0 : 0.0) - 2.0 * V[c] * V[c2];
            else if (!ku && !lu)
              hc = 2.0 * uu * (c == c2 ? 1.0 : 0.0) - 2.0 * U[c] * U[c2];
            else  // k in u-part, l in v-part (k <= l always puts u first)
              hc = 4.0 * U[c] * V[c2] - 2.0 * V[c] * U[c2] - 2.0 * uv * (c == c2 ? 1.0 : 0.0);
            hc *= sgn[k] * sgn[l];
            o.H[S12::at(i, j)] += kb1 * (gc[i] * gs[j] + gs[i] * gc[j]) + kB2 * gc[i] * gc[j] + kB1 * hc;
          }
  }
  if (project) project_translation_invariant(o.H);
}

// PSD projection of a packed 12x12 local Hessian whose null space holds the
// common translations of the 4 vertices: H = Q H9 Q^T with the 4-point
// Helmert basis Q (12x9), so H_+ = Q (H9)_+ Q^T.  In place.
__host__ __device__ inline void project_translation_invariant(double *H) {
  // H9 = Q^T H Q with Q[(k,c),(m,c)] = helm(m,k)
  double H9[45];
  {
    double T[9][12];  // T = Q^T H
#pragma unroll
    for (int mm = 0; mm < 3; ++mm)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < 12; ++j) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k) acc += helm(mm, k) * H[S12::at(3 * k + c, j)];
          T[3 * mm + c][j] = acc;
        }
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int mm = 0; mm < 3; ++mm)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int b = 3 * mm + c;
          if (b < a) continue;
          double acc = 0.0;
#pragma unroll
          for (int l = 0; l < 4; ++l) acc += T[a][3 * l + c] * helm(mm, l);
          H9[S9::at(a, b)] = acc;
        }
  }
  psd_project_packed<9>(H9);
  // H+ = Q H9+ Q^T
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int l = k; l < 4; ++l)
#pragma unroll
        for (int c2 = 0; c2 < 3; ++c2) {
          const int i = 3 * k + c, j = 3 * l + c2;
          if (j < i) continue;
          double acc = 0.0;
#pragma unroll
          for (int mm = 0; mm < 3; ++mm)
#pragma unroll
            for (int nn = 0; nn < 3; ++nn) acc += helm(mm, k) * helm(nn, l) * H9[S9::at(3 * mm + c, 3 * nn + c2)];
          H[S12::at(i, j)] = acc;
        }
}

}  // namespace abd_math
