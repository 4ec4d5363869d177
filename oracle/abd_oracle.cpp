// CPU reference ("oracle") for the affine-body contact path.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark load this library.  It shares no code with
// the GPU library and must never be called from the product path.
//
// Plain, slow, FP64 code written for checkability: every function follows
// one passage of Lan et al., "Affine Body Dynamics" (ABD), or the textbook
// definition that passage relies on, in the order the paper states it.
// Compiled with -O2 -ffp-contract=off -fno-fast-math so that the arithmetic
// written here is the arithmetic executed.  Per-pair loops run their pairs
// in parallel (OpenMP) where every pair's result is independent; sums over
// pairs are then taken in pair order, so every result is the same for any
// thread count.
//
// Derivatives of distances and barriers are NOT derived by hand here: a
// second-order forward-mode jet (value, gradient, full Hessian) is pushed
// through the closed-form distance of each case, so the oracle's
// derivatives are exact derivatives of the plain formulas.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include <omp.h>

namespace {

// ---------------------------------------------------------------- jets ----
constexpr int NJ = 12;  // 4 vertices x 3 coordinates

struct Jet {
  double v;
  double g[NJ];
  double h[NJ][NJ];
};

Jet jconst(double c) {
  Jet r;
  std::memset(&r, 0, sizeof(r));
  r.v = c;
  return r;
}
Jet jvar(double c, int i) {
  Jet r = jconst(c);
  r.g[i] = 1.0;
  return r;
}
Jet operator+(const Jet& a, const Jet& b) {
  Jet r;
  r.v = a.v + b.v;
  for (int i = 0; i < NJ; ++i) r.g[i] = a.g[i] + b.g[i];
  for (int i = 0; i < NJ; ++i)
    for (int j = 0; j < NJ; ++j) r.h[i][j] = a.h[i][j] + b.h[i][j];
  return r;
}
Jet operator-(const Jet& a, const Jet& b) {
  Jet r;
  r.v = a.v - b.v;
  for (int i = 0; i < NJ; ++i) r.g[i] = a.g[i] - b.g[i];
  for (int i = 0; i < NJ; ++i)
    for (int j = 0; j < NJ; ++j) r.h[i][j] = a.h[i][j] - b.h[i][j];
  return r;
}
Jet operator*(const Jet& a, const Jet& b) {
  Jet r;
  r.v = a.v * b.v;
  for (int i = 0; i < NJ; ++i) r.g[i] = a.v * b.g[i] + b.v * a.g[i];
  for (int i = 0; i < NJ; ++i)
    for (int j = 0; j < NJ; ++j)
      r.h[i][j] = a.v * b.h[i][j] + b.v * a.h[i][j] + a.g[i] * b.g[j] + b.g[i] * a.g[j];
  return r;
}
Jet scale(const Jet& a, double c) {
  Jet r;
  r.v = a.v * c;
  for (int i = 0; i < NJ; ++i) r.g[i] = a.g[i] * c;
  for (int i = 0; i < NJ; ++i)
    for (int j = 0; j < NJ; ++j) r.h[i][j] = a.h[i][j] * c;
  return r;
}
// f(a) given f(a.v), f'(a.v), f''(a.v)  (chain rule)
Jet unary(const Jet& a, double f, double df, double ddf) {
  Jet r;
  r.v = f;
  for (int i = 0; i < NJ; ++i) r.g[i] = df * a.g[i];
  for (int i = 0; i < NJ; ++i)
    for (int j = 0; j < NJ; ++j) r.h[i][j] = df * a.h[i][j] + ddf * a.g[i] * a.g[j];
  return r;
}
Jet operator/(const Jet& a, const Jet& b) {
  const double y = b.v;
  Jet inv = unary(b, 1.0 / y, -1.0 / (y * y), 2.0 / (y * y * y));
  return a * inv;
}
Jet jsqrt(const Jet& a) {
  const double s = std::sqrt(a.v);
  return unary(a, s, 0.5 / s, -0.25 / (s * a.v));
}
Jet jlog(const Jet& a) { return unary(a, std::log(a.v), 1.0 / a.v, -1.0 / (a.v * a.v)); }

// plain-double overloads so the distance formulas below are written once
inline double jsqrt(double a) { return std::sqrt(a); }
inline double scale(double a, double c) { return a * c; }

template <class T>
struct V3 {
  T x, y, z;
};
template <class T>
V3<T> sub(const V3<T>& a, const V3<T>& b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class T>
T dot(const V3<T>& a, const V3<T>& b) {
  return (a.x * b.x + a.y * b.y) + a.z * b.z;
}
template <class T>
V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// ------------------------------------------------------ distance cases ----
// Squared distance of each case as (numerator, denominator); the case's
// squared distance is num/den.  These are the closed forms of the distance
// between the affine hulls of the features involved.
template <class T>
void pp_nd(const V3<T>& a, const V3<T>& b, T& num, T& den, T one) {
  V3<T> d = sub(a, b);
  num = dot(d, d);
  den = one;
}
template <class T>
void pe_nd(const V3<T>& p, const V3<T>& e0, const V3<T>& e1, T& num, T& den) {
  V3<T> e = sub(e1, e0);
  V3<T> c = cross(sub(p, e0), e);
  num = dot(c, c);
  den = dot(e, e);
}
template <class T>
void ptf_nd(const V3<T>& p, const V3<T>& t0, const V3<T>& t1, const V3<T>& t2, T& num, T& den) {
  V3<T> n = cross(sub(t1, t0), sub(t2, t0));
  T h = dot(sub(p, t0), n);
  num = h * h;
  den = dot(n, n);
}
template <class T>
void ll_nd(const V3<T>& a0, const V3<T>& a1, const V3<T>& b0, const V3<T>& b1, T& num, T& den) {
  V3<T> n = cross(sub(a1, a0), sub(b1, b0));
  T h = dot(sub(b0, a0), n);
  num = h * h;
  den = dot(n, n);
}

// Distance case codes.  Local vertex slots: PT pair (p, t0, t1, t2) = 0..3,
// EE pair (a0, a1, b0, b1) = 0..3.
enum : int {
  PT_PP0 = 0, PT_PP1 = 1, PT_PP2 = 2, PT_PE01 = 3, PT_PE12 = 4, PT_PE02 = 5, PT_FACE = 6,
  EE_BASE = 16,  // 16 + 3k + sub, k = boundary side, sub 0/1 = PP with E0/E1, 2 = PE
  EE_LL = 28
};

// Case -> participating slots.  kind: 0 PP(i,j), 1 PE(i;j,k), 2 PT(0;1,2,3), 3 LL
struct CaseSlots {
  int kind, i, j, k, l;
};
CaseSlots case_slots(int type) {
  switch (type) {
    case PT_PP0: return {0, 0, 1, -1, -1};
    case PT_PP1: return {0, 0, 2, -1, -1};
    case PT_PP2: return {0, 0, 3, -1, -1};
    case PT_PE01: return {1, 0, 1, 2, -1};
    case PT_PE12: return {1, 0, 2, 3, -1};
    case PT_PE02: return {1, 0, 1, 3, -1};
    case PT_FACE: return {2, 0, 1, 2, 3};
    case EE_LL: return {3, 0, 1, 2, 3};
    default: break;
  }
  // EE boundary sides: k=0 point a0 vs segment (b0,b1); k=1 a1 vs (b0,b1);
  // k=2 b0 vs (a0,a1); k=3 b1 vs (a0,a1)
  const int k = (type - EE_BASE) / 3, sub = (type - EE_BASE) % 3;
  const int P[4] = {0, 1, 2, 3};
  const int E0[4] = {2, 2, 0, 0};
  const int E1[4] = {3, 3, 1, 1};
  if (sub == 0) return {0, P[k], E0[k], -1, -1};
  if (sub == 1) return {0, P[k], E1[k], -1, -1};
  return {1, P[k], E0[k], E1[k], -1};
}

template <class T>
void case_nd(int type, const V3<T> X[4], T& num, T& den, T one) {
  CaseSlots c = case_slots(type);
  switch (c.kind) {
    case 0: pp_nd(X[c.i], X[c.j], num, den, one); break;
    case 1: pe_nd(X[c.i], X[c.j], X[c.k], num, den); break;
    case 2: ptf_nd(X[0], X[1], X[2], X[3], num, den); break;
    default: ll_nd(X[0], X[1], X[2], X[3], num, den); break;
  }
}

typedef V3<double> D3;

// Point-triangle case classification: Voronoi regions of the triangle
// (vertex, edge, face) decided by sign tests of dot products, as in
// Ericson, Real-Time Collision Detection, sec. 5.1.5.  Ties go to the
// region tested first (vertices before edges before the face).
int classify_pt(const D3& p, const D3& t0, const D3& t1, const D3& t2) {
  D3 ab = sub(t1, t0), ac = sub(t2, t0);
  D3 ap = sub(p, t0);
  double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) return PT_PP0;
  D3 bp = sub(p, t1);
  double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) return PT_PP1;
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) return PT_PE01;
  D3 cp = sub(p, t2);
  double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) return PT_PP2;
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return PT_PE02;
  double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) return PT_PE12;
  return PT_FACE;
}

// point P vs segment (E0,E1): returns sub-case 0 (endpoint E0), 1 (E1), 2 (interior)
int classify_pseg(const D3& P, const D3& E0, const D3& E1) {
  D3 e = sub(E1, E0);
  double tn = dot(sub(P, E0), e);
  if (tn <= 0.0) return 0;
  if (tn >= dot(e, e)) return 1;
  return 2;
}

// Edge-edge case classification: if the unconstrained closest points of the
// two lines lie strictly inside both segments (and the lines are not
// parallel), the line-line case; otherwise the minimum over the four
// endpoint-versus-segment distances, compared without division, first
// minimum wins.
int classify_ee(const D3& a0, const D3& a1, const D3& b0, const D3& b1) {
  D3 u = sub(a1, a0), v = sub(b1, b0), w = sub(a0, b0);
  double a = dot(u, u), b = dot(u, v), c = dot(v, v), d = dot(u, w), e = dot(v, w);
  D3 n = cross(u, v);
  double nn = dot(n, n);
  double D = a * c - b * b;
  double sN = b * e - c * d, tN = a * e - b * d;
  if (nn > (1e-20 * a) * c && sN > 0.0 && sN < D && tN > 0.0 && tN < D) return EE_LL;
  const D3 X[4] = {a0, a1, b0, b1};
  int best = -1;
  double bn = 0.0, bd = 1.0;
  for (int k = 0; k < 4; ++k) {
    const int type = EE_BASE + 3 * k + classify_pseg(X[k], X[k < 2 ? 2 : 0], X[k < 2 ? 3 : 1]);
    double num, den;
    case_nd<double>(type, X, num, den, 1.0);
    if (best < 0 || num * bd < bn * den) {
      best = type;
      bn = num;
      bd = den;
    }
  }
  return best;
}

inline D3 ld3(const double* x, int v) { return {x[3 * v], x[3 * v + 1], x[3 * v + 2]}; }

// gathers the pair's 4 vertex ids in slot order
void pair_verts(int is_ee, const int32_t* pr, const int32_t* tris, const int32_t* edges, int vid[4]) {
  if (!is_ee) {
    const int t = pr[1];
    vid[0] = pr[0];
    vid[1] = tris[3 * t];
    vid[2] = tris[3 * t + 1];
    vid[3] = tris[3 * t + 2];
  } else {
    vid[0] = edges[2 * pr[0]];
    vid[1] = edges[2 * pr[0] + 1];
    vid[2] = edges[2 * pr[1]];
    vid[3] = edges[2 * pr[1] + 1];
  }
}

int classify(int is_ee, const D3 X[4]) {
  return is_ee ? classify_ee(X[0], X[1], X[2], X[3]) : classify_pt(X[0], X[1], X[2], X[3]);
}

double pair_dist(int is_ee, const D3 X[4]) {
  const int type = classify(is_ee, X);
  double num, den;
  case_nd<double>(type, X, num, den, 1.0);
  return std::sqrt(num / den);
}

// ---------------------------------------------------- symmetric eigen ----
// Cyclic Jacobi eigenvalue iteration (Golub & Van Loan, sec. 8.5): sweeps of
// plane rotations zeroing each off-diagonal entry in row order until the
// off-diagonal mass is negligible.  A is overwritten with (almost) diagonal
// form; V accumulates the rotations (columns are eigenvectors).
void jacobi_eig(int n, double* A, double* V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  double frob = 0.0;
  for (int i = 0; i < n * n; ++i) frob += A[i] * A[i];
  if (frob == 0.0) return;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off <= 1e-36 * frob) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        // symmetric 2x2 Schur decomposition
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t;
        if (std::fabs(theta) > 1e150)
          t = 0.5 / theta;
        else
          t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // A <- G^T A G with G the rotation in the (p,q) plane
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

// H <- sum over positive eigenvalues of lambda v v^T  (nearest PSD matrix in
// the Frobenius norm; projected Newton of IPC)
void psd_project(int n, double* H) {
  std::vector<double> A(H, H + n * n), V(n * n);
  jacobi_eig(n, A.data(), V.data());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) {
        const double lam = A[k * n + k];
        if (lam > 0.0) s += lam * V[i * n + k] * V[j * n + k];
      }
      H[i * n + j] = s;
    }
}

// ------------------------------------------------------------ barrier ----
// Clamped log barrier of the paper:  B(d) = -(d - dhat)^2 ln(d / dhat) on
// 0 < d < dhat, zero beyond.  Evaluated on a jet of d = sqrt(s).
Jet barrier_jet(const Jet& s, double dhat) {
  Jet d = jsqrt(s);
  Jet t = d - jconst(dhat);
  Jet l = jlog(scale(d, 1.0 / dhat));
  return scale(t * t * l, -1.0);
}

// EE mollifier (IPC): m(c) = (2 - c/eps) c/eps for c < eps, else 1, with
// c = |(a1-a0) x (b1-b0)|^2
Jet mollifier_jet(const V3<Jet> X[4], double eps) {
  V3<Jet> n = cross(sub(X[1], X[0]), sub(X[3], X[2]));
  Jet c = dot(n, n);
  if (c.v >= eps) return jconst(1.0);
  Jet r = scale(c, 1.0 / eps);
  return (jconst(2.0) - r) * r;
}

struct Scene {
  const double* xbar;
  const int32_t* vert_body;
  const int32_t* tris;
  const int32_t* edges;
  const uint8_t* fixed;
};

// Local (vertex-space) barrier energy, gradient, Hessian of one active pair.
void pair_local(int is_ee, int type, const D3 Xd[4], const double* xb4[4], double dhat, double kappa,
                double* e, double* g, double* H) {
  V3<Jet> X[4];
  for (int k = 0; k < 4; ++k)
    X[k] = {jvar(Xd[k].x, 3 * k), jvar(Xd[k].y, 3 * k + 1), jvar(Xd[k].z, 3 * k + 2)};
  Jet num, den;
  case_nd<Jet>(type, X, num, den, jconst(1.0));
  Jet s = num / den;
  Jet b = barrier_jet(s, dhat);
  if (is_ee) {
    // eps_x = 1e-3 |abar|^2 |bbar|^2 from rest-frame edge vectors
    double la = 0.0, lb = 0.0;
    {
      const double* a0 = xb4[0];
      const double* a1 = xb4[1];
      const double* b0 = xb4[2];
      const double* b1 = xb4[3];
      D3 u{a1[0] - a0[0], a1[1] - a0[1], a1[2] - a0[2]};
      D3 v{b1[0] - b0[0], b1[1] - b0[1], b1[2] - b0[2]};
      la = dot(u, u);
      lb = dot(v, v);
    }
    const double eps = (1e-3 * la) * lb;
    b = mollifier_jet(X, eps) * b;
  }
  b = scale(b, kappa);
  *e = b.v;
  for (int i = 0; i < NJ; ++i) g[i] = b.g[i];
  for (int i = 0; i < NJ; ++i)
    for (int j = 0; j < NJ; ++j) H[i * NJ + j] = b.h[i][j];
}

// J(xbar) of the kinematic map x = A xbar + p, with q = (p, a1, a2, a3) and
// a_i the rows of A:  row i has 1 at p_i and xbar^T at a_i.
void kin_jacobian(const double* xb, double J[3][12]) {
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 12; ++c) J[i][c] = 0.0;
  for (int i = 0; i < 3; ++i) {
    J[i][i] = 1.0;
    for (int m = 0; m < 3; ++m) J[i][3 + 3 * i + m] = xb[m];
  }
}

int find_off(const int32_t* keys, int64_t n_off, int a, int b) {
  // keys: [n_off][2] sorted (a<b) lexicographic
  int64_t lo = 0, hi = n_off;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    const int ka = keys[2 * mid], kb = keys[2 * mid + 1];
    if (ka < a || (ka == a && kb < b))
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < n_off && keys[2 * lo] == a && keys[2 * lo + 1] == b) return (int)lo;
  return -1;
}

}  // namespace

extern "C" {

// Threads the parallel loops below run on (OpenMP's current maximum).
int ora_threads() { return omp_get_max_threads(); }

// Mass properties (ABD, kinetic energy section, Eq. mass): M = int rho J^T J,
// needing m = int rho, the first moment h = int rho xbar and the second
// moment S = int rho xbar xbar^T, plus the volume nu (orthogonality
// potential).  Integrals by the divergence theorem: each outward-oriented
// triangle (v0,v1,v2) with the origin spans a signed tetrahedron of volume
// v0.(v1 x v2)/6, centroid-weighted first moment vol (v0+v1+v2)/4 and second
// moment vol/20 (sum v_i v_i^T + (sum v_i)(sum v_i)^T).
// out: mass[nb][10] = (m, h0,h1,h2, Sxx,Sxy,Sxz,Syy,Syz,Szz), volume[nb].
// Fixed bodies get zeros.
void ora_mass(int nb, const int32_t* body_tri_off, const int32_t* tris, const double* xbar,
              const double* density, const uint8_t* fixed, double* mass, double* volume) {
  for (int b = 0; b < nb; ++b) {
    double vol = 0.0, h[3] = {0, 0, 0}, S[3][3] = {{0}};
    if (!fixed[b]) {
      for (int t = body_tri_off[b]; t < body_tri_off[b + 1]; ++t) {
        D3 v0 = ld3(xbar, tris[3 * t]), v1 = ld3(xbar, tris[3 * t + 1]), v2 = ld3(xbar, tris[3 * t + 2]);
        const double vt = dot(v0, cross(v1, v2)) / 6.0;
        const double s[3] = {v0.x + v1.x + v2.x, v0.y + v1.y + v2.y, v0.z + v1.z + v2.z};
        const double a0[3] = {v0.x, v0.y, v0.z}, a1[3] = {v1.x, v1.y, v1.z}, a2[3] = {v2.x, v2.y, v2.z};
        vol += vt;
        for (int i = 0; i < 3; ++i) h[i] += vt * s[i] / 4.0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            S[i][j] += vt / 20.0 * (a0[i] * a0[j] + a1[i] * a1[j] + a2[i] * a2[j] + s[i] * s[j]);
      }
    }
    const double rho = fixed[b] ? 0.0 : density[b];
    double* o = mass + 10 * b;
    o[0] = rho * vol;
    o[1] = rho * h[0];
    o[2] = rho * h[1];
    o[3] = rho * h[2];
    o[4] = rho * S[0][0];
    o[5] = rho * S[0][1];
    o[6] = rho * S[0][2];
    o[7] = rho * S[1][1];
    o[8] = rho * S[1][2];
    o[9] = rho * S[2][2];
    volume[b] = fixed[b] ? 0.0 : vol;
  }
}

// Kinematic map (ABD Eq. kinematic): x_k = A_b xbar_k + p_b, component
// i evaluated as p_i + ((a_i0 xbar_0 + a_i1 xbar_1) + a_i2 xbar_2).
void ora_vertex_map(int nv, const double* xbar, const int32_t* vert_body, const double* q, double* x) {
  for (int k = 0; k < nv; ++k) {
    const double* qb = q + 12 * vert_body[k];
    const double* xb = xbar + 3 * k;
    for (int i = 0; i < 3; ++i) {
      const double* a = qb + 3 + 3 * i;
      x[3 * k + i] = qb[i] + ((a[0] * xb[0] + a[1] * xb[1]) + a[2] * xb[2]);
    }
  }
}

// Candidate pairs (ABD sec. 4.2, i-AABB culling; the set is defined by the
// primitive-box predicate, the culling only has to be exact for it).
// A primitive's box spans its vertices at x0 and x1; a pair is a candidate
// iff the primitives belong to different bodies of the same scene, not both
// fixed, and on every axis lo_a <= hi_b + inflate and lo_b <= hi_a + inflate.
// Here the exact filter is the same predicate applied to whole-body boxes,
// then every primitive pair of overlapping bodies is tested.
// PT output (v, t) for vertices of either body against triangles of the
// other; EE output (e_lo, e_hi).  Both sorted ascending.  Returns 0, or -2
// when a capacity is exceeded (counts still reported).
int ora_candidates(int nb, int nv, int nt, int ne, const int32_t* body_vert_off, const int32_t* body_tri_off,
                   const int32_t* body_edge_off, const int32_t* tris, const int32_t* edges, const uint8_t* fixed,
                   const int32_t* body_scene, const double* x0, const double* x1, double inflate, int32_t* pt,
                   int64_t cap_pt, int64_t* n_pt, int32_t* ee, int64_t cap_ee, int64_t* n_ee) {
  (void)nv;
  if (x1 == nullptr) x1 = x0;
  auto vbox = [&](int v, double lo[3], double hi[3]) {
    for (int i = 0; i < 3; ++i) {
      lo[i] = std::min(x0[3 * v + i], x1[3 * v + i]);
      hi[i] = std::max(x0[3 * v + i], x1[3 * v + i]);
    }
  };
  auto grow = [&](int v, double lo[3], double hi[3]) {
    double l[3], h[3];
    vbox(v, l, h);
    for (int i = 0; i < 3; ++i) {
      lo[i] = std::min(lo[i], l[i]);
      hi[i] = std::max(hi[i], h[i]);
    }
  };
  std::vector<double> tb(6 * (size_t)nt), eb(6 * (size_t)ne), vb(6 * (size_t)body_vert_off[nb]);
  for (int v = 0; v < body_vert_off[nb]; ++v) vbox(v, &vb[6 * v], &vb[6 * v + 3]);
  for (int t = 0; t < nt; ++t) {
    double* b = &tb[6 * (size_t)t];
    vbox(tris[3 * t], b, b + 3);
    grow(tris[3 * t + 1], b, b + 3);
    grow(tris[3 * t + 2], b, b + 3);
  }
  for (int e = 0; e < ne; ++e) {
    double* b = &eb[6 * (size_t)e];
    vbox(edges[2 * e], b, b + 3);
    grow(edges[2 * e + 1], b, b + 3);
  }
  auto overlap = [&](const double* a, const double* b) {
    for (int i = 0; i < 3; ++i) {
      if (!(a[i] <= b[3 + i] + inflate)) return false;
      if (!(b[i] <= a[3 + i] + inflate)) return false;
    }
    return true;
  };
  std::vector<double> bb(6 * (size_t)nb);
  for (int b = 0; b < nb; ++b) {
    double* o = &bb[6 * b];
    for (int i = 0; i < 3; ++i) {
      o[i] = INFINITY;
      o[3 + i] = -INFINITY;
    }
    for (int v = body_vert_off[b]; v < body_vert_off[b + 1]; ++v)
      for (int i = 0; i < 3; ++i) {
        o[i] = std::min(o[i], vb[6 * v + i]);
        o[3 + i] = std::max(o[3 + i], vb[6 * v + 3 + i]);
      }
  }
  // body pairs split over threads; the lists are sorted afterwards, so the
  // result does not depend on the split
  std::vector<std::pair<int32_t, int32_t>> P, E;
#pragma omp parallel if (nb >= 64)
  {
    std::vector<std::pair<int32_t, int32_t>> Pl, El;
#pragma omp for schedule(dynamic, 4) nowait
    for (int a = 0; a < nb; ++a)
      for (int b = a + 1; b < nb; ++b) {
        if (body_scene[a] != body_scene[b]) continue;
        if (fixed[a] && fixed[b]) continue;
        if (!overlap(&bb[6 * a], &bb[6 * b])) continue;
        for (int s = 0; s < 2; ++s) {
          const int bv = s ? b : a, bt = s ? a : b;
          for (int v = body_vert_off[bv]; v < body_vert_off[bv + 1]; ++v)
            for (int t = body_tri_off[bt]; t < body_tri_off[bt + 1]; ++t)
              if (overlap(&vb[6 * v], &tb[6 * (size_t)t])) Pl.push_back({v, t});
        }
        for (int e = body_edge_off[a]; e < body_edge_off[a + 1]; ++e)
          for (int f = body_edge_off[b]; f < body_edge_off[b + 1]; ++f)
            if (overlap(&eb[6 * (size_t)e], &eb[6 * (size_t)f])) El.push_back({std::min(e, f), std::max(e, f)});
      }
#pragma omp critical
    {
      P.insert(P.end(), Pl.begin(), Pl.end());
      E.insert(E.end(), El.begin(), El.end());
    }
  }
  std::sort(P.begin(), P.end());
  std::sort(E.begin(), E.end());
  *n_pt = (int64_t)P.size();
  *n_ee = (int64_t)E.size();
  if ((int64_t)P.size() > cap_pt || (int64_t)E.size() > cap_ee) return -2;
  for (size_t i = 0; i < P.size(); ++i) {
    pt[2 * i] = P[i].first;
    pt[2 * i + 1] = P[i].second;
  }
  for (size_t i = 0; i < E.size(); ++i) {
    ee[2 * i] = E[i].first;
    ee[2 * i + 1] = E[i].second;
  }
  return 0;
}

// Narrow phase: distance case, squared distance num/den and the active flag
// (num < dhat^2 den, i.e. d < dhat, decided without division).
void ora_classify(int64_t n, int is_ee, const int32_t* pairs, const int32_t* tris, const int32_t* edges,
                  const double* x, double dhat, uint8_t* type, double* d2, uint8_t* active) {
  const double dhat2 = dhat * dhat;
#pragma omp parallel for schedule(static) if (n >= 4096)
  for (int64_t i = 0; i < n; ++i) {
    int vid[4];
    pair_verts(is_ee, pairs + 2 * i, tris, edges, vid);
    D3 X[4];
    for (int k = 0; k < 4; ++k) X[k] = ld3(x, vid[k]);
    const int ty = classify(is_ee, X);
    double num, den;
    case_nd<double>(ty, X, num, den, 1.0);
    type[i] = (uint8_t)ty;
    d2[i] = num / den;
    active[i] = num < dhat2 * den ? 1 : 0;
  }
}

// Barrier term of one pair list (ABD Eq. barrier and Eq. clamped-b, EE
// mollified): energy kappa * sum m B(d); local gradient and PSD-projected
// local Hessian; J^T g and J^T H J (J of Eq. kinematic per vertex)
// accumulated into body gradient grad[nb][12], diagonal blocks diag[nb][144]
// and off-diagonal blocks off[n_off][144] keyed (a<b) by off_keys.
// Contributions to fixed bodies are dropped.  If `local_H` is non-null, the
// projected local Hessians (12x12) of every pair are stored there (zeros for
// inactive pairs), and `local_g` likewise.  project = 0 skips the PSD
// projection.  Returns the number of active pairs, or -3 when a pair has
// zero distance.
int64_t ora_barrier(int64_t n, int is_ee, const int32_t* pairs, const int32_t* vert_body, const int32_t* tris,
                    const int32_t* edges, const uint8_t* fixed, const double* xbar, const double* x, double dhat,
                    double kappa, int project, double* energy, double* grad, double* diag, double* off,
                    const int32_t* off_keys, int64_t n_off, double* local_g, double* local_H) {
  const double dhat2 = dhat * dhat;
  int64_t n_active = 0;
  double esum = 0.0;
  // pairs are evaluated a chunk at a time (in parallel), then their
  // contributions are added in pair order
  constexpr int64_t CH = 1024;
  struct PairOut {
    int status;  // 0 inactive, 1 active, -3 zero distance
    int ba, bo;
    double e, G[24], HH[24][24];
  };
  std::vector<PairOut> out((size_t)std::min<int64_t>(CH, std::max<int64_t>(n, 1)));
  for (int64_t c0 = 0; c0 < n; c0 += CH) {
    const int64_t m = std::min(CH, n - c0);
#pragma omp parallel for schedule(dynamic, 8) if (m >= 64)
    for (int64_t j = 0; j < m; ++j) {
      const int64_t i = c0 + j;
      PairOut& o = out[(size_t)j];
      int vid[4];
      pair_verts(is_ee, pairs + 2 * i, tris, edges, vid);
      D3 X[4];
      const double* xb4[4];
      for (int k = 0; k < 4; ++k) {
        X[k] = ld3(x, vid[k]);
        xb4[k] = xbar + 3 * vid[k];
      }
      const int ty = classify(is_ee, X);
      double num, den;
      case_nd<double>(ty, X, num, den, 1.0);
      if (local_H) std::memset(local_H + 144 * i, 0, 144 * sizeof(double));
      if (local_g) std::memset(local_g + 12 * i, 0, 12 * sizeof(double));
      o.status = 0;
      if (!(num < dhat2 * den)) continue;
      if (num == 0.0) {
        o.status = -3;
        continue;
      }
      o.status = 1;
      double g[12], H[144];
      pair_local(is_ee, ty, X, xb4, dhat, kappa, &o.e, g, H);
      if (project) psd_project(12, H);
      if (local_H) std::memcpy(local_H + 144 * i, H, sizeof(H));
      if (local_g) std::memcpy(local_g + 12 * i, g, sizeof(g));
      // 12 x 24 pair Jacobian: body slot 0 = body of vertex slot 0, slot 1 =
      // the other body
      const int ba = vert_body[vid[0]], bo = vert_body[vid[3]];
      o.ba = ba;
      o.bo = bo;
      double Jp[12][24];
      for (int r = 0; r < 12; ++r)
        for (int c = 0; c < 24; ++c) Jp[r][c] = 0.0;
      for (int k = 0; k < 4; ++k) {
        const int slot = vert_body[vid[k]] == ba ? 0 : 1;
        double J[3][12];
        kin_jacobian(xb4[k], J);
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 12; ++c) Jp[3 * k + r][12 * slot + c] = J[r][c];
      }
      for (int c = 0; c < 24; ++c) {
        double sum = 0.0;
        for (int r = 0; r < 12; ++r) sum += Jp[r][c] * g[r];
        o.G[c] = sum;
      }
      for (int c = 0; c < 24; ++c)
        for (int d = 0; d < 24; ++d) {
          double sum = 0.0;
          for (int r = 0; r < 12; ++r)
            for (int t = 0; t < 12; ++t) sum += Jp[r][c] * H[r * 12 + t] * Jp[t][d];
          o.HH[c][d] = sum;
        }
    }
    for (int64_t j = 0; j < m; ++j) {
      const PairOut& o = out[(size_t)j];
      if (o.status == -3) return -3;
      if (o.status == 0) continue;
      ++n_active;
      esum += o.e;
      const int bodies[2] = {o.ba, o.bo};
      for (int sa = 0; sa < 2; ++sa) {
        const int b = bodies[sa];
        if (fixed[b]) continue;
        for (int c = 0; c < 12; ++c) grad[12 * b + c] += o.G[12 * sa + c];
        for (int c = 0; c < 12; ++c)
          for (int d = 0; d < 12; ++d) diag[144 * b + 12 * c + d] += o.HH[12 * sa + c][12 * sa + d];
      }
      if (!fixed[o.ba] && !fixed[o.bo] && off) {
        const int lo = std::min(o.ba, o.bo), hi = std::max(o.ba, o.bo);
        const int k = find_off(off_keys, n_off, lo, hi);
        if (k < 0) return -1;
        const int sl = (lo == o.ba) ? 0 : 1, sh = 1 - sl;
        for (int c = 0; c < 12; ++c)
          for (int d = 0; d < 12; ++d) off[144 * (int64_t)k + 12 * c + d] += o.HH[12 * sl + c][12 * sh + d];
      }
    }
  }
  *energy += esum;
  return n_active;
}

// Barrier energy only (line search): kappa * sum m B(d) over active pairs.
double ora_barrier_energy(int64_t n, int is_ee, const int32_t* pairs, const int32_t* tris, const int32_t* edges,
                          const double* xbar, const double* x, double dhat, double kappa, int* status) {
  const double dhat2 = dhat * dhat;
  // per-pair terms in parallel (NaN marks a pair at zero distance), summed
  // in pair order
  std::vector<double> term((size_t)std::max<int64_t>(n, 1), 0.0);
#pragma omp parallel for schedule(static) if (n >= 1024)
  for (int64_t i = 0; i < n; ++i) {
    int vid[4];
    pair_verts(is_ee, pairs + 2 * i, tris, edges, vid);
    D3 X[4];
    const double* xb4[4];
    for (int k = 0; k < 4; ++k) {
      X[k] = ld3(x, vid[k]);
      xb4[k] = xbar + 3 * vid[k];
    }
    const int ty = classify(is_ee, X);
    double num, den;
    case_nd<double>(ty, X, num, den, 1.0);
    if (!(num < dhat2 * den)) continue;
    if (num == 0.0) {
      term[(size_t)i] = NAN;
      continue;
    }
    const double s = num / den, d = std::sqrt(s);
    double b = -(d - dhat) * (d - dhat) * std::log(d / dhat);
    if (is_ee) {
      D3 n3 = cross(sub(X[1], X[0]), sub(X[3], X[2]));
      const double c = dot(n3, n3);
      D3 u{xb4[1][0] - xb4[0][0], xb4[1][1] - xb4[0][1], xb4[1][2] - xb4[0][2]};
      D3 v{xb4[3][0] - xb4[2][0], xb4[3][1] - xb4[2][1], xb4[3][2] - xb4[2][2]};
      const double eps = (1e-3 * dot(u, u)) * dot(v, v);
      if (c < eps) {
        const double r = c / eps;
        b = (2.0 - r) * r * b;
      }
    }
    term[(size_t)i] = kappa * b;
  }
  double esum = 0.0;
  *status = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (std::isnan(term[(size_t)i])) {
      *status = -3;
      return INFINITY;
    }
    esum += term[(size_t)i];
  }
  return esum;
}

// Additive CCD (ACCD; Li et al. 2021, which ABD sec. 4.1 uses for all affine
// CCD) along the linear trajectories x + t dx of sec. 4.1.  The mean
// displacement of the 4 vertices is removed; l_p bounds the closing speed by
// the largest displacement on each side; t advances by safe increments
// (1-s) d0 / l_p first and 0.9 d / l_p after, until the distance falls
// below s d0 (the last safe t is returned) or t exceeds tmax (tmax is
// returned).  A capped iteration count returns the current (safe) t.
void ora_ccd(int64_t n, int is_ee, const int32_t* pairs, const int32_t* tris, const int32_t* edges,
             const double* x, const double* dx, double s, double tmax, int max_iter, double* tout,
             int32_t* iters_out) {
#pragma omp parallel for schedule(dynamic, 64) if (n >= 1024)
  for (int64_t i = 0; i < n; ++i) {
    int vid[4];
    pair_verts(is_ee, pairs + 2 * i, tris, edges, vid);
    D3 X[4], U[4];
    for (int k = 0; k < 4; ++k) {
      X[k] = ld3(x, vid[k]);
      U[k] = ld3(dx, vid[k]);
    }
    const D3 mean{((U[0].x + U[1].x) + (U[2].x + U[3].x)) * 0.25, ((U[0].y + U[1].y) + (U[2].y + U[3].y)) * 0.25,
                  ((U[0].z + U[1].z) + (U[2].z + U[3].z)) * 0.25};
    double len[4];
    for (int k = 0; k < 4; ++k) {
      U[k] = sub(U[k], mean);
      len[k] = std::sqrt(dot(U[k], U[k]));
    }
    double lp;
    if (!is_ee)
      lp = len[0] + std::max(len[1], std::max(len[2], len[3]));
    else
      lp = std::max(len[0], len[1]) + std::max(len[2], len[3]);
    if (iters_out) iters_out[i] = 0;
    if (lp == 0.0) {
      tout[i] = tmax;
      continue;
    }
    const double d0 = pair_dist(is_ee, X);
    if (d0 == 0.0) {
      tout[i] = 0.0;
      continue;
    }
    const double gap = s * d0;
    double t = 0.0, tl = (1.0 - s) * d0 / lp;
    int it = 0;
    for (;;) {
      for (int k = 0; k < 4; ++k) X[k] = {X[k].x + tl * U[k].x, X[k].y + tl * U[k].y, X[k].z + tl * U[k].z};
      const double d = pair_dist(is_ee, X);
      if (t > 0.0 && d < gap) break;
      t += tl;
      if (t > tmax) {
        t = tmax;
        break;
      }
      if (++it >= max_iter) break;
      tl = 0.9 * d / lp;
    }
    tout[i] = t;
    if (iters_out) iters_out[i] = it;
  }
}

// Orthogonality potential (ABD Eq. orthogonality, ortho-energy,
// ortho-poly): V = kappa nu (sum_i (a_i.a_i - 1)^2 + sum_{i!=j} (a_i.a_j)^2),
// gradient 4 kappa nu ((a_i.a_i - 1) a_i + sum_{j!=i} (a_i.a_j) a_j),
// diagonal blocks 2 kappa nu (4 a_i a_i^T + 2(|a_i|^2-1) I + 2 sum_{j!=i}
// a_j a_j^T), off-diagonal blocks 4 kappa nu ((a_i.a_j) I + a_j a_i^T).
// Scaled by `w` (dt^2 in the incremental potential).  The 9x9 A-block is
// PSD-projected when project != 0.  Accumulates; fixed bodies skipped.
void ora_orthogonality(int nb, const uint8_t* fixed, const double* volume, const double* q, double kappa, double w,
                       int project, double* energy, double* grad, double* diag) {
  double esum = 0.0;
  for (int b = 0; b < nb; ++b) {
    if (fixed[b]) continue;
    const double* A = q + 12 * b + 3;  // a_i = A + 3i
    const double kn = kappa * volume[b];
    double dots[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) dots[i][j] = (A[3 * i] * A[3 * j] + A[3 * i + 1] * A[3 * j + 1]) + A[3 * i + 2] * A[3 * j + 2];
    double V = 0.0;
    for (int i = 0; i < 3; ++i) V += (dots[i][i] - 1.0) * (dots[i][i] - 1.0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (i != j) V += dots[i][j] * dots[i][j];
    esum += w * kn * V;
    for (int i = 0; i < 3; ++i)
      for (int c = 0; c < 3; ++c) {
        double gi = (dots[i][i] - 1.0) * A[3 * i + c];
        for (int j = 0; j < 3; ++j)
          if (j != i) gi += dots[i][j] * A[3 * j + c];
        grad[12 * b + 3 + 3 * i + c] += w * 4.0 * kn * gi;
      }
    double H9[81];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) {
            double h;
            if (i == j) {
              h = 4.0 * A[3 * i + r] * A[3 * i + c] + (r == c ? 2.0 * (dots[i][i] - 1.0) : 0.0);
              for (int k = 0; k < 3; ++k)
                if (k != i) h += 2.0 * A[3 * k + r] * A[3 * k + c];
              h *= 2.0 * kn;
            } else {
              h = 4.0 * kn * ((r == c ? dots[i][j] : 0.0) + A[3 * j + r] * A[3 * i + c]);
            }
            H9[(3 * i + r) * 9 + 3 * j + c] = w * h;
          }
    if (project) psd_project(9, H9);
    for (int r = 0; r < 9; ++r)
      for (int c = 0; c < 9; ++c) diag[144 * b + 12 * (3 + r) + 3 + c] += H9[r * 9 + c];
  }
  *energy += esum;
}

// Orthogonality energy only.
double ora_orthogonality_energy(int nb, const uint8_t* fixed, const double* volume, const double* q, double kappa,
                                double w) {
  double esum = 0.0;
  for (int b = 0; b < nb; ++b) {
    if (fixed[b]) continue;
    const double* A = q + 12 * b + 3;
    double V = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double d = (A[3 * i] * A[3 * j] + A[3 * i + 1] * A[3 * j + 1]) + A[3 * i + 2] * A[3 * j + 2];
        V += (i == j) ? (d - 1.0) * (d - 1.0) : d * d;
      }
    esum += w * kappa * volume[b] * V;
  }
  return esum;
}

}  // extern "C"

namespace {

// ------------------------------------------------------------ friction ----
// Lagged friction (ABD sec. 4, friction potential V_F = sum mu lambda_j
// m_j(q) over the active pairs; details follow IPC's lagged model): at the
// step start x^t every active pair gets the normal-force magnitude
// lambda = -kappa m B'(d) (m = EE mollifier, held fixed), the closest-point
// weights w (the point on each primitive nearest the other, as weights of the
// 4 vertices with r = sum w_k x_k the closest-point difference) and a tangent
// basis T (3x2) orthogonal to r.  T: n = r/|r|; t1 = n x e_a / |n x e_a| with
// e_a the coordinate axis of smallest |n_a| (first on ties); t2 = n x t1.
void closest_weights(int type, const D3 X[4], double w[4]) {
  for (int k = 0; k < 4; ++k) w[k] = 0.0;
  CaseSlots c = case_slots(type);
  if (c.kind == 0) {
    w[c.i] = 1.0;
    w[c.j] = -1.0;
  } else if (c.kind == 1) {
    // closest point on the edge's line: parameter t of (x_i - x_j).e / e.e
    D3 e = sub(X[c.k], X[c.j]);
    const double t = dot(sub(X[c.i], X[c.j]), e) / dot(e, e);
    w[c.i] = 1.0;
    w[c.j] = -(1.0 - t);
    w[c.k] = -t;
  } else if (c.kind == 2) {
    // barycentric coordinates of the projection: normal equations
    D3 e1 = sub(X[2], X[1]), e2 = sub(X[3], X[1]), dp = sub(X[0], X[1]);
    const double a = dot(e1, e1), b = dot(e1, e2), cc = dot(e2, e2), f1 = dot(e1, dp), f2 = dot(e2, dp);
    const double det = a * cc - b * b;
    const double u = (cc * f1 - b * f2) / det, v = (a * f2 - b * f1) / det;
    w[0] = 1.0;
    w[1] = -(1.0 - u - v);
    w[2] = -u;
    w[3] = -v;
  } else {
    // closest points of the two lines: normal equations
    D3 u = sub(X[1], X[0]), v = sub(X[3], X[2]), r0 = sub(X[0], X[2]);
    const double a = dot(u, u), b = dot(u, v), cc = dot(v, v), d = dot(u, r0), e = dot(v, r0);
    const double den = a * cc - b * b;
    const double s = (b * e - cc * d) / den, t = (a * e - b * d) / den;
    w[0] = 1.0 - s;
    w[1] = s;
    w[2] = -(1.0 - t);
    w[3] = -t;
  }
}

void tangent_basis(const D3& r, double T[6]) {
  const double nr = std::sqrt(dot(r, r));
  const D3 n{r.x / nr, r.y / nr, r.z / nr};
  const double an[3] = {std::fabs(n.x), std::fabs(n.y), std::fabs(n.z)};
  int a = 0;
  if (an[1] < an[a]) a = 1;
  if (an[2] < an[a]) a = 2;
  const D3 ea{a == 0 ? 1.0 : 0.0, a == 1 ? 1.0 : 0.0, a == 2 ? 1.0 : 0.0};
  D3 t1 = cross(n, ea);
  const double l1 = std::sqrt(dot(t1, t1));
  t1 = {t1.x / l1, t1.y / l1, t1.z / l1};
  const D3 t2 = cross(n, t1);
  T[0] = t1.x, T[1] = t1.y, T[2] = t1.z;
  T[3] = t2.x, T[4] = t2.y, T[5] = t2.z;
}

// IPC's C1 mollified sliding norm with eps = eps_v dt:
// f0(y) = -y^3/(3 eps^2) + y^2/eps + eps/3 for y < eps, y beyond;
// f1 = f0' = -y^2/eps^2 + 2y/eps, 1 beyond.
double friction_f0(double y, double eps) {
  return y < eps ? -y * y * y / (3.0 * eps * eps) + y * y / eps + eps / 3.0 : y;
}
double friction_f1(double y, double eps) { return y < eps ? -y * y / (eps * eps) + 2.0 * y / eps : 1.0; }

}  // namespace

extern "C" {

// lagged quantities per pair at x^t: lambda (0 for inactive pairs), T [n][6]
// (columns t1, t2), w [n][4]
void ora_friction_lag(int64_t n, int is_ee, const int32_t* pairs, const int32_t* tris, const int32_t* edges,
                      const double* xbar, const double* xt, double dhat, double kappa, double* lam, double* T,
                      double* w) {
  const double dhat2 = dhat * dhat;
  for (int64_t i = 0; i < n; ++i) {
    int vid[4];
    pair_verts(is_ee, pairs + 2 * i, tris, edges, vid);
    D3 X[4];
    for (int k = 0; k < 4; ++k) X[k] = ld3(xt, vid[k]);
    const int ty = classify(is_ee, X);
    double num, den;
    case_nd<double>(ty, X, num, den, 1.0);
    lam[i] = 0.0;
    for (int k = 0; k < 6; ++k) T[6 * i + k] = 0.0;
    for (int k = 0; k < 4; ++k) w[4 * i + k] = 0.0;
    if (!(num < dhat2 * den) || num == 0.0) continue;
    const double d = std::sqrt(num / den);
    const double Bp = -2.0 * (d - dhat) * std::log(d / dhat) - (d - dhat) * (d - dhat) / d;
    double m = 1.0;
    if (is_ee) {
      D3 nn = cross(sub(X[1], X[0]), sub(X[3], X[2]));
      const double c = dot(nn, nn);
      const double* a0 = xbar + 3 * vid[0];
      const double* a1 = xbar + 3 * vid[1];
      const double* b0 = xbar + 3 * vid[2];
      const double* b1 = xbar + 3 * vid[3];
      D3 u{a1[0] - a0[0], a1[1] - a0[1], a1[2] - a0[2]}, v{b1[0] - b0[0], b1[1] - b0[1], b1[2] - b0[2]};
      const double eps = (1e-3 * dot(u, u)) * dot(v, v);
      if (c < eps) m = (2.0 - c / eps) * (c / eps);
    }
    lam[i] = -kappa * m * Bp;
    closest_weights(ty, X, w + 4 * i);
    D3 r{0, 0, 0};
    for (int k = 0; k < 4; ++k) {
      const double wk = w[4 * i + k];
      r = {r.x + wk * X[k].x, r.y + wk * X[k].y, r.z + wk * X[k].z};
    }
    tangent_basis(r, T + 6 * i);
  }
}

// Friction energy, gradient and Hessian of the lagged pairs at x.
// u = T^T sum_k w_k (x_k - x^t_k); D = mu lambda f0(|u|);
// grad = mu lambda f1(|u|)/|u| Gamma u, Hessian = mu lambda Gamma M Gamma^T
// with Gamma rows 3k..3k+2 = w_k T and
// M = (f1'(y) y - f1(y))/y^3 u u^T + f1(y)/y I  (y = |u|; M = 2/eps I at y = 0),
// PSD for this f1.  Accumulated like the barrier (J^T g, J^T H J).
int64_t ora_friction(int64_t n, int is_ee, const int32_t* pairs, const int32_t* vert_body, const int32_t* tris,
                     const int32_t* edges, const uint8_t* fixed, const double* xbar, const double* x, const double* xt,
                     const double* lam, const double* T, const double* w, double mu, double eps, double* energy,
                     double* grad, double* diag, double* off, const int32_t* off_keys, int64_t n_off, int want_hess) {
  double esum = 0.0;
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!(lam[i] > 0.0)) continue;
    ++cnt;
    int vid[4];
    pair_verts(is_ee, pairs + 2 * i, tris, edges, vid);
    double dl[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k)
      for (int c = 0; c < 3; ++c) dl[c] += w[4 * i + k] * (x[3 * vid[k] + c] - xt[3 * vid[k] + c]);
    const double* Ti = T + 6 * i;
    const double u[2] = {Ti[0] * dl[0] + Ti[1] * dl[1] + Ti[2] * dl[2], Ti[3] * dl[0] + Ti[4] * dl[1] + Ti[5] * dl[2]};
    const double y = std::sqrt(u[0] * u[0] + u[1] * u[1]);
    const double ml = mu * lam[i];
    esum += ml * friction_f0(y, eps);
    double M[2][2];
    double gs;  // f1(y)/y
    if (y == 0.0) {
      gs = 2.0 / eps;
      M[0][0] = M[1][1] = 2.0 / eps;
      M[0][1] = M[1][0] = 0.0;
    } else {
      gs = friction_f1(y, eps) / y;
      const double f1p = y < eps ? -2.0 * y / (eps * eps) + 2.0 / eps : 0.0;
      const double a = (f1p * y - friction_f1(y, eps)) / (y * y * y);
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) M[r][c] = a * u[r] * u[c] + (r == c ? gs : 0.0);
    }
    // Gamma (12 x 2)
    double G[12][2];
    for (int k = 0; k < 4; ++k)
      for (int c = 0; c < 3; ++c)
        for (int j = 0; j < 2; ++j) G[3 * k + c][j] = w[4 * i + k] * Ti[3 * j + c];
    double g[12], H[144];
    for (int r = 0; r < 12; ++r) g[r] = ml * gs * (G[r][0] * u[0] + G[r][1] * u[1]);
    for (int r = 0; r < 12; ++r)
      for (int c = 0; c < 12; ++c) {
        double s = 0.0;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) s += G[r][a] * M[a][b] * G[c][b];
        H[12 * r + c] = ml * s;
      }
    // J^T g, J^T H J (same as the barrier)
    const int ba = vert_body[vid[0]], bo = vert_body[vid[3]];
    double Jp[12][24];
    for (int r = 0; r < 12; ++r)
      for (int c = 0; c < 24; ++c) Jp[r][c] = 0.0;
    for (int k = 0; k < 4; ++k) {
      const int sl = vert_body[vid[k]] == ba ? 0 : 1;
      double J[3][12];
      kin_jacobian(xbar + 3 * vid[k], J);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 12; ++c) Jp[3 * k + r][12 * sl + c] = J[r][c];
    }
    const int bodies[2] = {ba, bo};
    double Gq[24], HH[24][24];
    for (int c = 0; c < 24; ++c) {
      double s = 0.0;
      for (int r = 0; r < 12; ++r) s += Jp[r][c] * g[r];
      Gq[c] = s;
    }
    if (want_hess)
      for (int c = 0; c < 24; ++c)
        for (int d = 0; d < 24; ++d) {
          double s = 0.0;
          for (int r = 0; r < 12; ++r)
            for (int t = 0; t < 12; ++t) s += Jp[r][c] * H[r * 12 + t] * Jp[t][d];
          HH[c][d] = s;
        }
    for (int sa = 0; sa < 2; ++sa) {
      const int b = bodies[sa];
      if (fixed[b]) continue;
      for (int c = 0; c < 12; ++c) grad[12 * b + c] += Gq[12 * sa + c];
      if (want_hess)
        for (int c = 0; c < 12; ++c)
          for (int d = 0; d < 12; ++d) diag[144 * b + 12 * c + d] += HH[12 * sa + c][12 * sa + d];
    }
    if (want_hess && !fixed[ba] && !fixed[bo] && off) {
      const int lo = std::min(ba, bo), hi = std::max(ba, bo);
      const int k = find_off(off_keys, n_off, lo, hi);
      if (k < 0) return -1;
      const int sl = (lo == ba) ? 0 : 1, sh = 1 - sl;
      for (int c = 0; c < 12; ++c)
        for (int d = 0; d < 12; ++d) off[144 * (int64_t)k + 12 * c + d] += HH[12 * sl + c][12 * sh + d];
    }
  }
  *energy += esum;
  return cnt;
}

}  // extern "C"

namespace {

// ------------------------------------------- friction lag, differentiated ----
// The lagged quantities as functions of the step-start positions x^t of a
// pair's 4 vertices (jets in those 12 coordinates): closest-point weights,
// normal force and tangent basis, with the case, the tangent axis and the
// mollifier branch fixed by the values (they are piecewise constant).
Jet jc(double c) { return jconst(c); }
Jet jneg(const Jet& a) { return scale(a, -1.0); }

void closest_weights_jet(int type, const V3<Jet> X[4], Jet w[4]) {
  for (int k = 0; k < 4; ++k) w[k] = jc(0.0);
  CaseSlots c = case_slots(type);
  if (c.kind == 0) {
    w[c.i] = jc(1.0);
    w[c.j] = jc(-1.0);
  } else if (c.kind == 1) {
    V3<Jet> e = sub(X[c.k], X[c.j]);
    const Jet t = dot(sub(X[c.i], X[c.j]), e) / dot(e, e);
    w[c.i] = jc(1.0);
    w[c.j] = t - jc(1.0);
    w[c.k] = jneg(t);
  } else if (c.kind == 2) {
    V3<Jet> e1 = sub(X[2], X[1]), e2 = sub(X[3], X[1]), dp = sub(X[0], X[1]);
    const Jet a = dot(e1, e1), b = dot(e1, e2), cc = dot(e2, e2), f1 = dot(e1, dp), f2 = dot(e2, dp);
    const Jet det = a * cc - b * b;
    const Jet u = (cc * f1 - b * f2) / det, v = (a * f2 - b * f1) / det;
    w[0] = jc(1.0);
    w[1] = u + v - jc(1.0);
    w[2] = jneg(u);
    w[3] = jneg(v);
  } else {
    V3<Jet> u = sub(X[1], X[0]), v = sub(X[3], X[2]), r0 = sub(X[0], X[2]);
    const Jet a = dot(u, u), b = dot(u, v), cc = dot(v, v), d = dot(u, r0), e = dot(v, r0);
    const Jet den = a * cc - b * b;
    const Jet s = (b * e - cc * d) / den, t = (a * e - b * d) / den;
    w[0] = jc(1.0) - s;
    w[1] = s;
    w[2] = t - jc(1.0);
    w[3] = jneg(t);
  }
}

}  // namespace

extern "C" {

// Adjoint term of the lag: for every lagged pair with lambda > 0,
// phi = v . g(x; lambda, T, w) with g the pair's friction gradient in vertex
// space at x (sliding displacement u = T^T sum_k w_k (x_k - x^t_k) held as
// data) and v = J l at the pair's vertices; the gradient of phi with respect
// to the pair's step-start positions (through lambda, T, w only) is mapped
// by J^T into out [nb][12] (accumulated; fixed bodies dropped).
void ora_friction_lag_vjp(int64_t n, int is_ee, const int32_t* pairs, const int32_t* vert_body, const int32_t* tris,
                          const int32_t* edges, const uint8_t* fixed, const double* xbar, const double* x,
                          const double* xt, const double* lam, double mu, double eps, double dhat, double kappa,
                          const double* l, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    if (!(lam[i] > 0.0)) continue;
    int vid[4];
    pair_verts(is_ee, pairs + 2 * i, tris, edges, vid);
    D3 Xd[4];
    for (int k = 0; k < 4; ++k) Xd[k] = ld3(xt, vid[k]);
    const int ty = classify(is_ee, Xd);
    V3<Jet> X[4];
    for (int k = 0; k < 4; ++k) X[k] = {jvar(Xd[k].x, 3 * k), jvar(Xd[k].y, 3 * k + 1), jvar(Xd[k].z, 3 * k + 2)};
    // lambda = -kappa m B'(d)
    Jet num, den;
    case_nd<Jet>(ty, X, num, den, jc(1.0));
    const Jet d = jsqrt(num / den);
    const Jet dm = d - jc(dhat);
    const Jet Bp = jneg(scale(dm * jlog(scale(d, 1.0 / dhat)), 2.0)) - dm * dm / d;
    Jet m = jc(1.0);
    if (is_ee) {
      V3<Jet> nn = cross(sub(X[1], X[0]), sub(X[3], X[2]));
      const Jet c = dot(nn, nn);
      const double* a0 = xbar + 3 * vid[0];
      const double* a1 = xbar + 3 * vid[1];
      const double* b0 = xbar + 3 * vid[2];
      const double* b1 = xbar + 3 * vid[3];
      D3 u{a1[0] - a0[0], a1[1] - a0[1], a1[2] - a0[2]}, v{b1[0] - b0[0], b1[1] - b0[1], b1[2] - b0[2]};
      const double ep = (1e-3 * dot(u, u)) * dot(v, v);
      if (c.v < ep) {
        const Jet r = scale(c, 1.0 / ep);
        m = (jc(2.0) - r) * r;
      }
    }
    const Jet L = jneg(scale(m * Bp, kappa));
    Jet w[4];
    closest_weights_jet(ty, X, w);
    V3<Jet> r{jc(0.0), jc(0.0), jc(0.0)};
    for (int k = 0; k < 4; ++k) r = {r.x + w[k] * X[k].x, r.y + w[k] * X[k].y, r.z + w[k] * X[k].z};
    const Jet nr = jsqrt(dot(r, r));
    V3<Jet> nv{r.x / nr, r.y / nr, r.z / nr};
    const double an[3] = {std::fabs(nv.x.v), std::fabs(nv.y.v), std::fabs(nv.z.v)};
    int ax = 0;
    if (an[1] < an[ax]) ax = 1;
    if (an[2] < an[ax]) ax = 2;
    V3<Jet> ea{jc(ax == 0 ? 1.0 : 0.0), jc(ax == 1 ? 1.0 : 0.0), jc(ax == 2 ? 1.0 : 0.0)};
    V3<Jet> t1 = cross(nv, ea);
    const Jet l1 = jsqrt(dot(t1, t1));
    t1 = {t1.x / l1, t1.y / l1, t1.z / l1};
    const V3<Jet> t2 = cross(nv, t1);
    // delta = sum w_k (x_k - x^t_k) (displacements are data), nu = sum w_k (J l)_k
    V3<Jet> delta{jc(0.0), jc(0.0), jc(0.0)}, nu{jc(0.0), jc(0.0), jc(0.0)};
    for (int k = 0; k < 4; ++k) {
      const double dx[3] = {x[3 * vid[k]] - xt[3 * vid[k]], x[3 * vid[k] + 1] - xt[3 * vid[k] + 1],
                            x[3 * vid[k] + 2] - xt[3 * vid[k] + 2]};
      double J[3][12];
      kin_jacobian(xbar + 3 * vid[k], J);
      const double* lb = l + 12 * vert_body[vid[k]];
      double vk[3];
      for (int c = 0; c < 3; ++c) {
        vk[c] = 0.0;
        for (int j = 0; j < 12; ++j) vk[c] += J[c][j] * lb[j];
      }
      delta = {delta.x + scale(w[k], dx[0]), delta.y + scale(w[k], dx[1]), delta.z + scale(w[k], dx[2])};
      nu = {nu.x + scale(w[k], vk[0]), nu.y + scale(w[k], vk[1]), nu.z + scale(w[k], vk[2])};
    }
    const Jet u0 = dot(t1, delta), u1 = dot(t2, delta);
    const Jet yy = u0 * u0 + u1 * u1;
    Jet gs;
    if (yy.v == 0.0) {
      gs = jc(2.0 / eps);
    } else {
      const Jet y = jsqrt(yy);
      gs = y.v < eps ? scale(y, -1.0 / (eps * eps)) + jc(2.0 / eps) : jc(1.0) / y;
    }
    const Jet coef = scale(L * gs, mu);
    const V3<Jet> f{coef * (t1.x * u0 + t2.x * u1), coef * (t1.y * u0 + t2.y * u1), coef * (t1.z * u0 + t2.z * u1)};
    const Jet phi = dot(nu, f);
    // J^T grad into the bodies
    for (int k = 0; k < 4; ++k) {
      const int b = vert_body[vid[k]];
      if (fixed[b]) continue;
      double J[3][12];
      kin_jacobian(xbar + 3 * vid[k], J);
      for (int j = 0; j < 12; ++j) {
        double sacc = 0.0;
        for (int c = 0; c < 3; ++c) sacc += J[c][j] * phi.g[3 * k + c];
        out[12 * b + j] += sacc;
      }
    }
  }
}

}  // extern "C"

namespace {
}  // namespace

extern "C" {
// Local 12x12 projection entry point (for pins of the eigen routine).
void ora_psd_project(int n, double* H) { psd_project(n, H); }

// Local barrier derivatives for explicit vertices (for pins): X[12], rest
// positions xb[12] (EE mollifier), returns energy, g[12], H[144].
int ora_pair_local(int is_ee, const double* X12, const double* xb12, double dhat, double kappa, double* e, double* g,
                   double* H) {
  D3 X[4];
  const double* xb4[4];
  for (int k = 0; k < 4; ++k) {
    X[k] = ld3(X12, k);
    xb4[k] = xb12 + 3 * k;
  }
  const int ty = classify(is_ee, X);
  pair_local(is_ee, ty, X, xb4, dhat, kappa, e, g, H);
  return ty;
}

// Distance and case for explicit vertices (for pins).
double ora_pair_distance(int is_ee, const double* X12, int* type) {
  D3 X[4];
  for (int k = 0; k < 4; ++k) X[k] = ld3(X12, k);
  *type = classify(is_ee, X);
  return pair_dist(is_ee, X);
}

}  // extern "C"
