// Per-vertex and per-body kernels: mass properties, the kinematic map, the
// inertia and orthogonality terms of the incremental potential.
#include "abd_internal.h"
#include "abd_jacobi.h"

namespace {

// Mass properties by the divergence theorem (one 64-lane wave per body;
// triangles strided over lanes, fixed-order wave reduction).
__global__ void __launch_bounds__(64) k_body_mass(int nb, const int32_t *tri_off, const int32_t *tris,
                                                  const double *xbar, const double *density, const uint8_t *fixed,
                                                  double *mass, double *volume) {
  const int b = blockIdx.x;
  if (b >= nb) return;
  double acc[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) acc[i] = 0.0;
  if (!fixed[b]) {
    for (int t = tri_off[b] + threadIdx.x; t < tri_off[b + 1]; t += 64) {
      const d3 v0 = ld3(xbar, tris[3 * t]), v1 = ld3(xbar, tris[3 * t + 1]), v2 = ld3(xbar, tris[3 * t + 2]);
      const d3 c12 = {v1.y * v2.z - v1.z * v2.y, v1.z * v2.x - v1.x * v2.z, v1.x * v2.y - v1.y * v2.x};
      const double vt = (v0.x * c12.x + v0.y * c12.y + v0.z * c12.z) / 6.0;
      const double s[3] = {v0.x + v1.x + v2.x, v0.y + v1.y + v2.y, v0.z + v1.z + v2.z};
      const double a0[3] = {v0.x, v0.y, v0.z}, a1[3] = {v1.x, v1.y, v1.z}, a2[3] = {v2.x, v2.y, v2.z};
      acc[0] += vt;
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[1 + i] += 0.25 * vt * s[i];
      int k = 4;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
          acc[k++] += (vt / 20.0) * (a0[i] * a0[j] + a1[i] * a1[j] + a2[i] * a2[j] + s[i] * s[j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 10; ++i) acc[i] = wave_sum(acc[i]);
  if (threadIdx.x == 0) {
    const double rho = fixed[b] ? 0.0 : density[b];
#pragma unroll
    for (int i = 0; i < 10; ++i) mass[10 * b + i] = rho * acc[i];
    volume[b] = fixed[b] ? 0.0 : acc[0];
  }
}

// x_k = p + A xbar_k, each component as p_i + ((a_i0 xb0 + a_i1 xb1) + a_i2 xb2)
// with contraction off: bit-identical to any IEEE evaluation in this order.
// (grid.y > 1: one map per trial, q and x advanced by qstride and 3 nv)
__global__ void __launch_bounds__(256) k_vertex_map(int nv, const double *__restrict__ xbar,
                                                    const int32_t *__restrict__ vert_body,
                                                    const double *__restrict__ q, double *__restrict__ x,
                                                    int64_t qstride = 0, const uint8_t *skip_scene = nullptr,
                                                    const int32_t *body_scene = nullptr) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nv) return;
  if (skip_scene && skip_scene[body_scene[vert_body[k]]]) return;
  q += blockIdx.y * qstride;
  x += blockIdx.y * 3 * (int64_t)nv;
  const double *qb = q + 12 * (int64_t)vert_body[k];
  const double xb0 = xbar[3 * k], xb1 = xbar[3 * k + 1], xb2 = xbar[3 * k + 2];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double *a = qb + 3 + 3 * i;
    x[3 * k + i] = qb[i] + ((a[0] * xb0 + a[1] * xb1) + a[2] * xb2);
  }
}

// Per-scene max_k |J_k p|_inf (p of fixed bodies is zero) as bit patterns
// of non-negative doubles, which order like the values (a NaN component, a
// failed solve, orders above +inf, so it reaches the result), at
// out[DISP_PAD * scene] (cleared to 0 first; one 128-byte line per scene,
// so that atomics on different scenes do not queue on one line).  A block
// whose vertices lie in one scene (vertices are scene-contiguous) folds to
// one atomic maximum, other blocks take one per wave and scene run; the
// maximum makes the result independent of order.
constexpr int DISP_PAD = 16;
__global__ void __launch_bounds__(256) k_disp_scene_max(int nv, const double *__restrict__ xbar,
                                                        const int32_t *__restrict__ vert_body,
                                                        const int32_t *__restrict__ body_scene,
                                                        const double *__restrict__ p, unsigned long long *out,
                                                        const uint8_t *skip_scene) {
  __shared__ unsigned long long sm[4];
  __shared__ int ss[4];
  const int k = blockIdx.x * 256 + threadIdx.x;
  unsigned long long m = 0ull;
  int sc = -1;
  if (k < nv) {
    const int b = vert_body[k];
    sc = body_scene[b];
  }
  if (k < nv && !(skip_scene && skip_scene[sc])) {
    const int b = vert_body[k];
    const double *qb = p + 12 * (int64_t)b;
    const double xb0 = xbar[3 * k], xb1 = xbar[3 * k + 1], xb2 = xbar[3 * k + 2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double *a = qb + 3 + 3 * i;
      const unsigned long long v =
          (unsigned long long)__double_as_longlong(fabs(qb[i] + ((a[0] * xb0 + a[1] * xb1) + a[2] * xb2)));
      m = v > m ? v : m;
    }
  }
  // (out-of-range lanes, sc = -1, are last in the block and carry 0)
  const int s0 = __shfl(sc, 0, 64);
  const bool uni = __all(sc == s0 || sc < 0);
  if (uni) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long v = (unsigned long long)__shfl_xor((long long)m, o, 64);
      m = v > m ? v : m;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[w] = m;
    ss[w] = uni ? s0 : -2;  // -2: this wave spans scenes
  }
  __syncthreads();
  const int b0 = ss[0];
  bool block_uni = b0 >= 0;
#pragma unroll
  for (int v = 1; v < 4; ++v) block_uni = block_uni && (ss[v] == b0 || ss[v] == -1);
  if (block_uni) {
    if (threadIdx.x == 0) {
      const unsigned long long a = sm[0] > sm[1] ? sm[0] : sm[1], c = sm[2] > sm[3] ? sm[2] : sm[3];
      atomicMax(out + DISP_PAD * b0, a > c ? a : c);
    }
  } else if (uni) {
    if ((threadIdx.x & 63) == 0 && s0 >= 0) atomicMax(out + DISP_PAD * s0, m);
  } else if (sc >= 0) {
    atomicMax(out + DISP_PAD * sc, m);
  }
}

__global__ void k_clear_u64n(int n, unsigned long long *a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0ull;
}


// (M dq) for one body, M = I_3 (x) [[m, h^T], [h, S]] in (p_i, a_i) groups
__device__ __forceinline__ void mass_apply(const double *mb, const double *dq, double *out) {
  const double m = mb[0], h[3] = {mb[1], mb[2], mb[3]};
  const double S[3][3] = {{mb[4], mb[5], mb[6]}, {mb[5], mb[7], mb[8]}, {mb[6], mb[8], mb[9]}};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double *a = dq + 3 + 3 * i;
    out[i] = m * dq[i] + h[0] * a[0] + h[1] * a[1] + h[2] * a[2];
#pragma unroll
    for (int r = 0; r < 3; ++r) out[3 + 3 * i + r] = h[r] * dq[i] + S[r][0] * a[0] + S[r][1] * a[1] + S[r][2] * a[2];
  }
}

// Orthogonality potential V = kn (sum_i (a_i.a_i - 1)^2 + sum_{i!=j} (a_i.a_j)^2)
// and its derivatives (ABD Eq. ortho-energy / ortho-poly; off-diagonal
// blocks 4 kn ((a_i.a_j) I + a_j a_i^T)), times w.
struct Ortho {
  double e;
  double g[9];
  double H[45];  // packed upper 9x9
};
__device__ __forceinline__ void ortho_eval(const double *A, double kn, double w, Ortho &o, bool want_h) {
  double dots[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dots[i][j] = A[3 * i] * A[3 * j] + A[3 * i + 1] * A[3 * j + 1] + A[3 * i + 2] * A[3 * j + 2];
  double V = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V += i == j ? (dots[i][i] - 1.0) * (dots[i][i] - 1.0) : dots[i][j] * dots[i][j];
  o.e = w * kn * V;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double gi = (dots[i][i] - 1.0) * A[3 * i + c];
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (j != i) gi += dots[i][j] * A[3 * j + c];
      o.g[3 * i + c] = w * 4.0 * kn * gi;
    }
  if (!want_h) return;
  using S = SymIdx<9>;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int j = i; j < 3; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (3 * j + c < 3 * i + r) continue;
          double h;
          if (i == j) {
            h = 4.0 * A[3 * i + r] * A[3 * i + c] + (r == c ? 2.0 * (dots[i][i] - 1.0) : 0.0);
#pragma unroll
            for (int k = 0; k < 3; ++k)
              if (k != i) h += 2.0 * A[3 * k + r] * A[3 * k + c];
            h *= 2.0 * kn;
          } else {
            h = 4.0 * kn * ((r == c ? dots[i][j] : 0.0) + A[3 * j + r] * A[3 * i + c]);
          }
          o.H[S::at(3 * i + r, 3 * j + c)] = w * h;
        }
}

// Projection of the orthogonality Hessian onto the PSD cone in closed form.
// V = ||G - I||_F^2 with G = A A^T depends on A only through its singular
// values (V = sum_k (sigma_k^2 - 1)^2), so with A = U diag(sigma) W^T the
// Hessian's eigenvectors are U E W^T for nine fixed 3x3 matrices E:
// e_k e_k^T (eigenvalue 4(3 sigma_k^2 - 1)) and, per pair i < j,
// (e_i e_j^T -/+ e_j e_i^T)/sqrt2 (eigenvalues 4(sigma_i^2 + sigma_j^2 -/+
// sigma_i sigma_j - 1)); the quadratic form of the Hessian in that basis is
// diagonal (second variation 4 sum_ij X_ij^2 (sigma_i^2 + sigma_j^2 - 1) +
// 4 sum_ij sigma_i sigma_j X_ij X_ji).  W and sigma^2 come from the 3x3
// eigenproblem of A^T A, U from A W / sigma (Gram-Schmidt).  H is kept when
// no eigenvalue is negative, else rebuilt from the clamped modes.  Returns
// false (leaving H alone) when A is too close to singular for U; the caller
// then projects numerically.  s = 4 w kn.
__device__ __forceinline__ bool ortho_project_closed(const double *A, double s, double *H) {
  using S3 = SymIdx<3>;
  double C[6];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = c; d < 3; ++d) C[S3::at(c, d)] = A[c] * A[d] + A[3 + c] * A[3 + d] + A[6 + c] * A[6 + d];
  double W[9];
  jacobi_eig<3>(C, W, 20, 1e-32);
  double s2[3], sg[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s2[k] = fmax(C[S3::at(k, k)], 0.0);
    sg[k] = sqrt(s2[k]);
  }
  const double smax = fmax(sg[0], fmax(sg[1], sg[2])), smin = fmin(sg[0], fmin(sg[1], sg[2]));
  if (!(smin > 1e-3 * smax)) return false;
  double lam[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) lam[k] = s * (3.0 * s2[k] - 1.0);
  // pairs (0,1), (0,2), (1,2): twist then flip
  lam[3] = s * (s2[0] + s2[1] - sg[0] * sg[1] - 1.0);
  lam[4] = s * (s2[0] + s2[1] + sg[0] * sg[1] - 1.0);
  lam[5] = s * (s2[0] + s2[2] - sg[0] * sg[2] - 1.0);
  lam[6] = s * (s2[0] + s2[2] + sg[0] * sg[2] - 1.0);
  lam[7] = s * (s2[1] + s2[2] - sg[1] * sg[2] - 1.0);
  lam[8] = s * (s2[1] + s2[2] + sg[1] * sg[2] - 1.0);
  bool neg = false;
#pragma unroll
  for (int m = 0; m < 9; ++m) neg = neg || lam[m] < 0.0;
  if (!neg) return true;
  // U: columns A w_k, orthonormalised in order
  double U[3][3];  // U[k][i] = component i of u_k
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) U[k][i] = A[3 * i] * W[k] + A[3 * i + 1] * W[3 + k] + A[3 * i + 2] * W[6 + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int j = 0; j < k; ++j) {
      const double d = U[j][0] * U[k][0] + U[j][1] * U[k][1] + U[j][2] * U[k][2];
#pragma unroll
      for (int i = 0; i < 3; ++i) U[k][i] -= d * U[j][i];
    }
    const double nr = 1.0 / sqrt(U[k][0] * U[k][0] + U[k][1] * U[k][1] + U[k][2] * U[k][2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) U[k][i] *= nr;
  }
  // modes v_m[3 i + c] = (U E_m W^T)_{ic}
  double V[9][9];
  const double r2 = 0.70710678118654752440;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int o = 3 * i + c;
#pragma unroll
      for (int k = 0; k < 3; ++k) V[k][o] = U[k][i] * W[3 * c + k];
      const double a01 = U[0][i] * W[3 * c + 1], a10 = U[1][i] * W[3 * c + 0];
      const double a02 = U[0][i] * W[3 * c + 2], a20 = U[2][i] * W[3 * c + 0];
      const double a12 = U[1][i] * W[3 * c + 2], a21 = U[2][i] * W[3 * c + 1];
      V[3][o] = r2 * (a01 - a10);
      V[4][o] = r2 * (a01 + a10);
      V[5][o] = r2 * (a02 - a20);
      V[6][o] = r2 * (a02 + a20);
      V[7][o] = r2 * (a12 - a21);
      V[8][o] = r2 * (a12 + a21);
    }
  using S9 = SymIdx<9>;
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = r; c < 9; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < 9; ++m) acc += fmax(lam[m], 0.0) * V[m][r] * V[m][c];
      H[S9::at(r, c)] = acc;
    }
  return true;
}

// Alternative rigidity potentials of A (sec. 3.2's ARAP, |A - R(A)|_F^2,
// and neo-Hookean with mu = lambda = 1: 1/2 (|A|_F^2 - 3) - ln J +
// 1/2 (ln J)^2, J = det A, infinite for J <= 0), times kn w, through A's
// signed singular value decomposition A = U diag(s) W^T (U, W rotations;
// s_3 < 0 when det A < 0).  Both are isotropic: Psi depends on s only, the
// gradient is U diag(psi) W^T (psi_i = dPsi/ds_i), and the Hessian's
// eigenvectors are U E W^T for: the three scaling modes, E = diag(z) with
// (z, lambda) the eigenpairs of d2Psi/ds2; per pair i < j the twist
// (e_i e_j^T - e_j e_i^T)/sqrt2 with eigenvalue (psi_i + psi_j)/(s_i + s_j)
// and the flip (e_i e_j^T + e_j e_i^T)/sqrt2 with (psi_i - psi_j)/(s_i -
// s_j), both in closed forms without the differences:
//   ARAP: psi_i = 2 (s_i - 1), d2Psi = 2 I, twist 2 - 4/(s_i + s_j), flip 2;
//   neo-Hookean: psi_i = s_i + (ln J - 1)/s_i,
//     d2Psi_ij = delta_ij (1 - (ln J - 1)/s_i^2) + 1/(s_i s_j),
//     twist 1 + (ln J - 1)/(s_i s_j), flip 1 - (ln J - 1)/(s_i s_j).
// W and s^2 come from the 3x3 eigenproblem of A^T A; the two larger
// singular directions give u = A w / s (Gram-Schmidt), the third u is their
// cross product and its s the signed length of A w along it.
struct IsoSvd {
  double U[3][3];  // U[k][i]: component i of u_k
  double W[3][3];  // W[k][c]: component c of w_k
  double s[3];
};
__device__ __forceinline__ void iso_svd(const double *A, IsoSvd &d) {
  using S3 = SymIdx<3>;
  double C[6], V[9];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int e = c; e < 3; ++e) C[S3::at(c, e)] = A[c] * A[e] + A[3 + c] * A[3 + e] + A[6 + c] * A[6 + e];
  jacobi_eig<3>(C, V, 20, 1e-32);
  // order: the two larger eigenvalues first, the smallest last
  double ev[3] = {C[S3::at(0, 0)], C[S3::at(1, 1)], C[S3::at(2, 2)]};
  int kmin = ev[0] <= ev[1] ? (ev[0] <= ev[2] ? 0 : 2) : (ev[1] <= ev[2] ? 1 : 2);
  const int ka = kmin == 0 ? 1 : 0, kb = kmin == 2 ? 1 : 2;
  const int ord[3] = {ka, kb, kmin};
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) d.W[k][c] = V[3 * c + ord[k]];
  // W a rotation
  const double detW = d.W[0][0] * (d.W[1][1] * d.W[2][2] - d.W[1][2] * d.W[2][1]) -
                      d.W[0][1] * (d.W[1][0] * d.W[2][2] - d.W[1][2] * d.W[2][0]) +
                      d.W[0][2] * (d.W[1][0] * d.W[2][1] - d.W[1][1] * d.W[2][0]);
  if (detW < 0.0)
#pragma unroll
    for (int c = 0; c < 3; ++c) d.W[2][c] = -d.W[2][c];
  double Aw[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) Aw[k][i] = A[3 * i] * d.W[k][0] + A[3 * i + 1] * d.W[k][1] + A[3 * i + 2] * d.W[k][2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double v[3] = {Aw[k][0], Aw[k][1], Aw[k][2]};
    if (k == 1) {
      const double dd = d.U[0][0] * v[0] + d.U[0][1] * v[1] + d.U[0][2] * v[2];
#pragma unroll
      for (int i = 0; i < 3; ++i) v[i] -= dd * d.U[0][i];
    }
    const double nr = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    d.s[k] = nr;
#pragma unroll
    for (int i = 0; i < 3; ++i) d.U[k][i] = v[i] / nr;
  }
  d.U[2][0] = d.U[0][1] * d.U[1][2] - d.U[0][2] * d.U[1][1];
  d.U[2][1] = d.U[0][2] * d.U[1][0] - d.U[0][0] * d.U[1][2];
  d.U[2][2] = d.U[0][0] * d.U[1][1] - d.U[0][1] * d.U[1][0];
  d.s[2] = d.U[2][0] * Aw[2][0] + d.U[2][1] * Aw[2][1] + d.U[2][2] * Aw[2][2];
  // (s_0, s_1: lengths after Gram-Schmidt; u_0 . A w_0 etc. are these)
}

// energy only of kind 2 (ARAP) or 3 (neo-Hookean), unscaled
__device__ __forceinline__ double iso_energy(const double *A, int kind) {
  if (kind == 3) {
    const double J = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(J > 0.0)) return INFINITY;
    double f2 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) f2 += A[i] * A[i];
    const double lj = log(J);
    return 0.5 * (f2 - 3.0) - lj + 0.5 * lj * lj;
  }
  IsoSvd d;
  iso_svd(A, d);
  return (d.s[0] - 1.0) * (d.s[0] - 1.0) + (d.s[1] - 1.0) * (d.s[1] - 1.0) + (d.s[2] - 1.0) * (d.s[2] - 1.0);
}

// energy, gradient and (projected when project) Hessian of kind 2 / 3,
// times c = kn w; H packed upper 9x9
__device__ __forceinline__ void iso_eval(const double *A, int kind, double c, Ortho &o, bool want_h, bool project) {
  IsoSvd d;
  iso_svd(A, d);
  const double *sv = d.s;
  double psi[3], hs[6], twist[3], flip[3];
  using S3 = SymIdx<3>;
  const int pi_[3] = {0, 0, 1}, pj_[3] = {1, 2, 2};
  if (kind == 2) {
    o.e = c * ((sv[0] - 1.0) * (sv[0] - 1.0) + (sv[1] - 1.0) * (sv[1] - 1.0) + (sv[2] - 1.0) * (sv[2] - 1.0));
#pragma unroll
    for (int k = 0; k < 3; ++k) psi[k] = 2.0 * (sv[k] - 1.0);
#pragma unroll
    for (int k = 0; k < 6; ++k) hs[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) hs[S3::at(k, k)] = 2.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      twist[m] = 2.0 - 4.0 / (sv[pi_[m]] + sv[pj_[m]]);
      flip[m] = 2.0;
    }
  } else {
    const double J = sv[0] * sv[1] * sv[2];
    if (!(J > 0.0)) {
      o.e = INFINITY;
#pragma unroll
      for (int i = 0; i < 9; ++i) o.g[i] = 0.0;
#pragma unroll
      for (int i = 0; i < 45; ++i) o.H[i] = 0.0;
      return;
    }
    const double lj = log(J), l1 = lj - 1.0;
    o.e = c * (0.5 * (sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2] - 3.0) - lj + 0.5 * lj * lj);
#pragma unroll
    for (int k = 0; k < 3; ++k) psi[k] = sv[k] + l1 / sv[k];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) hs[S3::at(a, b)] = (a == b ? 1.0 - l1 / (sv[a] * sv[a]) : 0.0) + 1.0 / (sv[a] * sv[b]);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double q = l1 / (sv[pi_[m]] * sv[pj_[m]]);
      twist[m] = 1.0 + q;
      flip[m] = 1.0 - q;
    }
  }
  // gradient U diag(psi) W^T (row-major in A's order)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      o.g[3 * i + cc] = c * (psi[0] * d.U[0][i] * d.W[0][cc] + psi[1] * d.U[1][i] * d.W[1][cc] +
                             psi[2] * d.U[2][i] * d.W[2][cc]);
  if (!want_h) return;
  // scaling modes: eigenpairs of d2Psi/ds2
  double Z[9];
  jacobi_eig<3>(hs, Z, 20, 1e-32);
  double lam[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) lam[k] = hs[S3::at(k, k)];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    lam[3 + 2 * m] = twist[m];
    lam[4 + 2 * m] = flip[m];
  }
  if (project)
#pragma unroll
    for (int m = 0; m < 9; ++m) lam[m] = fmax(lam[m], 0.0);
  double V[9][9];
  const double r2 = 0.70710678118654752440;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const int o_ = 3 * i + cc;
      double uw[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) uw[k] = d.U[k][i] * d.W[k][cc];
#pragma unroll
      for (int k = 0; k < 3; ++k) V[k][o_] = Z[k] * uw[0] + Z[3 + k] * uw[1] + Z[6 + k] * uw[2];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double aij = d.U[pi_[m]][i] * d.W[pj_[m]][cc], aji = d.U[pj_[m]][i] * d.W[pi_[m]][cc];
        V[3 + 2 * m][o_] = r2 * (aij - aji);
        V[4 + 2 * m][o_] = r2 * (aij + aji);
      }
    }
  using S9 = SymIdx<9>;
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int cc = r; cc < 9; ++cc) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < 9; ++m) acc += lam[m] * V[m][r] * V[m][cc];
      o.H[S9::at(r, cc)] = c * acc;
    }
}

// inertia + weighted orthogonality per body: energies to e_out[b], gradient
// and diagonal blocks accumulated (thread per body)
// DERIV = 0: energies only (the derivative code compiled out, so the
// energy-only launches of the line search do not carry its registers)
template <int DERIV>
__global__ void __launch_bounds__(64) k_body_terms(int nb, const uint8_t *fixed, const double *mass,
                                                  const double *volume, const double *q, const double *qt,
                                                  double kappa_o, double w, int do_inertia, int do_ortho,
                                                  int project, int want_grad, double *e_out, double *grad,
                                                  double *diag, int64_t estride = 0,
                                                  const uint8_t *skip_scene = nullptr,
                                                  const int32_t *body_scene = nullptr) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  // energy-only trials (grid.y > 1): trial t's q at q + 12 nb t, energies at
  // e_out + t estride (estride 0: nb)
  q += blockIdx.y * 12 * (int64_t)nb;
  e_out += blockIdx.y * (estride > 0 ? estride : (int64_t)nb);
  if (fixed[b] || (skip_scene && skip_scene[body_scene[b]])) {
    e_out[b] = 0.0;
    return;
  }
  const double *qb = q + 12 * (int64_t)b;
  double e = 0.0;
  if (do_inertia) {
    double dq[12], Mq[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) dq[i] = qb[i] - qt[12 * (int64_t)b + i];
    mass_apply(mass + 10 * (int64_t)b, dq, Mq);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 12; ++i) s += dq[i] * Mq[i];
    e += 0.5 * s;
    if (DERIV && want_grad)
#pragma unroll
      for (int i = 0; i < 12; ++i) grad[12 * (int64_t)b + i] += Mq[i];
    if (DERIV && diag) {
      const double *mb = mass + 10 * (int64_t)b;
      double *D = diag + 144 * (int64_t)b;
      const double S[3][3] = {{mb[4], mb[5], mb[6]}, {mb[5], mb[7], mb[8]}, {mb[6], mb[8], mb[9]}};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        D[12 * i + i] += mb[0];
#pragma unroll
        for (int n = 0; n < 3; ++n) {
          D[12 * i + 3 + 3 * i + n] += mb[1 + n];
          D[12 * (3 + 3 * i + n) + i] += mb[1 + n];
#pragma unroll
          for (int m = 0; m < 3; ++m) D[12 * (3 + 3 * i + m) + 3 + 3 * i + n] += S[m][n];
        }
      }
    }
  }
  if (do_ortho >= 2 && !DERIV) {
    e += w * kappa_o * volume[b] * iso_energy(qb + 3, do_ortho);
  } else if (do_ortho) {
    Ortho o;
    if (do_ortho == 1)
      ortho_eval(qb + 3, kappa_o * volume[b], w, o, DERIV && diag != nullptr);
    else
      iso_eval(qb + 3, do_ortho, w * kappa_o * volume[b], o, DERIV && diag != nullptr, project != 0);
    e += o.e;
    if (DERIV && want_grad)
#pragma unroll
      for (int i = 0; i < 9; ++i) grad[12 * (int64_t)b + 3 + i] += o.g[i];
    if (DERIV && diag) {
      if (do_ortho == 1 && project && !ortho_project_closed(qb + 3, 4.0 * w * kappa_o * volume[b], o.H))
        psd_project_packed<9>(o.H);
      using S = SymIdx<9>;
      double *D = diag + 144 * (int64_t)b;
#pragma unroll
      for (int r = 0; r < 9; ++r)
#pragma unroll
        for (int c = 0; c < 9; ++c) D[12 * (3 + r) + 3 + c] += o.H[S::at(r, c)];
    }
  }
  e_out[b] = e;
}

__global__ void k_q_tilde(int nb, const uint8_t *fixed, const double *q, const double *qd, double dt, double gx,
                          double gy, double gz, double *qt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * 12) return;
  const int b = i / 12, c = i % 12;
  if (fixed[b]) {
    qt[i] = q[i];
    return;
  }
  double v = q[i] + dt * qd[i];
  if (c < 3) v += dt * dt * (c == 0 ? gx : (c == 1 ? gy : gz));
  qt[i] = v;
}

}  // namespace

int op_vertex_map(abd_ctx *ctx, const abd_scene *sc, const double *q, double *x, hipStream_t s,
                  const uint8_t *skip_scene) {
  if (sc->n_verts <= 0) return ABD_OK;
  hipLaunchKernelGGL(k_vertex_map, dim3(grid_for(sc->n_verts, 256)), dim3(256), 0, s, sc->n_verts, sc->xbar,
                     sc->vert_body, q, x, (int64_t)0, skip_scene, sc->body_scene);
  return abd_hip_check(ctx, hipGetLastError(), "k_vertex_map");
}

// per-scene max_k |J_k p|_inf into out [n_scenes]
int op_max_abs_disp_scenes(abd_ctx *ctx, const abd_scene *sc, const double *p, const double **out, int *stride,
                           hipStream_t s, const uint8_t *skip_scene) {
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  unsigned long long *pad;
  ABD_TRY(ws(ctx, "disp_pad", DISP_PAD * (size_t)S, &pad, s));
  hipLaunchKernelGGL(k_clear_u64n, dim3(grid_for(DISP_PAD * S, 256)), dim3(256), 0, s, DISP_PAD * S, pad);
  if (sc->n_verts > 0)
    hipLaunchKernelGGL(k_disp_scene_max, dim3(grid_for(sc->n_verts, 256)), dim3(256), 0, s, sc->n_verts, sc->xbar,
                       sc->vert_body, sc->body_scene, p, pad, skip_scene);
  *out = reinterpret_cast<const double *>(pad);
  *stride = DISP_PAD;
  return abd_hip_check(ctx, hipGetLastError(), "k_disp_scene_max");
}

// (kappa_j > 0: the scene's joint penalties are added, times w)
static int body_terms(abd_ctx *ctx, const abd_scene *sc, const double *q, const double *qt, double kappa_o,
                      double w, int do_inertia, int do_ortho, int project, double *energy, double *grad,
                      double *diag, hipStream_t s, double kappa_j = 0.0, const uint8_t *skip_scene = nullptr) {
  if (sc->n_bodies <= 0) return ABD_OK;
  if (!sc->mass && do_inertia) return abd_fail(ctx, ABD_E_INVALID, "scene mass is NULL");
  if (!sc->volume && do_ortho) return abd_fail(ctx, ABD_E_INVALID, "scene volume is NULL");
  if (do_ortho < 0 || do_ortho > 3) return abd_fail(ctx, ABD_E_INVALID, "rigidity must be 0, 1 or 2");
  double *eb;
  ABD_TRY(ws(ctx, "body_e", sc->n_bodies, &eb, s));
  if (grad || diag)
    hipLaunchKernelGGL(k_body_terms<1>, dim3(grid_for(sc->n_bodies, 64)), dim3(64), 0, s, sc->n_bodies,
                       sc->body_fixed, sc->mass, sc->volume, q, qt, kappa_o, w, do_inertia, do_ortho, project,
                       grad != nullptr ? 1 : 0, eb, grad, diag, (int64_t)0, skip_scene, sc->body_scene);
  else
    hipLaunchKernelGGL(k_body_terms<0>, dim3(grid_for(sc->n_bodies, 64)), dim3(64), 0, s, sc->n_bodies,
                       sc->body_fixed, sc->mass, sc->volume, q, qt, kappa_o, w, do_inertia, do_ortho, project, 0, eb,
                       nullptr, nullptr, (int64_t)0);
  HIP_TRY(ctx, hipGetLastError());
  if (kappa_j > 0.0 && sc->n_joints > 0)
    ABD_TRY(op_joint_body(ctx, sc, kappa_j * w, q, 1, 0, eb, 0, grad, diag, s));
  if (energy) ABD_TRY(reduce_sum_f64(ctx, eb, sc->n_bodies, energy, s));
  return ABD_OK;
}

int op_body_terms(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, const double *qt,
                  double *energy, double *grad, double *diag, int project, hipStream_t s,
                  const uint8_t *skip_scene) {
  return body_terms(ctx, sc, q, qt, prm->kappa_o, prm->dt * prm->dt, 1, 1 + prm->rigidity, project, energy, grad, diag,
                    s, prm->kappa_j, skip_scene);
}

int op_body_energy(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, const double *qt,
                   double *energy, hipStream_t s) {
  return body_terms(ctx, sc, q, qt, prm->kappa_o, prm->dt * prm->dt, 1, 1 + prm->rigidity, 0, energy, nullptr, nullptr,
                    s, prm->kappa_j);
}


int op_body_energy_trials(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q,
                          const double *qt, int n_trials, double *energy, hipStream_t s, double *items,
                          int64_t estride, TrialSums *defer) {
  const int nb = sc->n_bodies;
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  if (nb <= 0 || n_trials <= 0) return ABD_OK;
  if (!sc->mass || !sc->volume) return abd_fail(ctx, ABD_E_INVALID, "scene mass or volume is NULL");
  double *eb = items;
  if (!eb) ABD_TRY(ws(ctx, "body_e_tr", (size_t)nb * n_trials, &eb, s));
  hipLaunchKernelGGL(k_body_terms<0>, dim3(grid_for(nb, 64), n_trials), dim3(64), 0, s, nb, sc->body_fixed, sc->mass,
                     sc->volume, q, qt, prm->kappa_o, prm->dt * prm->dt, 1, 1 + prm->rigidity, 0, 0, eb, nullptr, nullptr,
                     items ? estride : (int64_t)0, defer ? defer->skip : nullptr, sc->body_scene);
  HIP_TRY(ctx, hipGetLastError());
  if (prm->kappa_j > 0.0 && sc->n_joints > 0)
    ABD_TRY(op_joint_body(ctx, sc, prm->kappa_j * prm->dt * prm->dt, q, n_trials, 12 * (int64_t)nb, eb,
                          items ? estride : (int64_t)nb, nullptr, nullptr, s));
  if (items) return ABD_OK;
  if (defer) {
    defer->seg[defer->k++] = TrialSeg{eb, nb, nb, sc->body_scene};
    return ABD_OK;
  }
  return seg_sum_trials(ctx, eb, nb, nb, sc->body_scene, n_trials, S, energy, s);
}


int op_orthogonality(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, double weight,
                     double *energy, double *grad, double *diag, int project, hipStream_t s) {
  return body_terms(ctx, sc, q, nullptr, prm->kappa_o, weight, 0, 1 + prm->rigidity, project, energy, grad, diag, s);
}

int op_inertia(abd_ctx *ctx, const abd_scene *sc, const double *q, const double *qt, double *energy, double *grad,
               double *diag, hipStream_t s) {
  return body_terms(ctx, sc, q, qt, 0.0, 0.0, 1, 0, 0, energy, grad, diag, s);
}

// ------------------------------------------------------------------ ABI ----
extern "C" int abd_body_mass(abd_ctx *ctx, const abd_scene *sc, const double *density, double *mass,
                             double *volume, hipStream_t stream) {
  if (!ctx || !sc || !density || !mass || !volume) return abd_fail(ctx, ABD_E_INVALID, "abd_body_mass: null");
  if (sc->n_bodies <= 0) return ABD_OK;
  hipLaunchKernelGGL(k_body_mass, dim3(sc->n_bodies), dim3(64), 0, stream, sc->n_bodies, sc->body_tri_off, sc->tris,
                     sc->xbar, density, sc->body_fixed, mass, volume);
  return abd_hip_check(ctx, hipGetLastError(), "k_body_mass");
}

extern "C" int abd_vertex_map(abd_ctx *ctx, const abd_scene *sc, const double *q, double *x, hipStream_t stream) {
  if (!ctx || !sc || !q || !x) return abd_fail(ctx, ABD_E_INVALID, "abd_vertex_map: null");
  return op_vertex_map(ctx, sc, q, x, stream);
}

extern "C" int abd_orthogonality(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q,
                                 double weight, double *energy, double *grad, double *diag, int project_psd,
                                 hipStream_t stream) {
  if (!ctx || !sc || !prm || !q) return abd_fail(ctx, ABD_E_INVALID, "abd_orthogonality: null");
  return op_orthogonality(ctx, sc, prm, q, weight, energy, grad, diag, project_psd, stream);
}

extern "C" int abd_inertia(abd_ctx *ctx, const abd_scene *sc, const double *q, const double *q_tilde,
                           double *energy, double *grad, double *diag, hipStream_t stream) {
  if (!ctx || !sc || !q || !q_tilde) return abd_fail(ctx, ABD_E_INVALID, "abd_inertia: null");
  return op_inertia(ctx, sc, q, q_tilde, energy, grad, diag, stream);
}

extern "C" int abd_q_tilde(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q,
                           const double *qdot, double *q_tilde, hipStream_t stream) {
  if (!ctx || !sc || !prm || !q || !qdot || !q_tilde) return abd_fail(ctx, ABD_E_INVALID, "abd_q_tilde: null");
  const int n = sc->n_bodies * 12;
  if (n <= 0) return ABD_OK;
  hipLaunchKernelGGL(k_q_tilde, dim3(grid_for(n, 256)), dim3(256), 0, stream, sc->n_bodies, sc->body_fixed, q, qdot,
                     prm->dt, prm->gravity[0], prm->gravity[1], prm->gravity[2], q_tilde);
  return abd_hip_check(ctx, hipGetLastError(), "k_q_tilde");
}
