// Joints (ABD sec. 5.3): q maps linearly to any virtual tetrahedron's
// vertices (Eq. phi), and those vertices are material points p_i = A pbar_i
// + p, so a joint that fixes tetrahedron vertices is a linear equality
// between material points, x_a(q_a) = x_b(q_b) or = c for a world point.
// Enforced by the quadratic penalty w kappa_j / 2 |x_a - x_b|^2 (w = dt^2 in
// the incremental potential).  With x = J(xbar) q, J = [I | I (x) xbar^T],
// body a's gradient is w kappa J_a^T r (r = x_a - x_b), b's -w kappa J_b^T r,
// the diagonal blocks w kappa J^T J and the off-diagonal block of (a, b)
// -w kappa J_a^T J_b: constant, so the Hessian needs no projection.
//
// Sums are per body (thread per body over its joints, in joint order) and per
// body pair (thread per pair over its joints), so results are reproducible
// without atomics.
#include <algorithm>
#include <vector>

#include "abd_internal.h"

namespace {

// x = p + A xbar for the 12 DOFs q (rows a_i of A)
__device__ __forceinline__ void point_of(const double *q, const double *xb, double x[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) x[i] = q[i] + q[3 + 3 * i] * xb[0] + q[4 + 3 * i] * xb[1] + q[5 + 3 * i] * xb[2];
}

// energy (counted on the first free side), gradient and diagonal block per
// body; trial t (grid.y) reads q + t qstride and adds energies at
// e_out + t estride
template <int DERIV>
__global__ void k_joint_body(int nb, const uint8_t *fixed, const int32_t *joff, const int32_t *jent,
                             const int32_t *jbody, const double *jpoint, const double *q, int64_t qstride, double c,
                             double *e_out, int64_t estride, double *grad, double *diag) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb || fixed[b]) return;
  q += blockIdx.y * qstride;
  // J^T J summed over the body's joint points: m0 = sum 1, h = sum xbar,
  // M = sum xbar xbar^T (times c)
  double e = 0.0, g[12] = {0.0};
  double M[3][3] = {{0.0}}, h[3] = {0.0}, m0 = 0.0;
  for (int k = joff[b]; k < joff[b + 1]; ++k) {
    const int j = jent[k] >> 1, side = jent[k] & 1;
    const int a = jbody[2 * j], o = jbody[2 * j + 1];
    const double *pa = jpoint + 6 * (int64_t)j, *pb = pa + 3;
    double xa[3], xo[3];
    point_of(q + 12 * (int64_t)a, pa, xa);
    if (o >= 0)
      point_of(q + 12 * (int64_t)o, pb, xo);
    else
#pragma unroll
      for (int i = 0; i < 3; ++i) xo[i] = pb[i];
    double r[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) r[i] = xa[i] - xo[i];
    // the energy goes to the first free side
    const bool counts = side == 0 || fixed[a];
    if (counts) e += 0.5 * c * (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (DERIV) {
      const double sg = side == 0 ? c : -c;
      const double *xb = side == 0 ? pa : pb;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        g[i] += sg * r[i];
#pragma unroll
        for (int d = 0; d < 3; ++d) g[3 + 3 * i + d] += sg * r[i] * xb[d];
      }
      m0 += c;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        h[d] += c * xb[d];
#pragma unroll
        for (int f = 0; f < 3; ++f) M[d][f] += c * xb[d] * xb[f];
      }
    }
  }
  e_out[blockIdx.y * estride + b] += e;
  if (!DERIV) return;
  if (grad)
#pragma unroll
    for (int i = 0; i < 12; ++i) grad[12 * (int64_t)b + i] += g[i];
  if (diag) {
    double *Db = diag + 144 * (int64_t)b;
    // J^T J: [p_i][p_i] = 1, [p_i][a_i,d] = xbar_d, [a_i,d][a_i,f] = xbar_d xbar_f
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Db[12 * i + i] += m0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        Db[12 * i + 3 + 3 * i + d] += h[d];
        Db[12 * (3 + 3 * i + d) + i] += h[d];
#pragma unroll
        for (int f = 0; f < 3; ++f) Db[12 * (3 + 3 * i + d) + 3 + 3 * i + f] += M[d][f];
      }
    }
  }
}

__device__ __forceinline__ int64_t find_key(const int32_t *keys, int64_t n, int a, int b) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int ka = keys[2 * mid], kb = keys[2 * mid + 1];
    if (ka < a || (ka == a && kb < b))
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < n && keys[2 * lo] == a && keys[2 * lo + 1] == b) ? lo : -1;
}

// off-diagonal blocks: thread per body pair (lo < hi, both free), summing
// -c J_lo^T J_hi over its joints (in joint order) into the pair's block
__global__ void k_joint_off(int n_runs, const int32_t *run_off, const int32_t *run_joint, const int32_t *jbody,
                            const double *jpoint, double c, const int32_t *keys, int64_t n_keys, double *off,
                            int *err) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_runs) return;
  double P[4][4] = {{0.0}};  // sum over joints of u_lo u_hi^T, u = (1, xbar)
  int lo = 0, hi = 0;
  for (int k = run_off[r]; k < run_off[r + 1]; ++k) {
    const int j = run_joint[k];
    const int a = jbody[2 * j], b = jbody[2 * j + 1];
    const double *pa = jpoint + 6 * (int64_t)j, *pb = pa + 3;
    const bool swap = a > b;
    lo = swap ? b : a;
    hi = swap ? a : b;
    const double ul[4] = {1.0, swap ? pb[0] : pa[0], swap ? pb[1] : pa[1], swap ? pb[2] : pa[2]};
    const double uh[4] = {1.0, swap ? pa[0] : pb[0], swap ? pa[1] : pb[1], swap ? pa[2] : pb[2]};
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) P[u][v] += ul[u] * uh[v];
  }
  const int64_t kk = find_key(keys, n_keys, lo, hi);
  if (kk < 0) {
    atomicOr(err, 2);
    return;
  }
  double *O = off + 144 * kk;
  // rows: DOFs of lo (p_i -> u index 0, a_i,d -> 1 + d); the same i only
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    O[12 * i + i] -= c * P[0][0];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      O[12 * i + 3 + 3 * i + d] -= c * P[0][1 + d];
      O[12 * (3 + 3 * i + d) + i] -= c * P[1 + d][0];
#pragma unroll
      for (int f = 0; f < 3; ++f) O[12 * (3 + 3 * i + d) + 3 + 3 * i + f] -= c * P[1 + d][1 + f];
    }
  }
}

}  // namespace

// Per-scene joint tables (host-built once per context and joint arrays):
// per body its joint entries (joint << 1 | side) in joint order; the body
// pairs of joints between two free bodies (runs of joints per pair, pairs
// in (lo, hi) order); and one point-triangle-shaped pair per such joint
// (the first vertex of a, the first triangle of b) whose bodies the
// off-diagonal pattern marks.
int joint_tables(abd_ctx *ctx, const abd_scene *sc, JointTables **out, hipStream_t s) {
  *out = nullptr;
  if (sc->n_joints <= 0) return ABD_OK;
  if (!sc->joint_body || !sc->joint_point) return abd_fail(ctx, ABD_E_INVALID, "joints: null arrays");
  JointTables &T = ctx->joints;
  const std::vector<uintptr_t> key = {(uintptr_t)sc->joint_body, (uintptr_t)sc->joint_point,
                                      (uintptr_t)sc->n_joints, (uintptr_t)sc->n_bodies, (uintptr_t)sc->body_fixed};
  if (T.key != key) {
    const int nb = sc->n_bodies, nj = sc->n_joints;
    std::vector<int32_t> jb(2 * (size_t)nj), voff(nb + 1), toff(nb + 1), bscene(nb);
    std::vector<uint8_t> fx(nb);
    HIP_TRY(ctx, hipMemcpyAsync(jb.data(), sc->joint_body, jb.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(voff.data(), sc->body_vert_off, voff.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(toff.data(), sc->body_tri_off, toff.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(fx.data(), sc->body_fixed, fx.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(bscene.data(), sc->body_scene, bscene.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    std::vector<int32_t> cnt(nb + 1, 0);
    for (int j = 0; j < nj; ++j) {
      const int a = jb[2 * j], b = jb[2 * j + 1];
      if (a < 0 || a >= nb || b < -1 || b >= nb || a == b || (b >= 0 && bscene[a] != bscene[b]))
        return abd_fail(ctx, ABD_E_INVALID, "joint %d: bodies (%d, %d) invalid", j, a, b);
      ++cnt[a + 1];
      if (b >= 0) ++cnt[b + 1];
    }
    for (int b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
    std::vector<int32_t> ent(cnt[nb]), fill(cnt.begin(), cnt.end() - 1);
    for (int j = 0; j < nj; ++j) {
      ent[fill[jb[2 * j]]++] = 2 * j;
      if (jb[2 * j + 1] >= 0) ent[fill[jb[2 * j + 1]]++] = 2 * j + 1;
    }
    std::vector<int32_t> bb;  // joints between two free bodies, by (lo, hi) then joint
    for (int j = 0; j < nj; ++j)
      if (jb[2 * j + 1] >= 0 && !fx[jb[2 * j]] && !fx[jb[2 * j + 1]]) bb.push_back(j);
    auto lohi = [&](int j) {
      const int a = jb[2 * j], b = jb[2 * j + 1];
      return std::make_pair(std::min(a, b), std::max(a, b));
    };
    std::stable_sort(bb.begin(), bb.end(), [&](int x, int y) { return lohi(x) < lohi(y); });
    std::vector<int32_t> roff, pt;
    for (size_t k = 0; k < bb.size(); ++k) {
      if (k == 0 || lohi(bb[k]) != lohi(bb[k - 1])) roff.push_back((int32_t)k);
      const int a = jb[2 * bb[k]], b = jb[2 * bb[k] + 1];
      pt.push_back(voff[a]);
      pt.push_back(toff[b]);
    }
    roff.push_back((int32_t)bb.size());
    T.n_runs = (int)roff.size() - 1;
    T.n_pairs = (int64_t)bb.size();
    ABD_TRY(ws(ctx, "jt_off", nb + 1, &T.joff, s));
    ABD_TRY(ws(ctx, "jt_ent", ent.size() + 1, &T.jent, s));
    ABD_TRY(ws(ctx, "jt_roff", roff.size(), &T.run_off, s));
    ABD_TRY(ws(ctx, "jt_rj", bb.size() + 1, &T.run_joint, s));
    ABD_TRY(ws(ctx, "jt_pt", pt.size() + 2, &T.pairs, s));
    HIP_TRY(ctx, hipMemcpyAsync(T.joff, cnt.data(), cnt.size() * 4, hipMemcpyHostToDevice, s));
    if (!ent.empty()) HIP_TRY(ctx, hipMemcpyAsync(T.jent, ent.data(), ent.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(T.run_off, roff.data(), roff.size() * 4, hipMemcpyHostToDevice, s));
    if (!bb.empty()) {
      HIP_TRY(ctx, hipMemcpyAsync(T.run_joint, bb.data(), bb.size() * 4, hipMemcpyHostToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(T.pairs, pt.data(), pt.size() * 4, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(ctx, hipStreamSynchronize(s));  // (the host vectors go out of scope)
    T.key = key;
  }
  *out = &T;
  return ABD_OK;
}

int op_joint_body(abd_ctx *ctx, const abd_scene *sc, double c, const double *q, int n_trials, int64_t qstride,
                  double *e_items, int64_t estride, double *grad, double *diag, hipStream_t s) {
  JointTables *T;
  ABD_TRY(joint_tables(ctx, sc, &T, s));
  if (!T || n_trials <= 0) return ABD_OK;
  const int nb = sc->n_bodies;
  if (grad || diag)
    hipLaunchKernelGGL(k_joint_body<1>, dim3(grid_for(nb, 64), n_trials), dim3(64), 0, s, nb, sc->body_fixed, T->joff,
                       T->jent, sc->joint_body, sc->joint_point, q, qstride, c, e_items, estride, grad, diag);
  else
    hipLaunchKernelGGL(k_joint_body<0>, dim3(grid_for(nb, 64), n_trials), dim3(64), 0, s, nb, sc->body_fixed, T->joff,
                       T->jent, sc->joint_body, sc->joint_point, q, qstride, c, e_items, estride, nullptr, nullptr);
  return abd_hip_check(ctx, hipGetLastError(), "k_joint_body");
}

int op_joint_off(abd_ctx *ctx, const abd_scene *sc, double c, const int32_t *keys, int64_t n_keys, double *off,
                 hipStream_t s) {
  JointTables *T;
  ABD_TRY(joint_tables(ctx, sc, &T, s));
  if (!T || T->n_runs == 0 || !off) return ABD_OK;
  int *err;
  ABD_TRY(ws(ctx, "err_flag", 1, &err, s));
  hipLaunchKernelGGL(k_joint_off, dim3(grid_for(T->n_runs, 64)), dim3(64), 0, s, T->n_runs, T->run_off, T->run_joint,
                     sc->joint_body, sc->joint_point, c, keys, n_keys, off, err);
  return abd_hip_check(ctx, hipGetLastError(), "k_joint_off");
}
