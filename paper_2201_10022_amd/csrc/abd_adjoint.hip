// Reverse mode of the implicit-Euler time step (the differentiability that
// ABD's conclusion, sec. 6, claims).  q^{t+1} minimises the incremental
// potential E(q; q~, q^t) with q~ = q^t + dt qdot^t + dt^2 M^-1 f, so
// grad_q E(q^{t+1}) = 0.  Differentiating that condition (implicit
// function theorem), with H the unprojected Hessian of E at q^{t+1} and H_D
// the friction Hessian (the friction potential depends on q - q^t through
// the sliding displacement) and C_lag the derivative of the friction
// gradient through the lagged normal force, tangent basis and closest-point
// weights, themselves functions of q^t:
//     H dq^{t+1} = M dq~ + (H_D - C_lag) dq^t.
// With qdot^{t+1} = (q^{t+1} - q^t)/dt and a = qbar^{t+1} + qdbar^{t+1}/dt:
//     H l = a;  qbar^t = M l + H_D l - C_lag^T l - qdbar^{t+1}/dt;
//     qdbar^t = dt M l.
// C_lag^T l is the gradient with respect to the pairs' step-start
// positions of (J l) . g_D, taken with dual numbers one coordinate at a time.
// A rollout's gradient runs these steps backwards from checkpoints, re-running
// each segment's forward steps (the forward path is deterministic, so the
// re-run states equal the original ones bit for bit).
#include "abd_internal.h"

namespace {

__global__ void k_adj_rhs(int nb, const uint8_t *fixed, const double *qbar, const double *qdbar, double inv_dt,
                          double *a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 12 * nb) return;
  a[i] = fixed[i / 12] ? 0.0 : qbar[i] + qdbar[i] * inv_dt;
}

// qbar^t = M l + hdl - qdbar^{t+1}/dt, qdbar^t = dt M l (free bodies)
__global__ void k_adj_combine(int nb, const uint8_t *fixed, const double *mass, const double *l, const double *hdl,
                              const double *qdbar_next, double dt, double *qbar, double *qdbar) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double *qb = qbar + 12 * (int64_t)b, *qdb = qdbar + 12 * (int64_t)b;
  if (fixed[b]) {
    for (int i = 0; i < 12; ++i) qb[i] = qdb[i] = 0.0;
    return;
  }
  // M = I_3 (x) [[m, h^T], [h, S]] in (p_i, a_i) groups
  const double *mb = mass + 10 * (int64_t)b;
  const double *lb = l + 12 * (int64_t)b;
  const double m = mb[0], h[3] = {mb[1], mb[2], mb[3]};
  const double S[3][3] = {{mb[4], mb[5], mb[6]}, {mb[5], mb[7], mb[8]}, {mb[6], mb[8], mb[9]}};
  double Ml[12];
  for (int i = 0; i < 3; ++i) {
    const double *a = lb + 3 + 3 * i;
    Ml[i] = m * lb[i] + h[0] * a[0] + h[1] * a[1] + h[2] * a[2];
    for (int r = 0; r < 3; ++r) Ml[3 + 3 * i + r] = h[r] * lb[i] + S[r][0] * a[0] + S[r][1] * a[1] + S[r][2] * a[2];
  }
  const double *hd = hdl + 12 * (int64_t)b, *qn = qdbar_next + 12 * (int64_t)b;
  for (int i = 0; i < 12; ++i) {
    qb[i] = Ml[i] + hd[i] - qn[i] / dt;
    qdb[i] = dt * Ml[i];
  }
}

__global__ void k_sub_into(int n, const double *a, double *b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] -= a[i];
}

__global__ void k_zero_d(int64_t n, double *a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

int zero_d(abd_ctx *ctx, double *a, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_zero_d, dim3(grid_for(n, 256)), dim3(256), 0, s, n, a);
  return abd_hip_check(ctx, hipGetLastError(), "k_zero_d");
}

}  // namespace

// one reverse step; qbar_t / qdbar_t must not alias the inputs
int op_adjoint_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q_t, const double *qd_t,
                    const double *q_next, const double *qbar_next, const double *qdbar_next, double rtol,
                    int max_iter, double *qbar_t, double *qdbar_t, int *iters, hipStream_t s) {
  const int nb = sc->n_bodies, nv = sc->n_verts, n12 = 12 * nb;
  double *qt, *x, *g, *diag, *off, *a, *l, *hdl, *e;
  ABD_TRY(ws(ctx, "adj_qt", n12, &qt, s));
  ABD_TRY(ws(ctx, "adj_x", 3 * (size_t)nv, &x, s));
  ABD_TRY(ws(ctx, "adj_g", n12, &g, s));
  ABD_TRY(ws(ctx, "adj_diag", 144 * (size_t)nb, &diag, s));
  ABD_TRY(ws(ctx, "adj_a", n12, &a, s));
  ABD_TRY(ws(ctx, "adj_l", n12, &l, s));
  ABD_TRY(ws(ctx, "adj_hdl", n12, &hdl, s));
  ABD_TRY(ws(ctx, "adj_e", 2, &e, s));
  ABD_TRY(abd_q_tilde(ctx, sc, prm, q_t, qd_t, qt, s));
  // the step's friction, lagged at q^t as in the forward step
  struct FrictionScope {
    abd_ctx *c;
    bool on;
    ~FrictionScope() {
      if (on) abd_friction_end_step(c);
    }
  } fr_scope{ctx, false};
  if (prm->mu > 0.0) {
    ABD_TRY(abd_friction_begin_step(ctx, sc, prm, q_t, nullptr, s));
    fr_scope.on = true;
  }
  FrictionSet frs;
  bool fr_on = false;
  ABD_TRY(op_friction_state(ctx, sc, prm, &frs, &fr_on, s));
  const FrictionSet *fr = fr_on ? &frs : nullptr;

  // unprojected Hessian of E at q^{t+1}
  ABD_TRY(op_vertex_map(ctx, sc, q_next, x, s));
  int32_t *pt, *ee, *keys;
  int64_t npt, nee, nk;
  ABD_TRY(op_candidates(ctx, sc, x, nullptr, prm->dhat, &pt, &npt, &ee, &nee, "adj", s));
  ABD_TRY(op_offdiag(ctx, sc, pt, npt, ee, nee, &keys, &nk, "adj", s, fr ? fr->pt : nullptr, fr ? fr->n_pt : 0,
                     fr ? fr->ee : nullptr, fr ? fr->n_ee : 0));
  ABD_TRY(ws(ctx, "adj_off", 144 * (size_t)(nk + 1), &off, s));
  ABD_TRY(zero_d(ctx, g, n12, s));
  ABD_TRY(zero_d(ctx, diag, 144 * (int64_t)nb, s));
  ABD_TRY(zero_d(ctx, off, 144 * nk, s));
  ABD_TRY(zero_d(ctx, e, 1, s));
  ABD_TRY(op_body_terms(ctx, sc, prm, q_next, qt, e, g, diag, 0, s));
  ABD_TRY(op_barrier(ctx, sc, prm, x, pt, npt, ee, nee, keys, nk, e, g, diag, off, 0, nullptr, nullptr, s, fr));
  if (sc->n_joints > 0 && prm->kappa_j > 0.0)
    ABD_TRY(op_joint_off(ctx, sc, prm->kappa_j * prm->dt * prm->dt, keys, nk, off, s));
  ABD_TRY(op_read_err(ctx, s));

  // preconditioner: diagonal blocks of the projected (PSD) Hessian
  double *pre;
  ABD_TRY(ws(ctx, "adj_pre", 144 * (size_t)nb, &pre, s));
  ABD_TRY(zero_d(ctx, pre, 144 * (int64_t)nb, s));
  ABD_TRY(op_body_terms(ctx, sc, prm, q_next, qt, nullptr, nullptr, pre, 1, s));
  ABD_TRY(op_barrier(ctx, sc, prm, x, pt, npt, ee, nee, keys, nk, nullptr, nullptr, pre, nullptr, 1, nullptr, nullptr,
                     s, fr));
  ABD_TRY(op_read_err(ctx, s));

  // H l = qbar^{t+1} + qdbar^{t+1} / dt.  H is positive definite at a
  // strict local minimum, so conjugate gradients first (the solver of the
  // forward pass, its preconditioner from the projected diagonal blocks);
  // near contact the barrier's curvature can make H indefinite: if CG meets
  // a non-positive curvature or runs out of iterations, MINRES, which needs
  // symmetry only.
  hipLaunchKernelGGL(k_adj_rhs, dim3(grid_for(n12, 256)), dim3(256), 0, s, nb, sc->body_fixed, qbar_next, qdbar_next,
                     1.0 / prm->dt, a);
  int its = 0;
  // (environment ABD_ADJ_MINRES=1: MINRES alone)
  const char *only_mr = getenv("ABD_ADJ_MINRES");
  const bool cg_first = !(only_mr && only_mr[0] == '1');
  int *herr;
  ABD_TRY(pinned_get(ctx, 64, reinterpret_cast<void **>(&herr)));
  herr[0] = 0;
  if (cg_first) {
    ABD_TRY(op_pcg(ctx, sc, diag, off, keys, nk, a, l, rtol, max_iter, &its, s, nullptr, pre));
    ABD_TRY(err_enqueue(ctx, herr, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
  }
  if (!cg_first || (herr[0] & (4 | 8)) || its >= max_iter) {
    int *errf;
    ABD_TRY(ws(ctx, "err_flag", 1, &errf, s));
    HIP_TRY(ctx, hipMemsetAsync(errf, 0, sizeof(int), s));
    int its2 = 0;
    ABD_TRY(op_minres(ctx, sc, diag, off, keys, nk, pre, a, l, rtol, max_iter, &its2, s));
    its += its2;
  }
  ABD_TRY(op_read_err(ctx, s));
  if (iters) *iters = its;
  ABD_TRY(zero_d(ctx, hdl, n12, s));
  if (fr) {
    ABD_TRY(op_friction_hvp(ctx, sc, fr, x, l, hdl, s));
    // the lag's own dependence on q^t enters with the opposite sign
    double *lv;
    ABD_TRY(ws(ctx, "adj_lagv", n12, &lv, s));
    ABD_TRY(zero_d(ctx, lv, n12, s));
    ABD_TRY(op_friction_lag_vjp(ctx, sc, prm, fr, x, l, lv, s));
    hipLaunchKernelGGL(k_sub_into, dim3(grid_for(n12, 256)), dim3(256), 0, s, n12, lv, hdl);
  }
  hipLaunchKernelGGL(k_adj_combine, dim3(grid_for(nb, 64)), dim3(64), 0, s, nb, sc->body_fixed, sc->mass, l, hdl,
                     qdbar_next, prm->dt, qbar_t, qdbar_t);
  return abd_hip_check(ctx, hipGetLastError(), "k_adj_combine");
}

extern "C" int abd_adjoint_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q_t,
                                const double *qdot_t, const double *q_next, const double *qbar_next,
                                const double *qdbar_next, double rtol, double *qbar_t, double *qdbar_t,
                                int32_t *pcg_iters, hipStream_t stream) {
  if (!ctx || !sc || !prm || !q_t || !qdot_t || !q_next || !qbar_next || !qdbar_next || !qbar_t || !qdbar_t ||
      !sc->mass || !sc->volume)
    return abd_fail(ctx, ABD_E_INVALID, "abd_adjoint_step: null");
  if (prm->kappa_adaptive)
    return abd_fail(ctx, ABD_E_INVALID, "abd_adjoint_step: the adjoint takes a fixed barrier stiffness");
  if (qbar_t == qbar_next || qbar_t == qdbar_next || qdbar_t == qbar_next || qdbar_t == qdbar_next)
    return abd_fail(ctx, ABD_E_INVALID, "abd_adjoint_step: outputs alias inputs");
  int its = 0;
  ABD_TRY(op_adjoint_step(ctx, sc, prm, q_t, qdot_t, q_next, qbar_next, qdbar_next, rtol, prm->max_pcg, qbar_t,
                          qdbar_t, &its, stream));
  if (pcg_iters) *pcg_iters = its;
  return ABD_OK;
}

extern "C" int abd_rollout_forward(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, double *q,
                                   double *qdot, int32_t n_steps, int32_t checkpoint_every, double *checkpoints,
                                   int64_t *newton_iters, hipStream_t stream) {
  if (!ctx || !sc || !prm || !q || !qdot || !sc->mass || !sc->volume)
    return abd_fail(ctx, ABD_E_INVALID, "abd_rollout_forward: null");
  if (prm->kappa_adaptive)
    return abd_fail(ctx, ABD_E_INVALID, "abd_rollout_forward: the adjoint takes a fixed barrier stiffness");
  if (n_steps < 0 || checkpoint_every < 1) return abd_fail(ctx, ABD_E_INVALID, "abd_rollout_forward: bad sizes");
  hipStream_t s = stream;
  const int n12 = 12 * sc->n_bodies;
  const size_t vb = sizeof(double) * (size_t)n12;
  int64_t tot = 0;
  for (int t = 0; t < n_steps; ++t) {
    if (checkpoints && t % checkpoint_every == 0) {
      double *c = checkpoints + 2 * (size_t)n12 * (t / checkpoint_every);
      HIP_TRY(ctx, hipMemcpyAsync(c, q, vb, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(c + n12, qdot, vb, hipMemcpyDeviceToDevice, s));
    }
    abd_stats st;
    ABD_TRY(abd_time_step(ctx, sc, prm, q, qdot, &st, s));
    tot += st.newton_iters;
  }
  if (checkpoints) {  // the final state after the last checkpoint
    double *c = checkpoints + 2 * (size_t)n12 * ((n_steps + checkpoint_every - 1) / checkpoint_every);
    HIP_TRY(ctx, hipMemcpyAsync(c, q, vb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(c + n12, qdot, vb, hipMemcpyDeviceToDevice, s));
  }
  if (newton_iters) *newton_iters = tot;
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return ABD_OK;
}

extern "C" int abd_rollout_backward(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q0,
                                    const double *qdot0, int32_t n_steps, int32_t checkpoint_every,
                                    const double *checkpoints, const double *qbar_T, const double *qdbar_T,
                                    double rtol, double *qbar_0, double *qdbar_0, hipStream_t stream) {
  if (!ctx || !sc || !prm || !q0 || !qdot0 || !qbar_T || !qdbar_T || !qbar_0 || !qdbar_0 || !sc->mass ||
      !sc->volume)
    return abd_fail(ctx, ABD_E_INVALID, "abd_rollout_backward: null");
  if (prm->kappa_adaptive)
    return abd_fail(ctx, ABD_E_INVALID, "abd_rollout_backward: the adjoint takes a fixed barrier stiffness");
  if (n_steps < 0 || checkpoint_every < 1) return abd_fail(ctx, ABD_E_INVALID, "abd_rollout_backward: bad sizes");
  hipStream_t s = stream;
  const int n12 = 12 * sc->n_bodies;
  const size_t vb = sizeof(double) * (size_t)n12;
  const int K = checkpoint_every;
  const int n_ck = (n_steps + K - 1) / K;
  double *ckw, *seg, *q, *qd, *qb, *qdb, *qb2, *qdb2;
  const double *ck = checkpoints;
  if (!ck) ABD_TRY(ws(ctx, "ro_ck", 2 * (size_t)n12 * (n_ck + 1), &ckw, s));
  ABD_TRY(ws(ctx, "ro_seg", 2 * (size_t)n12 * (K + 1), &seg, s));
  ABD_TRY(ws(ctx, "ro_q", n12, &q, s));
  ABD_TRY(ws(ctx, "ro_qd", n12, &qd, s));
  ABD_TRY(ws(ctx, "ro_qb", n12, &qb, s));
  ABD_TRY(ws(ctx, "ro_qdb", n12, &qdb, s));
  ABD_TRY(ws(ctx, "ro_qb2", n12, &qb2, s));
  ABD_TRY(ws(ctx, "ro_qdb2", n12, &qdb2, s));
  if (!ck) {
    // forward, keeping (q, qdot) every K steps
    HIP_TRY(ctx, hipMemcpyAsync(q, q0, vb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(qd, qdot0, vb, hipMemcpyDeviceToDevice, s));
    ABD_TRY(abd_rollout_forward(ctx, sc, prm, q, qd, n_steps, K, ckw, nullptr, s));
    ck = ckw;
  }
  HIP_TRY(ctx, hipMemcpyAsync(qb, qbar_T, vb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(qdb, qdbar_T, vb, hipMemcpyDeviceToDevice, s));
  for (int c = n_ck - 1; c >= 0; --c) {
    const int t0 = c * K, t1 = (t0 + K < n_steps) ? t0 + K : n_steps;
    if (K == 1) {  // every state is a checkpoint: nothing to re-run
      const double *st = ck + 2 * (size_t)n12 * c, *sn = ck + 2 * (size_t)n12 * (c + 1);
      ABD_TRY(op_adjoint_step(ctx, sc, prm, st, st + n12, sn, qb, qdb, rtol, prm->max_pcg, qb2, qdb2, nullptr, s));
      std::swap(qb, qb2);
      std::swap(qdb, qdb2);
      continue;
    }
    // re-run the segment, keeping every state
    const double *cs = ck + 2 * (size_t)n12 * c;
    HIP_TRY(ctx, hipMemcpyAsync(seg, cs, vb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(seg + n12, cs + n12, vb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(q, cs, vb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(qd, cs + n12, vb, hipMemcpyDeviceToDevice, s));
    for (int t = t0; t < t1; ++t) {
      ABD_TRY(abd_time_step(ctx, sc, prm, q, qd, nullptr, s));
      double *dst = seg + 2 * (size_t)n12 * (t - t0 + 1);
      HIP_TRY(ctx, hipMemcpyAsync(dst, q, vb, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(dst + n12, qd, vb, hipMemcpyDeviceToDevice, s));
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const double *st = seg + 2 * (size_t)n12 * (t - t0), *sn = seg + 2 * (size_t)n12 * (t - t0 + 1);
      ABD_TRY(op_adjoint_step(ctx, sc, prm, st, st + n12, sn, qb, qdb, rtol, prm->max_pcg, qb2, qdb2, nullptr, s));
      std::swap(qb, qb2);
      std::swap(qdb, qdb2);
    }
  }
  HIP_TRY(ctx, hipMemcpyAsync(qbar_0, qb, vb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(qdbar_0, qdb, vb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return ABD_OK;
}
