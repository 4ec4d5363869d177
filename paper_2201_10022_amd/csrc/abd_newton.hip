// Newton iteration and implicit-Euler time step (ABD sec. 4: minimise the
// incremental potential E = sum_b E_b + V_C; sec. 4.1: CCD at every
// iteration keeps the line search intersection free).  Host orchestration of
// the device operations; scalars cross to the host only where a decision is
// taken (counts, convergence, step bound, line-search comparison).
#include <chrono>
#include <cmath>

#include <cstring>

#include "abd_internal.h"

namespace {

__global__ void k_axpy(int n, const double *a, double alpha, const double *b, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + alpha * b[i];
}
__global__ void k_neg(int n, const double *a, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = -a[i];
}
__global__ void k_velocity(int n, const uint8_t *fixed, const double *qn, const double *qo, double inv_dt,
                           double *qd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  qd[i] = fixed[i / 12] ? 0.0 : (qn[i] - qo[i]) * inv_dt;
}
__global__ void k_zero(int64_t n, double *a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

int zero(abd_ctx *ctx, double *a, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_zero, dim3(grid_for(n, 256)), dim3(256), 0, s, n, a);
  return abd_hip_check(ctx, hipGetLastError(), "k_zero");
}

// four arrays cleared by one launch (index i runs over their concatenation)
struct Zero4 {
  double *p[4];
  int64_t n[4];
};
__global__ void k_zero4(Zero4 z, int64_t total) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i < z.n[k]) {
      z.p[k][i] = 0.0;
      return;
    }
    i -= z.n[k];
  }
}
int zero4(abd_ctx *ctx, double *a, int64_t na, double *b, int64_t nb, double *c, int64_t nc, double *d, int64_t nd,
          hipStream_t s) {
  const Zero4 z = {{a, b, c, d}, {na, nb, nc, nd}};
  const int64_t total = na + nb + nc + nd;
  if (total > 0) hipLaunchKernelGGL(k_zero4, dim3(grid_for(total, 256)), dim3(256), 0, s, z, total);
  return abd_hip_check(ctx, hipGetLastError(), "k_zero4");
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

int op_read_err(abd_ctx *ctx, hipStream_t s) {
  int *h;
  ABD_TRY(pinned_get(ctx, 64, reinterpret_cast<void **>(&h)));
  ABD_TRY(err_enqueue(ctx, h, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return err_check(ctx, h[0], s);
}

int err_enqueue(abd_ctx *ctx, int *h_err, hipStream_t s) {
  int *err;
  ABD_TRY(ws(ctx, "err_flag", 1, &err, s));
  HIP_TRY(ctx, hipMemcpyAsync(h_err, err, sizeof(int), hipMemcpyDeviceToHost, s));
  return ABD_OK;
}

int err_check(abd_ctx *ctx, int e, hipStream_t s) {
  int *err;
  ABD_TRY(ws(ctx, "err_flag", 1, &err, s));
  if (e) HIP_TRY(ctx, hipMemsetAsync(err, 0, sizeof(int), s));
  if (e & 1) return abd_fail(ctx, ABD_E_INTERSECT, "pair at zero distance");
  if (e & 2) return abd_fail(ctx, ABD_E_INVALID, "pair's body pair missing from the off-diagonal keys");
  if (e & 4) return abd_fail(ctx, ABD_E_PCG, "diagonal block not positive definite");
  if (e & 8) return abd_fail(ctx, ABD_E_PCG, "PCG breakdown (non-positive curvature)");
  if (e & 16) return abd_fail(ctx, ABD_E_HIP, "scan: look-back wait exceeded its cap");
  return ABD_OK;
}

namespace {

// small results straight into mapped host memory (one launch instead of a
// copy per array): ha[0..na) = a[0, as, 2 as ..), hb[0..nb) = b, *he = *e
__global__ void k_to_host(const double *a, int na, const double *b, int nb, const int *e, double *ha, double *hb,
                          int *he, int as = 1) {
  for (int i = threadIdx.x; i < na; i += blockDim.x) ha[i] = a[(int64_t)as * i];
  for (int i = threadIdx.x; i < nb; i += blockDim.x) hb[i] = b[i];
  if (e && threadIdx.x == 0) *he = *e;
}

// per-body masks and per-scene step lengths
__global__ void k_neg_masked(int nb, const int32_t *body_scene, const uint8_t *done, const double *g, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 12 * nb) return;
  out[i] = done[body_scene[i / 12]] ? 0.0 : -g[i];
}
__global__ void k_zero_done(int nb, const int32_t *body_scene, const uint8_t *done, double *p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 12 * nb) return;
  if (done[body_scene[i / 12]]) p[i] = 0.0;
}
// the accepted step, in place: q += alpha[scene] p as one fused multiply-add
// per entry (the trial states' arithmetic); scenes with alpha 0 (done, or
// not accepted yet) keep q bit for bit
__global__ void k_step_scenes(int nb, const int32_t *body_scene, const double *alpha, const double *p, double *q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 12 * nb) return;
  const double al = alpha[body_scene[i / 12]];
  if (al != 0.0) q[i] = fma(al, p[i], q[i]);
}
// newly converged scenes: done[j] |= disp[j stride] <= tol (the host takes
// the same decision on the same values for its own copy of the flags).
// With cg_state (the solver's state, int[4]) only when the solve that made
// the direction has stopped every scene on its tolerance.
__global__ void k_done_update(int S, const double *disp, int stride, double tol, uint8_t *done,
                              const int *cg_state) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S || done[j]) return;
  if (cg_state && !(cg_state[1] >= S && cg_state[3] == 0)) return;
  if (disp[(int64_t)stride * j] <= tol) done[j] = 1;
}
// the first line-search batch's decision per scene: alpha[j] = the first
// trial step alpha_ccd 2^-t (t < kb) whose energy e[S + t S + j] does not
// exceed E(q) = e[j]; 0 for done scenes and scenes with no such trial
__global__ void k_ls_accept(int S, int kb, const uint8_t *done, const double *a_ccd, const double *e,
                            double *alpha) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S) return;
  double al = 0.0;
  if (!done[j]) {
    int t = 0;
    while (t < kb && !(e[S + (int64_t)t * S + j] <= e[j])) ++t;
    if (t < kb) al = ldexp(a_ccd[j], -t);
  }
  alpha[j] = al;
}
// The trial states of a line-search batch in one launch (trial in grid.y):
// blocks [0, nqb) form q_t = q + alpha_t p per entry with one fused
// multiply-add, as the accepted step does; the others (launched only when lagged friction
// reads vertex positions; the barrier maps its pairs' vertices from q_t
// itself) map every vertex, x_t = x(q_t), with the same arithmetic as the
// vertex map and q_t formed in place by that same fused multiply-add, so
// they need not wait for the first part.
__global__ void __launch_bounds__(256) k_trial_states(int nb, int S, const int32_t *body_scene, const double *q,
                                                      const double *alpha, const double *p, double *qn, int nv,
                                                      const double *xbar, const int32_t *vert_body, double *xn,
                                                      int nqb) {
#pragma clang fp contract(off)
  const int t = blockIdx.y;
  if ((int)blockIdx.x < nqb) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 12 * nb) return;
    qn[(int64_t)t * 12 * nb + i] = fma(alpha[(int64_t)t * S + body_scene[i / 12]], p[i], q[i]);
    return;
  }
  const int k = ((int)blockIdx.x - nqb) * 256 + threadIdx.x;
  if (k >= nv) return;
  const int64_t b = vert_body[k];
  const double al = alpha[(int64_t)t * S + body_scene[b]];
  double qb[12];
#pragma unroll
  for (int j = 0; j < 12; ++j) qb[j] = fma(al, p[12 * b + j], q[12 * b + j]);
  const double xb0 = xbar[3 * k], xb1 = xbar[3 * k + 1], xb2 = xbar[3 * k + 2];
  double *x = xn + (int64_t)t * 3 * nv;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double *a = qb + 3 + 3 * i;
    x[3 * k + i] = qb[i] + ((a[0] * xb0 + a[1] * xb1) + a[2] * xb2);
  }
}

// (one scene, one step length passed by value)
__global__ void k_axpy1(int n, const double *a, double alpha, const double *b, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + alpha * b[i];
}

// step lengths of the first line-search batch: row 0 is 0 (E(q) itself),
// row t >= 1 is alpha_ccd 2^-(t-1) (0 for scenes already done)
__global__ void k_ls_trials(int S, int n, const uint8_t *done, const double *a_ccd, double *a_tr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S * n) return;
  const int j = i % S, t = i / S;
  a_tr[i] = t == 0 || done[j] ? 0.0 : ldexp(a_ccd[j], -(t - 1));
}

// per-scene E(q + alpha_t p) for n trials (alpha [n][S] on the device) over
// the given (swept) candidates into e_dev [n][S]; all trials go through the
// same launches (a trial dimension in the grid), enqueued only
int energy_trials(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, const double *p,
                  const double *qt, const double *alpha, int n, const int32_t *pt, int64_t npt, const int32_t *ee,
                  int64_t nee, const FrictionSet *fr, double *e_dev, hipStream_t s,
                  const uint8_t *skip_scene = nullptr) {
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  const int nb = sc->n_bodies;
  const int64_t n12 = 12 * (int64_t)nb;
  double *qn, *xn = nullptr;
  ABD_TRY(ws(ctx, "ls_q", (size_t)n * n12, &qn, s));
  if (fr) ABD_TRY(ws(ctx, "ls_x", (size_t)n * 3 * sc->n_verts, &xn, s));
  // (one scene with items: the row sums below are assigned, not added; a
  // batch's per-scene sums are assigned by one launch over all segments)
  if (S == 1 && (int64_t)nb + npt + nee + (fr ? fr->n() : 0) == 0) ABD_TRY(zero(ctx, e_dev, (int64_t)n, s));
  {
    const int nqb = (int)grid_for(n12, 256);
    const int nvb = fr ? (int)grid_for(sc->n_verts, 256) : 0;
    hipLaunchKernelGGL(k_trial_states, dim3(nqb + nvb, n), dim3(256), 0, s, nb, S, sc->body_scene, q, alpha, p, qn,
                       sc->n_verts, sc->xbar, sc->vert_body, xn, nqb);
    HIP_TRY(ctx, hipGetLastError());
  }
  if (S > 1) {
    // (scenes already done: their energies are read by nobody)
    TrialSums ts;
    ts.skip = skip_scene;
    ABD_TRY(op_body_energy_trials(ctx, sc, prm, qn, qt, n, e_dev, s, nullptr, 0, &ts));
    ABD_TRY(op_barrier_energy_trials(ctx, sc, prm, qn, n, pt, npt, ee, nee, e_dev, s, nullptr, 0, &ts));
    if (fr) ABD_TRY(op_friction_energy_trials(ctx, sc, fr, xn, n, e_dev, s, nullptr, 0, &ts));
    return seg_sum_trials_multi(ctx, ts, n, S, e_dev, s);
  }
  // one scene: every item's energy of a trial in one row (bodies, barrier
  // pairs, friction pairs), one sum per row
  const int64_t nfr = fr ? fr->n() : 0;
  const int64_t nt = (int64_t)nb + npt + nee + nfr;
  double *items;
  ABD_TRY(ws(ctx, "ls_items", (size_t)n * nt, &items, s));
  ABD_TRY(op_body_energy_trials(ctx, sc, prm, qn, qt, n, nullptr, s, items, nt));
  if (npt + nee) ABD_TRY(op_barrier_energy_trials(ctx, sc, prm, qn, n, pt, npt, ee, nee, nullptr, s, items + nb, nt));
  if (nfr) ABD_TRY(op_friction_energy_trials(ctx, sc, fr, xn, n, nullptr, s, items + nb + npt + nee, nt));
  return seg_sum_trials(ctx, items, nt, nt, nullptr, n, 1, e_dev, s, true);
}

constexpr int LS_BATCH = 4;  // trial step lengths evaluated per line-search batch

}  // namespace

// One Newton iteration for every sub-scene not yet marked in done_dev
// (device [S], in/out).  Sub-scenes are independent problems: each has its
// own convergence test, CCD bound and line search (its own step length),
// and its own PCG scalars; a scene marked done keeps its q.
// done_mode: 0 read the done flags from done_dev, 1 they are all zero, 2 the
// staging area still holds them (the last call on this context wrote them)
int newton_iteration(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, double *q, const double *qt,
                     uint8_t *done_dev, abd_stats *st, hipStream_t s, bool reuse_sweep, int done_mode) {
  auto t_all = std::chrono::steady_clock::now();
  const int nb = sc->n_bodies, nv = sc->n_verts;
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  const int n12 = 12 * nb;
  double *x, *x1, *g, *diag, *off, *p, *qa, *alpha_dev;
  ABD_TRY(ws(ctx, "nt_x", 3 * (size_t)nv, &x, s));
  ABD_TRY(ws(ctx, "nt_x1", 3 * (size_t)nv, &x1, s));
  ABD_TRY(ws(ctx, "nt_g", n12, &g, s));
  ABD_TRY(ws(ctx, "nt_diag", 144 * (size_t)nb, &diag, s));
  ABD_TRY(ws(ctx, "nt_p", n12, &p, s));
  ABD_TRY(ws(ctx, "nt_qa", n12, &qa, s));
  ABD_TRY(ws(ctx, "nt_alpha", (size_t)(LS_BATCH + 1) * S, &alpha_dev, s));
  double *e_sc, *a_ccd;  // e_sc: E0 [S], then the trials' energies [LS_BATCH][S]
  ABD_TRY(ws(ctx, "nt_escene", (size_t)(LS_BATCH + 1) * S, &e_sc, s));
  ABD_TRY(ws(ctx, "nt_accd", S, &a_ccd, s));
  // host staging: error flag, done flags, per-scene disp / alpha / E0 / E1
  // (mapped memory: d_* are the device addresses of the same slots)
  double *h, *hd;
  ABD_TRY(pinned_get_nt(ctx, sizeof(double) * (8 + (4 + 2 * (size_t)LS_BATCH) * S), reinterpret_cast<void **>(&h),
                        reinterpret_cast<void **>(&hd)));
  int *h_err = reinterpret_cast<int *>(h), *d_err = reinterpret_cast<int *>(hd);
  double *h_disp = h + 8, *h_alpha = h_disp + S, *h_e0 = h_alpha + S, *h_e1 = h_e0 + S;  // h_e1 [LS_BATCH][S]
  double *d_disp = hd + 8, *d_alpha = d_disp + S, *d_e0 = d_alpha + S;
  double *h_atr = h_e1 + (size_t)LS_BATCH * S;                                          // [LS_BATCH][S]
  uint8_t *h_done = reinterpret_cast<uint8_t *>(h_atr + (size_t)LS_BATCH * S);
  if (done_mode == 0)
    HIP_TRY(ctx, hipMemcpyAsync(h_done, done_dev, S, hipMemcpyDeviceToHost, s));
  else if (done_mode == 1)
    std::memset(h_done, 0, S);

  // lagged friction of the current time step, if any
  FrictionSet frs;
  bool fr_on = false;
  ABD_TRY(op_friction_state(ctx, sc, prm, &frs, &fr_on, s));
  const FrictionSet *fr = fr_on ? &frs : nullptr;
  st->n_friction = fr_on ? frs.n() : 0;

  // gradient and projected Hessian at q
  auto t0 = std::chrono::steady_clock::now();
  // (without lagged friction no kernel of this iteration reads the vertices
  // of a scene already done, so they are not mapped)
  ABD_TRY(op_vertex_map(ctx, sc, q, x, s, done_mode == 1 || fr ? nullptr : done_dev));
  const int32_t *pt, *ee;
  int32_t *keys = nullptr;
  int64_t npt, nee, nk = 0;
  // The pairs whose activity is tested: after an accepted step, that step's
  // swept candidates (every pair within dhat at x lies in the sweep, since x
  // is on the swept segment, and the active pairs come out in the same
  // canonical order as from the static candidates at x); otherwise the
  // static candidates at x.  Scenes already done take no part (their
  // direction is zero).
  if (reuse_sweep && ctx->sw_valid) {
    pt = ctx->sw_pt;
    npt = ctx->sw_n_pt;
    ee = ctx->sw_ee;
    nee = ctx->sw_n_ee;
  } else {
    int32_t *cpt, *cee;
    ABD_TRY(op_candidates(ctx, sc, x, nullptr, prm->dhat, &cpt, &npt, &cee, &nee, "nt_st", s, done_dev));
    pt = cpt;
    ee = cee;
  }
  ctx->sw_valid = false;
  st->n_pt = npt;
  st->n_ee = nee;
  st->t_candidates_ms += ms_since(t0);
  // The off-diagonal pattern covers the active pairs (the only pairs with
  // Hessian blocks), the lagged friction pairs and the joints.  It is built
  // on the auxiliary stream, from the moment the active pairs are known,
  // while this stream runs the barrier's pair kernels, which do not read
  // it; the assembly joins it.
  KeyPattern pat;
  hipStream_t aux;
  ABD_TRY(aux_stream_get(ctx, &aux));
  {
    // (cached scene tables that both streams read are made here, before
    // the fork, so that their first build is ordered before every reader)
    const int32_t *sbo;
    ABD_TRY(op_scene_offsets(ctx, sc, &sbo, s));
    JointTables *jt = nullptr;
    if (sc->n_joints > 0) ABD_TRY(joint_tables(ctx, sc, &jt, s));
  }
  bool forked = false, joined = false;
  BarrierHooks hooks;
  hooks.active = [&](const int32_t *act, int64_t na, int64_t na_pt) -> int {
    HIP_TRY(ctx, hipEventRecord(ctx->ev_fork, s));
    HIP_TRY(ctx, hipStreamWaitEvent(aux, ctx->ev_fork, 0));
    // the body terms (they read q and q~ only; the assembly adds into the
    // same blocks after the join), then the pattern
    // (done scenes get a zero right-hand side: their body terms are not needed)
    ABD_TRY(zero4(ctx, g, n12, diag, 144 * (int64_t)nb, nullptr, 0, nullptr, 0, aux));
    ABD_TRY(op_body_terms(ctx, sc, prm, q, qt, nullptr, g, diag, 1, aux, done_dev));
    int32_t *apt, *aee;
    ABD_TRY(op_gather_active(ctx, act, na, na_pt, npt, pt, ee, &apt, &aee, aux));
    ABD_TRY(op_offdiag(ctx, sc, apt, na_pt, aee, na - na_pt, &keys, &nk, "nt_st", aux, fr ? fr->pt : nullptr,
                       fr ? fr->n_pt : 0, fr ? fr->ee : nullptr, fr ? fr->n_ee : 0, &pat, nullptr, 0, true));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_join, aux));
    forked = true;
    return ABD_OK;
  };
  hooks.join = [&](const int32_t **keys_j, int64_t *nk_j, double **off_j) -> int {
    if (!forked) ABD_TRY(hooks.active(nullptr, 0, 0));  // (no active pairs to hand over)
    if (!joined) {
      HIP_TRY(ctx, hipStreamSynchronize(aux));
      ABD_TRY(op_offdiag_count(ctx, &nk));
      HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->ev_join, 0));
      ABD_TRY(ws(ctx, "nt_off", 144 * (size_t)(nk + 1), &off, s));
      ABD_TRY(zero4(ctx, off, 144 * nk, nullptr, 0, nullptr, 0, nullptr, 0, s));
      joined = true;
    }
    if (keys_j) *keys_j = keys;
    if (nk_j) *nk_j = nk;
    if (off_j) *off_j = off;
    return ABD_OK;
  };
  // adaptive barrier stiffness: the doubling rule at this iterate, before
  // the barrier's derivatives and this iteration's energies
  if (ctx->kappa_sc) ABD_TRY(op_kappa_update(ctx, sc, prm, x, pt, npt, ee, nee, s));
  t0 = std::chrono::steady_clock::now();
  // (the energy at q comes with the line search's trials: none is summed
  // here; the body terms run in the hook)
  int64_t nap = 0, nae = 0;
  ABD_TRY(op_barrier(ctx, sc, prm, x, pt, npt, ee, nee, nullptr, 0, nullptr, g, diag, nullptr, 1, &nap, &nae, s, fr,
                     &hooks));
  ABD_TRY(hooks.join(nullptr, nullptr, nullptr));  // (when the barrier had nothing to assemble)
  st->n_offdiag = nk;
  if (sc->n_joints > 0 && prm->kappa_j > 0.0)
    ABD_TRY(op_joint_off(ctx, sc, prm->kappa_j * prm->dt * prm->dt, keys, nk, off, s));
  st->t_barrier_ms += ms_since(t0);
  st->n_active_pt = nap;
  st->n_active_ee = nae;

  // Newton direction (scenes already done get a zero right-hand side)
  t0 = std::chrono::steady_clock::now();
  double *rhs;
  ABD_TRY(ws(ctx, "nt_rhs", n12, &rhs, s));
  hipLaunchKernelGGL(k_neg_masked, dim3(grid_for(n12, 256)), dim3(256), 0, s, nb, sc->body_scene, done_dev, g, rhs);
  int its = 0;
  // (errors of the assembly and the solve are read with the displacement:
  // a failed assembly or block inverse leaves non-finite values that stop
  // the solve at once)
  // The displacement pass (per-scene max |J p|, errors, the done flags) is
  // enqueued behind each round of PCG replays, before the solver's own
  // synchronisation; its results stand when that round was the solve's
  // last (the flags change only then), else it runs again here.
  const double tol_disp = prm->newton_tol * prm->dt;
  auto disp_pass = [&](const int *cg_state) -> int {
    const double *dsp;
    int dstride;
    ABD_TRY(op_max_abs_disp_scenes(ctx, sc, p, &dsp, &dstride, s, done_dev));
    int *errf;
    ABD_TRY(ws(ctx, "err_flag", 1, &errf, s));
    hipLaunchKernelGGL(k_to_host, dim3(1), dim3(256), 0, s, dsp, S, nullptr, 0, errf, d_disp, nullptr, d_err,
                       dstride);
    hipLaunchKernelGGL(k_done_update, dim3(grid_for(S, 256)), dim3(256), 0, s, S, dsp, dstride, tol_disp, done_dev,
                       cg_state);
    return abd_hip_check(ctx, hipGetLastError(), "k_done_update");
  };
  // (below the check's tolerance the direction may change after the last
  // iterations: no early pass)
  const PcgHook pre_sync = disp_pass;
  bool disp_done = false;
  ABD_TRY(op_pcg(ctx, sc, diag, off, keys, nk, rhs, p, prm->pcg_rtol, prm->max_pcg, &its, s, nullptr, nullptr, &pat,
                 prm->pcg_rtol >= PCG_CHECK_RTOL ? &pre_sync : nullptr, &disp_done, done_dev));
  st->pcg_iters = its;
  st->t_solve_ms += ms_since(t0);
  if (!disp_done) {
    ABD_TRY(disp_pass(nullptr));
    HIP_TRY(ctx, hipStreamSynchronize(s));
  }
  ABD_TRY(err_check(ctx, h_err[0], s));
  double dmax = 0.0;
  int n_active = 0;
  for (int j = 0; j < S; ++j) {
    if (h_done[j]) continue;
    if (!std::isfinite(h_disp[j])) return abd_fail(ctx, ABD_E_PCG, "non-finite Newton direction (scene %d)", j);
    dmax = h_disp[j] > dmax ? h_disp[j] : dmax;
    if (h_disp[j] <= tol_disp) {
      h_done[j] = 1;
      ++st->newly_converged;
    } else {
      ++n_active;
    }
  }
  st->disp = dmax;
  if (n_active == 0) {
    st->converged = 1;
    st->alpha = 0.0;
    st->t_total_ms += ms_since(t_all);
    prof_flush(ctx);
    return ABD_OK;
  }
  st->converged = 0;
  hipLaunchKernelGGL(k_zero_done, dim3(grid_for(n12, 256)), dim3(256), 0, s, nb, sc->body_scene, done_dev, p);

  // CCD over the swept candidates of x(q) -> x(q + p)
  t0 = std::chrono::steady_clock::now();
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n12, 256)), dim3(256), 0, s, n12, q, 1.0, p, qa);
  // (the sweep and the CCD read no pair of a scene already done)
  ABD_TRY(op_vertex_map(ctx, sc, qa, x1, s, done_dev));
  int32_t *spt, *see;
  int64_t nspt, nsee;
  ABD_TRY(op_candidates(ctx, sc, x, x1, prm->dhat, &spt, &nspt, &see, &nsee, "nt_sw", s, done_dev));
  st->n_pt_swept = nspt;
  st->n_ee_swept = nsee;
  st->t_candidates_ms += ms_since(t0);
  t0 = std::chrono::steady_clock::now();
  ABD_TRY(op_ccd(ctx, sc, prm, x, nullptr, spt, nspt, see, nsee, nullptr, nullptr, a_ccd, s, x1));

  // backtracking line search, per scene: the trial step lengths
  // alpha 2^-j are evaluated in batches of K (K from the last iteration's
  // halvings) with one synchronisation per batch; each scene takes the
  // first trial that does not raise its energy, exactly as one-by-one
  // halving would.  E(q) and the first batch (its step lengths formed on
  // the device from the CCD bound) are enqueued behind the CCD, so one
  // synchronisation brings the bound, E(q) and the first batch's energies.
  int K = ctx->ls_hint + 1;
  K = K < 1 ? 1 : (K > LS_BATCH ? LS_BATCH : K);
  const int kb0 = K <= prm->max_ls ? K : (prm->max_ls > 0 ? prm->max_ls : 0);
  hipLaunchKernelGGL(k_ls_trials, dim3(grid_for((kb0 + 1) * S, 256)), dim3(256), 0, s, S, kb0 + 1, done_dev, a_ccd,
                     alpha_dev);
  ABD_TRY(energy_trials(ctx, sc, prm, q, p, qt, alpha_dev, kb0 + 1, spt, nspt, see, nsee, fr, e_sc, s, done_dev));
  hipLaunchKernelGGL(k_to_host, dim3(1), dim3(256), 0, s, a_ccd, S, e_sc, (kb0 + 1) * S, nullptr, d_alpha, d_e0,
                     nullptr);
  // (batches: the first batch's accepted steps are taken on the device
  // before the host has read the energies; it takes the same decisions)
  double *alpha_acc = nullptr;
  if (S > 1) {
    ABD_TRY(ws(ctx, "nt_alpha_acc", S, &alpha_acc, s));
    hipLaunchKernelGGL(k_ls_accept, dim3(grid_for(S, 256)), dim3(256), 0, s, S, kb0, done_dev, a_ccd, e_sc,
                       alpha_acc);
    hipLaunchKernelGGL(k_step_scenes, dim3(grid_for(n12, 256)), dim3(256), 0, s, nb, sc->body_scene, alpha_acc, p, q);
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  ABD_TRY(ws_collect(ctx));  // (the stream is idle here)
  st->t_ccd_ms += ms_since(t0);
  double amin = 1.0;
  for (int j = 0; j < S; ++j) {
    if (h_done[j]) h_alpha[j] = 0.0;
    else amin = h_alpha[j] < amin ? h_alpha[j] : amin;
  }
  st->alpha_ccd = amin;
  int k = 0;
  int max_halvings = 0;
  std::vector<int> halv(S, 0);
  std::vector<uint8_t> acc(S, 0), acc_first(S, 0);
  for (int j = 0; j < S; ++j) acc[j] = h_done[j];
  bool all_acc = false;
  while (k < prm->max_ls && !all_acc) {
    const int kb = k == 0 ? kb0 : (k + K <= prm->max_ls ? K : prm->max_ls - k);
    if (k > 0) {
      for (int t = 0; t < kb; ++t)
        for (int j = 0; j < S; ++j) h_atr[(size_t)t * S + j] = acc[j] ? 0.0 : std::ldexp(h_alpha[j], -t);
      HIP_TRY(ctx, hipMemcpyAsync(alpha_dev, h_atr, (size_t)kb * S * sizeof(double), hipMemcpyHostToDevice, s));
      ABD_TRY(energy_trials(ctx, sc, prm, q, p, qt, alpha_dev, kb, spt, nspt, see, nsee, fr, e_sc + S, s, done_dev));
      HIP_TRY(ctx, hipMemcpyAsync(h_e1, e_sc + S, (size_t)kb * S * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
    }
    all_acc = true;
    for (int j = 0; j < S; ++j) {
      if (acc[j]) continue;
      int t = 0;
      while (t < kb && !(h_e1[(size_t)t * S + j] <= h_e0[j])) ++t;
      if (t < kb) {
        acc[j] = 1;
        acc_first[j] = k == 0;
        h_alpha[j] = std::ldexp(h_alpha[j], -t);
        halv[j] += t;
        h_e1[j] = h_e1[(size_t)t * S + j];
      } else {
        h_alpha[j] = std::ldexp(h_alpha[j], -kb);
        halv[j] += kb;
        all_acc = false;
      }
    }
    if (kb <= 0) break;
    k += kb;
  }
  if (!all_acc) return abd_fail(ctx, ABD_E_LINESEARCH, "line search found no decrease");
  // the accepted point of every scene
  // (in place: each element reads q[i] before writing it)
  if (S == 1) {
    hipLaunchKernelGGL(k_axpy1, dim3(grid_for(n12, 256)), dim3(256), 0, s, n12, q, h_alpha[0], p, q);
  } else {
    // (scenes accepted in the first batch have taken their step already)
    bool later = false;
    for (int j = 0; j < S; ++j) {
      h_atr[j] = h_done[j] || acc_first[j] ? 0.0 : h_alpha[j];
      later = later || h_atr[j] != 0.0;
    }
    if (later) {
      HIP_TRY(ctx, hipMemcpyAsync(alpha_dev, h_atr, S * sizeof(double), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_step_scenes, dim3(grid_for(n12, 256)), dim3(256), 0, s, nb, sc->body_scene, alpha_dev,
                         p, q);
    }
  }
  double e0 = 0.0, e1 = 0.0, amin_acc = 1.0;
  for (int j = 0; j < S; ++j) {
    if (h_done[j]) continue;
    e0 += h_e0[j];
    e1 += h_e1[j];
    amin_acc = h_alpha[j] < amin_acc ? h_alpha[j] : amin_acc;
    max_halvings = halv[j] > max_halvings ? halv[j] : max_halvings;
  }
  st->ls_halvings = max_halvings;
  ctx->ls_hint = max_halvings;
  st->alpha = amin_acc;
  st->energy0 = e0;
  st->energy1 = e1;
  ctx->sw_valid = true;
  ctx->sw_pt = spt;
  ctx->sw_ee = see;
  ctx->sw_n_pt = nspt;
  ctx->sw_n_ee = nsee;
  st->t_total_ms += ms_since(t_all);
  prof_flush(ctx);
  return ABD_OK;
}

extern "C" int abd_newton_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, double *q,
                               const double *q_tilde, uint8_t *scene_done, abd_stats *stats, hipStream_t stream) {
  if (!ctx || !sc || !prm || !q || !q_tilde || !sc->mass || !sc->volume)
    return abd_fail(ctx, ABD_E_INVALID, "abd_newton_step: null");
  if (prm->kappa_adaptive)
    return abd_fail(ctx, ABD_E_INVALID, "abd_newton_step: the adaptive barrier stiffness runs inside abd_time_step");
  abd_stats local = {};
  abd_stats *st = stats ? stats : &local;
  *st = abd_stats{};
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  uint8_t *done = scene_done;
  if (!done) {
    ABD_TRY(ws(ctx, "ns_done", S, &done, stream));
    HIP_TRY(ctx, hipMemsetAsync(done, 0, S, stream));
  }
  ABD_TRY(newton_iteration(ctx, sc, prm, q, q_tilde, done, st, stream, false, scene_done ? 0 : 1));
  st->newton_iters = 1;
  return ABD_OK;
}

extern "C" int abd_time_step(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, double *q, double *qdot,
                             abd_stats *stats, hipStream_t stream) {
  if (!ctx || !sc || !prm || !q || !qdot || !sc->mass || !sc->volume)
    return abd_fail(ctx, ABD_E_INVALID, "abd_time_step: null");
  const int n12 = 12 * sc->n_bodies;
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  double *qt, *qo;
  uint8_t *done;
  ABD_TRY(ws(ctx, "ts_qt", n12, &qt, stream));
  ABD_TRY(ws(ctx, "ts_qo", n12, &qo, stream));
  ABD_TRY(ws(ctx, "ts_done", S, &done, stream));
  HIP_TRY(ctx, hipMemsetAsync(done, 0, S, stream));
  ABD_TRY(abd_q_tilde(ctx, sc, prm, q, qdot, qt, stream));
  HIP_TRY(ctx, hipMemcpyAsync(qo, q, sizeof(double) * n12, hipMemcpyDeviceToDevice, stream));
  // adaptive barrier stiffness: set at q^t (before friction is lagged with
  // it), read by the barrier kernels until the step returns
  struct KappaScope {
    abd_ctx *c;
    ~KappaScope() { c->kappa_sc = nullptr; }
  } kappa_scope{ctx};
  if (prm->kappa_adaptive) {
    if (!(prm->kappa_b > 0.0) || !(prm->kappa_max >= prm->kappa_b) || !(prm->kappa_eps_d >= 0.0))
      return abd_fail(ctx, ABD_E_INVALID, "abd_time_step: adaptive stiffness needs 0 < kappa_b <= kappa_max, eps_d >= 0");
    ABD_TRY(op_kappa_init(ctx, sc, prm, q, qt, stream));
    ABD_TRY(ws(ctx, "kappa_sc", S, &ctx->kappa_sc, stream));
  }
  // friction lagged once at q^t, released when the step returns
  struct FrictionScope {
    abd_ctx *c;
    ~FrictionScope() { abd_friction_end_step(c); }
  } fr_scope{ctx};
  int64_t n_fr = 0;
  if (prm->mu > 0.0) ABD_TRY(abd_friction_begin_step(ctx, sc, prm, q, &n_fr, stream));
  abd_stats total = {};
  total.n_friction = n_fr;
  int it = 0;
  int n_left = S;
  bool conv = false;
  for (; it < prm->max_newton; ++it) {
    abd_stats st = {};
    ABD_TRY(newton_iteration(ctx, sc, prm, q, qt, done, &st, stream, it > 0, it > 0 ? 2 : 1));
    // every scene still iterating ran this iteration
    total.scene_newton_iters += n_left;
    n_left -= st.newly_converged;
    total.n_pt = st.n_pt;
    total.n_ee = st.n_ee;
    total.n_active_pt += st.n_active_pt;
    total.n_active_ee += st.n_active_ee;
    total.n_pt_swept += st.n_pt_swept;
    total.n_ee_swept += st.n_ee_swept;
    total.n_offdiag = st.n_offdiag;
    total.pcg_iters += st.pcg_iters;
    total.ls_halvings += st.ls_halvings;
    total.t_barrier_ms += st.t_barrier_ms;
    total.t_ccd_ms += st.t_ccd_ms;
    total.t_candidates_ms += st.t_candidates_ms;
    total.t_solve_ms += st.t_solve_ms;
    total.t_total_ms += st.t_total_ms;
    total.disp = st.disp;
    if (st.converged) {
      conv = true;
      break;
    }
    total.alpha_ccd = st.alpha_ccd;
    total.alpha = st.alpha;
  }
  total.newton_iters = it + 1;
  total.converged = conv ? 1 : 0;
  if (stats) *stats = total;
  if (!conv) return abd_fail(ctx, ABD_E_NOT_CONVERGED, "Newton did not converge in %d iterations", prm->max_newton);
  hipLaunchKernelGGL(k_velocity, dim3(grid_for(n12, 256)), dim3(256), 0, stream, n12, sc->body_fixed, q, qo,
                     1.0 / prm->dt, qdot);
  return abd_hip_check(ctx, hipGetLastError(), "k_velocity");
}
