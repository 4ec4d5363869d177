// Narrow phase and barrier assembly (ABD sec. 4 Eq. barrier / clamped-b,
// sec. 4.3 contact-aware two-pass Hessian construction).
//
// Pass 1 (k_barrier_local, one lane per active pair): distance case, the
// case distance's gradient and Hessian, the clamped log barrier (EE pairs
// mollified), the 12x12 local Hessian and its PSD projection.  The
// projection runs on the 9x9 matrix of relative motions: the barrier of a
// pair is invariant under a common translation of its 4 vertices, so the
// translations span an exact null space of the local Hessian; with the
// orthonormal 4-point Helmert basis Q (12x9) the local Hessian is
// Q H9 Q^T and its PSD projection is Q (H9)_+ Q^T.
// Pass 2: every active pair emits up to three records (its two bodies'
// diagonal blocks and the body pair's off-diagonal block); records are
// stably sorted by block and each block's records are reduced in a fixed
// order (chunks of RCH records, then chunk partials in order), so the
// assembled matrix is bit-reproducible run to run.
#include "abd_barrier_math.h"

#include <mutex>

namespace {
using namespace abd_math;

// --------------------------------------------------------------- kernels ----
__device__ __forceinline__ void load_pair(int64_t idx, int64_t n_pt, const int32_t *pt, const int32_t *ee,
                                          const int32_t *tris, const int32_t *edges, const double *x, int &is_ee,
                                          int vid[4], d3 X[4]) {
  is_ee = idx >= n_pt;
  const int32_t *pr = is_ee ? ee + 2 * (idx - n_pt) : pt + 2 * idx;
  pair_vids(is_ee, pr, tris, edges, vid);
#pragma unroll
  for (int k = 0; k < 4; ++k) X[k] = ld3(x, vid[k]);
}

__global__ void __launch_bounds__(256) k_classify(int64_t n, int is_ee, const int32_t *pairs, const int32_t *tris,
                                                  const int32_t *edges, const double *x, double dhat2,
                                                  uint8_t *type, double *d2, uint8_t *active) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int vid[4];
  pair_vids(is_ee, pairs + 2 * i, tris, edges, vid);
  d3 X[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) X[k] = ld3(x, vid[k]);
  const int ty = classify_pair(is_ee, X);
  double num, den;
  case_nd(ty, X, num, den);
  if (type) type[i] = (uint8_t)ty;
  if (d2) d2[i] = num / den;
  if (active) active[i] = num < dhat2 * den ? 1 : 0;
}

// active flags over the combined PT+EE index space
__global__ void __launch_bounds__(256) k_active_flags(int64_t n_pt, int64_t n, const int32_t *pt, const int32_t *ee,
                                                      const int32_t *tris, const int32_t *edges, const double *x,
                                                      double dhat2, int64_t *flag) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int is_ee, vid[4];
  d3 X[4];
  load_pair(i, n_pt, pt, ee, tris, edges, x, is_ee, vid, X);
  const int ty = classify_pair(is_ee, X);
  double num, den;
  case_nd(ty, X, num, den);
  flag[i] = num < dhat2 * den ? 1 : 0;
}

__global__ void k_compact(int64_t n, const int64_t *flag, const int64_t *pos, int32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = (int32_t)i;
}

template <int BS>
__global__ void __launch_bounds__(BS) k_barrier_local(const int64_t *n_act_dev, const int32_t *act, int64_t n_pt,
                                                      const int32_t *pt, const int32_t *ee, const int32_t *tris,
                                                      const int32_t *edges, const int32_t *vert_body,
                                                      const double *x, const double *xbar, double dhat,
                                                      double kappa, int project, double *e_out, double *g_out,
                                                      double *H_out, PairInfo *info, int *err,
                                                      const double *kappa_sc, const int32_t *body_scene) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= *n_act_dev) return;
  const int64_t idx = act[a];
  int is_ee, vid[4];
  d3 X[4];
  load_pair(idx, n_pt, pt, ee, tris, edges, x, is_ee, vid, X);
  double xb4[12];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) xb4[3 * k + c] = xbar[3 * (int64_t)vid[k] + c];
  int ty;
  double num, den;
  {
#pragma clang fp contract(off)
    ty = classify_pair(is_ee, X);
    case_nd(ty, X, num, den);
  }
  PairInfo pi;
#pragma unroll
  for (int k = 0; k < 4; ++k) pi.vid[k] = vid[k];
  pi.body[0] = vert_body[vid[0]];
  pi.body[1] = vert_body[vid[3]];
  pi.is_ee = is_ee;
  pi.pad = ty;
  info[a] = pi;
  if (num == 0.0) {
    atomicOr(err, 1);
    e_out[a] = INFINITY;
#pragma unroll
    for (int i = 0; i < 12; ++i) g_out[12 * a + i] = 0.0;
#pragma unroll
    for (int i = 0; i < 78; ++i) H_out[78 * a + i] = 0.0;
    return;
  }
  LocalOut o;
  // (per-scene stiffness when it adapts)
  barrier_local(is_ee, ty, X, xb4, dhat, kappa_sc ? kappa_sc[body_scene[pi.body[0]]] : kappa, 0, o);
  // energy and gradient leave before the projection, whose eigen-solve
  // needs the registers
  e_out[a] = o.e;
#pragma unroll
  for (int i = 0; i < 12; ++i) g_out[12 * a + i] = o.g[i];
  if (project) project_translation_invariant(o.H);
#pragma unroll
  for (int i = 0; i < 78; ++i) H_out[78 * a + i] = o.H[i];
}

__device__ __forceinline__ int find_key(const int32_t *keys, int64_t n, int a, int b) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int ka = keys[2 * mid], kb = keys[2 * mid + 1];
    if (ka < a || (ka == a && kb < b))
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < n && keys[2 * lo] == a && keys[2 * lo + 1] == b) ? (int)lo : -1;
}

// records: key = block id (diag b -> b, off k -> nb + k), val = 4 a + role
//   role 0 diag of slot-0 body, 1 diag of slot-1 body,
//   2 off block with rows = slot-0 body, 3 off block with rows = slot-1 body
__global__ void k_records(int64_t n, const PairInfo *info, const uint8_t *fixed, int nb, const int32_t *keys,
                          int64_t n_keys, uint32_t *rkey, uint32_t *rval, int want_off, int *err) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const PairInfo pi = info[a];
  const int b0 = pi.body[0], b1 = pi.body[1];
  const bool f0 = fixed[b0] != 0, f1 = fixed[b1] != 0;
  // (records that belong to no block take key nb + n_keys, past the last
  // block, so that the sort needs only the bits of that value)
  const uint32_t none = (uint32_t)(nb + n_keys);
  rkey[3 * a] = f0 ? none : (uint32_t)b0;
  rval[3 * a] = (uint32_t)(4 * a + 0);
  rkey[3 * a + 1] = f1 ? none : (uint32_t)b1;
  rval[3 * a + 1] = (uint32_t)(4 * a + 1);
  uint32_t ko = none;
  if (want_off && !f0 && !f1) {
    const int k = find_key(keys, n_keys, min(b0, b1), max(b0, b1));
    if (k < 0)
      atomicOr(err, 2);
    else
      ko = (uint32_t)(nb + k);
  }
  rkey[3 * a + 2] = ko;
  rval[3 * a + 2] = (uint32_t)(4 * a + (b0 < b1 ? 2 : 3));
}

constexpr int RCH = 8;    // records per chunk (a short serial chain per wave)
constexpr int NENT = 156; // 144 block entries + 12 gradient entries

// chunk counts per block from the sorted keys (binary search)
__global__ void k_block_chunks(int64_t nblocks, const uint32_t *skey, int64_t nrec, int64_t *bstart) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nblocks) return;
  int64_t lo = 0, hi = nrec;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (skey[mid] < (uint32_t)b)
      lo = mid + 1;
    else
      hi = mid;
  }
  bstart[b] = lo;
}
__global__ void k_block_nchunk(int64_t nblocks, const int64_t *bstart, int64_t *nchunk) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblocks) return;
  const int64_t c = bstart[b + 1] - bstart[b];
  nchunk[b] = (c + RCH - 1) / RCH;
}

// one wave per chunk: entries strided over lanes, records staged in LDS
__global__ void __launch_bounds__(64) k_assemble_chunks(int64_t nblocks, const int64_t *chunk_off,
                                                        const int64_t *n_chunks_dev, const int64_t *bstart,
                                                        const uint32_t *sval, const PairInfo *info,
                                                        const double *g_loc, const double *H_loc,
                                                        const double *xbar, double *partial) {
  __shared__ double sH[78];
  __shared__ double sg[12];
  __shared__ double sx[4][4];  // xhat = (1, xbar) per slot
  __shared__ int srole, sis_ee;
  const int64_t ch = blockIdx.x;
  if (ch >= *n_chunks_dev) return;
  // block of this chunk: last b with chunk_off[b] <= ch
  int64_t lo = 0, hi = nblocks - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (chunk_off[mid] <= ch)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t blk = lo;
  const int64_t r0 = bstart[blk] + (ch - chunk_off[blk]) * RCH;
  const int64_t r1 = min(bstart[blk + 1], r0 + RCH);
  const int lane = threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t r = r0; r < r1; ++r) {
    const uint32_t val = sval[r];
    const int64_t a = val >> 2;
    if (lane < 78) sH[lane] = H_loc[78 * a + lane];
    if (lane + 64 < 78) sH[lane + 64] = H_loc[78 * a + lane + 64];
    if (lane < 12) sg[lane] = g_loc[12 * a + lane];
    if (lane < 16) {
      const int k = lane >> 2, c = lane & 3;
      sx[k][c] = c == 0 ? 1.0 : xbar[3 * (int64_t)info[a].vid[k] + c - 1];
    }
    if (lane == 0) {
      srole = (int)(val & 3u);
      sis_ee = info[a].is_ee;
    }
    __syncthreads();
    const int role = srole;
    // vertex slots of each body slot: PT {0} | {1,2,3}; EE {0,1} | {2,3}
    const int n0 = sis_ee ? 2 : 1;
    const int rb = (role == 0 || role == 2) ? 0 : 1;  // row body slot
    const int cb = (role == 0 || role == 3) ? 0 : 1;  // col body slot
    const int rk0 = rb == 0 ? 0 : n0, rk1 = rb == 0 ? n0 : 4;
    const int ck0 = cb == 0 ? 0 : n0, ck1 = cb == 0 ? n0 : 4;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int e = lane + 64 * q;
      if (e >= NENT) continue;
      double v = 0.0;
      if (e < 144) {
        const int rr = e / 12, cc = e % 12;
        const int i = rr < 3 ? rr : (rr - 3) / 3, mu = rr < 3 ? 0 : 1 + (rr - 3) % 3;
        const int j = cc < 3 ? cc : (cc - 3) / 3, nu = cc < 3 ? 0 : 1 + (cc - 3) % 3;
        for (int k = rk0; k < rk1; ++k)
          for (int l = ck0; l < ck1; ++l) v += sH[S12::at(3 * k + i, 3 * l + j)] * sx[k][mu] * sx[l][nu];
      } else if (role < 2) {
        const int rr = e - 144;
        const int i = rr < 3 ? rr : (rr - 3) / 3, mu = rr < 3 ? 0 : 1 + (rr - 3) % 3;
        for (int k = rk0; k < rk1; ++k) v += sg[3 * k + i] * sx[k][mu];
      }
      acc[q] += v;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int e = lane + 64 * q;
    if (e < NENT) partial[NENT * ch + e] = acc[q];
  }
}

// sum each block's chunk partials in order and add to the outputs
__global__ void k_assemble_final(int64_t nblocks, int nb, const int64_t *chunk_off, const int64_t *nchunk,
                                 const double *partial, const int32_t *keys, double *grad, double *diag,
                                 double *off) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblocks * NENT) return;
  const int64_t blk = t / NENT;
  const int e = (int)(t % NENT);
  const int64_t c0 = chunk_off[blk], nc = nchunk[blk];
  if (nc == 0) return;
  double v = 0.0;
  for (int64_t c = 0; c < nc; ++c) v += partial[NENT * (c0 + c) + e];
  if (blk < nb) {
    if (e < 144) {
      if (diag) diag[144 * blk + e] += v;
    } else if (grad) {
      grad[12 * blk + (e - 144)] += v;
    }
  } else if (e < 144 && off) {
    off[144 * (blk - nb) + e] += v;
  }
}

// pair energies; key_out (may be NULL) receives each pair's scene
// (grid.y > 1: trial t's positions at x + t xstride, energies at
// e_out + t estride, estride 0: n).  With qmap non-NULL the positions are
// mapped from the body states at qmap + t qstride instead (x unused): the
// pairs' vertices only, with the vertex map's arithmetic.
__global__ void k_energy_only(int64_t n_pt, int64_t n, const int32_t *pt, const int32_t *ee, const int32_t *tris,
                              const int32_t *edges, const double *x, const double *xbar, double dhat,
                              double kappa, double *e_out, const int32_t *vert_body, const int32_t *body_scene,
                              int32_t *key_out, int64_t xstride = 0, int64_t estride = 0,
                              const double *kappa_sc = nullptr, const double *qmap = nullptr, int64_t qstride = 0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  e_out += blockIdx.y * (estride > 0 ? estride : n);
  int is_ee, vid[4];
  d3 X[4];
  if (qmap) {
    is_ee = i >= n_pt;
    pair_vids(is_ee, is_ee ? ee + 2 * (i - n_pt) : pt + 2 * i, tris, edges, vid);
    qmap += blockIdx.y * qstride;
#pragma unroll
    for (int k = 0; k < 4; ++k) X[k] = map_vertex(qmap, vert_body, xbar, vid[k]);
  } else {
    load_pair(i, n_pt, pt, ee, tris, edges, x + blockIdx.y * xstride, is_ee, vid, X);
  }
  if (key_out && blockIdx.y == 0) key_out[i] = body_scene[vert_body[vid[0]]];
  int ty;
  double num, den;
  {
#pragma clang fp contract(off)
    ty = classify_pair(is_ee, X);
    case_nd(ty, X, num, den);
  }
  const double dhat2 = dhat * dhat;
  bool act;
  {
#pragma clang fp contract(off)
    act = num < dhat2 * den;
  }
  if (!act) {
    e_out[i] = 0.0;
    return;
  }
  if (num == 0.0) {
    e_out[i] = INFINITY;
    return;
  }
  const double s = num / den, d = sqrt(s);
  double b = -(d - dhat) * (d - dhat) * log(d / dhat);
  if (is_ee) {
    const d3 n3 = xcross(xsub(X[1], X[0]), xsub(X[3], X[2]));
    const double c = xdot(n3, n3);
    const d3 a0 = ld3(xbar, vid[0]), a1 = ld3(xbar, vid[1]), b0 = ld3(xbar, vid[2]), b1 = ld3(xbar, vid[3]);
    const d3 uu = xsub(a1, a0), vv = xsub(b1, b0);
    const double eps = (1e-3 * xdot(uu, uu)) * xdot(vv, vv);
    if (c < eps) {
      const double r = c / eps;
      b = (2.0 - r) * r * b;
    }
  }
  // (per-scene stiffness when it adapts)
  e_out[i] = (kappa_sc ? kappa_sc[body_scene[vert_body[vid[0]]]] : kappa) * b;
}

}  // namespace

namespace {
__global__ void k_gather_active(int64_t na, int64_t na_pt, int64_t n_pt, const int32_t *act, const int32_t *pt,
                                const int32_t *ee, int32_t *pt_out, int32_t *ee_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= na) return;
  const int64_t k = act[i];
  const int32_t *src = k < n_pt ? pt + 2 * k : ee + 2 * (k - n_pt);
  int32_t *dst = i < na_pt ? pt_out + 2 * i : ee_out + 2 * (i - na_pt);
  dst[0] = src[0];
  dst[1] = src[1];
}
}  // namespace

int op_gather_active(abd_ctx *ctx, const int32_t *act, int64_t na, int64_t na_pt, int64_t n_pt, const int32_t *pt,
                     const int32_t *ee, int32_t **pt_out, int32_t **ee_out, hipStream_t s) {
  ABD_TRY(ws(ctx, "ba_pt", 2 * (size_t)na_pt + 2, pt_out, s));
  ABD_TRY(ws(ctx, "ba_ee", 2 * (size_t)(na - na_pt) + 2, ee_out, s));
  if (na > 0)
    hipLaunchKernelGGL(k_gather_active, dim3(grid_for(na, 256)), dim3(256), 0, s, na, na_pt, n_pt, act, pt, ee,
                       *pt_out, *ee_out);
  return abd_hip_check(ctx, hipGetLastError(), "k_gather_active");
}

int op_barrier(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x, const int32_t *pt,
               int64_t n_pt, const int32_t *ee, int64_t n_ee, const int32_t *keys, int64_t n_keys, double *energy,
               double *grad, double *diag, double *off, int project, int64_t *n_active_pt, int64_t *n_active_ee,
               hipStream_t s, const FrictionSet *fr, const BarrierHooks *hooks) {
  const int64_t n = n_pt + n_ee;
  const int64_t nf = fr ? fr->n() : 0;
  if (n_active_pt) *n_active_pt = 0;
  if (n_active_ee) *n_active_ee = 0;
  if (n + nf == 0) return ABD_OK;
  const double dhat = prm->dhat, dhat2 = dhat * dhat;
  int64_t *flag, *pos, *nact;
  int32_t *act;
  int *err;
  ABD_TRY(ws(ctx, "br_flag", n, &flag, s));
  ABD_TRY(ws(ctx, "br_pos", n, &pos, s));
  ABD_TRY(ws(ctx, "br_nact", 2, &nact, s));
  ABD_TRY(ws(ctx, "br_act", n, &act, s));
  ABD_TRY(ws(ctx, "err_flag", 1, &err, s));
  int64_t na = 0, na_pt = 0;
  if (n > 0) {
    hipLaunchKernelGGL(k_active_flags, dim3(grid_for(n, 256)), dim3(256), 0, s, n_pt, n, pt, ee, sc->tris, sc->edges,
                       x, dhat2, flag);
    // active counts (total, and the PT part pos[n_pt]) written to mapped
    // host memory by the scan
    int64_t *hbuf, *hbuf_d;
    ABD_TRY(mirror_get(ctx, &hbuf, &hbuf_d));
    hbuf += MIR_COMPACT;
    ABD_TRY(scan_exclusive_i64(ctx, flag, pos, n, nact, s, hbuf_d + MIR_COMPACT, n_pt));
    hipLaunchKernelGGL(k_compact, dim3(grid_for(n, 256)), dim3(256), 0, s, n, flag, pos, act);
    HIP_TRY(ctx, hipStreamSynchronize(s));
    na = hbuf[0];
    na_pt = hbuf[1];
    ABD_TRY(mirror_counts_ok(ctx, {na, na_pt}, "barrier"));
  }
  if (n_active_pt) *n_active_pt = na_pt;
  if (n_active_ee) *n_active_ee = na - na_pt;
  const int64_t nl = na + nf;  // local records: active barrier pairs, then friction pairs
  if (nl == 0) return ABD_OK;
  if (hooks && hooks->active) ABD_TRY(hooks->active(act, na, na_pt));

  double *e_loc, *g_loc, *H_loc;
  PairInfo *info;
  ABD_TRY(ws(ctx, "br_e", nl, &e_loc, s));
  ABD_TRY(ws(ctx, "br_g", 12 * nl, &g_loc, s));
  ABD_TRY(ws(ctx, "br_H", 78 * nl, &H_loc, s));
  ABD_TRY(ws(ctx, "br_info", nl, &info, s));
  if (na > 0) {
    hipEvent_t pe = prof_begin(ctx, s);
    // (waves per block from the launch-shape table)
#define ABD_BARRIER_ARGS                                                                                          \
  nact, act, n_pt, pt, ee, sc->tris, sc->edges, sc->vert_body, x, sc->xbar, dhat, prm->kappa_b, project, e_loc, \
      g_loc, H_loc, info, err, ctx->kappa_sc, sc->body_scene
    const int wpb = ctx->tune.barrier_waves;
    if (wpb == 4)
      hipLaunchKernelGGL(k_barrier_local<256>, dim3(grid_for(na, 256)), dim3(256), 0, s, ABD_BARRIER_ARGS);
    else if (wpb == 2)
      hipLaunchKernelGGL(k_barrier_local<128>, dim3(grid_for(na, 128)), dim3(128), 0, s, ABD_BARRIER_ARGS);
    else
      hipLaunchKernelGGL(k_barrier_local<64>, dim3(grid_for(na, 64)), dim3(64), 0, s, ABD_BARRIER_ARGS);
#undef ABD_BARRIER_ARGS
    prof_end(ctx, pe, "barrier_local", na, s);
    HIP_TRY(ctx, hipGetLastError());
  }
  if (nf > 0) ABD_TRY(op_friction_local(ctx, sc, fr, x, e_loc + na, g_loc + 12 * na, H_loc + 78 * na, info + na, s));
  if (energy) ABD_TRY(reduce_sum_f64(ctx, e_loc, nl, energy, s));
  if (hooks && hooks->join) ABD_TRY(hooks->join(&keys, &n_keys, &off));
  if (!grad && !diag && !off) return ABD_OK;
  return op_assemble(ctx, sc, nl, info, g_loc, H_loc, keys, n_keys, grad, diag, off, s);
}

// records -> stable sort by block -> chunked fixed-order reduction
int op_assemble(abd_ctx *ctx, const abd_scene *sc, int64_t n, const PairInfo *info, const double *g_loc,
                const double *H_loc, const int32_t *keys, int64_t n_keys, double *grad, double *diag, double *off,
                hipStream_t s) {
  if (n == 0) return ABD_OK;
  int *err;
  ABD_TRY(ws(ctx, "err_flag", 1, &err, s));
  const int nb = sc->n_bodies;
  const int64_t nrec = 3 * n;
  const int64_t nblocks = nb + n_keys;
  uint32_t *rkey, *rval;
  ABD_TRY(ws(ctx, "br_rkey", nrec, &rkey, s));
  ABD_TRY(ws(ctx, "br_rval", nrec, &rval, s));
  hipLaunchKernelGGL(k_records, dim3(grid_for(n, 256)), dim3(256), 0, s, n, info, sc->body_fixed, nb, keys, n_keys,
                     rkey, rval, off != nullptr ? 1 : 0, err);
  int key_bits = 1;
  while (key_bits < 32 && (nblocks >> key_bits) != 0) ++key_bits;
  ABD_TRY(sort_pairs_u32(ctx, &rkey, &rval, nrec, key_bits, s));
  int64_t *bstart, *nchunk, *choff, *nch_tot;
  ABD_TRY(ws(ctx, "br_bstart", nblocks + 1, &bstart, s));
  ABD_TRY(ws(ctx, "br_nchunk", nblocks + 1, &nchunk, s));
  ABD_TRY(ws(ctx, "br_choff", nblocks + 1, &choff, s));
  ABD_TRY(ws(ctx, "br_nchtot", 1, &nch_tot, s));
  hipLaunchKernelGGL(k_block_chunks, dim3(grid_for(nblocks + 1, 256)), dim3(256), 0, s, nblocks, rkey, nrec, bstart);
  hipLaunchKernelGGL(k_block_nchunk, dim3(grid_for(nblocks, 256)), dim3(256), 0, s, nblocks, bstart, nchunk);
  ABD_TRY(scan_exclusive_i64(ctx, nchunk, choff, nblocks, nch_tot, s));
  // upper bound on chunks: every record alone plus one per block
  const int64_t max_chunks = (nrec + RCH - 1) / RCH + nblocks;
  double *partial;
  ABD_TRY(ws(ctx, "br_partial", (size_t)NENT * max_chunks, &partial, s));
  hipEvent_t pe = prof_begin(ctx, s);
  hipLaunchKernelGGL(k_assemble_chunks, dim3((unsigned)max_chunks), dim3(64), 0, s, nblocks, choff, nch_tot, bstart,
                     rval, info, g_loc, H_loc, sc->xbar, partial);
  prof_end(ctx, pe, "assemble_chunks", nrec, s);
  hipLaunchKernelGGL(k_assemble_final, dim3(grid_for(nblocks * NENT, 256)), dim3(256), 0, s, nblocks, nb, choff, nchunk,
                     partial, keys, grad, diag, off);
  return abd_hip_check(ctx, hipGetLastError(), "barrier assemble");
}

int op_barrier_energy(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x, const int32_t *pt,
                      int64_t n_pt, const int32_t *ee, int64_t n_ee, double *energy, hipStream_t s) {
  const int64_t n = n_pt + n_ee;
  if (n == 0) return ABD_OK;
  double *e;
  ABD_TRY(ws(ctx, "be_e", n, &e, s));
  hipEvent_t pe = prof_begin(ctx, s);
  const int eb = ctx->tune.energy_block;
  hipLaunchKernelGGL(k_energy_only, dim3(grid_for(n, eb)), dim3(eb), 0, s, n_pt, n, pt, ee, sc->tris, sc->edges, x,
                     sc->xbar, prm->dhat, prm->kappa_b, e, sc->vert_body, sc->body_scene, nullptr, 0, 0,
                     ctx->kappa_sc);
  prof_end(ctx, pe, "energy_only", n, s);
  HIP_TRY(ctx, hipGetLastError());
  return reduce_sum_f64(ctx, e, n, energy, s);
}


int op_barrier_energy_trials(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q,
                             int n_trials, const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee,
                             double *energy, hipStream_t s, double *items, int64_t estride, TrialSums *defer) {
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  const int64_t n = n_pt + n_ee;
  if (n == 0 || n_trials <= 0) return ABD_OK;
  double *e = items;
  int32_t *key = nullptr;
  if (!e) ABD_TRY(ws(ctx, "be_e_tr", (size_t)n * n_trials, &e, s));
  if (!items) ABD_TRY(ws(ctx, "be_key", n, &key, s));
  hipEvent_t pe = prof_begin(ctx, s);
  const int eb = ctx->tune.energy_block;
  hipLaunchKernelGGL(k_energy_only, dim3(grid_for(n, eb), n_trials), dim3(eb), 0, s, n_pt, n, pt, ee, sc->tris,
                     sc->edges, nullptr, sc->xbar, prm->dhat, prm->kappa_b, e, sc->vert_body, sc->body_scene, key,
                     (int64_t)0, items ? estride : 0, ctx->kappa_sc, q, 12 * (int64_t)sc->n_bodies);
  prof_end(ctx, pe, "energy_only", n * n_trials, s);
  HIP_TRY(ctx, hipGetLastError());
  if (items) return ABD_OK;
  // PT and EE lists are each ordered by scene
  if (defer) {
    if (n_pt) defer->seg[defer->k++] = TrialSeg{e, n, n_pt, key};
    if (n_ee) defer->seg[defer->k++] = TrialSeg{e + n_pt, n, n_ee, key + n_pt};
    return ABD_OK;
  }
  if (n_pt) ABD_TRY(seg_sum_trials(ctx, e, n, n_pt, key, n_trials, S, energy, s));
  if (n_ee) ABD_TRY(seg_sum_trials(ctx, e + n_pt, n, n_ee, key + n_pt, n_trials, S, energy, s));
  return ABD_OK;
}

// ------------------------------------------------------------------ ABI ----
extern "C" int abd_classify(abd_ctx *ctx, const abd_scene *sc, const double *x, double dhat, const int32_t *pairs,
                            int64_t n, int is_ee, uint8_t *type, double *d2, uint8_t *active, hipStream_t stream) {
  if (!ctx || !sc || !x || (n && !pairs)) return abd_fail(ctx, ABD_E_INVALID, "abd_classify: null");
  if (n <= 0) return ABD_OK;
  hipLaunchKernelGGL(k_classify, dim3(grid_for(n, 256)), dim3(256), 0, stream, n, is_ee, pairs, sc->tris, sc->edges, x,
                     dhat * dhat, type, d2, active);
  return abd_hip_check(ctx, hipGetLastError(), "k_classify");
}

extern "C" int abd_barrier_grad_hess(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x,
                                     const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee,
                                     const int32_t *keys, int64_t n_keys, double *energy, double *grad, double *diag,
                                     double *off, int project_psd, hipStream_t stream) {
  if (!ctx || !sc || !prm || !x || (n_pt && !pt) || (n_ee && !ee) || !grad || (off && n_keys && !keys))
    return abd_fail(ctx, ABD_E_INVALID, "abd_barrier_grad_hess: null");
  return op_barrier(ctx, sc, prm, x, pt, n_pt, ee, n_ee, keys, n_keys, energy, grad, diag, off, project_psd, nullptr,
                    nullptr, stream);
}

// ----------------------------------------- allocation-free barrier energy ----
// Scratch of abd_barrier_energy_noalloc: the per-pair energies, then the
// reduction's block partials.  One copy per GPU, held until the process
// ends; every call on a GPU shares it, so calls that overlap on one GPU
// race.  Host code uses the device address taken once per device below,
// never the array's name.
static __device__ __align__(256) double scratch[ABD_NOALLOC_MAX_PAIRS + REDUCE_MAX_PARTS];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[NOALLOC_MAX_DEVICES] = {};
}  // namespace

int noalloc_scratch_init(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return ABD_E_INVALID;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return ABD_OK;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return ABD_E_HIP;
  }
  g_scratch[device] = static_cast<double *>(ptr);
  return ABD_OK;
}

extern "C" int abd_barrier_energy_noalloc(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm,
                                          const double *x, const int32_t *pt, int64_t n_pt, const int32_t *ee,
                                          int64_t n_ee, double *energy, hipStream_t stream) {
  if (!ctx || !sc || !prm || !x || !energy || n_pt < 0 || n_ee < 0 || (n_pt && !pt) || (n_ee && !ee))
    return abd_fail(ctx, ABD_E_INVALID, "abd_barrier_energy_noalloc: null or negative count");
  const int64_t n = n_pt + n_ee;
  if (n > ABD_NOALLOC_MAX_PAIRS)
    return abd_fail(ctx, ABD_E_CAPACITY, "abd_barrier_energy_noalloc: %lld pairs exceed the scratch capacity of %d",
                    (long long)n, (int)ABD_NOALLOC_MAX_PAIRS);
  if (n == 0) return ABD_OK;
  double *scr = g_scratch[ctx->device];
  if (!scr) return abd_fail(ctx, ABD_E_HIP, "abd_barrier_energy_noalloc: scratch address not set for this device");
  // the kernels and the summation order of abd_barrier_energy
  double *e = scr, *part = scr + ABD_NOALLOC_MAX_PAIRS;
  const int eb = ctx->tune.energy_block;
  hipLaunchKernelGGL(k_energy_only, dim3(grid_for(n, eb)), dim3(eb), 0, stream, n_pt, n, pt, ee, sc->tris,
                     sc->edges, x, sc->xbar, prm->dhat, prm->kappa_b, e, sc->vert_body, sc->body_scene, nullptr);
  reduce_sum_f64_into(e, n, part, energy, stream);
  return abd_hip_check(ctx, hipGetLastError(), "abd_barrier_energy_noalloc");
}

extern "C" int abd_barrier_energy(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x,
                                  const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, double *energy,
                                  hipStream_t stream) {
  if (!ctx || !sc || !prm || !x || !energy || (n_pt && !pt) || (n_ee && !ee))
    return abd_fail(ctx, ABD_E_INVALID, "abd_barrier_energy: null");
  return op_barrier_energy(ctx, sc, prm, x, pt, n_pt, ee, n_ee, energy, stream);
}
