// Block-Jacobi preconditioned conjugate gradients on the symmetric
// 12x12-block system H p = rhs (diagonal blocks per body, off-diagonal
// blocks per contacting body pair, fixed bodies removed).
//
// Default: one kernel per iteration (Chronopoulos and Gear's recurrences,
// one reduction point per iteration), with the products B_bc = H_bc P_c
// formed once per solve.  Its result is then checked against a freshly
// computed residual by iteration 0 of the two-kernel form below, which
// carries on for any scene the check rejects (ABD_PCG_CG=0 runs the
// two-kernel form alone).
//
// Two-kernel form.  The first kernel forms the search direction
// p_new = z + beta p_old on the fly (p is double-buffered, so no block reads
// a vector another block is writing), multiplies by H (one wave per body)
// and writes per-block partials of p.Hp; the second updates x, r, z = P r and
// writes per-block partials of r.z and r.r.
//
// In both forms each kernel starts by folding the previous kernel's
// partials in a fixed order; every block does the same fold, so all blocks
// take the same decisions (alpha, beta, stop) without fences, atomics or
// separate reduction launches, and results are run-to-run reproducible.
// Iterations are replayed from captured hipGraphs of a short or a long run
// of iterations (even counts from the launch-shape table: the p buffers
// alternate; long replays while the last solve's count says many remain); once
// a scene's stop flag is set its remaining kernels return at once, and the
// host reads the flags once per replay.
#include <cstdlib>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "abd_internal.h"

namespace {


// inverse of each free body's diagonal block via Cholesky (thread per
// body); bodies of the scenes skip_scene marks (may be NULL) get zeros
__global__ void __launch_bounds__(64) k_block_inverse(int nb, const uint8_t *fixed, const double *diag, double *inv,
                                                      int *err, const uint8_t *skip_scene = nullptr,
                                                      const int32_t *body_scene = nullptr) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double *Iv = inv + 144 * (int64_t)b;
  if (fixed[b] || (skip_scene && skip_scene[body_scene[b]])) {
    for (int i = 0; i < 144; ++i) Iv[i] = 0.0;
    return;
  }
  const double *A = diag + 144 * (int64_t)b;
  double L[12][12];
#pragma unroll
  for (int i = 0; i < 12; ++i)
#pragma unroll
    for (int j = 0; j < 12; ++j) L[i][j] = 0.0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    double d = 0.5 * (A[12 * j + j] + A[12 * j + j]);
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) {
      ok = false;
      d = 1.0;
    }
    const double ljj = sqrt(d);
    L[j][j] = ljj;
#pragma unroll
    for (int i = j + 1; i < 12; ++i) {
      double v = 0.5 * (A[12 * i + j] + A[12 * j + i]);
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / ljj;
    }
  }
  if (!ok) atomicOr(err, 4);
  // inverse of L (lower), then A^-1 = L^-T L^-1
  double M[12][12];
#pragma unroll
  for (int i = 0; i < 12; ++i)
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      if (j > i) {
        M[i][j] = 0.0;
        continue;
      }
      if (i == j) {
        M[i][i] = 1.0 / L[i][i];
        continue;
      }
      double v = 0.0;
#pragma unroll
      for (int k = j; k < i; ++k) v -= L[i][k] * M[k][j];
      M[i][j] = v / L[i][i];
    }
#pragma unroll
  for (int i = 0; i < 12; ++i)
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      double v = 0.0;
#pragma unroll
      for (int k = (i > j ? i : j); k < 12; ++k) v += M[k][i] * M[k][j];
      Iv[12 * i + j] = v;
    }
}

// row structure: for body b the off-diagonal blocks with b as row (lo side,
// contiguous in the sorted keys) and as column (hi side, via the transposed
// order)
__global__ void k_row_ranges(int nb, int64_t nk, const int32_t *keys, const uint64_t *tkeys, int64_t *lo_beg,
                             int64_t *hi_beg) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nb) return;
  int64_t lo = 0, hi = nk;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[2 * mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  lo_beg[b] = lo;
  lo = 0;
  hi = nk;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int)(tkeys[mid] >> 40) < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  hi_beg[b] = lo;
}

__global__ void k_tkeys(int64_t nk, const int32_t *keys, uint64_t *tk, uint32_t *tv) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  // (hi, lo) ordering key; 24 bits per body id
  tk[k] = ((uint64_t)keys[2 * k + 1] << 40) | ((uint64_t)keys[2 * k] << 16);
  tv[k] = (uint32_t)k;
}


constexpr int PB = 192;  // init / update: 16 bodies x 12 rows per block
constexpr int PBB = PB / 12;
constexpr int SWB = 256;  // SpMV-shaped blocks: four 64-lane waves
constexpr int SWBB = SWB / 64;
constexpr int CBB = 5 * SWBB;  // SpMV-shaped kernels: five bodies per wave, 12 lanes each

// Sub-scenes are independent systems (the matrix is block diagonal by
// scene), each with its own CG scalars and stop test.  Blocks never span
// two scenes: scene s owns update blocks [u_off[s], u_off[s+1]) and spmv
// blocks [s_off[s], s_off[s+1]), so a block folds only its scene's
// partials.  Iteration k runs in lockstep for all scenes; a stopped scene's
// blocks return at once.
//
// Device-side iteration state.  Every value is written by one designated
// block of one kernel (block 0 for the global counters, the scene's first
// block for a scene's scalars) and read only by later kernels, so no fences
// are needed; the one atomic counts stopped scenes for the host.
struct PcgState {
  int it_done;    // iterations completed (written by update's block 0)
  int k_cur;      // iteration being run (written by spmv's block 0)
  int n_stopped;  // scenes stopped so far
  int max_final;  // largest iteration count of a stopped scene
};
struct PcgScene {
  double *rz;      // [2 S] r.z of the iterations with parity 0 / 1
  double *bb;      // [S] initial r.r
  int *stop;       // [S]
  int *it_final;   // [S] iterations run by the scene
};

// fixed-order sum of n per-block partials (stride `stride`, offset `off`),
// identical in every block that calls it
__device__ __forceinline__ double fold(const double *part, int n, int stride, int off, double *sh) {
  double v = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) v += part[stride * j + off];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  __syncthreads();
  return s;
}

// blocks per scene (update and spmv mappings)
__global__ void k_pcg_scene_blocks(int S, const int32_t *sbo, int64_t *ucnt, int64_t *scnt) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const int n = sbo[s + 1] - sbo[s];
  ucnt[s] = (n + PBB - 1) / PBB;
  scnt[s] = (n + CBB - 1) / CBB;
}
// the four steps below in one block, for up to SETUP_T scenes: per-scene
// block counts, their exclusive scans (u_off, s_off) and the scene of
// every update and SpMV block
constexpr int SETUP_T = 1024;
__global__ void __launch_bounds__(SETUP_T) k_pcg_scene_setup(int S, const int32_t *sbo, int64_t nblk_u,
                                                             int64_t nblk_s, int64_t *u_off, int64_t *s_off,
                                                             int32_t *u_scene, int32_t *s_scene) {
  __shared__ int64_t su[SETUP_T + 1], ss[SETUP_T + 1];
  const int t = threadIdx.x;
  int64_t cu = 0, cs = 0;
  if (t < S) {
    const int n = sbo[t + 1] - sbo[t];
    cu = (n + PBB - 1) / PBB;
    cs = (n + CBB - 1) / CBB;
  }
  su[t + 1] = cu;
  ss[t + 1] = cs;
  if (t == 0) su[0] = ss[0] = 0;
  __syncthreads();
  // inclusive scan of su[1..], ss[1..] (Hillis-Steele)
  for (int o = 1; o < SETUP_T; o <<= 1) {
    const int64_t a = t >= o ? su[t + 1 - o] : 0, b = t >= o ? ss[t + 1 - o] : 0;
    __syncthreads();
    su[t + 1] += a;
    ss[t + 1] += b;
    __syncthreads();
  }
  for (int k = t; k <= S; k += SETUP_T) {
    u_off[k] = su[k];
    s_off[k] = ss[k];
  }
  for (int64_t j = t; j < nblk_u; j += SETUP_T) {
    int lo = 0, hi = S;
    if (j >= su[S]) {
      u_scene[j] = -1;
      continue;
    }
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (su[mid] <= j) lo = mid; else hi = mid - 1;
    }
    u_scene[j] = lo;
  }
  for (int64_t j = t; j < nblk_s; j += SETUP_T) {
    int lo = 0, hi = S;
    if (j >= ss[S]) {
      s_scene[j] = -1;
      continue;
    }
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ss[mid] <= j) lo = mid; else hi = mid - 1;
    }
    s_scene[j] = lo;
  }
}

// one more mapping (bpb bodies per block) the same way: per-scene block
// counts (cnt, S > SETUP_T) or, for up to SETUP_T scenes, everything in one
// block (counts, their exclusive scan `off`, the scene of every block)
__global__ void k_pcg_scene_count(int S, const int32_t *sbo, int bpb, int64_t *cnt) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  cnt[s] = (sbo[s + 1] - sbo[s] + bpb - 1) / bpb;
}
__global__ void __launch_bounds__(SETUP_T) k_pcg_scene_map(int S, const int32_t *sbo, int bpb, int64_t nblk,
                                                           int64_t *off, int32_t *tab) {
  __shared__ int64_t sc_[SETUP_T + 1];
  const int t = threadIdx.x;
  sc_[t + 1] = t < S ? (sbo[t + 1] - sbo[t] + bpb - 1) / bpb : 0;
  if (t == 0) sc_[0] = 0;
  __syncthreads();
  for (int o = 1; o < SETUP_T; o <<= 1) {
    const int64_t a = t >= o ? sc_[t + 1 - o] : 0;
    __syncthreads();
    sc_[t + 1] += a;
    __syncthreads();
  }
  for (int k = t; k <= S; k += SETUP_T) off[k] = sc_[k];
  for (int64_t j = t; j < nblk; j += SETUP_T) {
    if (j >= sc_[S]) {
      tab[j] = -1;
      continue;
    }
    int lo = 0, hi = S;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sc_[mid] <= j) lo = mid; else hi = mid - 1;
    }
    tab[j] = lo;
  }
}

// scene of every block (-1 beyond the last scene's blocks)
__global__ void k_pcg_block_scene(int S, int64_t nblk, const int64_t *off, int32_t *tab) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nblk) return;
  int lo = 0, hi = S;  // last s with off[s] <= j, if j < off[S]
  if (j >= off[S]) {
    tab[j] = -1;
    return;
  }
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  tab[j] = lo;
}


// r = rhs - H x0 (free bodies; Hx0 NULL: x0 = 0), x = x0, z = P r, p_old = 0;
// partials of r.z, r.r and rhs.rhs
__global__ void __launch_bounds__(PB) k_pcg_init(const int32_t *u_scene, const int64_t *u_off, const int32_t *sbo,
                                                const uint8_t *fixed, const double *inv, const double *rhs,
                                                const double *x0, const double *Hx0, double *x, double *r,
                                                double *z, double *p_old, double *part2) {
  __shared__ double sr[PBB][12];
  __shared__ double sh[PB / 64];
  const int sc = u_scene[blockIdx.x];
  if (sc < 0) return;
  const int lb = threadIdx.x / 12, i = threadIdx.x % 12;
  const int b = sbo[sc] + (int)(blockIdx.x - u_off[sc]) * PBB + lb;
  const bool ok = lb < PBB && b < sbo[sc + 1];
  double rv = 0.0, bv = 0.0;
  if (ok) {
    const int64_t o = 12 * (int64_t)b + i;
    bv = fixed[b] ? 0.0 : rhs[o];
    rv = Hx0 && !fixed[b] ? bv - Hx0[o] : bv;
    x[o] = Hx0 && !fixed[b] ? x0[o] : 0.0;
    r[o] = rv;
    p_old[o] = 0.0;
  }
  sr[lb][i] = rv;
  __syncthreads();
  double zv = 0.0;
  if (ok) {
    const double *M = inv + 144 * (int64_t)b + 12 * i;
#pragma unroll
    for (int j = 0; j < 12; ++j) zv += M[j] * sr[lb][j];
    z[12 * (int64_t)b + i] = zv;
  }
  const double rz = block_sum(rv * zv, sh), rr = block_sum(rv * rv, sh), bb = block_sum(bv * bv, sh);
  if (threadIdx.x == 0) {
    part2[3 * blockIdx.x] = rz;
    part2[3 * blockIdx.x + 1] = rr;
    part2[3 * blockIdx.x + 2] = bb;
  }
}

// Per-block constants of one iteration kernel, loaded in one go: the
// block's scene, body range and the range of the other kernel's partials it
// folds.
struct alignas(16) PcgBlk {
  int32_t sc, first, last, is_first;
  int32_t fold_lo, fold_n;
  int32_t pad[2];
};

// per body: its matrix entries (the diagonal block first, then the
// off-diagonal blocks with the body as row, then as column)
// entry = (block index, column body | transposed << 30); block -1 = diagonal
// (body b's entries start at b + lo_beg[b] + hi_beg[b]: one diagonal entry
// per earlier body plus the earlier rows' and columns' keys; ent_off gets
// these offsets, nb + 1 of them)
__global__ void k_pcg_entries(int nb, const int64_t *lo_beg, const int64_t *hi_beg, const uint32_t *tperm,
                              const int32_t *keys, int64_t *ent_off, int2 *ent) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == nb) ent_off[nb] = nb + lo_beg[nb] + hi_beg[nb];
  if (b >= nb) return;
  int64_t o = b + lo_beg[b] + hi_beg[b];
  ent_off[b] = o;
  ent[o++] = make_int2(-1, b);
  for (int64_t kk = lo_beg[b]; kk < lo_beg[b + 1]; ++kk) ent[o++] = make_int2((int)kk, keys[2 * kk + 1]);
  for (int64_t h = hi_beg[b]; h < hi_beg[b + 1]; ++h) {
    const int kk = (int)tperm[h];
    ent[o++] = make_int2(kk, keys[2 * kk] | (1 << 30));
  }
}
// block constants of a mapping with `bpb` bodies per block; up to three
// mappings per launch (thread index over their concatenation)
struct BlkJob {
  int64_t nblk;
  int bpb;
  const int32_t *tab;
  const int64_t *off, *fold_off;
  PcgBlk *out;
};
struct BlkJobs {
  BlkJob j[3];
};
__global__ void k_pcg_blk(BlkJobs J, const int32_t *sbo, int S, PcgState *st, PcgScene scs) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // (the two-kernel form's state reset rides along)
  if (j == 0) {
    st->it_done = 0;
    st->k_cur = 0;
    st->n_stopped = 0;
    st->max_final = 0;
  }
  for (int64_t q = j; q < S; q += (int64_t)gridDim.x * blockDim.x) {
    scs.stop[q] = 0;
    scs.it_final[q] = 0;
  }
  int m = 0;
  while (m < 3 && j >= J.j[m].nblk) j -= J.j[m++].nblk;
  if (m == 3) return;
  const int64_t nblk = J.j[m].nblk;
  const int bpb = J.j[m].bpb;
  const int32_t *tab = J.j[m].tab;
  const int64_t *off = J.j[m].off, *fold_off = J.j[m].fold_off;
  PcgBlk *out = J.j[m].out;
  if (j >= nblk) return;
  PcgBlk r;
  r.pad[0] = r.pad[1] = 0;
  const int s = tab[j];
  r.sc = s;
  if (s < 0) {
    r.first = r.last = r.is_first = r.fold_lo = r.fold_n = 0;
    out[j] = r;
    return;
  }
  r.first = sbo[s] + (int)(j - off[s]) * bpb;
  r.last = sbo[s + 1];
  r.is_first = j == off[s];
  r.fold_lo = (int)fold_off[s];
  r.fold_n = (int)(fold_off[s + 1] - fold_off[s]);
  out[j] = r;
}

// Iteration k (k = it_done): fold the scene's r.z, r.r of the previous
// update, decide its stop, beta = rz_k / rz_{k-1}; p_new = z + beta p_old;
// Ap = H p_new with one wave per body: lane = (entry slot 0..4, row 0..11),
// five entries per pass.  Latency is what bounds this kernel at 12k DOFs, so
// the dependent loads are cut to three round trips (block constants; entry
// list, partials and stop flag; matrix rows and column vectors) and the
// matrix work does not wait for beta (H z and H p_old are accumulated
// separately and combined after the fold).  Per-row sums over slots in
// fixed order.
__global__ void __launch_bounds__(SWB) k_pcg_spmv(const PcgBlk *blk, const int64_t *eoff, const int2 *ent,
                                                 const uint8_t *fixed, const double *diag, const double *off,
                                                 const double *p_old, const double *z, double *p_new, double *Ap,
                                                 const double *part2, double *part, PcgState *st, PcgScene scs,
                                                 double rtol2, int max_iter) {
  __shared__ double sh[SWB / 64];
  const int k = st->it_done;
  const PcgBlk bi = blk[blockIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) st->k_cur = k;
  if (bi.sc < 0) return;
  const int sc = bi.sc;
  // five bodies per wave (lanes 12 h .. 12 h + 11: rows of body h)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int hb = lane / 12, i = lane - 12 * hb;
  const int b = bi.first + 5 * wv + hb;
  const bool ok = hb < 5 && b < bi.last;
  int64_t e0 = 0;
  int E = 0;
  if (ok) {
    e0 = eoff[b];
    E = (int)(eoff[b + 1] - e0);
  }
  // round trip 2: stop flag, partials, the bodies' own vectors
  const int stopped = scs.stop[sc];
  double prz = 0.0, prr = 0.0, pbb = 0.0;
  for (int j = threadIdx.x; j < bi.fold_n; j += SWB) {
    prz += part2[3 * (bi.fold_lo + j)];
    prr += part2[3 * (bi.fold_lo + j) + 1];
    if (k == 0) pbb += part2[3 * (bi.fold_lo + j) + 2];
  }
  const double own_z = ok ? z[12 * (int64_t)b + i] : 0.0, own_p = ok ? p_old[12 * (int64_t)b + i] : 0.0;
  if (stopped) return;  // uniform over the block (one scene)
  // H z and H p_old kept apart so that no load waits for beta; each
  // entry's product added in entry order
  double vz = 0.0, vp = 0.0;
  for (int e = 0; e < E; ++e) {
    const int2 en = ent[e0 + e];
    const int c = en.y & ((1 << 30) - 1);
    const bool tr = (en.y >> 30) & 1;
    const double *rp = en.x < 0 ? diag + 144 * (int64_t)b + 12 * i
                                : (tr ? off + 144 * (int64_t)en.x + i : off + 144 * (int64_t)en.x + 12 * i);
    const int stride = tr ? 12 : 1;
    double pz = 0.0, pp = 0.0;
#pragma unroll
    for (int jj = 0; jj < 12; ++jj) {
      pz = fma(rp[stride * jj], z[12 * (int64_t)c + jj], pz);
      pp = fma(rp[stride * jj], p_old[12 * (int64_t)c + jj], pp);
    }
    vz += pz;
    vp += pp;
  }
  double rz = wave_sum(prz), rr = wave_sum(prr), b0 = wave_sum(pbb);
  if (lane == 0) sh[wv] = rz;
  __syncthreads();
  rz = 0.0;
  for (int w = 0; w < SWB / 64; ++w) rz += sh[w];
  __syncthreads();
  if (lane == 0) sh[wv] = rr;
  __syncthreads();
  rr = 0.0;
  for (int w = 0; w < SWB / 64; ++w) rr += sh[w];
  __syncthreads();
  if (k == 0) {
    if (lane == 0) sh[wv] = b0;
    __syncthreads();
    b0 = 0.0;
    for (int w = 0; w < SWB / 64; ++w) b0 += sh[w];
    __syncthreads();
  }
  // |r| <= rtol |b| with b the right-hand side (x0 may be non-zero)
  const double bb = k == 0 ? b0 : scs.bb[sc];
  const double beta = k == 0 ? 0.0 : rz / scs.rz[2 * sc + ((k - 1) & 1)];
  const bool stop = !(bb > 0.0) || rr <= rtol2 * bb || k >= max_iter || rz == 0.0;
  if (bi.is_first && threadIdx.x == 0) {
    scs.rz[2 * sc + (k & 1)] = rz;
    if (k == 0) scs.bb[sc] = bb;
    if (stop) {
      scs.stop[sc] = 1;
      scs.it_final[sc] = k;
      atomicMax(&st->max_final, k);
      atomicAdd(&st->n_stopped, 1);
    }
  }
  if (stop) return;
  double dot = 0.0;
  if (ok) {
    const int64_t o = 12 * (int64_t)b + i;
    const double av = fixed[b] ? 0.0 : vz + beta * vp;
    const double pown = own_z + beta * own_p;
    Ap[o] = av;
    p_new[o] = pown;
    dot = av * pown;
  }
  const double sdot = block_sum(dot, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = sdot;
}

// alpha = rz_k / p.Ap (folded from the scene's spmv partials); x += alpha p;
// r -= alpha Ap; z = P r = P r_old - alpha P Ap (both products formed
// before alpha is known); partials of r.z, r.r for the next spmv
__global__ void __launch_bounds__(PB) k_pcg_update(const PcgBlk *blk, const double *inv, const double *p,
                                                  const double *Ap, double *x, double *r, double *z,
                                                  const double *part, double *part2, PcgState *st, PcgScene scs,
                                                  int *err) {
  __shared__ double sr[PBB][12], sa[PBB][12];
  __shared__ double sh[PB / 64];
  const int k = st->k_cur;
  const PcgBlk bi = blk[blockIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) st->it_done = k + 1;
  if (bi.sc < 0) return;
  const int sc = bi.sc;
  const int lb = threadIdx.x / 12, i = threadIdx.x % 12;
  const int b = bi.first + lb;
  const bool ok = b < bi.last;
  const int64_t o = 12 * (int64_t)b + i;
  // round trip 2: stop flag, partials, the row's data
  const int stopped = scs.stop[sc];
  double pp = 0.0;
  for (int j = threadIdx.x; j < bi.fold_n; j += PB) pp += part[bi.fold_lo + j];
  double pv = 0.0, av = 0.0, xv = 0.0, rv = 0.0, M[12];
#pragma unroll
  for (int j = 0; j < 12; ++j) M[j] = 0.0;
  if (ok) {
    pv = p[o];
    av = Ap[o];
    xv = x[o];
    rv = r[o];
    const double *Mi = inv + 144 * (int64_t)b + 12 * i;
#pragma unroll
    for (int j = 0; j < 12; ++j) M[j] = Mi[j];
  }
  if (stopped) return;  // uniform over the block
  const double rz = scs.rz[2 * sc + (k & 1)];
  sr[lb][i] = rv;
  sa[lb][i] = av;
  double pap = wave_sum(pp);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = pap;
  __syncthreads();
  pap = 0.0;
  for (int w = 0; w < PB / 64; ++w) pap += sh[w];
  double zr = 0.0, za = 0.0;
#pragma unroll
  for (int j = 0; j < 12; ++j) {
    zr += M[j] * sr[lb][j];
    za += M[j] * sa[lb][j];
  }
  __syncthreads();
  if (!(pap > 0.0)) {
    if (bi.is_first && threadIdx.x == 0) {
      scs.stop[sc] = 1;
      scs.it_final[sc] = k;
      atomicMax(&st->max_final, k);
      atomicAdd(&st->n_stopped, 1);
      if (!(pap == 0.0 && rz == 0.0)) atomicOr(err, 8);
    }
    return;
  }
  const double a = rz / pap;
  double rn = 0.0, zn = 0.0;
  if (ok) {
    x[o] = xv + a * pv;
    rn = rv - a * av;
    zn = zr - a * za;
    r[o] = rn;
    z[o] = zn;
  }
  const double rzp = block_sum(rn * zn, sh), rrp = block_sum(rn * rn, sh);
  if (threadIdx.x == 0) {
    part2[3 * blockIdx.x] = rzp;
    part2[3 * blockIdx.x + 1] = rrp;
  }
}

// ------------------------------------------------ one kernel per iteration ----
// Chronopoulos and Gear's form of preconditioned CG: with u = P r, w = H u,
// p = u + beta p, s = w + beta s (s = H p), the two inner products of an
// iteration, gamma = r.u and delta = w.u, come from one reduction:
//   beta_i = gamma_i / gamma_{i-1};  alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1});
//   x += alpha p_i;  r_{i+1} = r_i - alpha s_i;  u_{i+1} = P r_{i+1};  w_{i+1} = H u_{i+1}.
// One kernel per iteration folds the previous kernel's partials and forms
// the products H u_{i+1} of its bodies; the new u of each neighbour is
// recomputed on the fly from the neighbour's r_i, w_i, s_{i-1} and its
// preconditioner block with the very arithmetic its owner uses (one helper,
// fused multiply-adds written out), so every wave sees the same values.
// r, w, s and the partials alternate between two buffers by the parity of
// the iteration; per-scene gamma and alpha are stored by parity.
struct CgScene {
  double *gam;  // [2S] gamma of the iterations with parity 0 / 1
  double *alp;  // [2S] alpha, by parity
  double *bb;   // [S] rhs.rhs
  int *stop, *it_final;
};
struct CgState {
  int base;  // iteration of the first kernel of a replay
  int n_stopped;
  int max_final;  // largest iteration count of a stopped scene
  int n_bad;      // scenes stopped by the iteration cap or a breakdown, not by the tolerance
};
static_assert(sizeof(CgState) == 4 * sizeof(int), "the pre-sync hook reads the state as int[4]");

__device__ __forceinline__ void cg_step(double r, double w, double s_prev, double alpha, double beta, double &s_new,
                                        double &r_new) {
  s_new = fma(beta, s_prev, w);
  r_new = fma(-alpha, s_new, r);
}


// r = rhs - H x0 (free bodies; Hx0 NULL: x0 = 0), x = x0, u = P r,
// p = 0, s_prev = 0
__global__ void __launch_bounds__(PB) k_cg_init1(const PcgBlk *blk, const uint8_t *fixed, const double *inv,
                                                const double *rhs, const double *x0, const double *Hx0, double *x,
                                                double *r, double *u, double *p, double *s_prev) {
  __shared__ double sr[PBB][12];
  const PcgBlk bi = blk[blockIdx.x];
  if (bi.sc < 0) return;
  const int lb = threadIdx.x / 12, i = threadIdx.x % 12;
  const int b = bi.first + lb;
  const bool ok = b < bi.last;
  double rv = 0.0;
  if (ok) {
    const int64_t o = 12 * (int64_t)b + i;
    const double bv = fixed[b] ? 0.0 : rhs[o];
    rv = Hx0 && !fixed[b] ? bv - Hx0[o] : bv;
    x[o] = Hx0 && !fixed[b] ? x0[o] : 0.0;
    r[o] = rv;
    p[o] = 0.0;
    s_prev[o] = 0.0;
  }
  sr[lb][i] = rv;
  __syncthreads();
  if (ok) {
    const double *M = inv + 144 * (int64_t)b + 12 * i;
    double uv = 0.0;
#pragma unroll
    for (int j = 0; j < 12; ++j) uv = fma(M[j], sr[lb][j], uv);
    u[12 * (int64_t)b + i] = uv;
  }
}

// The one-kernel iteration's mapping: five bodies per wave (lanes 12 h .. 12 h
// + 11 hold rows 0..11 of body h; lanes 60..63 idle), CBB bodies per block,
// a body's matrix entries taken one at a time in entry order (the row sums
// add the entries' products in that order).  The piles this solver runs on
// have few entries per body (one, the diagonal block, for a body touching
// only fixed geometry), so a wave per body left most lanes idle and made
// the launch a sequence of occupancy-limited rounds of waves.
// w_0 = H u_0; partials of gamma_0, delta_0, rho_0 = r.r and rhs.rhs
__global__ void __launch_bounds__(SWB) k_cg_init2(const PcgBlk *blk, const int64_t *eoff, const int2 *ent,
                                                 const uint8_t *fixed, const double *diag, const double *off,
                                                 const double *rhs, const double *r, const double *u, double *w,
                                                 double *part) {
  __shared__ double sh[SWB / 64];
  const PcgBlk bi = blk[blockIdx.x];
  if (bi.sc < 0) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int hb = lane / 12, i = lane - 12 * hb;
  const int b = bi.first + 5 * wv + hb;
  const bool ok = hb < 5 && b < bi.last;
  int64_t e0 = 0;
  int E = 0;
  if (ok) {
    e0 = eoff[b];
    E = (int)(eoff[b + 1] - e0);
  }
  double v = 0.0;
  for (int e = 0; e < E; ++e) {
    const int2 en = ent[e0 + e];
    const int c = en.y & ((1 << 30) - 1);
    const bool tr = (en.y >> 30) & 1;
    const double *rp = en.x < 0 ? diag + 144 * (int64_t)b + 12 * i
                                : (tr ? off + 144 * (int64_t)en.x + i : off + 144 * (int64_t)en.x + 12 * i);
    const int stride = tr ? 12 : 1;
    double pe = 0.0;
#pragma unroll
    for (int jj = 0; jj < 12; ++jj) pe = fma(rp[stride * jj], u[12 * (int64_t)c + jj], pe);
    v += pe;
  }
  double g = 0.0, d = 0.0, rr = 0.0, bb = 0.0;
  if (ok) {
    const int64_t o = 12 * (int64_t)b + i;
    const double wv_ = fixed[b] ? 0.0 : v;
    w[o] = wv_;
    const double rv = r[o], uv = u[o], bv = fixed[b] ? 0.0 : rhs[o];
    g = rv * uv;
    d = wv_ * uv;
    rr = rv * rv;
    bb = bv * bv;
  }
  g = block_sum(g, sh);
  d = block_sum(d, sh);
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = g;
    part[4 * blockIdx.x + 1] = d;
    part[4 * blockIdx.x + 2] = rr;
    part[4 * blockIdx.x + 3] = bb;
  }
}

// Per matrix entry (row body b, column body c) the product B_bc = H_bc P_c
// with the column body's preconditioner block, stored in entry order
// (144 doubles per entry), so that w = H u = H P r = sum_c B_bc r_c needs
// the column bodies' residuals only.  One thread per output element over
// all entries (an entry's row of H and column of P are shared by 12
// threads each, through the cache); the diagonal entry of body b is
// (-1, b), so no entry needs its row body.
__global__ void __launch_bounds__(256) k_cg_bmat(int64_t n_out, const int2 *ent, const double *diag,
                                                const double *off, const double *inv, double *B, int S, CgState *st,
                                                CgScene scs) {
  if (blockIdx.x == 0) {  // (the iteration state's reset rides along)
    if (threadIdx.x == 0) {
      st->base = 0;
      st->n_stopped = 0;
      st->max_final = 0;
      st->n_bad = 0;
    }
    for (int q = threadIdx.x; q < S; q += blockDim.x) {
      scs.stop[q] = 0;
      scs.it_final[q] = 0;
    }
  }
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_out) return;
  // (32-bit index arithmetic: n_out < 2^32, checked by the caller)
  const uint32_t tu = (uint32_t)t, eu = tu / 144u, ij = tu - 144u * eu;
  const int64_t e = eu;
  const int i = (int)(ij / 12u), j = (int)(ij - 12u * (ij / 12u));
  const int2 en = ent[e];
  const int kk = en.x, c = en.y & ((1 << 30) - 1);
  const bool tr = (en.y >> 30) & 1;
  const double *rp = kk < 0 ? diag + 144 * (int64_t)c + 12 * i
                            : (tr ? off + 144 * (int64_t)kk + i : off + 144 * (int64_t)kk + 12 * i);
  const int stride = tr ? 12 : 1;
  const double *Mc = inv + 144 * (int64_t)c + j;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 12; ++q) acc = fma(rp[stride * q], Mc[12 * q], acc);
  B[t] = acc;
}

// Operands of one entry of one lane: the column body's r_k, w_k, s_{k-1}
// components and row i of B_bc.
struct CgOps {
  double r, w, s, B[12];
};
__device__ __forceinline__ void cg_fetch(bool live, int c, int64_t eg, int i, const double *Bm, const double *r_in,
                                         const double *w_in, const double *s_in, CgOps &o) {
  if (!live) {
    o.r = o.w = o.s = 0.0;
#pragma unroll
    for (int j = 0; j < 12; ++j) o.B[j] = 0.0;
    return;
  }
  const int64_t oc = 12 * (int64_t)c + i;
  o.r = r_in[oc];
  o.w = w_in[oc];
  o.s = s_in[oc];
  const double *Bi = Bm + 144 * eg + 12 * i;
#pragma unroll
  for (int j = 0; j < 12; ++j) o.B[j] = Bi[j];
}

// column body of a body's entry e (entries below 12 from the lanes' copies)
__device__ __forceinline__ int cg_col(int my_c, int g0, int e, bool live, const int2 *ent, int64_t e0) {
  const int cs = __shfl(my_c, (g0 + (e < 12 ? e : 0)) & 63, 64);
  return !live ? 0 : (e < 12 ? cs : (ent[e0 + e].y & ((1 << 30) - 1)));
}

// Iteration k = base + jloc of every scene not yet stopped: fold gamma_k,
// delta_k, rho_k = r_k.r_k, decide the stop, alpha_k and beta_k; then per
// body p_k, x_{k+1}, s_k, r_{k+1}, u_{k+1} = P r_{k+1} and w_{k+1} =
// sum_c B_bc r_{k+1,c}, each entry's column body's s_k and r_{k+1} formed
// with the owner's arithmetic (so every wave that reads the body computes
// the same values); partials of gamma, delta, rho for the next iteration.
// Five bodies per wave (see CBB); a body's entries one at a time, the next
// entry's operands loaded while the current one is used.  The first
// entry's operands are loaded before the fold; the fold and the closing
// reduction take one barrier each.
__global__ void __launch_bounds__(SWB) k_cg_iter(int jloc, const PcgBlk *blk, const int64_t *eoff, const int2 *ent,
                                                const uint8_t *fixed, const double *Bm, const double *inv,
                                                const double *r_in, const double *w_in, const double *s_in,
                                                double *r_out, double *w_out, double *s_out, double *x, double *u,
                                                double *p, const double *part_in, double *part_out, CgState *st,
                                                CgScene scs, double rtol2, int max_iter, int batch) {
  __shared__ double shf[SWBB][4], she[SWBB][3];
  const int k = st->base + jloc;
  const PcgBlk bi = blk[blockIdx.x];
  if (bi.sc < 0) return;
  // In a batch, scenes stop at different iterations of a replay: a stopped
  // scene's blocks leave before loading anything more.  (One scene: its
  // stop comes once, at the end, so the flag is read with the other first
  // loads instead of ahead of them.)
  if (batch && scs.stop[bi.sc]) return;
  const int sc = bi.sc;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int hb = lane / 12, i = lane - 12 * hb, g0 = 12 * hb;
  const int b = bi.first + 5 * wv + hb;
  const bool ok = hb < 5 && b < bi.last;
  int64_t e0 = 0;
  int E = 0;
  if (ok) {
    e0 = eoff[b];
    E = (int)(eoff[b + 1] - e0);
  }
  const int stopped = scs.stop[sc];
  double pg = 0.0, pd = 0.0, pr = 0.0, pb = 0.0;
  for (int j = threadIdx.x; j < bi.fold_n; j += SWB) {
    const double *q = part_in + 4 * (int64_t)(bi.fold_lo + j);
    pg += q[0];
    pd += q[1];
    pr += q[2];
    if (k == 0) pb += q[3];
  }
  int my_c = 0;
  if (ok && i < E) my_c = ent[e0 + i].y & ((1 << 30) - 1);
  const int64_t oo = 12 * (int64_t)b + i;
  const double own_x = ok ? x[oo] : 0.0, own_u = ok ? u[oo] : 0.0, own_p = ok ? p[oo] : 0.0;
  const bool own_fixed = ok && fixed[b];
  // the scene's scalars of iteration k - 1 (parity buffers) and rhs.rhs
  const double gam_prev = scs.gam[2 * sc + ((k - 1) & 1)], alp_prev = scs.alp[2 * sc + ((k - 1) & 1)];
  const double bb_prev = scs.bb[sc];
  if (stopped) return;  // uniform over the block (one scene)
  // the wave's entry passes: its bodies' largest entry count
  int Emax = E;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) Emax = max(Emax, __shfl_xor(Emax, o, 64));
  CgOps op;
  cg_fetch(ok && E > 0, cg_col(my_c, g0, 0, ok && E > 0, ent, e0), e0, i, Bm, r_in, w_in, s_in, op);
  pg = wave_sum(pg);
  pd = wave_sum(pd);
  pr = wave_sum(pr);
  pb = wave_sum(pb);
  if (lane == 0) {
    shf[wv][0] = pg;
    shf[wv][1] = pd;
    shf[wv][2] = pr;
    shf[wv][3] = pb;
  }
  __syncthreads();
  double gam = 0.0, del = 0.0, rho = 0.0, b0 = 0.0;
#pragma unroll
  for (int w = 0; w < SWBB; ++w) {
    gam += shf[w][0];
    del += shf[w][1];
    rho += shf[w][2];
    b0 += shf[w][3];
  }
  // |r| <= rtol |b| with b the right-hand side (x0 may be non-zero)
  const double bb = k == 0 ? b0 : bb_prev;
  bool stop = !(bb > 0.0) || rho <= rtol2 * bb || k >= max_iter || gam == 0.0;
  double beta = 0.0, alpha = 0.0;
  if (!stop) {
    beta = k == 0 ? 0.0 : gam / gam_prev;
    const double den = k == 0 ? del : del - beta * gam / alp_prev;
    if (den > 0.0)
      alpha = gam / den;
    else
      stop = true;  // p.Hp lost to rounding (or H indefinite): the check that follows decides
  }
  if (bi.is_first && threadIdx.x == 0) {
    scs.gam[2 * sc + (k & 1)] = gam;
    scs.alp[2 * sc + (k & 1)] = alpha;
    if (k == 0) scs.bb[sc] = bb;
    if (stop) {
      scs.stop[sc] = 1;
      scs.it_final[sc] = k;
      atomicMax(&st->max_final, k);
      atomicAdd(&st->n_stopped, 1);
      if (bb > 0.0 && gam != 0.0 && !(rho <= rtol2 * bb)) atomicAdd(&st->n_bad, 1);
    }
  }
  if (stop) return;
  // row i of the body's preconditioner block, for u_{k+1} = P_b r_{k+1}
  double Mown[12];
  {
    const double *Mi = inv + 144 * (int64_t)(ok ? b : 0) + 12 * i;
#pragma unroll
    for (int j = 0; j < 12; ++j) Mown[j] = ok ? Mi[j] : 0.0;
  }
  double v = 0.0, own_r = 0.0, own_s = 0.0;
  for (int e = 0; e < Emax; ++e) {
    CgOps nx;
    {
      const int en = e + 1;
      const bool live = ok && en < E;
      cg_fetch(live, cg_col(my_c, g0, en, live, ent, e0), e0 + en, i, Bm, r_in, w_in, s_in, nx);
    }
    double rn, sn;
    cg_step(op.r, op.w, op.s, alpha, beta, sn, rn);
    double pe = 0.0;
#pragma unroll
    for (int j = 0; j < 12; ++j) pe = fma(op.B[j], __shfl(rn, (g0 + j) & 63, 64), pe);
    v += pe;  // (entries past E have zero operands)
    if (e == 0) {  // entry 0 is the body itself
      own_r = rn;
      own_s = sn;
    }
    op = nx;
  }
  double own_un = 0.0;
#pragma unroll
  for (int j = 0; j < 12; ++j) own_un = fma(Mown[j], __shfl(own_r, (g0 + j) & 63, 64), own_un);
  double g = 0.0, d = 0.0, rr = 0.0;
  if (ok) {
    const double pn = fma(beta, own_p, own_u);
    x[oo] = fma(alpha, pn, own_x);
    p[oo] = pn;
    const double wn = own_fixed ? 0.0 : v;
    r_out[oo] = own_r;
    s_out[oo] = own_s;
    u[oo] = own_un;
    w_out[oo] = wn;
    g = own_r * own_un;
    d = wn * own_un;
    rr = own_r * own_r;
  }
  g = wave_sum(g);
  d = wave_sum(d);
  rr = wave_sum(rr);
  if (lane == 0) {
    she[wv][0] = g;
    she[wv][1] = d;
    she[wv][2] = rr;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < SWBB; ++w) t += she[w][threadIdx.x];
    part_out[4 * blockIdx.x + threadIdx.x] = t;
  }
}

// Between replays of a batch: the blocks of scenes still iterating move to
// the front of the block list, in order, with their partials (a scene's fold
// range moves with its blocks), and the tail is marked empty (sc = -1), so
// that once most scenes have stopped an iteration launch reads and runs only
// the remaining scenes' blocks instead of every scene's constants,
// preconditioner blocks and vectors.  One block walks the list in segments
// of CT entries: a segment is read whole before any of it is written, and
// entries only move to lower indices, so nothing unread is overwritten.
constexpr int CT = 1024;
__global__ void __launch_bounds__(CT) k_cg_compact(PcgBlk *blk, int nblk, double *part, CgScene scs) {
  __shared__ int wsum[CT / 64];
  __shared__ int base_sh;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) base_sh = 0;
  __syncthreads();
  for (int seg = 0; seg < nblk; seg += CT) {
    const int j = seg + (int)threadIdx.x;
    PcgBlk r;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
    bool live = false;
    if (j < nblk) {
      r = blk[j];
      live = r.sc >= 0 && !scs.stop[r.sc];
      if (live) {
        p0 = part[4 * (int64_t)j];
        p1 = part[4 * (int64_t)j + 1];
        p2 = part[4 * (int64_t)j + 2];
        p3 = part[4 * (int64_t)j + 3];
      }
    }
    const unsigned long long m = __ballot(live);
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int before = base_sh, total = 0;
    for (int q = 0; q < CT / 64; ++q) {
      before += q < w ? wsum[q] : 0;
      total += wsum[q];
    }
    __syncthreads();  // every entry of the segment, base_sh and wsum read
    if (live) {
      const int np = before + __popcll(m & ((1ull << lane) - 1ull));
      r.fold_lo = np - (j - r.fold_lo);
      blk[np] = r;
      part[4 * (int64_t)np] = p0;
      part[4 * (int64_t)np + 1] = p1;
      part[4 * (int64_t)np + 2] = p2;
      part[4 * (int64_t)np + 3] = p3;
    }
    if (threadIdx.x == 0) base_sh += total;
    __syncthreads();
  }
  for (int j = base_sh + (int)threadIdx.x; j < nblk; j += CT) blk[j].sc = -1;
}

// closes a replay: advances the base and copies the state the host reads
// Algorithmic HBM bytes of a finished solve, added to the profile's device
// total: per scene its iteration count (it_final, or `done` for one scene)
// times its matrix and preconditioner blocks once ((2 n_b + n_k) 12x12
// blocks) and nvec 12-vectors per body; one block, fixed-order sum.
__global__ void __launch_bounds__(256) k_pcg_bytes(int S, const int *it_final, int done, const int32_t *sbo,
                                                   const int64_t *lo_beg, int nvec, unsigned long long *acc) {
  __shared__ unsigned long long sh[256];
  unsigned long long t = 0;
  for (int j = threadIdx.x; j < S; j += 256) {
    const int64_t nbs = sbo[j + 1] - sbo[j], nks = lo_beg[sbo[j + 1]] - lo_beg[sbo[j]];
    const int64_t it = S == 1 ? done : it_final[j];
    t += (unsigned long long)(it * ((2 * nbs + nks) * 1152 + (int64_t)nvec * 96 * nbs));
  }
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *acc += sh[0];
}

// (base, n_stopped, max_final) to mapped host memory
__global__ void k_cg_advance(CgState *st, int n, int *host) {
  st->base += n;
  host[0] = st->base;
  host[1] = st->n_stopped;
  host[2] = st->max_final;
  host[3] = st->n_bad;
}

// y = sx H x (plain block SpMV; five bodies per wave, CBB per block, each
// entry's product added in entry order)
__global__ void __launch_bounds__(SWB) k_bsr_spmv(int nb, const uint8_t *fixed, const double *diag, const double *off,
                                                 const int32_t *keys, const uint32_t *tperm, const int64_t *lo_beg,
                                                 const int64_t *hi_beg, const double *xv, double sx, double *y) {
  const int lane = threadIdx.x & 63;
  const int hb = lane / 12, i = lane - 12 * hb;
  const int b = blockIdx.x * CBB + 5 * (threadIdx.x >> 6) + hb;
  if (hb >= 5 || b >= nb) return;
  const int64_t l0 = lo_beg[b], nlo = lo_beg[b + 1] - l0;
  const int64_t h0 = hi_beg[b], nhi = hi_beg[b + 1] - h0;
  const int64_t E = 1 + nlo + nhi;
  double v = 0.0;
  for (int64_t e = 0; e < E; ++e) {
    const double *row;
    int64_t c;
    int stride;
    if (e == 0) {
      row = diag + 144 * (int64_t)b + 12 * i;
      c = b;
      stride = 1;
    } else if (e <= nlo) {
      const int64_t kk = l0 + e - 1;
      row = off + 144 * kk + 12 * i;
      c = keys[2 * kk + 1];
      stride = 1;
    } else {
      const int64_t kk = tperm[h0 + e - 1 - nlo];
      row = off + 144 * kk + i;
      c = keys[2 * kk];
      stride = 12;
    }
    const double *xc = xv + 12 * c;
    double pe = 0.0;
#pragma unroll
    for (int jj = 0; jj < 12; ++jj) pe = fma(row[stride * jj], xc[jj], pe);
    v += pe;
  }
  y[12 * (int64_t)b + i] = fixed[b] ? 0.0 : sx * v;
}

// The iteration loop of the one-kernel form (set-up shared with op_pcg).
int cg_solve(abd_ctx *ctx, const abd_scene *sc, int S, int nb, int64_t n_keys, const double *diag, const double *off,
             const int32_t *keys, const uint32_t *tv2, const int64_t *lo_beg, const int64_t *hi_beg,
             const double *inv, const double *rhs, const double *x0, const double *Hx0, double *x_out,
             const PcgBlk *ublk, int nblk_u, const int32_t *s_scene, const int64_t *s_off, const int32_t *sbo,
             const int64_t *eoff, const int2 *ent, int nblk_c, double rtol2, int max_iter, int *iters,
             hipStream_t s, int *n_bad, const PcgHook *pre_sync) {
  const int iter_g[2] = {ctx->tune.pcg_short, ctx->tune.pcg_long};
  double *rv[2], *wv[2], *sv[2], *pt[2], *u, *p;
  PcgBlk *cblk;
  CgState *st;
  CgScene scs;
  ABD_TRY(ws(ctx, "cg_r0", 12 * (size_t)nb, &rv[0], s));
  ABD_TRY(ws(ctx, "cg_r1", 12 * (size_t)nb, &rv[1], s));
  ABD_TRY(ws(ctx, "cg_w0", 12 * (size_t)nb, &wv[0], s));
  ABD_TRY(ws(ctx, "cg_w1", 12 * (size_t)nb, &wv[1], s));
  ABD_TRY(ws(ctx, "cg_s0", 12 * (size_t)nb, &sv[0], s));
  ABD_TRY(ws(ctx, "cg_s1", 12 * (size_t)nb, &sv[1], s));
  ABD_TRY(ws(ctx, "cg_u", 12 * (size_t)nb, &u, s));
  ABD_TRY(ws(ctx, "cg_p", 12 * (size_t)nb, &p, s));
  ABD_TRY(ws(ctx, "cg_part0", 4 * (size_t)nblk_c, &pt[0], s));
  ABD_TRY(ws(ctx, "cg_part1", 4 * (size_t)nblk_c, &pt[1], s));
  ABD_TRY(ws(ctx, "cg_blk", nblk_c, &cblk, s));
  double *Bm;
  ABD_TRY(ws(ctx, "cg_bmat", 144 * ((size_t)nb + 2 * (size_t)n_keys), &Bm, s));
  ABD_TRY(ws(ctx, "cg_state", 1, &st, s));
  ABD_TRY(ws(ctx, "cg_s_gam", 2 * (size_t)S, &scs.gam, s));
  ABD_TRY(ws(ctx, "cg_s_alp", 2 * (size_t)S, &scs.alp, s));
  ABD_TRY(ws(ctx, "cg_s_bb", S, &scs.bb, s));
  ABD_TRY(ws(ctx, "cg_s_stop", S, &scs.stop, s));
  ABD_TRY(ws(ctx, "cg_s_final", S, &scs.it_final, s));
  // (cblk, the iteration blocks' constants, folding their own mapping's
  // partials, come from the caller's launch)
  {
    const int64_t n_out = 144 * ((int64_t)nb + 2 * n_keys);  // (entries: one diagonal per body, each key twice)
    if (n_out >= (1ll << 32)) return abd_fail(ctx, ABD_E_INVALID, "pcg: too many matrix entries");
    hipLaunchKernelGGL(k_cg_bmat, dim3(grid_for(n_out, 256)), dim3(256), 0, s, n_out, ent, diag, off, inv, Bm, S, st,
                       scs);
  }
  hipLaunchKernelGGL(k_cg_init1, dim3(nblk_u), dim3(PB), 0, s, ublk, sc->body_fixed, inv, rhs, x0, Hx0, x_out, rv[0],
                     u, p, sv[0]);
  hipLaunchKernelGGL(k_cg_init2, dim3(nblk_c), dim3(SWB), 0, s, cblk, eoff, ent, sc->body_fixed, diag, off, rhs,
                     rv[0], u, wv[0], pt[0]);
  HIP_TRY(ctx, hipGetLastError());
  int64_t *mir_h, *mir_d;
  ABD_TRY(mirror_get(ctx, &mir_h, &mir_d));
  int *hst_d = reinterpret_cast<int *>(mir_d + MIR_PCG);
  const int *hst = reinterpret_cast<const int *>(mir_h + MIR_PCG);
  // n iterations (n even: the parity of k is that of the local index)
  auto enqueue = [&](hipStream_t q, int n) {
    for (int j = 0; j < n; ++j) {
      const int a = j & 1, o = a ^ 1;
      hipLaunchKernelGGL(k_cg_iter, dim3(nblk_c), dim3(SWB), 0, q, j, cblk, eoff, ent, sc->body_fixed, Bm, inv,
                         rv[a], wv[a], sv[a], rv[o], wv[o], sv[o], x_out, u, p, pt[a], pt[o], st, scs, rtol2,
                         max_iter, S > 1 ? 1 : 0);
    }
    // (n is even: the next replay's first iteration folds pt[0])
    if (S > 1) hipLaunchKernelGGL(k_cg_compact, dim3(1), dim3(CT), 0, q, cblk, nblk_c, pt[0], scs);
    hipLaunchKernelGGL(k_cg_advance, dim3(1), dim3(1), 0, q, st, n, hst_d);
  };
  const char *env = getenv("ABD_PCG_GRAPH");
  const bool use_graph = !(env && env[0] == '0');
  // every value baked into the captured kernels' arguments is part of a
  // replay's key (rtol2 by its bit pattern), with its length
  uint64_t rtol_bits;
  std::memcpy(&rtol_bits, &rtol2, sizeof(rtol_bits));
  const std::vector<uintptr_t> key = {
      (uintptr_t)Bm,       (uintptr_t)off,      (uintptr_t)inv,          (uintptr_t)x_out,      (uintptr_t)u,
      (uintptr_t)p,        (uintptr_t)rv[0],    (uintptr_t)rv[1],        (uintptr_t)wv[0],      (uintptr_t)wv[1],
      (uintptr_t)sv[0],    (uintptr_t)sv[1],    (uintptr_t)pt[0],        (uintptr_t)pt[1],      (uintptr_t)cblk,
      (uintptr_t)ent,      (uintptr_t)st,       (uintptr_t)sc->body_fixed, (uintptr_t)eoff,
      (uintptr_t)nblk_c,   (uintptr_t)max_iter, (uintptr_t)rtol_bits,    (uintptr_t)scs.gam,    (uintptr_t)scs.alp,
      (uintptr_t)scs.bb,   (uintptr_t)scs.stop, (uintptr_t)scs.it_final, (uintptr_t)hst_d, (uintptr_t)S, (uintptr_t)1};
  // replay L iterations (L a power of two in [2, 256]): its captured graph,
  // captured on first use, or the launches themselves without graphs
  auto replay = [&](int L) -> int {
    if (!use_graph) {
      enqueue(s, L);
      return ABD_OK;
    }
    int k = 0;
    while ((2 << k) < L) ++k;
    std::vector<uintptr_t> kk = key;
    kk.push_back((uintptr_t)L);
    if (ctx->cg_exec[k] == nullptr || ctx->cg_key[k] != kk) {
      HostTimer ht(ctx, "pcg_capture", L);
      if (!ctx->capture_stream)
        HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
      if (ctx->cg_exec[k]) HIP_TRY(ctx, hipGraphExecDestroy(ctx->cg_exec[k]));
      ctx->cg_exec[k] = nullptr;
      hipGraph_t g = nullptr;
      HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
      enqueue(ctx->capture_stream, L);
      HIP_TRY(ctx, hipStreamEndCapture(ctx->capture_stream, &g));
      HIP_TRY(ctx, hipGraphInstantiate(&ctx->cg_exec[k], g, nullptr, nullptr, 0));
      HIP_TRY(ctx, hipGraphDestroy(g));
      ctx->cg_key[k] = kk;
    }
    HIP_TRY(ctx, hipGraphLaunch(ctx->cg_exec[k], s));
    return ABD_OK;
  };
  // Replay lengths are powers of two from Lmin (pcg_short) to Lmax
  // (pcg_long).  A round covers the last solve's iteration count (once
  // that count is passed, as many iterations again as done so far, at
  // least Lmin) with the fewest replays whose total overshoots it by at
  // most half: launches past a scene's stop return at once but still cost
  // a launch, and each round costs a host round trip.
  int Lmin = 2, Lmax = 2;
  while (Lmin < iter_g[0] && Lmin < 256) Lmin <<= 1;
  while (2 * Lmax <= iter_g[1] && Lmax < 256) Lmax <<= 1;
  if (Lmax < Lmin) Lmax = Lmin;
  auto pick = [&](int target) {
    int L = Lmin;
    while (L < target && L < Lmax) L <<= 1;
    if (L > Lmin && L - target > target / 2) L >>= 1;
    return L;
  };
  const int max_rounds = max_iter / Lmin + 2;
  int done = 0;
  bool all = false;
  bool profiled = false;
  for (int round = 0; round < max_rounds && !all;) {
    int target = ctx->pcg_hint - done;
    if (target < Lmin) target = done > Lmin ? done : Lmin;
    int planned = 0;
    do {
      const int L = pick(target - planned);
      hipEvent_t pe = prof_begin(ctx, s);
      profiled = profiled || pe != nullptr;
      ABD_TRY(replay(L));
      prof_end(ctx, pe, "pcg_round", 0, s);
      HIP_TRY(ctx, hipGetLastError());
      planned += L;
      ++round;
    } while (round < max_rounds && planned < target);
    if (pre_sync) ABD_TRY((*pre_sync)(reinterpret_cast<const int *>(st)));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    all = hst[1] >= S;
    done = all ? hst[2] : hst[0];  // iterations: the largest count over the scenes
  }
  *iters = done;
  *n_bad = all ? hst[3] : S;
  ctx->pcg_hint = done;
  if (profiled && all) {
    // (the profile's device total; the query reads it)
    unsigned long long *acc;
    ABD_TRY(prof_pcg_bytes(ctx, &acc, s));
    hipLaunchKernelGGL(k_pcg_bytes, dim3(1), dim3(256), 0, s, S, scs.it_final, done, sbo, lo_beg, 12, acc);
    HIP_TRY(ctx, hipGetLastError());
  }
  (void)n_keys;
  (void)keys;
  (void)tv2;
  (void)hi_beg;
  return ABD_OK;
}

}  // namespace


int op_pcg(abd_ctx *ctx, const abd_scene *sc, const double *diag, const double *off, const int32_t *keys,
           int64_t n_keys, const double *rhs, double *x_out, double rtol, int max_iter, int *iters, hipStream_t s,
           const double *x0, const double *pre_diag, const KeyPattern *pat, const PcgHook *pre_sync,
           bool *pre_sync_final, const uint8_t *skip_scene) {
  if (pre_sync_final) *pre_sync_final = false;
  const int nb = sc->n_bodies;
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  const int iter_g[2] = {ctx->tune.pcg_short, ctx->tune.pcg_long};
  *iters = 0;
  if (nb <= 0) return ABD_OK;
  if (n_keys >= (1ll << 31) || nb >= (1 << 24)) return abd_fail(ctx, ABD_E_INVALID, "pcg: too many blocks");
  double *inv, *r, *z, *pa, *pb, *Ap, *part, *part2;
  int64_t *lo_beg, *hi_beg, *ucnt, *scnt, *u_off, *s_off;
  int32_t *u_scene, *s_scene;
  uint64_t *tk, *tk2;
  uint32_t *tv, *tv2;
  int *err;
  PcgState *st;
  PcgScene scs;
  // block counts: at most one partly filled block per scene
  const int nblk_u = (int)grid_for((int64_t)nb, PBB) + S;
  const int nblk_s = (int)grid_for(nb, CBB) + S;
  const int nblk_c = (int)grid_for(nb, CBB) + S;
  const int32_t *sbo;
  ABD_TRY(op_scene_offsets(ctx, sc, &sbo, s));
  ABD_TRY(ws(ctx, "pcg_inv", 144 * (size_t)nb, &inv, s));
  ABD_TRY(ws(ctx, "pcg_r", 12 * (size_t)nb, &r, s));
  ABD_TRY(ws(ctx, "pcg_z", 12 * (size_t)nb, &z, s));
  ABD_TRY(ws(ctx, "pcg_pa", 12 * (size_t)nb, &pa, s));
  ABD_TRY(ws(ctx, "pcg_pb", 12 * (size_t)nb, &pb, s));
  ABD_TRY(ws(ctx, "pcg_Ap", 12 * (size_t)nb, &Ap, s));
  ABD_TRY(ws(ctx, "pcg_part", nblk_s, &part, s));
  ABD_TRY(ws(ctx, "pcg_part2", 3 * (size_t)nblk_u, &part2, s));
  ABD_TRY(ws(ctx, "pcg_lob", nb + 1, &lo_beg, s));
  ABD_TRY(ws(ctx, "pcg_hib", nb + 1, &hi_beg, s));
  ABD_TRY(ws(ctx, "pcg_tk", n_keys + 1, &tk, s));
  ABD_TRY(ws(ctx, "pcg_tk2", n_keys + 1, &tk2, s));
  ABD_TRY(ws(ctx, "pcg_tv", n_keys + 1, &tv, s));
  ABD_TRY(ws(ctx, "pcg_tv2", n_keys + 1, &tv2, s));
  ABD_TRY(ws(ctx, "pcg_ucnt", S, &ucnt, s));
  ABD_TRY(ws(ctx, "pcg_scnt", S, &scnt, s));
  ABD_TRY(ws(ctx, "pcg_uoff", S + 1, &u_off, s));
  ABD_TRY(ws(ctx, "pcg_soff", S + 1, &s_off, s));
  ABD_TRY(ws(ctx, "pcg_usc", nblk_u, &u_scene, s));
  ABD_TRY(ws(ctx, "pcg_ssc", nblk_s, &s_scene, s));
  int64_t *c_off;
  int32_t *c_scene;
  ABD_TRY(ws(ctx, "pcg_coff", S + 1, &c_off, s));
  ABD_TRY(ws(ctx, "pcg_csc", nblk_c, &c_scene, s));
  ABD_TRY(ws(ctx, "pcg_state", 1, &st, s));
  ABD_TRY(ws(ctx, "pcg_s_rz", 2 * (size_t)S, &scs.rz, s));
  ABD_TRY(ws(ctx, "pcg_s_bb", S, &scs.bb, s));
  ABD_TRY(ws(ctx, "pcg_s_stop", S, &scs.stop, s));
  ABD_TRY(ws(ctx, "pcg_s_final", S, &scs.it_final, s));
  ABD_TRY(ws(ctx, "err_flag", 1, &err, s));
  hipLaunchKernelGGL(k_block_inverse, dim3(grid_for(nb, 64)), dim3(64), 0, s, nb, sc->body_fixed,
                     pre_diag ? pre_diag : diag, inv, err, skip_scene, sc->body_scene);
  // (the block-to-scene maps depend on the scene alone)
  if (scene_table_cached(ctx, sc, "pcg_scene_maps", c_scene)) {
  } else if (S <= SETUP_T) {
    hipLaunchKernelGGL(k_pcg_scene_setup, dim3(1), dim3(SETUP_T), 0, s, S, sbo, (int64_t)nblk_u, (int64_t)nblk_s,
                       u_off, s_off, u_scene, s_scene);
    hipLaunchKernelGGL(k_pcg_scene_map, dim3(1), dim3(SETUP_T), 0, s, S, sbo, CBB, (int64_t)nblk_c, c_off, c_scene);
  } else {
    hipLaunchKernelGGL(k_pcg_scene_blocks, dim3(grid_for(S, 256)), dim3(256), 0, s, S, sbo, ucnt, scnt);
    ABD_TRY(scan_exclusive_i64(ctx, ucnt, u_off, S, u_off + S, s));
    ABD_TRY(scan_exclusive_i64(ctx, scnt, s_off, S, s_off + S, s));
    hipLaunchKernelGGL(k_pcg_block_scene, dim3(grid_for(nblk_u, 256)), dim3(256), 0, s, S, (int64_t)nblk_u, u_off,
                       u_scene);
    hipLaunchKernelGGL(k_pcg_block_scene, dim3(grid_for(nblk_s, 256)), dim3(256), 0, s, S, (int64_t)nblk_s, s_off,
                       s_scene);
    int64_t *ccnt;
    ABD_TRY(ws(ctx, "pcg_ccnt", S, &ccnt, s));
    hipLaunchKernelGGL(k_pcg_scene_count, dim3(grid_for(S, 256)), dim3(256), 0, s, S, sbo, CBB, ccnt);
    ABD_TRY(scan_exclusive_i64(ctx, ccnt, c_off, S, c_off + S, s));
    hipLaunchKernelGGL(k_pcg_block_scene, dim3(grid_for(nblk_c, 256)), dim3(256), 0, s, S, (int64_t)nblk_c, c_off,
                       c_scene);
  }
  if (pat && pat->valid) {
    // row structure built with the keys
    lo_beg = const_cast<int64_t *>(pat->lo_beg);
    hi_beg = const_cast<int64_t *>(pat->hi_beg);
    tv2 = const_cast<uint32_t *>(pat->tperm);
  } else {
    if (n_keys > 0) {
      hipLaunchKernelGGL(k_tkeys, dim3(grid_for(n_keys, 256)), dim3(256), 0, s, n_keys, keys, tk, tv);
      size_t tmp_bytes = 0;
      HIP_TRY(ctx, rocprim::radix_sort_pairs(nullptr, tmp_bytes, tk, tk2, tv, tv2, (size_t)n_keys, 0, 64, s));
      void *tmp;
      ABD_TRY(ws_get(ctx, "pcg_sort_tmp", tmp_bytes + 16, &tmp, s));
      HIP_TRY(ctx, rocprim::radix_sort_pairs(tmp, tmp_bytes, tk, tk2, tv, tv2, (size_t)n_keys, 0, 64, s));
    }
    hipLaunchKernelGGL(k_row_ranges, dim3(grid_for(nb + 1, 256)), dim3(256), 0, s, nb, n_keys, keys, tk2, lo_beg,
                       hi_beg);
  }
  // entry lists per body and per-block constants
  int64_t *eoff;
  int2 *ent;
  PcgBlk *sblk, *ublk;
  ABD_TRY(ws(ctx, "pcg_eoff", nb + 1, &eoff, s));
  ABD_TRY(ws(ctx, "pcg_ent", nb + 2 * n_keys + 1, &ent, s));
  ABD_TRY(ws(ctx, "pcg_sblk", nblk_s, &sblk, s));
  ABD_TRY(ws(ctx, "pcg_ublk", nblk_u, &ublk, s));
  hipLaunchKernelGGL(k_pcg_entries, dim3(grid_for(nb + 1, 256)), dim3(256), 0, s, nb, lo_beg, hi_beg, tv2, keys, eoff,
                     ent);
  // block constants of the three mappings: two-kernel SpMV blocks (folding
  // the update blocks' partials), update blocks (folding the SpMV blocks'),
  // one-kernel iteration blocks (folding their own)
  PcgBlk *cblk;
  ABD_TRY(ws(ctx, "cg_blk", nblk_c, &cblk, s));
  {
    BlkJobs J;
    J.j[0] = BlkJob{(int64_t)nblk_s, CBB, s_scene, s_off, u_off, sblk};
    J.j[1] = BlkJob{(int64_t)nblk_u, PBB, u_scene, u_off, s_off, ublk};
    J.j[2] = BlkJob{(int64_t)nblk_c, CBB, c_scene, c_off, c_off, cblk};
    const int64_t tot = (int64_t)nblk_s + nblk_u + nblk_c;
    hipLaunchKernelGGL(k_pcg_blk, dim3(grid_for(tot, 256)), dim3(256), 0, s, J, sbo, S, st, scs);
  }
  const double *Hx0 = nullptr;
  if (x0) {
    // warm start: r = rhs - H x0 (Ap as scratch)
    hipLaunchKernelGGL(k_bsr_spmv, dim3(grid_for(nb, CBB)), dim3(SWB), 0, s, nb, sc->body_fixed, diag, off, keys, tv2,
                       lo_beg, hi_beg, x0, 1.0, Ap);
    Hx0 = Ap;
  }
  const double rtol2 = rtol * rtol;
  const char *cg_env = getenv("ABD_PCG_CG");
  int it0 = 0;
  const bool one_kernel = !(cg_env && cg_env[0] == '0');
  if (one_kernel) {
    int n_bad = 0;
    ABD_TRY(cg_solve(ctx, sc, S, nb, n_keys, diag, off, keys, tv2, lo_beg, hi_beg, inv, rhs, x0, Hx0, x_out, ublk,
                     nblk_u, s_scene, s_off, sbo, eoff, ent, nblk_c, rtol2, max_iter, &it0, s, &n_bad,
                     pre_sync));
    // At a tolerance of 1e-6 or looser, a recursive residual that drifted
    // by the one-reduction form's rounding (about 1e-12 of |b|) cannot turn
    // a stop on the tolerance into a wrong one, so when every scene stopped
    // on it the check below is skipped.
    if (rtol >= PCG_CHECK_RTOL && n_bad == 0) {
      *iters = it0;
      ctx->pcg_hint = it0;
      if (pre_sync_final) *pre_sync_final = pre_sync != nullptr;
      return ABD_OK;
    }
    // The one-reduction recurrences may stop on a recursive residual that
    // has drifted from rhs - H x (w is formed as (H P) r rather than
    // H (P r), and p.Hp as a difference that cancels near the attainable
    // floor), so the iterate is checked against a freshly computed
    // residual: iteration 0 of the two-reduction form, started from it,
    // stops every scene that meets the tolerance and carries on with the
    // others.
    hipLaunchKernelGGL(k_bsr_spmv, dim3(grid_for(nb, CBB)), dim3(SWB), 0, s, nb, sc->body_fixed, diag, off, keys, tv2,
                       lo_beg, hi_beg, x_out, 1.0, Ap);
    x0 = x_out;
    Hx0 = Ap;
  }
  // (after the check's iteration, which runs outside the captured graphs,
  // the graphs must again start from p in pa)
  hipLaunchKernelGGL(k_pcg_init, dim3(nblk_u), dim3(PB), 0, s, u_scene, u_off, sbo, sc->body_fixed, inv, rhs, x0, Hx0,
                     x_out, r, z, one_kernel ? pb : pa, part2);
  HIP_TRY(ctx, hipGetLastError());
  if (one_kernel) {
    hipLaunchKernelGGL(k_pcg_spmv, dim3(nblk_s), dim3(SWB), 0, s, sblk, eoff, ent, sc->body_fixed, diag, off, pb, z, pa, Ap,
                       part2, part, st, scs, rtol2, max_iter);
    hipLaunchKernelGGL(k_pcg_update, dim3(nblk_u), dim3(PB), 0, s, ublk, inv, pa, Ap, x_out, r, z, part, part2, st,
                       scs, err);
    HIP_TRY(ctx, hipGetLastError());
    int *hv;
    ABD_TRY(pinned_get(ctx, sizeof(int) * (4 + (size_t)S), reinterpret_cast<void **>(&hv)));
    HIP_TRY(ctx, hipMemcpyAsync(hv, st, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (hv[2] >= S) {
      *iters = it0;
      ctx->pcg_hint = it0;
      return ABD_OK;
    }
  }
  // n iterations: p alternates pa -> pb -> pa ... (n is even)
  auto enqueue = [&](hipStream_t q, int n) {
    for (int k = 0; k < n; ++k) {
      double *p_old = (k % 2 == 0) ? pa : pb, *p_new = (k % 2 == 0) ? pb : pa;
      hipLaunchKernelGGL(k_pcg_spmv, dim3(nblk_s), dim3(SWB), 0, q, sblk, eoff, ent, sc->body_fixed, diag, off, p_old, z,
                         p_new, Ap, part2, part, st, scs, rtol2, max_iter);
      hipLaunchKernelGGL(k_pcg_update, dim3(nblk_u), dim3(PB), 0, q, ublk, inv, p_new, Ap, x_out, r, z, part, part2,
                         st, scs, err);
    }
  };
  const char *env = getenv("ABD_PCG_GRAPH");
  const bool use_graph = !(env && env[0] == '0');
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  if (use_graph) {
    // every value baked into the captured kernels' arguments is part of the
    // key (rtol2 by its bit pattern)
    uint64_t rtol_bits;
    std::memcpy(&rtol_bits, &rtol2, sizeof(rtol_bits));
    const std::vector<uintptr_t> key = {
        (uintptr_t)diag, (uintptr_t)off, (uintptr_t)keys, (uintptr_t)tv2, (uintptr_t)lo_beg, (uintptr_t)hi_beg,
        (uintptr_t)inv, (uintptr_t)x_out, (uintptr_t)r, (uintptr_t)z, (uintptr_t)pa, (uintptr_t)pb,
        (uintptr_t)Ap, (uintptr_t)part, (uintptr_t)part2, (uintptr_t)st, (uintptr_t)err,
        (uintptr_t)sc->body_fixed, (uintptr_t)nb, (uintptr_t)max_iter, (uintptr_t)rtol_bits,
        (uintptr_t)S, (uintptr_t)sbo, (uintptr_t)u_scene, (uintptr_t)s_scene, (uintptr_t)u_off, (uintptr_t)s_off,
        (uintptr_t)scs.rz, (uintptr_t)scs.bb, (uintptr_t)scs.stop, (uintptr_t)scs.it_final,
        (uintptr_t)nblk_u, (uintptr_t)nblk_s, (uintptr_t)sblk, (uintptr_t)ublk, (uintptr_t)ent,
        (uintptr_t)iter_g[0], (uintptr_t)iter_g[1]};
    if (!ctx->capture_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    for (int gi = 0; gi < 2; ++gi) {
      if (ctx->pcg_exec[gi] == nullptr || ctx->pcg_key[gi] != key) {
        HostTimer ht(ctx, "pcg_capture", iter_g[gi]);
        if (ctx->pcg_exec[gi]) HIP_TRY(ctx, hipGraphExecDestroy(ctx->pcg_exec[gi]));
        ctx->pcg_exec[gi] = nullptr;
        hipGraph_t g = nullptr;
        HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        enqueue(ctx->capture_stream, iter_g[gi]);
        HIP_TRY(ctx, hipStreamEndCapture(ctx->capture_stream, &g));
        HIP_TRY(ctx, hipGraphInstantiate(&ctx->pcg_exec[gi], g, nullptr, nullptr, 0));
        HIP_TRY(ctx, hipGraphDestroy(g));
        ctx->pcg_key[gi] = key;
      }
      exec[gi] = ctx->pcg_exec[gi];
    }
  }
  int *h;  // [0..3] state counters
  ABD_TRY(pinned_get(ctx, sizeof(int) * 4, reinterpret_cast<void **>(&h)));
  const int max_rounds = max_iter / iter_g[0] + 2;
  // algorithmic HBM bytes of one iteration of a scene: every 12x12 block of
  // its matrix and of its preconditioner once, plus the 12-vectors read and
  // written by the two kernels (spmv: z, p_old in, p_new, Ap out; update:
  // p, Ap, x, r in, x, r, z out)
  int done = 0;
  bool all = false;
  bool profiled = false;
  // (after the one-kernel form, the iterations left are few and unknown)
  const int hint = one_kernel ? 0 : ctx->pcg_hint;
  for (int round = 0; round < max_rounds && !all; ++round) {
    // a long replay while the last solve's count says at least that many
    // iterations remain, else a short one
    const int gi = hint - done >= iter_g[1] ? 1 : 0;
    hipEvent_t pe = prof_begin(ctx, s);
    profiled = profiled || pe != nullptr;
    if (exec[gi])
      HIP_TRY(ctx, hipGraphLaunch(exec[gi], s));
    else
      enqueue(s, iter_g[gi]);
    prof_end(ctx, pe, "pcg_round", 0, s);
    HIP_TRY(ctx, hipGetLastError());
    // it_done, k_cur, n_stopped, max_final
    HIP_TRY(ctx, hipMemcpyAsync(h, st, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    all = h[2] >= S;
    done = all ? h[3] : h[0];  // iterations: the largest count over the scenes
  }
  *iters = it0 + done;
  ctx->pcg_hint = one_kernel ? it0 : done;
  if (profiled && all) {
    // (the profile's device total; the query reads it)
    unsigned long long *acc;
    ABD_TRY(prof_pcg_bytes(ctx, &acc, s));
    hipLaunchKernelGGL(k_pcg_bytes, dim3(1), dim3(256), 0, s, S, scs.it_final, done, sbo, lo_beg, 11, acc);
    HIP_TRY(ctx, hipGetLastError());
  }
  return ABD_OK;
}

// --------------------------------------------------------------- MINRES ----
// Preconditioned MINRES (Paige and Saunders; the formulation of Elman,
// Silvester and Wathen) for symmetric systems that may be indefinite, such
// as the unprojected Hessian of the adjoint: one SpMV and one block-Jacobi
// application per iteration, the short scalar recurrence on the host.  The
// preconditioner must be symmetric positive definite (its diagonal blocks
// are given separately).
namespace {

__global__ void k_block_apply(int nb, const double *inv, const double *v, double *z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 12 * nb) return;
  const int b = t / 12, i = t % 12;
  const double *M = inv + 144 * (int64_t)b + 12 * i;
  const double *vb = v + 12 * (int64_t)b;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 12; ++j) s += M[j] * vb[j];
  z[t] = s;
}

__global__ void k_vmul(int n, const double *a, const double *b, double *o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i] * b[i];
}

// v_next = Az - a v - b v_prev
__global__ void k_minres_v(int n, const double *Az, const double *v, const double *vp, double a, double b,
                           double *vn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) vn[i] = Az[i] - a * v[i] - b * vp[i];
}

// w_next = (zs z - a3 w_prev - a2 w) / a1 (written over w_prev); x += cx w_next
__global__ void k_minres_wx(int n, const double *z, double zs, double *wp, const double *w, double a3, double a2,
                            double a1, double cx, double *x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double wn = (zs * z[i] - a3 * wp[i] - a2 * w[i]) / a1;
  wp[i] = wn;
  x[i] += cx * wn;
}

__global__ void k_vzero(int n, double *a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

// MINRES scalars on the device (Paige and Saunders' recurrences with the
// preconditioner's inner product), so that iterations are queued without a
// host round trip; the host reads `done` once per batch.  An iteration
// begun after `done` is set changes nothing: apply = 0 for it.
struct MrState {
  double gam, gam_prev, eta, c, c_prev, sn, s_prev, g1, rtol;
  double delta;                       // (A z / gam) . (z / gam) of the iteration
  double inv_gam, va, vb;             // v_next = inv_gam A z - va v - vb v_prev
  double wz, wa3, wa2, wa1, wcx;      // w_next = (wz z - wa3 w_prev - wa2 w) / wa1; x += wcx w_next
  int done, apply, iters, err;        // err: 1 preconditioner not SPD, 2 breakdown
};
constexpr int MR_T = 1024;
__device__ __forceinline__ double mr_block_dot(const double *a, const double *b, int n, double *sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += MR_T) v += a[i] * b[i];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < MR_T / 64; ++w) r += sh[w];
  return r;  // (thread 0)
}
// delta = (A z / gam) . (z / gam) from the unscaled A z
__global__ void __launch_bounds__(MR_T) k_mr_delta(const double *Az, const double *z, int n, MrState *st) {
  __shared__ double sh[MR_T / 64];
  if (st->done) return;
  const double dz = mr_block_dot(Az, z, n, sh);
  if (threadIdx.x == 0) {
    const double gam = st->gam;
    const double delta = dz / gam / gam;
    st->inv_gam = 1.0 / gam;
    st->va = delta / gam;
    st->vb = gam / st->gam_prev;
    st->delta = delta;
  }
}
// gamma_next from z_next . v_next, the Givens rotation, the w / x update
// coefficients, the residual estimate and the stop test
__global__ void __launch_bounds__(MR_T) k_mr_rot(const double *zn, const double *vn, int n, MrState *st) {
  __shared__ double sh[MR_T / 64];
  if (st->done) {
    if (threadIdx.x == 0) st->apply = 0;
    return;
  }
  const double gn2 = mr_block_dot(zn, vn, n, sh);
  if (threadIdx.x != 0) return;
  if (!(gn2 >= 0.0)) {
    st->err = 1;
    st->done = 1;
    st->apply = 0;
    return;
  }
  const double gam = st->gam, delta = st->delta, c = st->c, c_prev = st->c_prev, sn = st->sn, s_prev = st->s_prev;
  const double gn = sqrt(gn2);
  const double a0 = c * delta - c_prev * sn * gam;
  const double a1 = sqrt(a0 * a0 + gn * gn);
  const double a2 = sn * delta + c_prev * c * gam;
  const double a3 = s_prev * gam;
  if (!(a1 > 0.0)) {
    st->err = 2;
    st->done = 1;
    st->apply = 0;
    return;
  }
  const double c_n = a0 / a1, s_n = gn / a1;
  st->wz = 1.0 / gam;
  st->wa3 = a3;
  st->wa2 = a2;
  st->wa1 = a1;
  st->wcx = c_n * st->eta;
  st->apply = 1;
  st->eta = -s_n * st->eta;
  st->gam_prev = gam;
  st->gam = gn;
  st->c_prev = c;
  st->c = c_n;
  st->s_prev = sn;
  st->sn = s_n;
  st->iters += 1;
  if (fabs(st->eta) <= st->rtol * st->g1 || gn == 0.0) st->done = 1;
}
// One launch for the element-wise work between the two reductions of an
// iteration: the previous iteration's w / x update (its coefficients were
// fixed by that iteration's k_mr_rot; skipped on the first iteration and
// once stopped), then v_next = inv_gam A z - va v - vb v_prev and
// z_next = P v_next.  A block covers whole bodies (MV_B of them), so P's
// 12 x 12 block product reads v_next from LDS.
constexpr int MV_B = 16;
__global__ void __launch_bounds__(12 * MV_B) k_mr_vz(int nb, const double *Az, const double *v, const double *vp,
                                                    const double *inv, MrState *st, double *vn, double *zn,
                                                    int first, const double *z_prev, double *wp, const double *w,
                                                    double *x) {
  __shared__ double sv[12 * MV_B];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = 12 * nb;
  if (!first && st->apply && t < n) {
    const double wn = (st->wz * z_prev[t] - st->wa3 * wp[t] - st->wa2 * w[t]) / st->wa1;
    wp[t] = wn;
    x[t] += st->wcx * wn;
  }
  if (st->done) return;  // (uniform over the grid)
  const double val = t < n ? st->inv_gam * Az[t] - st->va * v[t] - st->vb * vp[t] : 0.0;
  if (t < n) vn[t] = val;
  sv[threadIdx.x] = val;
  __syncthreads();
  if (t >= n) return;
  const int lb = threadIdx.x / 12, i = threadIdx.x % 12;
  const double *M = inv + 144 * (int64_t)(t / 12) + 12 * i;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < 12; ++j) acc += M[j] * sv[12 * lb + j];
  zn[t] = acc;
}

__global__ void k_mr_wx(int n, const double *z, double *wp, const double *w, const MrState *st, double *x) {
  if (!st->apply) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double wn = (st->wz * z[i] - st->wa3 * wp[i] - st->wa2 * w[i]) / st->wa1;
  wp[i] = wn;
  x[i] += st->wcx * wn;
}

}  // namespace

int op_minres(abd_ctx *ctx, const abd_scene *sc, const double *diag, const double *off, const int32_t *keys,
              int64_t n_keys, const double *pre_diag, const double *rhs, double *x_out, double rtol, int max_iter,
              int *iters, hipStream_t s) {
  const int nb = sc->n_bodies, n12 = 12 * nb;
  *iters = 0;
  if (nb <= 0) return ABD_OK;
  double *inv, *v0, *v1, *v2, *z, *Az, *w0, *w1, *tmp, *dot;
  int64_t *lo_beg, *hi_beg;
  uint64_t *tk, *tk2;
  uint32_t *tv, *tv2;
  int *err;
  ABD_TRY(ws(ctx, "mr_inv", 144 * (size_t)nb, &inv, s));
  ABD_TRY(ws(ctx, "mr_v0", n12, &v0, s));
  ABD_TRY(ws(ctx, "mr_v1", n12, &v1, s));
  ABD_TRY(ws(ctx, "mr_v2", n12, &v2, s));
  ABD_TRY(ws(ctx, "mr_z", n12, &z, s));
  ABD_TRY(ws(ctx, "mr_Az", n12, &Az, s));
  ABD_TRY(ws(ctx, "mr_w0", n12, &w0, s));
  ABD_TRY(ws(ctx, "mr_w1", n12, &w1, s));
  ABD_TRY(ws(ctx, "mr_tmp", n12, &tmp, s));
  ABD_TRY(ws(ctx, "mr_dot", 2, &dot, s));
  ABD_TRY(ws(ctx, "mr_lob", nb + 1, &lo_beg, s));
  ABD_TRY(ws(ctx, "mr_hib", nb + 1, &hi_beg, s));
  ABD_TRY(ws(ctx, "mr_tk", n_keys + 1, &tk, s));
  ABD_TRY(ws(ctx, "mr_tk2", n_keys + 1, &tk2, s));
  ABD_TRY(ws(ctx, "mr_tv", n_keys + 1, &tv, s));
  ABD_TRY(ws(ctx, "mr_tv2", n_keys + 1, &tv2, s));
  ABD_TRY(ws(ctx, "err_flag", 1, &err, s));
  hipLaunchKernelGGL(k_block_inverse, dim3(grid_for(nb, 64)), dim3(64), 0, s, nb, sc->body_fixed, pre_diag, inv, err);
  if (n_keys > 0) {
    hipLaunchKernelGGL(k_tkeys, dim3(grid_for(n_keys, 256)), dim3(256), 0, s, n_keys, keys, tk, tv);
    size_t tmp_bytes = 0;
    HIP_TRY(ctx, rocprim::radix_sort_pairs(nullptr, tmp_bytes, tk, tk2, tv, tv2, (size_t)n_keys, 0, 64, s));
    void *stmp;
    ABD_TRY(ws_get(ctx, "mr_sort_tmp", tmp_bytes + 16, &stmp, s));
    HIP_TRY(ctx, rocprim::radix_sort_pairs(stmp, tmp_bytes, tk, tk2, tv, tv2, (size_t)n_keys, 0, 64, s));
  }
  hipLaunchKernelGGL(k_row_ranges, dim3(grid_for(nb + 1, 256)), dim3(256), 0, s, nb, n_keys, keys, tk2, lo_beg,
                     hi_beg);
  const unsigned gv = grid_for(n12, 256), gs = grid_for(nb, CBB);
  double *h;
  ABD_TRY(pinned_get(ctx, 64, reinterpret_cast<void **>(&h)));
  auto dotp = [&](const double *a, const double *b, double *out) -> int {
    hipLaunchKernelGGL(k_vmul, dim3(gv), dim3(256), 0, s, n12, a, b, tmp);
    HIP_TRY(ctx, hipMemsetAsync(dot, 0, sizeof(double), s));
    ABD_TRY(reduce_sum_f64(ctx, tmp, n12, dot, s));
    HIP_TRY(ctx, hipMemcpyAsync(h, dot, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *out = h[0];
    return ABD_OK;
  };
  // x = 0, v_prev = 0, v = rhs on free bodies, z = P v
  hipLaunchKernelGGL(k_vzero, dim3(gv), dim3(256), 0, s, n12, x_out);
  hipLaunchKernelGGL(k_vzero, dim3(gv), dim3(256), 0, s, n12, v0);
  hipLaunchKernelGGL(k_vzero, dim3(gv), dim3(256), 0, s, n12, w0);
  hipLaunchKernelGGL(k_vzero, dim3(gv), dim3(256), 0, s, n12, w1);
  hipLaunchKernelGGL(k_block_apply, dim3(gv), dim3(256), 0, s, nb, inv, rhs, z);  // P is zero on fixed bodies
  HIP_TRY(ctx, hipMemcpyAsync(v1, rhs, sizeof(double) * n12, hipMemcpyDeviceToDevice, s));
  ABD_TRY(op_read_err(ctx, s));
  double g2;
  ABD_TRY(dotp(z, v1, &g2));
  if (!(g2 >= 0.0)) return abd_fail(ctx, ABD_E_PCG, "MINRES: preconditioner not positive definite");
  double gam = std::sqrt(g2), gam_prev = 1.0;
  const double g1 = gam;
  if (g1 == 0.0) return ABD_OK;
  // device scalars; iterations queued in batches of MR_BATCH, the host
  // reading the stop flag, the count and the error after each batch
  MrState h0 = {};
  h0.gam = gam;
  h0.gam_prev = gam_prev;
  h0.eta = gam;
  h0.c = h0.c_prev = 1.0;
  h0.sn = h0.s_prev = 0.0;
  h0.g1 = g1;
  h0.rtol = rtol;
  MrState *st;
  ABD_TRY(ws(ctx, "mr_state", 1, &st, s));
  MrState *hs;
  ABD_TRY(pinned_get(ctx, sizeof(MrState), reinterpret_cast<void **>(&hs)));
  *hs = h0;
  HIP_TRY(ctx, hipMemcpyAsync(st, hs, sizeof(MrState), hipMemcpyHostToDevice, s));
  double *z2, *z3;
  ABD_TRY(ws(ctx, "mr_z2", n12, &z2, s));
  ABD_TRY(ws(ctx, "mr_z3", n12, &z3, s));
  double *vp = v0, *vc = v1, *vn = v2, *wp = w0, *wc = w1, *zc = z, *zn = z2;
  constexpr int MR_BATCH = 16;
  int j = 0;
  // per iteration: A z; delta; [previous w / x update, v_next, z_next];
  // gamma_next and the rotation.  The w / x update of an iteration runs in
  // the next iteration's element-wise launch (or after the loop), with the
  // z of its own iteration (zp).
  const unsigned gvz = grid_for(nb, MV_B);
  double *zp = nullptr;
  bool first = true;
  while (j < max_iter) {
    const int nbat = max_iter - j < MR_BATCH ? max_iter - j : MR_BATCH;
    for (int q = 0; q < nbat; ++q) {
      hipLaunchKernelGGL(k_bsr_spmv, dim3(gs), dim3(SWB), 0, s, nb, sc->body_fixed, diag, off, keys, tv2, lo_beg,
                         hi_beg, zc, 1.0, Az);
      hipLaunchKernelGGL(k_mr_delta, dim3(1), dim3(MR_T), 0, s, Az, zc, n12, st);
      hipLaunchKernelGGL(k_mr_vz, dim3(gvz), dim3(12 * MV_B), 0, s, nb, Az, vc, vp, inv, st, vn, zn, first ? 1 : 0,
                         zp, wp, wc, x_out);
      if (!first) std::swap(wp, wc);  // (the update wrote w_next over w_prev)
      first = false;
      hipLaunchKernelGGL(k_mr_rot, dim3(1), dim3(MR_T), 0, s, zn, vn, n12, st);
      // rotate (data independent, so queued iterations agree with the device)
      double *t = vp;
      vp = vc;
      vc = vn;
      vn = t;
      // z of this iteration, needed by its w / x update next time; its
      // buffer is free again once that update has run
      double *zold = zp;
      zp = zc;
      zc = zn;
      zn = zold ? zold : z3;
    }
    j += nbat;
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(hs, st, sizeof(MrState), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (hs->err == 1) return abd_fail(ctx, ABD_E_PCG, "MINRES: preconditioner not positive definite");
    if (hs->err == 2) return abd_fail(ctx, ABD_E_PCG, "MINRES breakdown (singular system)");
    if (hs->done) break;
  }
  // the last iteration's w / x update
  if (!first) hipLaunchKernelGGL(k_mr_wx, dim3(gv), dim3(256), 0, s, n12, zp, wp, wc, st, x_out);
  HIP_TRY(ctx, hipGetLastError());
  j = hs->iters;
  *iters = j;
  return abd_hip_check(ctx, hipGetLastError(), "minres");
}

extern "C" int abd_pcg_solve(abd_ctx *ctx, const abd_scene *sc, const double *diag, const double *off,
                             const int32_t *keys, int64_t n_keys, const double *rhs, const double *x0, double *p,
                             double rtol, int32_t max_iter, int32_t *iters, hipStream_t stream) {
  if (!ctx || !sc || !diag || !rhs || !p || !iters || (n_keys && (!off || !keys)))
    return abd_fail(ctx, ABD_E_INVALID, "abd_pcg_solve: null");
  int it = 0;
  ABD_TRY(op_pcg(ctx, sc, diag, off, keys, n_keys, rhs, p, rtol, max_iter, &it, stream, x0));
  *iters = it;
  return ABD_OK;
}
