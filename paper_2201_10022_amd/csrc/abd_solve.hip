// Block-Jacobi preconditioned conjugate gradients on the symmetric
// 12x12-block system H p = rhs (diagonal blocks per body, off-diagonal
// blocks per contacting body pair, fixed bodies removed).  Scalars (alpha,
// beta, r.z) stay on the device; the host reads the residual only every
// CHECK iterations.  All dot products are fixed-order tree reductions.
#include <rocprim/device/device_radix_sort.hpp>

#include "abd_internal.h"

namespace {

constexpr int CHECK = 8;

// inverse of each free body's diagonal block via Cholesky (thread per body)
__global__ void __launch_bounds__(64) k_block_inverse(int nb, const uint8_t *fixed, const double *diag, double *inv,
                                                      int *err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double *Iv = inv + 144 * (int64_t)b;
  if (fixed[b]) {
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

// y = H x (thread per body row component); partial dot x.y per block
constexpr int SB = 192;  // 16 bodies x 12 rows
__global__ void __launch_bounds__(SB) k_spmv(int nb, const uint8_t *fixed, const double *diag, const double *off,
                                            const int32_t *keys, const uint32_t *tperm, const int64_t *lo_beg,
                                            const int64_t *hi_beg, const double *x, double *y, double *part) {
  __shared__ double sh[SB / 64];
  const int t = blockIdx.x * SB + threadIdx.x;
  const int b = t / 12, i = t % 12;
  double v = 0.0, dotv = 0.0;
  if (b < nb && !fixed[b]) {
    const double *D = diag + 144 * (int64_t)b + 12 * i;
    const double *xb = x + 12 * (int64_t)b;
#pragma unroll
    for (int j = 0; j < 12; ++j) v += D[j] * xb[j];
    for (int64_t k = lo_beg[b]; k < lo_beg[b + 1]; ++k) {
      const double *O = off + 144 * k + 12 * i;
      const double *xc = x + 12 * (int64_t)keys[2 * k + 1];
#pragma unroll
      for (int j = 0; j < 12; ++j) v += O[j] * xc[j];
    }
    for (int64_t m = hi_beg[b]; m < hi_beg[b + 1]; ++m) {
      const int64_t k = tperm[m];
      const double *O = off + 144 * k + i;  // column i of block (lo, b)
      const double *xc = x + 12 * (int64_t)keys[2 * k];
#pragma unroll
      for (int j = 0; j < 12; ++j) v += O[12 * j] * xc[j];
    }
    y[12 * (int64_t)b + i] = v;
    dotv = v * x[12 * (int64_t)b + i];
  } else if (b < nb) {
    y[12 * (int64_t)b + i] = 0.0;
  }
  dotv = wave_sum(dotv);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = dotv;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + sh[2];
}

// scalars: [0] rz, [1] pAp, [2] alpha, [3] beta, [4] rr, [5] bb, [6] rz_new, [7] stop flag
__global__ void k_fold_alpha(const double *part, int np, double *sc, int *err) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += 64) v += part[i];
  v = wave_sum(v);
  if (threadIdx.x == 0) {
    sc[1] = v;
    double a = 0.0;
    if (sc[7] == 0.0) {
      if (v > 0.0)
        a = sc[0] / v;
      else {
        sc[7] = 1.0;
        if (!(v == 0.0 && sc[0] == 0.0)) atomicOr(err, 8);
      }
    }
    sc[2] = a;
  }
}

// x += alpha p; r -= alpha Ap; z = P r; partials of r.z and r.r
__global__ void __launch_bounds__(SB) k_update_xr(int nb, const double *inv, const double *p, const double *Ap,
                                                 double *x, double *r, double *z, const double *sc, double *part2) {
  __shared__ double sr[16][12];
  __shared__ double sh[2][SB / 64];
  const int t = blockIdx.x * SB + threadIdx.x;
  const int b = t / 12, i = t % 12, lb = threadIdx.x / 12;
  const double a = sc[2];
  double rv = 0.0;
  if (b < nb) {
    const int64_t o = 12 * (int64_t)b + i;
    x[o] += a * p[o];
    rv = r[o] - a * Ap[o];
    r[o] = rv;
  }
  sr[lb][i] = rv;
  __syncthreads();
  double zv = 0.0;
  if (b < nb) {
    const double *M = inv + 144 * (int64_t)b + 12 * i;
#pragma unroll
    for (int j = 0; j < 12; ++j) zv += M[j] * sr[lb][j];
    z[12 * (int64_t)b + i] = zv;
  }
  double rz = wave_sum(rv * zv), rr = wave_sum(rv * rv);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = rz;
    sh[1][threadIdx.x >> 6] = rr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part2[2 * blockIdx.x] = (sh[0][0] + sh[0][1]) + sh[0][2];
    part2[2 * blockIdx.x + 1] = (sh[1][0] + sh[1][1]) + sh[1][2];
  }
}

__global__ void k_fold_beta(const double *part2, int np, double *sc) {
  double rz = 0.0, rr = 0.0;
  for (int i = threadIdx.x; i < np; i += 64) {
    rz += part2[2 * i];
    rr += part2[2 * i + 1];
  }
  rz = wave_sum(rz);
  rr = wave_sum(rr);
  if (threadIdx.x == 0) {
    double beta = 0.0;
    if (sc[7] == 0.0 && sc[0] != 0.0) beta = rz / sc[0];
    if (sc[7] == 0.0) sc[0] = rz;
    sc[3] = beta;
    sc[4] = rr;
  }
}

__global__ void k_update_p(int n, const double *z, double *p, const double *sc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (sc[7] != 0.0) return;
  p[i] = z[i] + sc[3] * p[i];
}

// initial: r = rhs (x = 0), z = P r, p = z, rz, rr, bb
__global__ void __launch_bounds__(SB) k_pcg_init(int nb, const uint8_t *fixed, const double *inv, const double *rhs,
                                                double *x, double *r, double *z, double *p, double *part2) {
  __shared__ double sr[16][12];
  __shared__ double sh[2][SB / 64];
  const int t = blockIdx.x * SB + threadIdx.x;
  const int b = t / 12, i = t % 12, lb = threadIdx.x / 12;
  double rv = 0.0;
  if (b < nb) {
    const int64_t o = 12 * (int64_t)b + i;
    rv = fixed[b] ? 0.0 : rhs[o];
    x[o] = 0.0;
    r[o] = rv;
  }
  sr[lb][i] = rv;
  __syncthreads();
  double zv = 0.0;
  if (b < nb) {
    const double *M = inv + 144 * (int64_t)b + 12 * i;
#pragma unroll
    for (int j = 0; j < 12; ++j) zv += M[j] * sr[lb][j];
    z[12 * (int64_t)b + i] = zv;
    p[12 * (int64_t)b + i] = zv;
  }
  double rz = wave_sum(rv * zv), rr = wave_sum(rv * rv);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = rz;
    sh[1][threadIdx.x >> 6] = rr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part2[2 * blockIdx.x] = (sh[0][0] + sh[0][1]) + sh[0][2];
    part2[2 * blockIdx.x + 1] = (sh[1][0] + sh[1][1]) + sh[1][2];
  }
}

__global__ void k_fold_init(const double *part2, int np, double *sc) {
  double rz = 0.0, rr = 0.0;
  for (int i = threadIdx.x; i < np; i += 64) {
    rz += part2[2 * i];
    rr += part2[2 * i + 1];
  }
  rz = wave_sum(rz);
  rr = wave_sum(rr);
  if (threadIdx.x == 0) {
    sc[0] = rz;
    sc[4] = rr;
    sc[5] = rr;
    sc[7] = rr == 0.0 ? 1.0 : 0.0;
  }
}

}  // namespace

int op_pcg(abd_ctx *ctx, const abd_scene *sc, const double *diag, const double *off, const int32_t *keys,
           int64_t n_keys, const double *rhs, double *p_out, double rtol, int max_iter, int *iters, hipStream_t s) {
  const int nb = sc->n_bodies;
  *iters = 0;
  if (nb <= 0) return ABD_OK;
  if (n_keys >= (1ll << 31) || nb >= (1 << 24)) return abd_fail(ctx, ABD_E_INVALID, "pcg: too many blocks");
  double *inv, *r, *z, *p, *Ap, *scal, *part, *part2;
  int64_t *lo_beg, *hi_beg;
  uint64_t *tk, *tk2;
  uint32_t *tv, *tv2;
  int *err;
  const int nblk = (int)grid_for((int64_t)nb * 12, SB);
  ABD_TRY(ws(ctx, "pcg_inv", 144 * (size_t)nb, &inv, s));
  ABD_TRY(ws(ctx, "pcg_r", 12 * (size_t)nb, &r, s));
  ABD_TRY(ws(ctx, "pcg_z", 12 * (size_t)nb, &z, s));
  ABD_TRY(ws(ctx, "pcg_p", 12 * (size_t)nb, &p, s));
  ABD_TRY(ws(ctx, "pcg_Ap", 12 * (size_t)nb, &Ap, s));
  ABD_TRY(ws(ctx, "pcg_sc", 8, &scal, s));
  ABD_TRY(ws(ctx, "pcg_part", nblk, &part, s));
  ABD_TRY(ws(ctx, "pcg_part2", 2 * nblk, &part2, s));
  ABD_TRY(ws(ctx, "pcg_lob", nb + 1, &lo_beg, s));
  ABD_TRY(ws(ctx, "pcg_hib", nb + 1, &hi_beg, s));
  ABD_TRY(ws(ctx, "pcg_tk", n_keys + 1, &tk, s));
  ABD_TRY(ws(ctx, "pcg_tk2", n_keys + 1, &tk2, s));
  ABD_TRY(ws(ctx, "pcg_tv", n_keys + 1, &tv, s));
  ABD_TRY(ws(ctx, "pcg_tv2", n_keys + 1, &tv2, s));
  ABD_TRY(ws(ctx, "err_flag", 1, &err, s));
  hipLaunchKernelGGL(k_block_inverse, dim3(grid_for(nb, 64)), dim3(64), 0, s, nb, sc->body_fixed, diag, inv, err);
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
  hipLaunchKernelGGL(k_pcg_init, dim3(nblk), dim3(SB), 0, s, nb, sc->body_fixed, inv, rhs, p_out, r, z, p, part2);
  hipLaunchKernelGGL(k_fold_init, dim3(1), dim3(64), 0, s, part2, nblk, scal);
  HIP_TRY(ctx, hipGetLastError());
  double *h;
  ABD_TRY(pinned_get(ctx, 64, reinterpret_cast<void **>(&h)));
  const double rtol2 = rtol * rtol;
  int it = 0;
  for (; it < max_iter;) {
    for (int k = 0; k < CHECK && it < max_iter; ++k, ++it) {
      hipEvent_t pe = prof_begin(ctx, s);
      hipLaunchKernelGGL(k_spmv, dim3(nblk), dim3(SB), 0, s, nb, sc->body_fixed, diag, off, keys, tv2, lo_beg, hi_beg,
                         p, Ap, part);
      prof_end(ctx, pe, "spmv", nb + 2 * n_keys, s);
      hipLaunchKernelGGL(k_fold_alpha, dim3(1), dim3(64), 0, s, part, nblk, scal, err);
      hipLaunchKernelGGL(k_update_xr, dim3(nblk), dim3(SB), 0, s, nb, inv, p, Ap, p_out, r, z, scal, part2);
      hipLaunchKernelGGL(k_fold_beta, dim3(1), dim3(64), 0, s, part2, nblk, scal);
      hipLaunchKernelGGL(k_update_p, dim3(grid_for(12 * nb, 256)), dim3(256), 0, s, 12 * nb, z, p, scal);
    }
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(h, scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h[7] != 0.0 || h[4] <= rtol2 * h[5]) break;
  }
  *iters = it;
  return ABD_OK;
}

extern "C" int abd_pcg_solve(abd_ctx *ctx, const abd_scene *sc, const double *diag, const double *off,
                             const int32_t *keys, int64_t n_keys, const double *rhs, double *p, double rtol,
                             int32_t max_iter, int32_t *iters, hipStream_t stream) {
  if (!ctx || !sc || !diag || !rhs || !p || !iters || (n_keys && (!off || !keys)))
    return abd_fail(ctx, ABD_E_INVALID, "abd_pcg_solve: null");
  int it = 0;
  ABD_TRY(op_pcg(ctx, sc, diag, off, keys, n_keys, rhs, p, rtol, max_iter, &it, stream));
  *iters = it;
  return ABD_OK;
}
