// Context, workspace, errors and device-wide primitives (scan, sort,
// deterministic reductions) of the gfx950 ABD library.
#include <cstdarg>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "abd_internal.h"
#include "abd_lookback.h"

int abd_fail(abd_ctx *ctx, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return code;
}

int abd_hip_check(abd_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return ABD_OK;
  return abd_fail(ctx, ABD_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int ws_get(abd_ctx *ctx, const char *name, size_t bytes, void **out, hipStream_t stream) {
  DevBuf &b = ctx->bufs[name];
  if (b.bytes < bytes) {
    HostTimer ht(ctx, "ws_grow", (int64_t)bytes);
    // The old buffer may still be read by queued work: it is kept until the
    // next idle point.  Growing to twice the request (at least 256 KiB)
    // keeps the number of growths logarithmic in the final size when
    // counts rise step after step (contacts forming).
    if (b.ptr) {
      ctx->ws_old.push_back(b.ptr);
      ctx->ws_old_bytes += b.bytes;
      b.ptr = nullptr;
      b.bytes = 0;
      if (ctx->ws_old_bytes > ((size_t)1 << 30)) ABD_TRY(ws_collect(ctx));
    }
    size_t nb = bytes < ((size_t)128 << 10) ? ((size_t)256 << 10) : 2 * bytes;
    nb = (nb + 4095) & ~(size_t)4095;
    HIP_TRY(ctx, hipMalloc(&b.ptr, nb));
    HIP_TRY(ctx, hipMemsetAsync(b.ptr, 0, nb, stream));
    b.bytes = nb;
  }
  *out = b.ptr;
  return ABD_OK;
}

int ws_collect(abd_ctx *ctx) {
  if (ctx->ws_old.empty()) return ABD_OK;
  HIP_TRY(ctx, hipDeviceSynchronize());
  for (void *p : ctx->ws_old) HIP_TRY(ctx, hipFree(p));
  ctx->ws_old.clear();
  ctx->ws_old_bytes = 0;
  return ABD_OK;
}

int pinned_get(abd_ctx *ctx, size_t bytes, void **out) {
  if (ctx->pinned_bytes < bytes) {
    // growing waits for any queued copy into the old area
    if (ctx->pinned) {
      HIP_TRY(ctx, hipDeviceSynchronize());
      HIP_TRY(ctx, hipHostFree(ctx->pinned));
    }
    ctx->pinned = nullptr;
    size_t nb = bytes < 4096 ? 4096 : bytes;
    HIP_TRY(ctx, hipHostMalloc(&ctx->pinned, nb, hipHostMallocDefault));
    ctx->pinned_bytes = nb;
  }
  *out = ctx->pinned;
  return ABD_OK;
}

int pinned_get_nt(abd_ctx *ctx, size_t bytes, void **out, void **dev) {
  if (ctx->pinned_nt_bytes < bytes) {
    // growing waits for queued work that may still write the old area
    if (ctx->pinned_nt) {
      HIP_TRY(ctx, hipDeviceSynchronize());
      HIP_TRY(ctx, hipHostFree(ctx->pinned_nt));
    }
    ctx->pinned_nt = ctx->pinned_nt_d = nullptr;
    size_t nb = bytes < 4096 ? 4096 : bytes;
    HIP_TRY(ctx, hipHostMalloc(&ctx->pinned_nt, nb, hipHostMallocMapped | hipHostMallocCoherent));
    HIP_TRY(ctx, hipHostGetDevicePointer(&ctx->pinned_nt_d, ctx->pinned_nt, 0));
    ctx->pinned_nt_bytes = nb;
  }
  *out = ctx->pinned_nt;
  if (dev) *dev = ctx->pinned_nt_d;
  return ABD_OK;
}

int mirror_counts_ok(abd_ctx *ctx, std::initializer_list<int64_t> counts, const char *where) {
  for (int64_t c : counts)
    if (c < 0) return abd_fail(ctx, ABD_E_HIP, "%s: a look-back scan did not complete", where);
  return ABD_OK;
}

int mirror_get(abd_ctx *ctx, int64_t **host, int64_t **dev) {
  if (!ctx->mirror_h) {
    void *h = nullptr, *d = nullptr;
    HIP_TRY(ctx, hipHostMalloc(&h, MIRROR_SLOTS * sizeof(int64_t), hipHostMallocMapped | hipHostMallocCoherent));
    const hipError_t e = hipHostGetDevicePointer(&d, h, 0);
    if (e != hipSuccess) {
      hipHostFree(h);
      return abd_hip_check(ctx, e, "hipHostGetDevicePointer");
    }
    ctx->mirror_h = static_cast<int64_t *>(h);
    ctx->mirror_d = static_cast<int64_t *>(d);
  }
  *host = ctx->mirror_h;
  *dev = ctx->mirror_d;
  return ABD_OK;
}

// total and split value of a scan done by the library (single thread)
__global__ void k_scan_tail(const int64_t *out, const int64_t *last_in, int64_t n, int64_t *total, int64_t *host,
                            int64_t split) {
  const int64_t v = out[n - 1] + *last_in;
  if (total) *total = v;
  if (host) {
    host[0] = v;
    if (split >= 0) host[1] = split < n ? out[split] : v;
  }
}

// Exclusive scan of up to SCAN1_SMALL values by one block (one launch; the
// scans here are mostly per body or per scene): each thread sums a
// contiguous chunk, the chunk sums are scanned across the block, then each
// thread rewrites its chunk.  Works in place; `total` may be out + n.
constexpr int SCAN1_T = 1024;
constexpr int SCAN1_U = 8;  // loads in flight per thread
constexpr int64_t SCAN1_SMALL = 1 << 12;  // larger scans: k_scan_lb
__global__ void __launch_bounds__(SCAN1_T) k_scan1(const int64_t *in, int64_t *out, int64_t n, int64_t *total,
                                                   int64_t *host, int64_t split) {
  __shared__ int64_t sw[SCAN1_T / 64 + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t per = (n + SCAN1_T - 1) / SCAN1_T;
  const int64_t lo = t * per < n ? t * per : n, hi = lo + per < n ? lo + per : n;
  // each thread's range is read in groups of SCAN1_U independent loads
  int64_t own = 0;
  for (int64_t i0 = lo; i0 < hi; i0 += SCAN1_U) {
    int64_t v[SCAN1_U];
#pragma unroll
    for (int k = 0; k < SCAN1_U; ++k) v[k] = i0 + k < hi ? in[i0 + k] : 0;
#pragma unroll
    for (int k = 0; k < SCAN1_U; ++k) own += v[k];
  }
  int64_t x = own;  // inclusive scan over the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sw[w] = x;
  __syncthreads();
  if (t == 0) {
    int64_t acc = 0;
    for (int j = 0; j < SCAN1_T / 64; ++j) {
      const int64_t v = sw[j];
      sw[j] = acc;
      acc += v;
    }
    sw[SCAN1_T / 64] = acc;
  }
  __syncthreads();
  int64_t run = sw[w] + x - own;
  for (int64_t i0 = lo; i0 < hi; i0 += SCAN1_U) {
    int64_t v[SCAN1_U];
#pragma unroll
    for (int k = 0; k < SCAN1_U; ++k) v[k] = i0 + k < hi ? in[i0 + k] : 0;
#pragma unroll
    for (int k = 0; k < SCAN1_U; ++k) {
      if (i0 + k < hi) {
        out[i0 + k] = run;  // (in place: the group's inputs are already read)
        if (host && i0 + k == split) host[1] = run;
      }
      run += v[k];
    }
  }
  if (t == 0) {
    const int64_t tot = sw[SCAN1_T / 64];
    if (total) *total = tot;
    if (host) {
      host[0] = tot;
      if (split == n) host[1] = tot;
    }
  }
}

// Exclusive scan of more values in one pass, by decoupled look-back over
// tiles of LB_TILE values (abd_lookback.h).
constexpr int LB_T = 256, LB_U = 8;
constexpr int64_t LB_TILE = (int64_t)LB_T * LB_U;
__global__ void __launch_bounds__(LB_T) k_scan_lb(const int64_t *in, int64_t *out, int64_t n, int64_t *total,
                                                  int64_t *host, int64_t split, unsigned long long *status,
                                                  unsigned long long *counter, unsigned int tag, int *err) {
  __shared__ int64_t sw[LB_T / 64];
  __shared__ int64_t s_agg, s_prefix;
  __shared__ unsigned int s_tile;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) s_tile = lb_claim(counter, tag, err);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t i0 = tile * LB_TILE + (int64_t)t * LB_U;
  int64_t v[LB_U];
  int64_t own = 0;
#pragma unroll
  for (int k = 0; k < LB_U; ++k) {
    v[k] = i0 + k < n ? in[i0 + k] : 0;
    own += v[k];
  }
  int64_t x = own;  // inclusive scan over the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sw[w] = x;
  __syncthreads();
  if (t == 0) {
    int64_t acc = 0;
    for (int j = 0; j < LB_T / 64; ++j) {
      const int64_t a = sw[j];
      sw[j] = acc;
      acc += a;
    }
    s_agg = acc;
  }
  __syncthreads();
  if (w == 0) {
    const int64_t p = lb_lookback(status, tile, s_agg, tag, err);
    if (lane == 0) s_prefix = p;
  }
  __syncthreads();
  int64_t run = s_prefix + sw[w] + x - own;
#pragma unroll
  for (int k = 0; k < LB_U; ++k) {
    if (i0 + k < n) {
      out[i0 + k] = run;
      if (host && i0 + k == split) host[1] = s_prefix < 0 ? -1 : run;  // (-1: a failed look-back)
    }
    run += v[k];
  }
  if (t == 0 && (tile + 1) * LB_TILE >= n) {  // the last tile
    const int64_t tot = s_prefix < 0 ? -1 : s_prefix + s_agg;
    if (total) *total = tot;
    if (host) {
      host[0] = tot;
      if (split == n) host[1] = tot;
    }
  }
}

int lb_prepare(abd_ctx *ctx, int64_t words, unsigned long long **status, unsigned int *tag, hipStream_t s) {
  abd_ctx::LbState &lb = ctx->lb[s != nullptr && s == ctx->aux_stream ? 1 : 0];
  if (lb.words < words) {
    // status words start untagged (tag 0 is never used)
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (lb.status) HIP_TRY(ctx, hipFree(lb.status));
    lb.status = nullptr;
    const int64_t cap = words + words / 2 + 64;
    HIP_TRY(ctx, hipMalloc(&lb.status, cap * sizeof(unsigned long long)));
    HIP_TRY(ctx, hipMemsetAsync(lb.status, 0, cap * sizeof(unsigned long long), s));
    lb.words = cap;
  }
  if (++lb.tag >= (1u << LB_TAG_BITS)) {
    // tags wrap: clear the words so that none carries a reused tag
    lb.tag = 1;
    HIP_TRY(ctx, hipMemsetAsync(lb.status, 0, lb.words * sizeof(unsigned long long), s));
  }
  *status = lb.status;
  *tag = lb.tag;
  return ABD_OK;
}

int aux_stream_get(abd_ctx *ctx, hipStream_t *aux) {
  if (!ctx->aux_stream) {
    HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->aux_stream, hipStreamNonBlocking));
    HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  }
  *aux = ctx->aux_stream;
  return ABD_OK;
}

int scan_exclusive_i64(abd_ctx *ctx, const int64_t *in, int64_t *out, int64_t n, int64_t *total, hipStream_t s,
                       int64_t *host, int64_t split) {
  if (n < 0) n = 0;
  if (split > n) split = -1;
  if (n <= SCAN1_SMALL) {
    // (n == 0 reads nothing and writes the zero total)
    hipLaunchKernelGGL(k_scan1, dim3(1), dim3(SCAN1_T), 0, s, in, out, n, total, host, split);
    return abd_hip_check(ctx, hipGetLastError(), "k_scan1");
  }
  const int64_t tiles = (n + LB_TILE - 1) / LB_TILE;
  if (tiles < (1ll << 31) && n < (1ll << 42)) {
    unsigned long long *st;
    unsigned int tag;
    ABD_TRY(lb_prepare(ctx, tiles + 1, &st, &tag, s));
    int *err;
    ABD_TRY(ws(ctx, "err_flag", 1, &err, s));
    // the counter is the word after the tiles' status words
    hipLaunchKernelGGL(k_scan_lb, dim3((unsigned)tiles), dim3(LB_T), 0, s, in, out, n, total, host, split, st,
                       st + tiles, tag, err);
    return abd_hip_check(ctx, hipGetLastError(), "k_scan_lb");
  }
  // the last input for the total: a copy only when the scan is in place
  const bool aux = s != nullptr && s == ctx->aux_stream;  // (its own scratch)
  const int64_t *last = in + n - 1;
  if ((total || host) && in == out) {
    int64_t *keep;
    ABD_TRY(ws(ctx, aux ? "scan_last_aux" : "scan_last", 1, &keep, s));
    HIP_TRY(ctx, hipMemcpyAsync(keep, in + n - 1, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    last = keep;
  }
  size_t tmp_bytes = 0;
  HIP_TRY(ctx, rocprim::exclusive_scan(nullptr, tmp_bytes, in, out, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), s));
  void *tmp = nullptr;
  ABD_TRY(ws_get(ctx, "scan_tmp", tmp_bytes + 16, &tmp, s));
  HIP_TRY(ctx, rocprim::exclusive_scan(tmp, tmp_bytes, in, out, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), s));
  if (total || host) {
    // total = out[n-1] + in[n-1]
    hipLaunchKernelGGL(k_scan_tail, dim3(1), dim3(1), 0, s, out, last, n, total, host, split);
  }
  return abd_hip_check(ctx, hipGetLastError(), "scan tail");
}

int sort_pairs_u32(abd_ctx *ctx, uint32_t **keys, uint32_t **vals, int64_t n, int key_bits, hipStream_t s) {
  if (n <= 1) return ABD_OK;
  uint32_t *k2, *v2;
  ABD_TRY(ws(ctx, "sort_k2", n, &k2, s));
  ABD_TRY(ws(ctx, "sort_v2", n, &v2, s));
  size_t tmp_bytes = 0;
  HIP_TRY(ctx, rocprim::radix_sort_pairs(nullptr, tmp_bytes, *keys, k2, *vals, v2, (size_t)n, 0, key_bits, s));
  void *tmp = nullptr;
  ABD_TRY(ws_get(ctx, "sort_tmp", tmp_bytes + 16, &tmp, s));
  HIP_TRY(ctx, rocprim::radix_sort_pairs(tmp, tmp_bytes, *keys, k2, *vals, v2, (size_t)n, 0, key_bits, s));
  *keys = k2;
  *vals = v2;
  return ABD_OK;
}

// ---------------------------------------------------------- reductions ----
namespace {
constexpr int RB = 256;

template <int OP>  // 0 sum, 1 min
__global__ void __launch_bounds__(RB) k_reduce_pass(const double *in, int64_t n, double init, double *out) {
  __shared__ double sh[RB / 64];
  double v = init;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    const double a = in[i];
    v = OP == 0 ? v + a : fmin(v, a);
  }
  v = OP == 0 ? wave_sum(v) : wave_min(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < RB / 64; ++w) r = OP == 0 ? r + sh[w] : fmin(r, sh[w]);
    out[blockIdx.x] = r;
  }
}

template <int OP>
__global__ void __launch_bounds__(RB) k_reduce_final(const double *part, int np, double init, double *out,
                                                     int accumulate) {
  __shared__ double sh[RB / 64];
  double v = init;
  for (int i = threadIdx.x; i < np; i += RB) v = OP == 0 ? v + part[i] : fmin(v, part[i]);
  v = OP == 0 ? wave_sum(v) : wave_min(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < RB / 64; ++w) r = OP == 0 ? r + sh[w] : fmin(r, sh[w]);
    if (OP == 0)
      *out = accumulate ? *out + r : r;
    else
      *out = accumulate ? fmin(*out, r) : r;
  }
}

// one block for small inputs (one launch)
constexpr int R1 = 1024;
template <int OP>
__global__ void __launch_bounds__(R1) k_reduce1(const double *in, int64_t n, double init, double *out,
                                               int accumulate) {
  __shared__ double sh[R1 / 64];
  double v = init;
  for (int64_t i = threadIdx.x; i < n; i += R1) {
    const double a = in[i];
    v = OP == 0 ? v + a : fmin(v, a);
  }
  v = OP == 0 ? wave_sum(v) : wave_min(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < R1 / 64; ++w) r = OP == 0 ? r + sh[w] : fmin(r, sh[w]);
    if (OP == 0)
      *out = accumulate ? *out + r : r;
    else
      *out = accumulate ? fmin(*out, r) : r;
  }
}

// partial blocks of the two-pass form (n > 16 R1)
int reduce_blocks(int64_t n) {
  int nblk = (int)((n + RB * 4 - 1) / (RB * 4));
  if (nblk < 1) nblk = 1;
  if (nblk > REDUCE_MAX_PARTS) nblk = REDUCE_MAX_PARTS;
  return nblk;
}

// the launches of a reduction; part holds reduce_blocks(n) doubles (unused
// for n <= 16 R1)
template <int OP>
void reduce_launch(const double *in, int64_t n, double init, double *part, double *out, int accumulate,
                   hipStream_t s) {
  if (n <= 16 * R1) {
    hipLaunchKernelGGL(k_reduce1<OP>, dim3(1), dim3(R1), 0, s, in, n, init, out, accumulate);
    return;
  }
  const int nblk = reduce_blocks(n);
  hipLaunchKernelGGL(k_reduce_pass<OP>, dim3(nblk), dim3(RB), 0, s, in, n, init, part);
  hipLaunchKernelGGL(k_reduce_final<OP>, dim3(1), dim3(RB), 0, s, part, nblk, init, out, accumulate);
}

template <int OP>
int reduce_f64(abd_ctx *ctx, const double *in, int64_t n, double init, double *out, int accumulate, hipStream_t s) {
  double *part = nullptr;
  if (n > 16 * R1) ABD_TRY(ws(ctx, OP == 0 ? "red_sum" : "red_min", reduce_blocks(n), &part, s));
  reduce_launch<OP>(in, n, init, part, out, accumulate, s);
  return ABD_OK;
}
}  // namespace

void reduce_sum_f64_into(const double *in, int64_t n, double *part, double *out_accum, hipStream_t s) {
  reduce_launch<0>(in, n, 0.0, part, out_accum, 1, s);
}

int reduce_sum_f64(abd_ctx *ctx, const double *in, int64_t n, double *out_accum, hipStream_t s) {
  return reduce_f64<0>(ctx, in, n, 0.0, out_accum, 1, s);
}
int reduce_min_f64(abd_ctx *ctx, const double *in, int64_t n, double init, double *out, hipStream_t s) {
  return reduce_f64<1>(ctx, in, n, init, out, 0, s);
}

// ------------------------------------------------- per-scene reductions ----
namespace {
constexpr int SB = 512;

__device__ __forceinline__ int64_t lower_bound_i32(const int32_t *a, int64_t n, int v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// scene s's body range starts at the first body with body_scene >= s
__global__ void k_scene_offsets(int nb, const int32_t *body_scene, int n_scenes, int32_t *off) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > n_scenes) return;
  off[s] = (int32_t)lower_bound_i32(body_scene, nb, s);
}

// Trial-major values (trial t's items at vals + t * stride): one block per
// (trial, scene) sums the scene's items in fixed order into out[t S + s].
__global__ void __launch_bounds__(SB) k_seg_reduce_trials(const double *vals, int64_t stride, int64_t n,
                                                          const int32_t *keys, int S, double *out) {
  __shared__ double sh[SB / 64];
  const int t = blockIdx.x / S, s = blockIdx.x % S;
  const int64_t lo = lower_bound_i32(keys, n, s), hi = lower_bound_i32(keys, n, s + 1);
  const double *v = vals + (int64_t)t * stride;
  double a = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += SB) a += v[i];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < SB / 64; ++w) r += sh[w];
    out[blockIdx.x] += r;
  }
}

// Several segments per (trial, scene) block, each reduced exactly as
// k_seg_reduce_trials reduces it, accumulated in segment order.
__global__ void __launch_bounds__(SB) k_seg_reduce_trials_multi(TrialSums ts, int S, double *out) {
  __shared__ double sh[SB / 64];
  __shared__ int64_t bound[10];
  const int t = blockIdx.x / S, s = blockIdx.x % S;
  if (ts.skip && ts.skip[s]) {  // (uniform over the block)
    if (threadIdx.x == 0) out[blockIdx.x] = 0.0;
    return;
  }
  // every segment's range of the scene, one binary search per thread
  if ((int)threadIdx.x < 2 * ts.k) {
    const TrialSeg g = ts.seg[threadIdx.x >> 1];
    bound[threadIdx.x] = lower_bound_i32(g.keys, g.n, s + (int)(threadIdx.x & 1));
  }
  __syncthreads();
  double acc = 0.0;
  for (int j = 0; j < ts.k; ++j) {
    const TrialSeg g = ts.seg[j];
    const int64_t lo = bound[2 * j], hi = bound[2 * j + 1];
    const double *v = g.vals + (int64_t)t * g.stride;
    double a = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += SB) a += v[i];
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = sh[0];
      for (int w = 1; w < SB / 64; ++w) r += sh[w];
      acc += r;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// One scene: per trial, blocks of TRB*4 items into partials, then one
// block per trial folds them (both in fixed order).
constexpr int TRB = 256;
__global__ void __launch_bounds__(TRB) k_trial_pass(const double *vals, int64_t stride, int64_t n, double *part) {
  __shared__ double sh[TRB / 64];
  const double *v = vals + (int64_t)blockIdx.y * stride;
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TRB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TRB) a += v[i];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < TRB / 64; ++w) r += sh[w];
    part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = r;
  }
}
__global__ void __launch_bounds__(TRB) k_trial_final(const double *part, int np, double *out, int assign) {
  __shared__ double sh[TRB / 64];
  const double *pp = part + (int64_t)blockIdx.x * np;
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += TRB) a += pp[i];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < TRB / 64; ++w) r += sh[w];
    if (assign)
      out[blockIdx.x] = r;
    else
      out[blockIdx.x] += r;
  }
}
}  // namespace

int seg_sum_trials(abd_ctx *ctx, const double *vals, int64_t stride, int64_t n, const int32_t *keys, int n_trials,
                   int n_scenes, double *out_accum, hipStream_t s, bool assign) {
  if (n <= 0 || n_trials <= 0) return ABD_OK;
  if (assign && n_scenes > 1) return abd_fail(ctx, ABD_E_INVALID, "seg_sum_trials: assign needs one scene");
  if (n_scenes > 1) {
    hipLaunchKernelGGL(k_seg_reduce_trials, dim3(n_trials * n_scenes), dim3(SB), 0, s, vals, stride, n, keys, n_scenes,
                       out_accum);
    return abd_hip_check(ctx, hipGetLastError(), "k_seg_reduce_trials");
  }
  int nblk = (int)((n + TRB * 4 - 1) / (TRB * 4));
  nblk = nblk < 1 ? 1 : (nblk > 256 ? 256 : nblk);
  double *part;
  ABD_TRY(ws(ctx, "trial_part", (size_t)nblk * n_trials, &part, s));
  hipLaunchKernelGGL(k_trial_pass, dim3(nblk, n_trials), dim3(TRB), 0, s, vals, stride, n, part);
  hipLaunchKernelGGL(k_trial_final, dim3(n_trials), dim3(TRB), 0, s, part, nblk, out_accum, assign ? 1 : 0);
  return abd_hip_check(ctx, hipGetLastError(), "k_trial_pass");
}

int seg_sum_trials_multi(abd_ctx *ctx, const TrialSums &ts, int n_trials, int n_scenes, double *out,
                         hipStream_t s) {
  if (n_trials <= 0) return ABD_OK;
  if (n_scenes <= 1) return abd_fail(ctx, ABD_E_INVALID, "seg_sum_trials_multi: needs several scenes");
  hipLaunchKernelGGL(k_seg_reduce_trials_multi, dim3(n_trials * n_scenes), dim3(SB), 0, s, ts, n_scenes, out);
  return abd_hip_check(ctx, hipGetLastError(), "k_seg_reduce_trials_multi");
}

bool scene_table_cached(abd_ctx *ctx, const abd_scene *sc, const char *name, const void *buf) {
  const std::vector<uintptr_t> key = {(uintptr_t)sc->body_scene, (uintptr_t)sc->n_bodies, (uintptr_t)sc->n_scenes,
                                      (uintptr_t)buf};
  std::vector<uintptr_t> &k = ctx->scene_tables[name];
  if (k == key) return true;
  k = key;
  return false;
}

int op_scene_offsets(abd_ctx *ctx, const abd_scene *sc, const int32_t **off, hipStream_t s) {
  int32_t *o;
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  ABD_TRY(ws(ctx, "scene_body_off", S + 1, &o, s));
  *off = o;
  if (scene_table_cached(ctx, sc, "scene_body_off", o)) return ABD_OK;
  hipLaunchKernelGGL(k_scene_offsets, dim3(grid_for(S + 1, 256)), dim3(256), 0, s, sc->n_bodies, sc->body_scene, S,
                     o);
  return abd_hip_check(ctx, hipGetLastError(), "k_scene_offsets");
}

// ----------------------------------------------------------- profiling ----
static hipEvent_t pool_get(abd_ctx *ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipEvent_t prof_begin(abd_ctx *ctx, hipStream_t s) {
  if (!ctx->profiling) return nullptr;
  hipEvent_t a = pool_get(ctx);
  if (a) hipEventRecord(a, s);
  return a;
}

void prof_end(abd_ctx *ctx, hipEvent_t a, const char *name, int64_t units, hipStream_t s) {
  if (!a) return;
  hipEvent_t b = pool_get(ctx);
  if (!b) return;
  hipEventRecord(b, s);
  ctx->pending.push_back({a, b, name, units});
}

HostTimer::~HostTimer() {
  if (!ctx->profiling) return;
  KStat &k = ctx->kstats[name];
  k.ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  k.launches += 1;
  k.units += units;
}

namespace {
__global__ void k_clear_u64(unsigned long long *a) { *a = 0ull; }
}  // namespace

int prof_pcg_bytes(abd_ctx *ctx, unsigned long long **acc, hipStream_t s) {
  ABD_TRY(ws(ctx, "prof_pcg_bytes", 1, acc, s));
  if (ctx->prof_pcg_clear) hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(1), 0, s, *acc);
  ctx->prof_pcg_clear = false;
  return abd_hip_check(ctx, hipGetLastError(), "k_clear_u64");
}

void prof_flush(abd_ctx *ctx) {
  for (auto &p : ctx->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      KStat &k = ctx->kstats[p.name];
      k.ms += ms;
      k.launches += 1;
      k.units += p.units;
    }
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
}

extern "C" int abd_profile(abd_ctx *ctx, int enable, int reset) {
  if (!ctx) return ABD_E_INVALID;
  prof_flush(ctx);
  if (reset) {
    ctx->kstats.clear();
    ctx->prof_box_tests_clear = true;
    ctx->prof_pcg_clear = true;
  }
  ctx->profiling = enable != 0;
  ctx->count_box_tests = enable == 2;
  return ABD_OK;
}

extern "C" int abd_profile_query(abd_ctx *ctx, const char *kernel, double *ms, int64_t *launches, int64_t *units) {
  if (!ctx || !kernel || !ms || !launches || !units) return abd_fail(ctx, ABD_E_INVALID, "abd_profile_query: null");
  hipDeviceSynchronize();
  prof_flush(ctx);
  auto it = ctx->kstats.find(kernel);
  const std::string kn(kernel);
  if (it != ctx->kstats.end() && (kn == "box_tests" || kn == "box_tests_single_level")) {
    // (device sums: the units of the two entries)
    auto b = ctx->bufs.find("prof_box_tests");
    double h[2] = {0.0, 0.0};
    if (b != ctx->bufs.end() && b->second.ptr)
      HIP_TRY(ctx, hipMemcpy(h, b->second.ptr, sizeof h, hipMemcpyDeviceToHost));
    it->second.units = (int64_t)h[kn == "box_tests" ? 0 : 1];
  }
  if (it != ctx->kstats.end() && kn == "pcg_round") {
    auto b = ctx->bufs.find("prof_pcg_bytes");
    unsigned long long h = 0;
    if (b != ctx->bufs.end() && b->second.ptr) HIP_TRY(ctx, hipMemcpy(&h, b->second.ptr, sizeof h, hipMemcpyDeviceToHost));
    it->second.units = (int64_t)h;
  }
  *ms = it == ctx->kstats.end() ? 0.0 : it->second.ms;
  *launches = it == ctx->kstats.end() ? 0 : it->second.launches;
  *units = it == ctx->kstats.end() ? 0 : it->second.units;
  return ABD_OK;
}

// ------------------------------------------------------------ ABI: ctx ----
extern "C" int abd_create(abd_ctx **out, int device) {
  if (!out) return ABD_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return ABD_E_HIP;
  if (device < 0 || device >= n) return ABD_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return ABD_E_HIP;
  if (noalloc_scratch_init(device) != ABD_OK) return ABD_E_HIP;
  abd_ctx *c = new abd_ctx();
  c->device = device;
  for (auto &e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      for (auto &d : c->ev)
        if (d) hipEventDestroy(d);
      delete c;
      return ABD_E_HIP;
    }
  *out = c;
  return ABD_OK;
}

extern "C" int abd_destroy(abd_ctx *ctx) {
  if (!ctx) return ABD_OK;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto &kv : ctx->bufs)
    if (kv.second.ptr) hipFree(kv.second.ptr);
  for (void *p : ctx->ws_old) hipFree(p);
  if (ctx->pinned) hipHostFree(ctx->pinned);
  if (ctx->pinned_nt) hipHostFree(ctx->pinned_nt);
  if (ctx->mirror_h) hipHostFree(ctx->mirror_h);
  for (auto &lb : ctx->lb)
    if (lb.status) hipFree(lb.status);
  if (ctx->aux_stream) hipStreamDestroy(ctx->aux_stream);
  if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
  for (auto &e : ctx->ev)
    if (e) hipEventDestroy(e);
  prof_flush(ctx);
  for (auto &e : ctx->ev_pool) hipEventDestroy(e);
  for (int g = 0; g < 2; ++g)
    if (ctx->pcg_exec[g]) hipGraphExecDestroy(ctx->pcg_exec[g]);
  for (auto &e : ctx->cg_exec)
    if (e) hipGraphExecDestroy(e);
  if (ctx->capture_stream) hipStreamDestroy(ctx->capture_stream);
  delete ctx;
  return ABD_OK;
}

extern "C" const char *abd_last_error(const abd_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }
