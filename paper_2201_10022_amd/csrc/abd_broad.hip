// Broad phase (ABD sec. 4.2): swept, inflated primitive boxes -> body boxes
// -> overlapping body pairs -> per body pair the primitives inside the
// other body's box (the i-AABB cull) -> tiled primitive-pair box tests with
// wave ballot compaction.  Count and write passes run the same tests, so
// the output order is a pure function of the candidate set.
#include <rocprim/device/device_radix_sort.hpp>

#include "abd_internal.h"

namespace {

// Box of a primitive: lo = min over its vertices at x0 and x1, hi' =
// max(...) + inflate (rounded once; max commutes with the monotone rounding
// so body boxes built from hi' equal body max + inflate).
struct Box {
  double lo[3], hi[3];
};

__device__ __forceinline__ bool box_overlap(const double *a, const double *b) {
  // a, b: [lo0 lo1 lo2 hi'0 hi'1 hi'2]
  return a[0] <= b[3] && b[0] <= a[3] && a[1] <= b[4] && b[1] <= a[4] && a[2] <= b[5] && b[2] <= a[5];
}

// The culling step (primitives inside the other body's box) only narrows
// the rows and columns of the exact primitive-pair test, which implies it
// (a primitive box overlapping one inside the other body's box overlaps
// that box), so it may keep extra primitives: it reads single-precision
// copies of the boxes rounded outwards, half the bytes of the exact ones.
__device__ __forceinline__ void store_box32(float *o, const double *b) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o[i] = __double2float_rd(b[i]);
    o[3 + i] = __double2float_ru(b[3 + i]);
  }
}
__device__ __forceinline__ bool box_overlap32(const float *a, const double *b) {
  return (double)a[0] <= b[3] && b[0] <= (double)a[3] && (double)a[1] <= b[4] && b[1] <= (double)a[4] &&
         (double)a[2] <= b[5] && b[2] <= (double)a[5];
}

// list capacities are rounded up to multiples of 64 (chunk alignment)
__device__ __forceinline__ int64_t round64(int64_t n) { return (n + 63) & ~(int64_t)63; }

// swept box of vertex v over x0 -> x1, inflated upwards
__device__ __forceinline__ void vert_box(int64_t v, const double *x0, const double *x1, double inflate, double b[6]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double a = x0[3 * v + i], c = x1[3 * v + i];
    b[i] = fmin(a, c);
    b[3 + i] = fmax(a, c) + inflate;
  }
}

// exact swept box of a primitive (kind 0 vertex, 1 triangle, 2 edge):
// min / max of its vertices' boxes, the same arithmetic as a vertex's
__device__ __forceinline__ void prim_box(int kind, int64_t i, const int32_t *tris, const int32_t *edges,
                                         const double *x0, const double *x1, double inflate, double b[6]) {
  if (kind == 0) {
    vert_box(i, x0, x1, inflate, b);
    return;
  }
  const int K = kind == 1 ? 3 : 2;
  const int32_t *prim = kind == 1 ? tris + 3 * i : edges + 2 * i;
  vert_box(prim[0], x0, x1, inflate, b);
  for (int q = 1; q < K; ++q) {
    double o[6];
    vert_box(prim[q], x0, x1, inflate, o);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      b[c] = fmin(b[c], o[c]);
      b[3 + c] = fmax(b[3 + c], o[3 + c]);
    }
  }
}

// single-precision culling box of a primitive from its vertices' culling
// boxes (rounding outwards is monotone, so this equals the primitive's exact
// box rounded outwards)
__device__ __forceinline__ void prim_box32(int kind, int64_t i, const int32_t *tris, const int32_t *edges,
                                           const float *vb32, float b[6]) {
  const int K = kind == 0 ? 1 : (kind == 1 ? 3 : 2);
  const int32_t v0 = kind == 0 ? (int32_t)i : (kind == 1 ? tris[3 * i] : edges[2 * i]);
#pragma unroll
  for (int c = 0; c < 6; ++c) b[c] = vb32[6 * (int64_t)v0 + c];
  for (int q = 1; q < K; ++q) {
    const int32_t v = kind == 1 ? tris[3 * i + q] : edges[2 * i + q];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      b[c] = fminf(b[c], vb32[6 * (int64_t)v + c]);
      b[3 + c] = fmaxf(b[3 + c], vb32[6 * (int64_t)v + 3 + c]);
    }
  }
}

// Body boxes (min / max over the body's vertex boxes), one wave per body;
// clears the body's mark of being in an overlapping body pair.
// (bodies of the scenes skip_scene marks, which take part in no pair, get
// no box)
__global__ void __launch_bounds__(256) k_body_boxes(int nb, const int32_t *voff, const double *x0,
                                                    const double *x1, double inflate, double *bb,
                                                    uint8_t *involved, const uint8_t *skip_scene,
                                                    const int32_t *body_scene) {
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b >= nb) return;  // (uniform over the wave)
  if (skip_scene && skip_scene[body_scene[b]]) {
    if (lane == 0) involved[b] = 0;
    return;
  }
  double m[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int v = voff[b] + lane; v < voff[b + 1]; v += 64) {
    double vbx[6];
    vert_box(v, x0, x1, inflate, vbx);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      m[i] = fmin(m[i], vbx[i]);
      m[3 + i] = fmax(m[3 + i], vbx[3 + i]);
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    m[i] = wave_min(m[i]);
    m[3 + i] = wave_max(m[3 + i]);
  }
  if (lane < 6) {
    double r = m[0];
#pragma unroll
    for (int i = 1; i < 6; ++i) r = lane == i ? m[i] : r;
    bb[6 * (int64_t)b + lane] = r;
  }
  if (lane == 0) involved[b] = 0;
}

// Single-precision culling boxes of the vertices of the bodies that are in
// at least one overlapping body pair (triangle and edge boxes are formed
// from them where the culling reads them; the exact pair test forms its
// boxes from the positions).
__global__ void __launch_bounds__(256) k_vert_boxes(int nv, const int32_t *vert_body, const uint8_t *involved,
                                                    const double *x0, const double *x1, double inflate,
                                                    float *vb32) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= nv || !involved[vert_body[k]]) return;
  double box[6];
  vert_box(k, x0, x1, inflate, box);
  store_box32(vb32 + 6 * k, box);
}

// body pairs (a < b) in one sub-scene, not both fixed, boxes overlapping.
// Pass 0 counts per a, pass 1 writes in (a, b) order.
template <int WRITE>
__global__ void __launch_bounds__(64) k_body_pairs(int nb, const int32_t *body_scene, const uint8_t *fixed,
                                                   const double *bb, const int32_t *scene_end_of_body,
                                                   const uint8_t *skip_scene, int64_t *cnt, const int64_t *off,
                                                   int32_t *pairs, int64_t cap = 0) {
  const int a = blockIdx.x;
  if (a >= nb) return;
  if (skip_scene && skip_scene[body_scene[a]]) {
    if (!WRITE && threadIdx.x == 0) cnt[a] = 0;
    return;
  }
  const int end = scene_end_of_body[a];
  double ba[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) ba[i] = bb[6 * (int64_t)a + i];
  const bool fa = fixed[a] != 0;
  int64_t base = WRITE ? off[a] : 0;
  int64_t c = 0;
  // BPU chunks of 64 candidates per trip: their box loads are issued
  // together, so the wave of body 0 (the longest scan) waits on one load
  // latency per BPU chunks rather than per chunk
  constexpr int BPU = 4;
  for (int b0 = a + 1; b0 < end; b0 += 64 * BPU) {
    bool ok[BPU];
#pragma unroll
    for (int u = 0; u < BPU; ++u) {
      // (loads from a clamped index, so none waits on a test)
      const int b = b0 + 64 * u + (int)threadIdx.x;
      const int bl = b < end ? b : a;
      double o[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) o[i] = bb[6 * (int64_t)bl + i];
      const bool fb = fixed[bl] != 0;
      const bool ov = (ba[0] <= o[3]) & (o[0] <= ba[3]) & (ba[1] <= o[4]) & (o[1] <= ba[4]) & (ba[2] <= o[5]) &
                      (o[2] <= ba[5]);
      ok[u] = (b < end) & !(fa & fb) & ov;
    }
#pragma unroll
    for (int u = 0; u < BPU; ++u) {
      const int b = b0 + 64 * u + (int)threadIdx.x;
      const unsigned long long m = __ballot(ok[u]);
      if (WRITE && ok[u]) {
        const int64_t pos = base + c + __popcll(m & ((1ull << threadIdx.x) - 1ull));
        if (pos < cap) {  // (beyond the capacity the caller sizes again and repeats)
          pairs[2 * pos] = a;
          pairs[2 * pos + 1] = b;
        }
      }
      c += __popcll(m);
    }
  }
  if (!WRITE && threadIdx.x == 0) cnt[a] = c;
}

__global__ void k_scene_end(int nb, const int32_t *body_scene, int32_t *end) {
  // end of the sub-scene containing body b (body_scene is non-decreasing)
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int s = body_scene[b];
  int lo = b, hi = nb;  // first index with scene > s
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (body_scene[mid] > s)
      hi = mid;
    else
      lo = mid + 1;
  }
  end[b] = lo;
}

// List kinds per body pair (a,b):
//   0: vertices of a in box(b)   1: triangles of b in box(a)
//   2: vertices of b in box(a)   3: triangles of a in box(b)
//   4: edges of a in box(b)      5: edges of b in box(a)
// Capacity of each list = primitive count of its body rounded up to 64;
// region offsets per body pair from a scan of the summed capacities.  Runs over a buffer of
// n_cap slots; slots at or beyond the body-pair count (device) get 0.  Also
// marks both bodies of every pair as involved (their primitive boxes are
// then computed).
__global__ void k_list_caps(int64_t n_cap, const int64_t *nbp_dev, const int32_t *bpairs, const int32_t *voff,
                            const int32_t *toff, const int32_t *eoff, int64_t *cap, uint8_t *involved) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_cap) return;
  if (p >= *nbp_dev) {
    cap[p] = 0;
    return;
  }
  const int a = bpairs[2 * p], b = bpairs[2 * p + 1];
  involved[a] = 1;  // (every writer stores the same value)
  involved[b] = 1;
  // (each list's capacity rounded up to 64, so lists start at multiples of 64)
  cap[p] = round64(voff[a + 1] - voff[a]) + round64(toff[b + 1] - toff[b]) + round64(voff[b + 1] - voff[b]) +
           round64(toff[a + 1] - toff[a]) + round64(eoff[a + 1] - eoff[a]) + round64(eoff[b + 1] - eoff[b]);
}


__global__ void k_clear_f64(int n, double *a) {
  if ((int)threadIdx.x < n) a[threadIdx.x] = 0.0;
}

// Three-level i-AABB tree (sec. 4.2, Fig. iBVH).  Every culled column
// list is cut, in its index order, into blocks of 256 positions, and each
// block is the root of a binary AABB tree of three levels: the block, its
// two 128-position halves and their four 64-position chunks (the leaves).
// A node's box is the union of its primitives' culling boxes.  A tile of
// rows tests the box of its rows against each block's tree top-down and
// runs the primitive-pair tests only in the chunks it reaches; a column
// whose exact box overlaps a row's lies in such a chunk (every node box
// contains its primitives' boxes), and skipping a chunk drops only columns
// that no row of the tile meets, so the output is the single-level one,
// pair for pair.  Lists start at multiples of 64 in the list buffer, so
// chunk k of a list starting at s is record (s >> 6) + k of the chunk
// records: its leaf box, the box of the 128-node that starts at it (even k)
// and of the 256-node that starts at it (k % 4 == 0).
constexpr int CREC = 18;  // floats per chunk record
__device__ __forceinline__ void box32_union(float *o, const float *a, const float *b) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o[c] = fminf(a[c], b[c]);
    o[3 + c] = fmaxf(a[3 + c], b[3 + c]);
  }
}
// lane 0 stores the wave-uniform box b
__device__ __forceinline__ void store_box_lanes(float *dst, const float *b, int lane) {
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) dst[c] = b[c];
  }
}
// a node's single-precision box against a tile's double-precision box
__device__ __forceinline__ bool node_meets(const float *n, const double *t) {
  return (double)n[0] <= t[3] && t[0] <= (double)n[3] && (double)n[1] <= t[4] && t[1] <= (double)n[4] &&
         (double)n[2] <= t[5] && t[2] <= (double)n[5];
}
// is chunk k of a column list (first record g0) reached from the tile box
__device__ __forceinline__ bool chunk_reached(const float *crec, int64_t g0, int k, const double *tb) {
  return node_meets(crec + CREC * (g0 + (k & ~3)) + 12, tb) && node_meets(crec + CREC * (g0 + (k & ~1)) + 6, tb) &&
         node_meets(crec + CREC * (g0 + k), tb);
}

// One wave per body pair p and sub-problem sub (0: a's vertices x b's
// triangles, 1: b's vertices x a's triangles, 2: a's edges x b's edges):
// the two lists of primitives inside the other body's box (kinds 2 sub and
// 2 sub + 1), each in index order by ballot compaction in chunks of 64,
// then the sub-problem's tile count (trows rows x all columns per tile).
// With crec (three-level tree): the column list's chunk records.  tests
// (optional, profiling) gets the sub-problem's primitive-pair box tests of
// a single-level cull.
__global__ void __launch_bounds__(64) k_cull_lists(const int32_t *bpairs, const int64_t *region,
                                                    const int32_t *voff, const int32_t *toff, const int32_t *eoff,
                                                    const double *bb, const float *vb32, const int32_t *tris,
                                                    const int32_t *edges, int32_t *lists, int64_t *list_start,
                                                    int32_t *list_len, int64_t *tiles_pt, int64_t *tiles_ee,
                                                    int trows, float *crec, double *tests, const int64_t *nbp_dev,
                                                    int64_t cap_lists, int64_t *masks_pt, int64_t *masks_ee) {
  const int64_t p = blockIdx.x;
  const int sub = blockIdx.y;
  const int lane = threadIdx.x;
  // (the grid covers a capacity: slots past the device count, and body
  // pairs whose lists would end past the list capacity, which the caller
  // detects from the total and repeats at the exact size, record no tiles)
  bool skip = p >= *nbp_dev;
  int a = 0, b = 0;
  if (!skip) {
    a = bpairs[2 * p];
    b = bpairs[2 * p + 1];
  }
  const int la = voff[a + 1] - voff[a], lb = voff[b + 1] - voff[b];
  const int ta = toff[a + 1] - toff[a], tb = toff[b + 1] - toff[b];
  const int ea = eoff[a + 1] - eoff[a], eb = eoff[b + 1] - eoff[b];
  // list starts inside the body pair's region (capacities rounded to 64)
  const int64_t s1 = round64(la), s2 = s1 + round64(tb), s3 = s2 + round64(lb), s4 = s3 + round64(ta),
                s5 = s4 + round64(ea);
  // (a failed look-back scan leaves negative offsets: nothing is written
  // and the host rejects the poisoned total)
  skip = skip || region[p] < 0 || region[p] + s5 + round64(eb) > cap_lists;
  if (skip) {
    if (lane == 0) {
      list_len[6 * p + 2 * sub] = 0;
      list_len[6 * p + 2 * sub + 1] = 0;
      if (sub < 2) {
        tiles_pt[2 * p + sub] = 0;
        masks_pt[2 * p + sub] = 0;
      } else {
        tiles_ee[p] = 0;
        masks_ee[p] = 0;
      }
      if (tests) tests[3 * p + sub] = 0.0;
    }
    return;
  }
  int len[2], pkh[2];
  int64_t sth[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int kind = 2 * sub + h;
    // (body owning the primitives, body whose box culls them)
    const int own = (kind == 0 || kind == 3 || kind == 4) ? a : b;
    const int oth = own == a ? b : a;
    const int32_t *offs = (kind == 0 || kind == 2) ? voff : (kind == 1 || kind == 3) ? toff : eoff;
    const int pk = (kind == 0 || kind == 2) ? 0 : (kind == 1 || kind == 3) ? 1 : 2;  // vertex, triangle, edge
    // start of this list inside the body pair's region
    const int64_t start =
        region[p] + (kind == 0 ? 0 : kind == 1 ? s1 : kind == 2 ? s2 : kind == 3 ? s3 : kind == 4 ? s4 : s5);
    double ob[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ob[i] = bb[6 * (int64_t)oth + i];
    int total = 0;
    // four chunks of 64 per trip (their loads in flight together), then
    // compacted in order
    constexpr int CU = 4;
    const int hi = offs[own + 1];
    for (int c0 = offs[own]; c0 < hi; c0 += 64 * CU) {
      bool ok[CU];
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const int i = c0 + 64 * u + lane;
        ok[u] = false;
        if (i < hi) {
          float fb[6];
          prim_box32(pk, i, tris, edges, vb32, fb);
          ok[u] = box_overlap32(fb, ob);
        }
      }
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const unsigned long long m = __ballot(ok[u]);
        if (ok[u]) lists[start + total + __popcll(m & ((1ull << lane) - 1ull))] = c0 + 64 * u + lane;
        total += __popcll(m);
      }
    }
    if (lane == 0) {
      list_start[6 * p + kind] = start;
      list_len[6 * p + kind] = total;
    }
    len[h] = total;
    pkh[h] = pk;
    sth[h] = start;
  }
  if (crec) {
    // chunk records of the column list (kind 2 sub + 1)
    const int n = len[1];
    const int64_t g0 = sth[1] >> 6;
    float n128[6], n256[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      n128[c] = n256[c] = INFINITY;
      n128[3 + c] = n256[3 + c] = -INFINITY;
    }
    for (int k = 0; 64 * k < n; ++k) {
      float fb[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
      if (64 * k + lane < n) prim_box32(pkh[1], lists[sth[1] + 64 * k + lane], tris, edges, vb32, fb);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          fb[c] = fminf(fb[c], __shfl_xor(fb[c], o, 64));
          fb[3 + c] = fmaxf(fb[3 + c], __shfl_xor(fb[3 + c], o, 64));
        }
      store_box_lanes(crec + CREC * (g0 + k), fb, lane);
      box32_union(n128, n128, fb);
      box32_union(n256, n256, fb);
      const bool last = 64 * (k + 1) >= n;
      if ((k & 1) || last) {
        store_box_lanes(crec + CREC * (g0 + (k & ~1)) + 6, n128, lane);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          n128[c] = INFINITY;
          n128[3 + c] = -INFINITY;
        }
      }
      if ((k & 3) == 3 || last) {
        store_box_lanes(crec + CREC * (g0 + (k & ~3)) + 12, n256, lane);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          n256[c] = INFINITY;
          n256[3 + c] = -INFINITY;
        }
      }
    }
  }
  if (lane == 0) {
    const int64_t t = len[1] > 0 ? (len[0] + trows - 1) / trows : 0;
    // (masks of the sub-problem's tiles: its rows x its column chunks)
    const int64_t mk = t > 0 ? (int64_t)len[0] * ((len[1] + 63) / 64) : 0;
    if (sub < 2) {
      tiles_pt[2 * p + sub] = t;
      masks_pt[2 * p + sub] = mk;
    } else {
      tiles_ee[p] = t;
      masks_ee[p] = mk;
    }
    if (tests) tests[3 * p + sub] = (double)len[0] * len[1];
  }
}


// (sub-problem, tile index within it) of every tile.  The 3 nbp
// sub-problems' tile counts are scanned as one array: PT sub-problems
// [0, 2 nbp) first, then EE; an EE tile's index is counted from the first
// EE tile (off[2 nbp]).
__global__ void k_tile_sub(int64_t nbp, const int64_t *cnt, const int64_t *off, int2 *tsub_pt, int64_t cap_pt,
                           int2 *tsub_ee, int64_t cap_ee) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 3 * nbp) return;
  const bool ee = j >= 2 * nbp;
  const int64_t o = ee ? off[j] - off[2 * nbp] : off[j], cap = ee ? cap_ee : cap_pt;
  if (off[j] < 0 || (ee && off[2 * nbp] < 0)) return;  // (a failed scan: the host rejects its total)
  int2 *ts = ee ? tsub_ee : tsub_pt;
  const int sub = (int)(ee ? j - 2 * nbp : j);
  for (int64_t t = 0; t < cnt[j] && o + t < cap; ++t) ts[o + t] = make_int2(sub, (int)t);
}

// One wave per tile of trows (<= 64) rows x all columns.  WRITE=0 counts the
// passing tests of the tile, WRITE=1 writes them row-major at the tile's
// offset.  is_ee selects the sub-problem family.  The tile's row boxes
// (one per lane) and the lane's boxes of the first CPRE column chunks are
// loaded up front, so the row loop runs on registers and shuffles; columns
// beyond CPRE chunks are loaded in the loop.
constexpr int CPRE = 8;
// Hit masks: the count pass stores, per tile row and column chunk, the
// ballot of its box tests (masks + mask_off[sub-problem] + row-major
// (row, chunk)), when the tile's range lies inside the mask capacity; the
// write pass then emits the same pairs from the masks without the tests.
struct TileMasks {
  unsigned long long *m;
  const int64_t *off;  // per sub-problem, in the tile-count layout
  int64_t cap;
  int64_t ee_base;  // index of the first EE sub-problem in that layout
};
template <int WRITE>
__device__ __forceinline__ void pair_tile(int is_ee, int64_t tile, const int2 *tile_sub, int64_t n_tiles,
                                          const int64_t *list_start, const int32_t *list_len, const int32_t *lists,
                                          const int32_t *tris, const int32_t *edges, const double *x0,
                                          const double *x1, double inflate, int64_t *tile_cnt, int64_t pos0,
                                          int32_t *out, int64_t n_tiles_valid, int trows, const float *crec,
                                          double *tile_tests, TileMasks tm) {
  // rows: vertices (PT) or edges (EE); columns: triangles (PT) or edges (EE)
  const int rk = is_ee ? 2 : 0, ck = is_ee ? 2 : 1;
  // (the count pass runs over a capacity: tiles beyond the device count
  // record 0 so that the scan over the capacity stays exact)
  if (!WRITE && tile < n_tiles && tile >= n_tiles_valid) {
    if (threadIdx.x == 0) {
      tile_cnt[tile] = 0;
      if (tile_tests) tile_tests[tile] = 0.0;
    }
    return;
  }
  if (tile >= n_tiles) return;
  const int2 ts = tile_sub[tile];  // (sub-problem, tile within it)
  const int64_t s = ts.x;
  const int64_t p = is_ee ? s : s / 2;
  const int li = is_ee ? 4 : 2 * (int)(s % 2);
  const int64_t rstart = list_start[6 * p + li], cstart = list_start[6 * p + li + 1];
  const int nr = list_len[6 * p + li], nc = list_len[6 * p + li + 1];
  const int r0 = ts.y * trows;
  const int r1 = min(nr, r0 + trows);
  const int lane = threadIdx.x;
  const int nch = (nc + 63) / 64;
  // this tile's masks (row-major over its rows and the column chunks)
  unsigned long long *tmask = nullptr;
  if (tm.m) {
    const int64_t mb = tm.off[is_ee ? tm.ee_base + s : s];
    const int64_t m0 = mb + (int64_t)r0 * nch, m1 = m0 + (int64_t)(r1 - r0) * nch;
    if (mb >= 0 && m1 <= tm.cap) tmask = tm.m + m0;
  }
  if (WRITE && tmask) {
    // the pairs from the count pass's masks, in the same order
    int64_t cnt = 0;
    for (int r = r0; r < r1; ++r) {
      const int rp = lists[rstart + r];
      const unsigned long long *mr = tmask + (int64_t)(r - r0) * nch;
      for (int k = 0; k < nch; ++k) {
        const unsigned long long m = mr[k];
        if (m == 0ull) continue;  // (uniform over the wave)
        if ((m >> lane) & 1ull) {
          const int64_t o = pos0 + cnt + __popcll(m & ((1ull << lane) - 1ull));
          out[2 * o] = rp;
          out[2 * o + 1] = lists[cstart + 64 * k + lane];
        }
        cnt += __popcll(m);
      }
    }
    return;
  }
  // row r0 + lane (lanes < trows) and the lane's first CPRE column chunks
  int my_rp = 0;
  double my_rb[6];
  if (r0 + lane < r1) my_rp = lists[rstart + r0 + lane];
  int cpv[CPRE];
  double cb[CPRE][6];
  if (r0 + lane < r1) {
    prim_box(rk, my_rp, tris, edges, x0, x1, inflate, my_rb);
  } else {
#pragma unroll
    for (int i = 0; i < 6; ++i) my_rb[i] = 0.0;
  }
  // three-level tree: the tile's box (union of its row boxes) and the
  // column chunks it reaches (bit k of `live` for the first CPRE chunks)
  double tb[6];
  const int64_t g0 = cstart >> 6;
  unsigned live = 0xFFFFFFFFu;
  if (crec) {
    const bool own = r0 + lane < r1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      tb[c] = own ? my_rb[c] : INFINITY;
      tb[3 + c] = own ? my_rb[3 + c] : -INFINITY;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        tb[c] = fmin(tb[c], __shfl_xor(tb[c], o, 64));
        tb[3 + c] = fmax(tb[3 + c], __shfl_xor(tb[3 + c], o, 64));
      }
    live = 0;
#pragma unroll
    for (int k = 0; k < CPRE; ++k)
      if (k < nch && chunk_reached(crec, g0, k, tb)) live |= 1u << k;
  }
#pragma unroll
  for (int k = 0; k < CPRE; ++k) {
    const int c = 64 * k + lane;
    cpv[k] = c < nc && ((live >> k) & 1) ? lists[cstart + c] : -1;
  }
#pragma unroll
  for (int k = 0; k < CPRE; ++k) {
    if (cpv[k] >= 0) {
      prim_box(ck, cpv[k], tris, edges, x0, x1, inflate, cb[k]);
    } else {
#pragma unroll
      for (int i = 0; i < 6; ++i) cb[k][i] = 0.0;
    }
  }
  int64_t pos = WRITE ? pos0 : 0;
  int64_t cnt = 0;
  for (int r = r0; r < r1; ++r) {
    const int src = r - r0;
    const int rp = __shfl(my_rp, src, 64);
    double rb[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) rb[i] = __shfl(my_rb[i], src, 64);
#pragma unroll
    for (int k = 0; k < CPRE; ++k) {
      if (k < nch) {  // uniform over the wave
        const bool ok = cpv[k] >= 0 && box_overlap(rb, cb[k]);
        const unsigned long long m = __ballot(ok);
        if (!WRITE && tmask && lane == 0) tmask[(int64_t)src * nch + k] = m;
        if (WRITE && ok) {
          const int64_t o = pos + cnt + __popcll(m & ((1ull << lane) - 1ull));
          out[2 * o] = rp;
          out[2 * o + 1] = cpv[k];
        }
        cnt += __popcll(m);
      }
    }
    for (int c0 = 64 * CPRE; c0 < nc; c0 += 64) {
      if (crec && !chunk_reached(crec, g0, c0 >> 6, tb)) {  // (uniform over the wave)
        if (!WRITE && tmask && lane == 0) tmask[(int64_t)src * nch + (c0 >> 6)] = 0ull;
        continue;
      }
      const int c = c0 + lane;
      int cp = 0;
      bool ok = false;
      if (c < nc) {
        cp = lists[cstart + c];
        double cbx[6];
        prim_box(ck, cp, tris, edges, x0, x1, inflate, cbx);
        ok = box_overlap(rb, cbx);
      }
      const unsigned long long m = __ballot(ok);
      if (!WRITE && tmask && lane == 0) tmask[(int64_t)src * nch + (c0 >> 6)] = m;
      if (WRITE && ok) {
        const int64_t o = pos + cnt + __popcll(m & ((1ull << lane) - 1ull));
        out[2 * o] = rp;
        out[2 * o + 1] = cp;
      }
      cnt += __popcll(m);
    }
  }
  if (!WRITE && lane == 0) {
    tile_cnt[tile] = cnt;
    if (tile_tests) {
      // primitive-pair box tests of the tile: its rows x the columns of the
      // chunks it reaches
      int cols = 0;
      for (int k = 0; k < nch; ++k)
        if (!crec || (k < CPRE ? (live >> k) & 1 : chunk_reached(crec, g0, k, tb))) cols += min(64, nc - 64 * k);
      tile_tests[tile] = (double)(r1 - r0) * cols;
    }
  }
}

// Both families in one launch: blocks [0, n_pt_blocks) take PT tiles, the
// rest EE tiles.  Count pass (WRITE=0): n_pt_blocks / n_ee_blocks are the
// capacities, the valid tile counts come from the device (toff, the scan
// of the per-sub-problem tile counts over 3 nbp, and its total), and the
// counts go to cnt[0, cap_pt) (PT) and cnt[cap_pt, cap_pt + cap_ee) (EE).
// Write pass: the blocks are the exact tile counts and off is the scan of
// cnt (EE offsets counted from off[cap_pt]).
template <int WRITE>
__global__ void __launch_bounds__(64) k_pair_tiles(int64_t nbp, int64_t n_pt_blocks, int64_t n_ee_blocks,
                                                   int64_t cap_pt, const int2 *tsub_pt, const int2 *tsub_ee,
                                                   const int64_t *toff, const int64_t *ttotal,
                                                   const int64_t *list_start, const int32_t *list_len,
                                                   const int32_t *lists, const int32_t *tris, const int32_t *edges,
                                                   const double *x0, const double *x1, double inflate,
                                                   int64_t *cnt, const int64_t *off, int32_t *out_pt,
                                                   int32_t *out_ee, int trows, const float *crec,
                                                   double *tile_tests, TileMasks tm) {
  const int64_t b = blockIdx.x;
  if (b < n_pt_blocks) {
    const int64_t valid = WRITE ? n_pt_blocks : toff[2 * nbp];
    pair_tile<WRITE>(0, b, tsub_pt, n_pt_blocks, list_start, list_len, lists, tris, edges, x0, x1, inflate, cnt,
                     WRITE ? off[b] : 0, out_pt, valid, trows, crec, tile_tests, tm);
  } else if (b < n_pt_blocks + n_ee_blocks) {
    const int64_t t = b - n_pt_blocks;
    const int64_t valid = WRITE ? n_ee_blocks : *ttotal - toff[2 * nbp];
    pair_tile<WRITE>(1, t, tsub_ee, n_ee_blocks, list_start, list_len, lists, tris, edges, x0, x1, inflate,
                     cnt + cap_pt, WRITE ? off[cap_pt + t] - off[cap_pt] : 0, out_ee, valid, trows, crec,
                     tile_tests ? tile_tests + cap_pt : nullptr, tm);
  }
}

}  // namespace

int op_candidates(abd_ctx *ctx, const abd_scene *sc, const double *x0, const double *x1, double inflate,
                  int32_t **pt_out, int64_t *n_pt, int32_t **ee_out, int64_t *n_ee, const char *tag,
                  hipStream_t s, const uint8_t *skip_scene) {
  const int nb = sc->n_bodies, nv = sc->n_verts, nt = sc->n_tris, ne = sc->n_edges;
  if (!x1) x1 = x0;
  *n_pt = *n_ee = 0;
  if (nb <= 1 || nv <= 0) return ABD_OK;
  double *bbox;
  ABD_TRY(ws(ctx, "bp_bbox", 6 * (size_t)nb, &bbox, s));
  float *vbox32;
  ABD_TRY(ws(ctx, "bp_vbox32", 6 * (size_t)nv, &vbox32, s));
  uint8_t *involved;
  ABD_TRY(ws(ctx, "bp_involved", nb, &involved, s));
  hipLaunchKernelGGL(k_body_boxes, dim3(grid_for(nb, 4)), dim3(256), 0, s, nb, sc->body_vert_off, x0, x1, inflate,
                     bbox, involved, skip_scene, sc->body_scene);
  HIP_TRY(ctx, hipGetLastError());

  // body pairs
  int32_t *send;
  int64_t *bcnt, *boff, *btot;
  ABD_TRY(ws(ctx, "bp_send", nb, &send, s));
  ABD_TRY(ws(ctx, "bp_bcnt", nb, &bcnt, s));
  ABD_TRY(ws(ctx, "bp_boff", nb, &boff, s));
  ABD_TRY(ws(ctx, "bp_btot", 8, &btot, s));  // totals: body pairs, lists, tiles (2), pairs (2)
  if (!scene_table_cached(ctx, sc, "bp_send", send))
    hipLaunchKernelGGL(k_scene_end, dim3(grid_for(nb, 256)), dim3(256), 0, s, nb, sc->body_scene, send);
  hipLaunchKernelGGL(k_body_pairs<0>, dim3(nb), dim3(64), 0, s, nb, sc->body_scene, sc->body_fixed, bbox, send,
                     skip_scene, bcnt, nullptr, nullptr);
  // the totals' scans also write them to mapped host memory (hbuf, slot
  // for slot like btot), so reading them needs no copy
  int64_t *hbuf, *hbuf_d;
  ABD_TRY(mirror_get(ctx, &hbuf, &hbuf_d));
  hbuf += MIR_BROAD;
  hbuf_d += MIR_BROAD;
  ABD_TRY(scan_exclusive_i64(ctx, bcnt, boff, nb, btot, s, hbuf_d));
  // Body pairs, their list regions and the culled lists are sized by the
  // last call's counts (with room to grow); the search's one
  // synchronisation, after the tile counts, reads every total, and a count
  // beyond its capacity repeats the search from here at the exact sizes.
  const std::string key_bp = std::string(tag) + "_bp", key_lt = std::string(tag) + "_lt";
  // (twice the last counts: contact counts rise step after step while
  // bodies land, and an overflow repeats the whole search)
  int64_t cap_bp = ctx->cap_hint[key_bp], cap_lt = ctx->cap_hint[key_lt];
  cap_bp = 2 * cap_bp + 256;
  cap_lt = 2 * cap_lt + 4096;
  int64_t nbp = 0, list_total = 0;
  const int trows = ctx->tune.tile_rows;
  for (int attempt = 0;; ++attempt) {
  int32_t *bpairs;
  int64_t *cap, *region, *rtot = btot + 1;
  ABD_TRY(ws(ctx, "bp_pairs", 2 * cap_bp + 2, &bpairs, s));
  ABD_TRY(ws(ctx, "bp_cap", cap_bp + 1, &cap, s));
  ABD_TRY(ws(ctx, "bp_region", cap_bp + 1, &region, s));
  hipLaunchKernelGGL(k_body_pairs<1>, dim3(nb), dim3(64), 0, s, nb, sc->body_scene, sc->body_fixed, bbox, send,
                     skip_scene, nullptr, boff, bpairs, cap_bp);
  hipLaunchKernelGGL(k_list_caps, dim3(grid_for(cap_bp, 256)), dim3(256), 0, s, cap_bp, btot, bpairs,
                     sc->body_vert_off, sc->body_tri_off, sc->body_edge_off, cap, involved);
  ABD_TRY(scan_exclusive_i64(ctx, cap, region, cap_bp, rtot, s, hbuf_d + 1));
  // culling boxes of the vertices of bodies in overlapping pairs only
  hipLaunchKernelGGL(k_vert_boxes, dim3(grid_for(nv, 256)), dim3(256), 0, s, nv, sc->vert_body, involved, x0, x1,
                     inflate, vbox32);
  HIP_TRY(ctx, hipGetLastError());

  // culled primitive lists per body pair
  int32_t *lists, *llen;
  int64_t *lstart;
  ABD_TRY(ws(ctx, "bp_lists", cap_lt + 1, &lists, s));
  ABD_TRY(ws(ctx, "bp_llen", 6 * cap_bp, &llen, s));
  ABD_TRY(ws(ctx, "bp_lstart", 6 * cap_bp, &lstart, s));

  // tiles: the count pass is sized like the body pairs.  Tile counts per
  // sub-problem: PT [0, 2 cap_bp), EE [2 cap_bp, 3 cap_bp), scanned as one
  // array (slots past the body-pair count hold 0).
  int64_t *tcnt, *toff, *ttot = btot + 2, *otot = btot + 4;
  ABD_TRY(ws(ctx, "bp_tcnt", 3 * cap_bp, &tcnt, s));
  ABD_TRY(ws(ctx, "bp_toff", 3 * cap_bp + 1, &toff, s));
  float *crec = nullptr;  // three-level tree: chunk records of the column lists
  if (ctx->tune.cull_levels == 3) ABD_TRY(ws(ctx, "bp_crec", CREC * (cap_lt / 64 + 1), &crec, s));
  double *tests = nullptr;  // box-test counting: single-level tests per sub-problem
  if (ctx->count_box_tests) ABD_TRY(ws(ctx, "bp_tests", 3 * cap_bp, &tests, s));
  // hit masks of the tiles (per sub-problem counts in the tile-count layout,
  // their offsets, and the masks on a capacity of twice the last total)
  int64_t *mcnt, *moff;
  ABD_TRY(ws(ctx, "bp_mcnt", 3 * cap_bp, &mcnt, s));
  ABD_TRY(ws(ctx, "bp_moff", 3 * cap_bp + 1, &moff, s));
  const std::string key_mk = std::string(tag) + "_mk";
  const int64_t cap_mk = 2 * ctx->cap_hint[key_mk] + 4096;
  unsigned long long *masks;
  ABD_TRY(ws(ctx, "bp_masks", cap_mk, &masks, s));
  const TileMasks tm{masks, moff, cap_mk, 2 * cap_bp};
  hipLaunchKernelGGL(k_cull_lists, dim3((unsigned)cap_bp, 3), dim3(64), 0, s, bpairs, region, sc->body_vert_off,
                     sc->body_tri_off, sc->body_edge_off, bbox, vbox32, sc->tris, sc->edges, lists, lstart, llen,
                     tcnt, tcnt + 2 * cap_bp, trows, crec, tests, btot, cap_lt, mcnt, mcnt + 2 * cap_bp);
  // hbuf[2] = all tiles, hbuf[3] = PT tiles; hbuf[6] = all masks
  ABD_TRY(scan_exclusive_i64(ctx, tcnt, toff, 3 * cap_bp, ttot, s, hbuf_d + 2, 2 * cap_bp));
  ABD_TRY(scan_exclusive_i64(ctx, mcnt, moff, 3 * cap_bp, btot + 6, s, hbuf_d + 6));
  const std::string key_tp = std::string(tag) + "_tpt", key_te = std::string(tag) + "_tee";
  int64_t cap_tp = ctx->cap_hint[key_tp], cap_te = ctx->cap_hint[key_te];
  cap_tp = cap_tp + cap_tp / 4 + 256;
  cap_te = cap_te + cap_te / 4 + 256;
  int64_t ntile_pt = 0, ntile_ee = 0;
  int64_t *ccnt, *coff;
  double *tile_tests = nullptr;
  int2 *tsub_pt, *tsub_ee;
  for (int pass = 0;; ++pass) {
    // pair counts per tile: PT tiles [0, cap_tp), EE tiles [cap_tp, cap_tp + cap_te)
    ABD_TRY(ws(ctx, "bp_ccnt", cap_tp + cap_te + 1, &ccnt, s));
    ABD_TRY(ws(ctx, "bp_coff", cap_tp + cap_te + 1, &coff, s));
    ABD_TRY(ws(ctx, "bp_tsub_pt", cap_tp + 1, &tsub_pt, s));
    ABD_TRY(ws(ctx, "bp_tsub_ee", cap_te + 1, &tsub_ee, s));
    hipLaunchKernelGGL(k_tile_sub, dim3(grid_for(3 * cap_bp, 256)), dim3(256), 0, s, cap_bp, tcnt, toff, tsub_pt,
                       cap_tp, tsub_ee, cap_te);
    if (tests) ABD_TRY(ws(ctx, "bp_tile_tests", cap_tp + cap_te, &tile_tests, s));
    hipLaunchKernelGGL(k_pair_tiles<0>, dim3((unsigned)(cap_tp + cap_te)), dim3(64), 0, s, cap_bp, cap_tp, cap_te,
                       cap_tp, tsub_pt, tsub_ee, toff, ttot, lstart, llen, lists, sc->tris, sc->edges, x0, x1,
                       inflate, ccnt, nullptr, nullptr, nullptr, trows, crec, tile_tests, tm);
    // hbuf[4] = all pairs, hbuf[5] = PT pairs
    ABD_TRY(scan_exclusive_i64(ctx, ccnt, coff, cap_tp + cap_te, otot, s, hbuf_d + 4, cap_tp));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    ABD_TRY(mirror_counts_ok(ctx, {hbuf[0], hbuf[1], hbuf[2], hbuf[3], hbuf[4], hbuf[5], hbuf[6]}, "candidates"));
    nbp = hbuf[0];
    list_total = hbuf[1];
    if (nbp > cap_bp || list_total > cap_lt) break;  // (the search repeats at the exact sizes)
    ntile_pt = hbuf[3];
    ntile_ee = hbuf[2] - hbuf[3];
    if (ntile_pt <= cap_tp && ntile_ee <= cap_te) break;
    if (pass > 0) return abd_fail(ctx, ABD_E_INVALID, "candidates: tile count changed between passes");
    cap_tp = ntile_pt > cap_tp ? ntile_pt : cap_tp;
    cap_te = ntile_ee > cap_te ? ntile_ee : cap_te;
  }
  if (nbp > cap_bp || list_total > cap_lt) {
    // (a list total read with too few body pairs covers only those: one
    // more pass then sizes the lists)
    if (attempt > 1) return abd_fail(ctx, ABD_E_INVALID, "candidates: body-pair or list count changed between passes");
    cap_bp = nbp > cap_bp ? nbp : cap_bp;
    cap_lt = list_total > cap_lt ? list_total : cap_lt;
    continue;
  }
  ctx->cap_hint[key_bp] = nbp;
  ctx->cap_hint[key_lt] = list_total;
  ctx->cap_hint[key_mk] = hbuf[6];
  ctx->cap_hint[key_tp] = ntile_pt;
  ctx->cap_hint[key_te] = ntile_ee;
  if (tests) {
    // primitive-pair box tests (the tiles' with the table's culling, and a
    // single-level cull's), summed on the device over the profiled calls
    double *acc;
    ABD_TRY(ws(ctx, "prof_box_tests", 2, &acc, s));
    if (ctx->prof_box_tests_clear) hipLaunchKernelGGL(k_clear_f64, dim3(1), dim3(64), 0, s, 2, acc);
    ctx->prof_box_tests_clear = false;
    ABD_TRY(reduce_sum_f64(ctx, tile_tests, cap_tp + cap_te, acc, s));
    ABD_TRY(reduce_sum_f64(ctx, tests, 3 * cap_bp, acc + 1, s));
    ctx->kstats["box_tests"].launches += 1;
    ctx->kstats["box_tests_single_level"].launches += 1;
  }
  *n_pt = hbuf[5];
  *n_ee = hbuf[4] - hbuf[5];
  std::string tpt_name = std::string(tag) + "_pt", tee_name = std::string(tag) + "_ee";
  ABD_TRY(ws(ctx, tpt_name.c_str(), 2 * (*n_pt) + 2, pt_out, s));
  ABD_TRY(ws(ctx, tee_name.c_str(), 2 * (*n_ee) + 2, ee_out, s));
  hipEvent_t pe = prof_begin(ctx, s);
  if (*n_pt + *n_ee > 0)
    hipLaunchKernelGGL(k_pair_tiles<1>, dim3((unsigned)(ntile_pt + ntile_ee)), dim3(64), 0, s, cap_bp, ntile_pt,
                       ntile_ee, cap_tp, tsub_pt, tsub_ee, toff, ttot, lstart, llen, lists, sc->tris, sc->edges, x0,
                       x1, inflate, nullptr, coff, *pt_out, *ee_out, trows, crec, nullptr, tm);
  prof_end(ctx, pe, "pair_tiles_write", ntile_pt + ntile_ee, s);
  return abd_hip_check(ctx, hipGetLastError(), "candidates");
  }
}

// ----------------------------------------------------- off-diag pattern ----
namespace {
__global__ void k_pair_keys(int64_t n, int is_ee, const int32_t *pairs, const int32_t *vert_body,
                            const int32_t *tri_body, const int32_t *edge_body, const uint8_t *fixed, uint64_t *keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = is_ee ? edge_body[pairs[2 * i]] : vert_body[pairs[2 * i]];
  const int b = is_ee ? edge_body[pairs[2 * i + 1]] : tri_body[pairs[2 * i + 1]];
  uint64_t k = ~0ull;
  if (!fixed[a] && !fixed[b] && a != b) {
    const uint64_t lo = (uint64_t)min(a, b), hi = (uint64_t)max(a, b);
    k = (lo << 32) | hi;
  }
  keys[i] = k;
}
__global__ void k_unique_flags(int64_t n, const uint64_t *k, int64_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (k[i] != ~0ull && (i == 0 || k[i] != k[i - 1])) ? 1 : 0;
}
__global__ void k_unique_write(int64_t n, const uint64_t *k, const int64_t *flag, const int64_t *pos, int32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  out[2 * pos[i]] = (int32_t)(k[i] >> 32);
  out[2 * pos[i] + 1] = (int32_t)(k[i] & 0xffffffffu);
}

// Dense variant: the body pairs of every scene are marked in the scene's own
// n_s x n_s byte matrix (the matrices of a batch side by side, scene s at
// foff[s]; every writer stores 1, so races are harmless), then each row a
// writes its marked columns b > a in order, which gives the same sorted,
// unique keys as sorting the pair keys (a scene's bodies are contiguous and
// scenes are in order).  Used while the matrices fit in OD_DENSE_BYTES.
constexpr int64_t OD_DENSE_BYTES = 64ll << 20;
__global__ void k_od_clear(int64_t n16, uint4 *f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) f[i] = make_uint4(0u, 0u, 0u, 0u);
}
// a body's scene matrix: base of its row, scene size, local index
struct OdRow {
  int64_t base;
  int n, loc, first;
};
__device__ __forceinline__ OdRow od_row(int a, const int32_t *body_scene, const int32_t *sbo, const int64_t *foff) {
  const int sc = body_scene[a];
  OdRow r;
  r.first = sbo[sc];
  r.n = sbo[sc + 1] - r.first;
  r.loc = a - r.first;
  r.base = foff[sc] + (int64_t)r.loc * r.n;
  return r;
}
// the four pair lists (PT, EE, extra PT, extra EE) marked by one launch;
// both (a, b) and (b, a) are marked, so that row b also lists the rows
// a < b of its column
struct MarkLists {
  const int32_t *p[5];
  int64_t end[5];  // cumulative counts (point-triangle, edge-edge, pt2, ee2, pt3)
};
__global__ void k_od_mark(MarkLists L, const int32_t *vert_body, const int32_t *tri_body, const int32_t *edge_body,
                          const uint8_t *fixed, const int32_t *body_scene, const int32_t *sbo, const int64_t *foff,
                          uint8_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.end[4]) return;
  int l = 0;
  while (i >= L.end[l]) ++l;
  if (l > 0) i -= L.end[l - 1];
  const int32_t *pairs = L.p[l];
  const int is_ee = l & 1;
  const int a = is_ee ? edge_body[pairs[2 * i]] : vert_body[pairs[2 * i]];
  const int b = is_ee ? edge_body[pairs[2 * i + 1]] : tri_body[pairs[2 * i + 1]];
  if (!fixed[a] && !fixed[b] && a != b) {  // (a and b are bodies of one scene)
    const OdRow ra = od_row(a, body_scene, sbo, foff), rb = od_row(b, body_scene, sbo, foff);
    flags[ra.base + rb.loc] = 1;
    flags[rb.base + ra.loc] = 1;
  }
}
// one wave per row: count (WRITE 0) or write (WRITE 1) the marked columns
// b > a: the keys in (row, column) order.  With the pattern requested, the
// count pass also counts the marked columns b < a (keys with column a) and
// the write pass stores each key's index at the transposed position of the
// scene matrix of kidx (laid out like the flags).
template <int WRITE>
__global__ void __launch_bounds__(64) k_od_row(int nb, const uint8_t *flags, const int32_t *body_scene,
                                               const int32_t *sbo, const int64_t *foff, int64_t *cnt,
                                               const int64_t *off, int32_t *keys, int64_t *lcnt, int32_t *kidx) {
  const int a = blockIdx.x;
  if (a >= nb) return;
  const OdRow ra = od_row(a, body_scene, sbo, foff);
  const uint8_t *row = flags + ra.base;
  int64_t c = 0, base = WRITE ? off[a] : 0;
  for (int b0 = ra.loc + 1; b0 < ra.n; b0 += 64) {
    const int b = b0 + (int)threadIdx.x;
    const bool on = b < ra.n && row[b];
    const unsigned long long m = __ballot(on);
    if (WRITE && on) {
      const int64_t o = base + c + __popcll(m & ((1ull << threadIdx.x) - 1ull));
      keys[2 * o] = a;
      keys[2 * o + 1] = ra.first + b;
      if (kidx) kidx[ra.base - (int64_t)ra.loc * ra.n + (int64_t)b * ra.n + ra.loc] = (int32_t)o;
    }
    c += __popcll(m);
  }
  if (!WRITE && threadIdx.x == 0) cnt[a] = c;
  if (!WRITE && lcnt) {
    int64_t cl = 0;
    for (int b0 = 0; b0 < ra.loc; b0 += 64) {
      const int b = b0 + (int)threadIdx.x;
      cl += __popcll(__ballot(b < ra.loc && row[b]));
    }
    if (threadIdx.x == 0) lcnt[a] = cl;
  }
}
// one wave per body c: the indices of the keys (b, c), b < c, in order of
// b (the keys sorted by (column, row))
__global__ void __launch_bounds__(64) k_od_lower(int nb, const uint8_t *flags, const int32_t *body_scene,
                                                 const int32_t *sbo, const int64_t *foff, const int64_t *loff,
                                                 const int32_t *kidx, uint32_t *tperm) {
  const int c = blockIdx.x;
  if (c >= nb) return;
  const OdRow rc = od_row(c, body_scene, sbo, foff);
  const uint8_t *row = flags + rc.base;
  int64_t o = loff[c];
  for (int b0 = 0; b0 < rc.loc; b0 += 64) {
    const int b = b0 + (int)threadIdx.x;
    const bool on = b < rc.loc && row[b];
    const unsigned long long m = __ballot(on);
    if (on) tperm[o + __popcll(m & ((1ull << threadIdx.x) - 1ull))] = (uint32_t)kidx[rc.base + b];
    o += __popcll(m);
  }
}
}  // namespace

// Byte offsets of the scenes' dense pair matrices (device [S+1]) and their
// total, from the scene's body-to-scene map, read once per scene arrays
// and kept in the context.
int dense_layout(abd_ctx *ctx, const abd_scene *sc, const int64_t **foff, int64_t *total, hipStream_t s) {
  const int S = sc->n_scenes > 0 ? sc->n_scenes : 1;
  const std::vector<uintptr_t> key = {(uintptr_t)sc->body_scene, (uintptr_t)sc->n_bodies, (uintptr_t)S};
  int64_t *f;
  ABD_TRY(ws(ctx, "od_foff", S + 1, &f, s));
  if (ctx->od_key != key) {
    std::vector<int32_t> bs(sc->n_bodies);
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (sc->n_bodies > 0)
      HIP_TRY(ctx, hipMemcpy(bs.data(), sc->body_scene, sizeof(int32_t) * bs.size(), hipMemcpyDeviceToHost));
    std::vector<int64_t> n(S, 0), h(S + 1, 0);
    for (int32_t v : bs) {
      if (v < 0 || v >= S) return abd_fail(ctx, ABD_E_INVALID, "offdiag: body scene %d out of range", v);
      ++n[v];
    }
    for (int k = 0; k < S; ++k) h[k + 1] = h[k] + n[k] * n[k];
    HIP_TRY(ctx, hipMemcpy(f, h.data(), sizeof(int64_t) * h.size(), hipMemcpyHostToDevice));
    ctx->od_key = key;
    ctx->od_total = h[S];
  }
  *foff = f;
  *total = ctx->od_total;
  return ABD_OK;
}

int op_offdiag_count(abd_ctx *ctx, int64_t *n_keys) {
  int64_t *hbuf, *hbuf_d;
  ABD_TRY(mirror_get(ctx, &hbuf, &hbuf_d));
  *n_keys = hbuf[MIR_OFFDIAG];
  return mirror_counts_ok(ctx, {*n_keys}, "offdiag");
}

int op_offdiag(abd_ctx *ctx, const abd_scene *sc, const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee,
               int32_t **keys_out, int64_t *n_keys, const char *tag, hipStream_t s, const int32_t *pt2,
               int64_t n_pt2, const int32_t *ee2, int64_t n_ee2, KeyPattern *pat, const int32_t *pt3,
               int64_t n_pt3, bool defer) {
  // (a scene's joints between two free bodies join the pattern)
  if (!pt3 && sc->n_joints > 0) {
    JointTables *jt = nullptr;
    ABD_TRY(joint_tables(ctx, sc, &jt, s));
    if (jt) {
      pt3 = jt->pairs;
      n_pt3 = jt->n_pairs;
    }
  }
  const int64_t n = n_pt + n_ee + n_pt2 + n_ee2 + n_pt3;
  *n_keys = 0;
  if (pat) *pat = KeyPattern{};
  std::string nm = std::string(tag) + "_keys";
  ABD_TRY(ws(ctx, nm.c_str(), 2 * n + 2, keys_out, s));
  if (n == 0) {
    if (defer) {
      // (the count the caller will read)
      int64_t *hbuf, *hbuf_d;
      ABD_TRY(mirror_get(ctx, &hbuf, &hbuf_d));
      hbuf[MIR_OFFDIAG] = 0;
    }
    return ABD_OK;
  }
  uint64_t *k, *k2;
  int64_t *flag, *pos, *tot;
  ABD_TRY(ws(ctx, "od_k", n, &k, s));
  ABD_TRY(ws(ctx, "od_k2", n, &k2, s));
  ABD_TRY(ws(ctx, "od_flag", n, &flag, s));
  ABD_TRY(ws(ctx, "od_pos", n, &pos, s));
  ABD_TRY(ws(ctx, "od_tot", 1, &tot, s));
  const int32_t *lists[5] = {pt, ee, pt2, ee2, pt3};
  const int64_t counts[5] = {n_pt, n_ee, n_pt2, n_ee2, n_pt3};
  const int nb = sc->n_bodies;
  const int64_t *foff;
  int64_t fbytes;
  ABD_TRY(dense_layout(ctx, sc, &foff, &fbytes, s));
  if (fbytes <= OD_DENSE_BYTES) {
    const int32_t *sbo;
    ABD_TRY(op_scene_offsets(ctx, sc, &sbo, s));
    const int64_t nbb = (fbytes + 15) / 16 * 16;
    uint8_t *flags;
    int64_t *rcnt, *roff;
    ABD_TRY(ws(ctx, "od_flags", nbb, &flags, s));
    ABD_TRY(ws(ctx, "od_rcnt", nb, &rcnt, s));
    ABD_TRY(ws(ctx, "od_roff", nb + 1, &roff, s));
    hipLaunchKernelGGL(k_od_clear, dim3(grid_for(nbb / 16, 256)), dim3(256), 0, s, nbb / 16,
                       reinterpret_cast<uint4 *>(flags));
    MarkLists ml;
    int64_t acc = 0;
    for (int l = 0; l < 5; ++l) {
      ml.p[l] = lists[l];
      acc += counts[l];
      ml.end[l] = acc;
    }
    hipLaunchKernelGGL(k_od_mark, dim3(grid_for(n, 256)), dim3(256), 0, s, ml, sc->vert_body, sc->tri_body,
                       sc->edge_body, sc->body_fixed, sc->body_scene, sbo, foff, flags);
    int64_t *hbuf, *hbuf_d;
    ABD_TRY(mirror_get(ctx, &hbuf, &hbuf_d));
    int64_t *lcnt = nullptr, *loff = nullptr;
    int32_t *kidx = nullptr;
    uint32_t *tperm = nullptr;
    if (pat) {
      ABD_TRY(ws(ctx, "od_lcnt", nb, &lcnt, s));
      ABD_TRY(ws(ctx, "od_loff", nb + 1, &loff, s));
      ABD_TRY(ws(ctx, "od_kidx", (size_t)fbytes + 1, &kidx, s));
      ABD_TRY(ws(ctx, "od_tperm", n + 1, &tperm, s));
    }
    hipLaunchKernelGGL(k_od_row<0>, dim3(nb), dim3(64), 0, s, nb, flags, sc->body_scene, sbo, foff, rcnt, nullptr,
                       nullptr, lcnt, nullptr);
    ABD_TRY(scan_exclusive_i64(ctx, rcnt, roff, nb, roff + nb, s, hbuf_d + MIR_OFFDIAG));
    hipLaunchKernelGGL(k_od_row<1>, dim3(nb), dim3(64), 0, s, nb, flags, sc->body_scene, sbo, foff, nullptr, roff,
                       *keys_out, nullptr, kidx);
    if (pat) {
      ABD_TRY(scan_exclusive_i64(ctx, lcnt, loff, nb, loff + nb, s));
      hipLaunchKernelGGL(k_od_lower, dim3(nb), dim3(64), 0, s, nb, flags, sc->body_scene, sbo, foff, loff, kidx,
                         tperm);
      pat->lo_beg = roff;
      pat->hi_beg = loff;
      pat->tperm = tperm;
      pat->valid = true;
    }
    if (defer) return abd_hip_check(ctx, hipGetLastError(), "offdiag");
    HIP_TRY(ctx, hipStreamSynchronize(s));
    ABD_TRY(op_offdiag_count(ctx, n_keys));
    return abd_hip_check(ctx, hipGetLastError(), "offdiag");
  }
  int64_t at = 0;
  for (int l = 0; l < 5; ++l) {
    if (counts[l] > 0)
      hipLaunchKernelGGL(k_pair_keys, dim3(grid_for(counts[l], 256)), dim3(256), 0, s, counts[l], l & 1, lists[l],
                         sc->vert_body, sc->tri_body, sc->edge_body, sc->body_fixed, k + at);
    at += counts[l];
  }
  size_t tmp_bytes = 0;
  HIP_TRY(ctx, rocprim::radix_sort_keys(nullptr, tmp_bytes, k, k2, (size_t)n, 0, 64, s));
  void *tmp;
  ABD_TRY(ws_get(ctx, "od_tmp", tmp_bytes + 16, &tmp, s));
  HIP_TRY(ctx, rocprim::radix_sort_keys(tmp, tmp_bytes, k, k2, (size_t)n, 0, 64, s));
  hipLaunchKernelGGL(k_unique_flags, dim3(grid_for(n, 256)), dim3(256), 0, s, n, k2, flag);
  int64_t *hbuf, *hbuf_d;
  ABD_TRY(mirror_get(ctx, &hbuf, &hbuf_d));
  ABD_TRY(scan_exclusive_i64(ctx, flag, pos, n, tot, s, hbuf_d + MIR_OFFDIAG));
  hipLaunchKernelGGL(k_unique_write, dim3(grid_for(n, 256)), dim3(256), 0, s, n, k2, flag, pos, *keys_out);
  if (defer) return abd_hip_check(ctx, hipGetLastError(), "offdiag");
  HIP_TRY(ctx, hipStreamSynchronize(s));
  ABD_TRY(op_offdiag_count(ctx, n_keys));
  return abd_hip_check(ctx, hipGetLastError(), "offdiag");
}

// ------------------------------------------------ static subset of a sweep ----
// The candidates at positions x inside a swept segment x0 -> x1 are a subset
// of that segment's swept candidates (every static box lies inside the
// swept box), so they are the swept list filtered by the static predicate:
// the same vertex boxes [x, x + inflate] and the same box test.  Filtering
// keeps the canonical order, so the result equals a full broad phase.
namespace {
template <int K>
__device__ __forceinline__ void static_box(const int32_t *vid, const double *x, double inflate, double b[6]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double a = x[3 * (int64_t)vid[0] + i];
    b[i] = fmin(a, a);
    b[3 + i] = fmax(a, a) + inflate;
  }
#pragma unroll
  for (int k = 1; k < K; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double a = x[3 * (int64_t)vid[k] + i];
      b[i] = fmin(b[i], a);
      b[3 + i] = fmax(b[3 + i], a + inflate);
    }
}

__global__ void k_static_flags(int64_t n_pt, int64_t n, const int32_t *pt, const int32_t *ee, const int32_t *tris,
                               const int32_t *edges, const double *x, double inflate, int64_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a[6], b[6];
  if (i < n_pt) {
    const int32_t v = pt[2 * i];
    static_box<1>(&v, x, inflate, a);
    static_box<3>(tris + 3 * (int64_t)pt[2 * i + 1], x, inflate, b);
  } else {
    const int64_t j = i - n_pt;
    static_box<2>(edges + 2 * (int64_t)ee[2 * j], x, inflate, a);
    static_box<2>(edges + 2 * (int64_t)ee[2 * j + 1], x, inflate, b);
  }
  flag[i] = box_overlap(a, b) ? 1 : 0;
}

__global__ void k_static_compact(int64_t n_pt, int64_t n, const int32_t *pt, const int32_t *ee, const int64_t *flag,
                                 const int64_t *pos, const int64_t *n_keep_pt, int32_t *opt, int32_t *oee) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const int64_t j = pos[i];
  if (i < n_pt) {
    opt[2 * j] = pt[2 * i];
    opt[2 * j + 1] = pt[2 * i + 1];
  } else {
    const int64_t je = j - *n_keep_pt;
    oee[2 * je] = ee[2 * (i - n_pt)];
    oee[2 * je + 1] = ee[2 * (i - n_pt) + 1];
  }
}
}  // namespace

int op_candidates_within(abd_ctx *ctx, const abd_scene *sc, const double *x, double inflate, const int32_t *spt,
                         int64_t n_spt, const int32_t *see, int64_t n_see, int32_t **pt_out, int64_t *n_pt,
                         int32_t **ee_out, int64_t *n_ee, const char *tag, hipStream_t s) {
  const int64_t n = n_spt + n_see;
  const std::string pn = std::string(tag) + "_pt", en = std::string(tag) + "_ee";
  *n_pt = *n_ee = 0;
  int64_t *flag, *pos, *tot;
  ABD_TRY(ws(ctx, "cw_flag", n + 1, &flag, s));
  ABD_TRY(ws(ctx, "cw_pos", n + 1, &pos, s));
  ABD_TRY(ws(ctx, "cw_tot", 2, &tot, s));
  if (n == 0) {
    ABD_TRY(ws(ctx, pn.c_str(), 2, pt_out, s));
    ABD_TRY(ws(ctx, en.c_str(), 2, ee_out, s));
    return ABD_OK;
  }
  hipLaunchKernelGGL(k_static_flags, dim3(grid_for(n, 256)), dim3(256), 0, s, n_spt, n, spt, see, sc->tris, sc->edges,
                     x, inflate, flag);
  // total and the PT part pos[n_spt], written to mapped host memory by the scan
  int64_t *h, *h_d;
  ABD_TRY(mirror_get(ctx, &h, &h_d));
  h += MIR_COMPACT;
  ABD_TRY(scan_exclusive_i64(ctx, flag, pos, n, tot, s, h_d + MIR_COMPACT, n_spt));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  const int64_t keep = h[0], keep_pt = h[1];
  ABD_TRY(mirror_counts_ok(ctx, {keep, keep_pt}, "candidates_within"));
  ABD_TRY(ws(ctx, pn.c_str(), 2 * keep_pt + 2, pt_out, s));
  ABD_TRY(ws(ctx, en.c_str(), 2 * (keep - keep_pt) + 2, ee_out, s));
  const int64_t *nkp = n_see > 0 ? pos + n_spt : tot;
  hipLaunchKernelGGL(k_static_compact, dim3(grid_for(n, 256)), dim3(256), 0, s, n_spt, n, spt, see, flag, pos, nkp,
                     *pt_out, *ee_out);
  *n_pt = keep_pt;
  *n_ee = keep - keep_pt;
  return abd_hip_check(ctx, hipGetLastError(), "candidates within sweep");
}

// ------------------------------------------------------------------ ABI ----
extern "C" int abd_candidates(abd_ctx *ctx, const abd_scene *sc, const double *x0, const double *x1,
                              double inflate, int32_t *pt, int64_t cap_pt, int64_t *n_pt, int32_t *ee,
                              int64_t cap_ee, int64_t *n_ee, hipStream_t stream) {
  if (!ctx || !sc || !x0 || !n_pt || !n_ee) return abd_fail(ctx, ABD_E_INVALID, "abd_candidates: null");
  int32_t *ipt, *iee;
  ABD_TRY(op_candidates(ctx, sc, x0, x1, inflate, &ipt, n_pt, &iee, n_ee, "abi_cand", stream));
  if (*n_pt > cap_pt || *n_ee > cap_ee)
    return abd_fail(ctx, ABD_E_CAPACITY, "candidates need pt %lld ee %lld", (long long)*n_pt, (long long)*n_ee);
  if (*n_pt) HIP_TRY(ctx, hipMemcpyAsync(pt, ipt, 2 * sizeof(int32_t) * *n_pt, hipMemcpyDeviceToDevice, stream));
  if (*n_ee) HIP_TRY(ctx, hipMemcpyAsync(ee, iee, 2 * sizeof(int32_t) * *n_ee, hipMemcpyDeviceToDevice, stream));
  return ABD_OK;
}

extern "C" int abd_candidates_within(abd_ctx *ctx, const abd_scene *sc, const double *x, double inflate,
                                     const int32_t *spt, int64_t n_spt, const int32_t *see, int64_t n_see, int32_t *pt,
                                     int64_t cap_pt, int64_t *n_pt, int32_t *ee, int64_t cap_ee, int64_t *n_ee,
                                     hipStream_t stream) {
  if (!ctx || !sc || !x || !n_pt || !n_ee || (n_spt && !spt) || (n_see && !see))
    return abd_fail(ctx, ABD_E_INVALID, "abd_candidates_within: null");
  int32_t *ipt, *iee;
  ABD_TRY(op_candidates_within(ctx, sc, x, inflate, spt, n_spt, see, n_see, &ipt, n_pt, &iee, n_ee, "abi_cw", stream));
  if (*n_pt > cap_pt || *n_ee > cap_ee)
    return abd_fail(ctx, ABD_E_CAPACITY, "candidates need pt %lld ee %lld", (long long)*n_pt, (long long)*n_ee);
  if (*n_pt) HIP_TRY(ctx, hipMemcpyAsync(pt, ipt, 2 * sizeof(int32_t) * *n_pt, hipMemcpyDeviceToDevice, stream));
  if (*n_ee) HIP_TRY(ctx, hipMemcpyAsync(ee, iee, 2 * sizeof(int32_t) * *n_ee, hipMemcpyDeviceToDevice, stream));
  return ABD_OK;
}

extern "C" int abd_offdiag_pattern(abd_ctx *ctx, const abd_scene *sc, const int32_t *pt, int64_t n_pt,
                                   const int32_t *ee, int64_t n_ee, int32_t *keys, int64_t cap, int64_t *n_keys,
                                   hipStream_t stream) {
  if (!ctx || !sc || !n_keys || (n_pt && !pt) || (n_ee && !ee))
    return abd_fail(ctx, ABD_E_INVALID, "abd_offdiag_pattern: null");
  int32_t *k;
  ABD_TRY(op_offdiag(ctx, sc, pt, n_pt, ee, n_ee, &k, n_keys, "abi_od", stream));
  if (*n_keys > cap) return abd_fail(ctx, ABD_E_CAPACITY, "offdiag needs %lld", (long long)*n_keys);
  if (*n_keys) HIP_TRY(ctx, hipMemcpyAsync(keys, k, 2 * sizeof(int32_t) * *n_keys, hipMemcpyDeviceToDevice, stream));
  return ABD_OK;
}
