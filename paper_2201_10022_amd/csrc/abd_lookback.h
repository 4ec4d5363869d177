// Decoupled look-back: tiles claimed in order from a counter publish their
// own sum, then the sum of everything before and including them; a tile
// finds its exclusive prefix from the nearest earlier tile whose inclusive
// prefix is published, adding the sums of the tiles in between.  Each
// status word packs (call tag, flag, value) into one 64-bit atomic, so no
// fence orders a flag against its value; a tag new on every launch makes
// the words of earlier launches read as not yet published, and the counter
// restarts when a block finds it tagged with an earlier launch.  A tile
// waits only on tiles claimed before it, whose blocks are running and
// publish their own sum without waiting, so every wait ends; a spin cap
// (error bit 16) bounds the waits regardless.  A tile that hits the cap
// publishes the poison value LB_VAL_MASK as its inclusive prefix, and every
// tile after it that reads a poisoned word returns the prefix -1, so a scan
// whose look-back failed ends with a total of -1 that the host rejects
// instead of sizing buffers from it.  Values must stay below 2^42 - 1.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

constexpr int LB_TAG_BITS = 20;
constexpr unsigned long long LB_VAL_MASK = (1ull << 42) - 1;
constexpr int LB_SPIN_CAP = 1 << 24;

__device__ __forceinline__ int64_t lb_wave_sum(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// next tile of this launch (one thread).  The counter word carries the tag
// where a status word does (bits 44 and up), so a word left by any earlier
// launch, counter or status, reads as another launch's and is restarted.
__device__ __forceinline__ unsigned int lb_claim(unsigned long long *counter, unsigned int tag, int *err) {
  const unsigned long long T = tag;
  for (int spin = 0;; ++spin) {
    const unsigned long long v = __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((v >> 44) != T) {
      if (atomicCAS(counter, v, (T << 44) | 1ull) == v) return 0;
      if (spin > LB_SPIN_CAP) {  // (cannot happen: some CAS succeeds)
        atomicOr(err, 16);
        return 0;
      }
    } else {
      return (unsigned int)(atomicAdd(counter, 1ull) & ((1ull << 44) - 1ull));
    }
  }
}

__device__ __forceinline__ void lb_publish(unsigned long long *word, unsigned int tag, int inclusive, int64_t v) {
  __hip_atomic_store(word,
                     ((unsigned long long)tag << 44) | ((inclusive ? 2ull : 1ull) << 42) |
                         ((unsigned long long)v & LB_VAL_MASK),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by one whole wave with the tile's sum agg (same on every lane):
// publishes the tile, looks back 64 tiles at a time (one per lane) and
// returns the exclusive prefix on every lane.
__device__ __forceinline__ int64_t lb_lookback(unsigned long long *status, int64_t tile, int64_t agg,
                                               unsigned int tag, int *err) {
  const int lane = threadIdx.x & 63;
  const unsigned long long T = tag;
  if (tile == 0) {
    if (lane == 0) lb_publish(status, tag, 1, agg);
    return 0;
  }
  if (lane == 0) lb_publish(status + tile, tag, 0, agg);
  int64_t p = 0, j0 = tile - 1;
  bool poisoned = false;
  for (int spin = 0;;) {
    const int64_t j = j0 - lane;
    bool ready = true;
    int flag = 2;
    int64_t val = 0;
    if (j >= 0) {  // (before tile 0: a published prefix of 0)
      const unsigned long long st = __hip_atomic_load(status + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ready = (st >> 44) == T;
      flag = (int)((st >> 42) & 3ull);
      val = (int64_t)(st & LB_VAL_MASK);
    }
    const unsigned long long pre = __ballot(ready && flag == 2);
    const int first = pre ? __ffsll((long long)pre) - 1 : 64;
    const unsigned long long need = first >= 63 ? ~0ull : ((1ull << (first + 1)) - 1ull);
    if (__ballot(!ready) & need) {
      if (++spin > LB_SPIN_CAP) {
        if (lane == 0) atomicOr(err, 16);
        poisoned = true;
        break;
      }
      continue;
    }
    if (__ballot(lane <= first && val == (int64_t)LB_VAL_MASK)) {
      poisoned = true;
      break;
    }
    p += lb_wave_sum(lane <= first ? val : 0);
    if (first < 64) break;
    j0 -= 64;
  }
  if (lane == 0) lb_publish(status + tile, tag, 1, poisoned ? (int64_t)LB_VAL_MASK : p + agg);
  return poisoned ? -1 : p;
}
