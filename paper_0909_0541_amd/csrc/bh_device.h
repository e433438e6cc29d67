// Device-side helpers shared by the kernels of libbh (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bh_internal.h"

namespace bh {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// One value per wavefront from an atomic counter: every lane executes the
// atomic (lane 0 adds one, the others zero) so that no divergent branch
// precedes the broadcast of lane 0's result.  Call with all lanes active and
// a counter address the compiler can see is the same on every lane (derive
// a computed index with readfirstlane): only then is the atomic issued as
// one request; 64 requests on one counter serialise behind each other, which
// once made the walk ten times slower.
__device__ __forceinline__ int take_one(int *counter, int lane) {
  const int t = atomicAdd(counter, lane == 0 ? 1 : 0);
  return __builtin_amdgcn_readfirstlane(t);
}

// Number of set bits of m below this lane.
__device__ __forceinline__ int rank_below(unsigned long long m) {
  return (int)__popcll(m & __lanemask_lt());
}

// Inclusive prefix sum and maximum over the 64 lanes of a wave, in data-
// parallel-primitive (DPP) moves between lanes instead of LDS permutes:
// shifts by 1, 2, 4 and 8 lanes within each row of 16 (a Hillis-Steele scan
// of the row), then row 15's last lane broadcast into rows 1 and 3 and lane
// 31 into rows 2 and 3.  Lanes whose source lies outside the row take the
// identity.  Call with all lanes active.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

__device__ __forceinline__ int wave_inclusive_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr1, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr2, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr4, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr8, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowBcast15, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowBcast31, 0xc, 0xf, false);
  return v;
}

__device__ __forceinline__ int wave_inclusive_max(int v) {
  constexpr int kId = -2147483647 - 1;
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, kDppRowShr1, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, kDppRowShr2, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, kDppRowShr4, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, kDppRowShr8, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, kDppRowBcast15, 0xa, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, kDppRowBcast31, 0xc, 0xf, false));
  return v;
}

__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
  int2 a = *reinterpret_cast<int2 *>(&v);
  a.x = __shfl_xor(a.x, mask, kWave);
  a.y = __shfl_xor(a.y, mask, kWave);
  return *reinterpret_cast<double *>(&a);
}

// Octal digits shared by two 63-bit keys (21 when equal).
__device__ __forceinline__ int common_digits(uint64_t a, uint64_t b) {
  uint64_t x = a ^ b;
  if (x == 0) return kKeyLevels;
  int hb = 63 - __clzll((long long)x);
  return 20 - hb / 3;
}

// Octant (0..7) of a key at level l (1..21).
__device__ __forceinline__ int key_digit(uint64_t k, int l) {
  return (int)((k >> (3 * (kKeyLevels - l))) & 7u);
}

// Shift that keeps the first l octal digits of a key.
__device__ __forceinline__ int prefix_shift(int l) { return 3 * (kKeyLevels - l); }

// First index in [lo, hi) whose key prefix (k >> sh) is >= p (keys sorted).
__device__ __forceinline__ int lower_bound_prefix(const uint64_t *__restrict__ keys, int lo, int hi, uint64_t p,
                                                  int sh) {
  while (lo < hi) {
    int mid = lo + ((hi - lo) >> 1);
    if ((keys[mid] >> sh) < p) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// First index in [lo, hi) whose key prefix is > p.
__device__ __forceinline__ int upper_bound_prefix(const uint64_t *__restrict__ keys, int lo, int hi, uint64_t p,
                                                  int sh) {
  while (lo < hi) {
    int mid = lo + ((hi - lo) >> 1);
    if ((keys[mid] >> sh) <= p) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Galloping searches around a known position j whose key prefix equals p:
// steps of 1, 2, 4, ... away from j, then a binary search in the last step,
// so that small cells cost a few cached loads instead of a search over the
// whole system.
// First index in [lo, j] whose prefix equals p.
__device__ __forceinline__ int gallop_first(const uint64_t *__restrict__ keys, int lo, int j, uint64_t p, int sh) {
  int good = j, bad = lo - 1;
  for (int step = 1;; step <<= 1) {
    const int probe = good - step;
    if (probe < lo) break;
    if ((keys[probe] >> sh) < p) {
      bad = probe;
      break;
    }
    good = probe;
  }
  return lower_bound_prefix(keys, bad + 1, good, p, sh);
}

// First index in (j, hi) whose prefix exceeds p (hi if none).
__device__ __forceinline__ int gallop_past(const uint64_t *__restrict__ keys, int j, int hi, uint64_t p, int sh) {
  int good = j, bad = hi;
  for (int step = 1;; step <<= 1) {
    const int probe = good + step;
    if (probe >= hi) break;
    if ((keys[probe] >> sh) > p) {
      bad = probe;
      break;
    }
    good = probe;
  }
  return upper_bound_prefix(keys, good + 1, bad, p, sh);
}

// System owning Morton position j (systems occupy consecutive ranges).
__device__ __forceinline__ int system_of(const SysInfo *__restrict__ sys, int nsys, int j) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sys[mid].first <= j) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Cell coordinates (21 bits per axis) of a Morton key.
__device__ __forceinline__ void key_cells(uint64_t k, uint32_t q[3]) {
  q[0] = q[1] = q[2] = 0;
#pragma unroll 1
  for (int b = 0; b < kKeyLevels; ++b) {
    q[0] |= (uint32_t)((k >> (3 * b + 2)) & 1) << b;
    q[1] |= (uint32_t)((k >> (3 * b + 1)) & 1) << b;
    q[2] |= (uint32_t)((k >> (3 * b)) & 1) << b;
  }
}

}  // namespace bh
