// Stable LSD radix sort of (u64 Morton key, u32 index) pairs, 8-bit digits.
//
// Key passes: the digit counts of every pass are taken in one read of the
// keys; then one kernel per pass ranks each tile's keys stably (ballot-based
// peer masks, per-wave digit counters in LDS), finds the tile's offset within
// each digit from the tiles before it by decoupled look-back (a tile posts its
// own digit counts, then adds its predecessors' posts until it meets an
// inclusive prefix, and posts its own inclusive prefix), and scatters.  Tiles
// take their index from a counter in the order they start, so a tile only
// waits for tiles that are already running and have posted or will post
// without waiting for it; the wait is bounded all the same, and a timeout is
// reported as an error rather than hanging.  The tile is staged in LDS in
// digit order so that the writes to HBM are runs of consecutive addresses.
// Passes on an external digit (the system of a row) use a per-tile histogram
// table and a scan instead.
// A tile is 4 waves x 16 chunks x 64 keys = 4096 keys; keys of wave w, chunk
// c, lane l sit at tile offset w*1024 + c*64 + l, so (w, c, l) order is input
// order and the sort is stable.
#include <algorithm>

#include "bh_device.h"

namespace bh {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortChunks = 16;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kSortTile = kSortThreads * kSortChunks;
constexpr int kRadix = 256;

// Digit of a (key, value) pair: 8 bits of the key ...
struct KeyDigit {
  int bit;
  __device__ __forceinline__ int of(uint64_t k, uint32_t) const { return (int)((k >> bit) & 255u); }
};

// ... or 8 bits of the system of the input row the value names.
struct SysDigit {
  const int32_t *sys_in;
  int shift;
  __device__ __forceinline__ int of(uint64_t, uint32_t v) const {
    return (int)(((uint32_t)sys_in[v] >> shift) & 255u);
  }
};

template <class Digit>
__global__ __launch_bounds__(kSortThreads) void k_hist(const uint64_t *__restrict__ keys,
                                                       const uint32_t *__restrict__ vals, int64_t n, Digit dig,
                                                       int64_t ntiles, uint32_t *__restrict__ hist) {
  __shared__ uint32_t cnt[kSortWaves][kRadix];
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortThreads) (&cnt[0][0])[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)w * (kSortChunks * kWave);
#pragma unroll 4
  for (int c = 0; c < kSortChunks; ++c) {
    int64_t i = base + c * kWave + lane;
    if (i < n) atomicAdd(&cnt[w][dig.of(keys[i], vals[i])], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
    uint32_t s = 0;
    for (int k = 0; k < kSortWaves; ++k) s += cnt[k][d];
    hist[(int64_t)d * ntiles + blockIdx.x] = s;
  }
}

template <class Digit>
__global__ __launch_bounds__(kSortThreads) void k_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                          uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                          int64_t n, Digit dig, int64_t ntiles,
                                                          const uint32_t *__restrict__ offs) {
  __shared__ uint32_t cnt[kSortWaves][kRadix];
  __shared__ uint32_t dstart[kRadix];  // tile-local start of each digit
  __shared__ uint64_t skey[kSortTile];
  __shared__ uint32_t sval[kSortTile];
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortThreads) (&cnt[0][0])[d] = 0;
  __syncthreads();
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  const int64_t base = tile0 + (int64_t)w * (kSortChunks * kWave);
  const int tile_n = (int)min((int64_t)kSortTile, n - tile0);
  uint64_t key[kSortChunks];
  uint32_t val[kSortChunks];
  int rank[kSortChunks];
  int digit[kSortChunks];
#pragma unroll
  for (int c = 0; c < kSortChunks; ++c) {
    int64_t i = base + c * kWave + lane;
    bool ok = i < n;
    key[c] = ok ? kin[i] : 0;
    val[c] = ok ? vin[i] : 0;
    int d = ok ? dig.of(key[c], val[c]) : 0;
    digit[c] = d;
    unsigned long long valid = __ballot(ok);
    unsigned long long peers = valid;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      unsigned long long m = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    if (!ok) peers = 0;
    // all peers read the running count before the lowest peer advances it
    uint32_t before = ok ? cnt[w][d] : 0;
    rank[c] = (int)before + rank_below(peers);
    __builtin_amdgcn_wave_barrier();
    if (ok && rank_below(peers) == 0) cnt[w][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // tile-local offsets: digits in order, within a digit the waves in order
  if (threadIdx.x < kRadix) {
    const int d = threadIdx.x;
    uint32_t tot = 0;
    for (int k = 0; k < kSortWaves; ++k) {
      uint32_t c = cnt[k][d];
      cnt[k][d] = tot;
      tot += c;
    }
    dstart[d] = tot;  // digit total for now, turned into a start below
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    // exclusive scan of the 256 digit totals by one wave (4 per lane)
    uint32_t v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = dstart[4 * threadIdx.x + q];
      s += v[q];
    }
    const uint32_t inc = (uint32_t)wave_inclusive_sum((int)s);
    uint32_t run = inc - s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      dstart[4 * threadIdx.x + q] = run;
      run += v[q];
    }
  }
  __syncthreads();
  // stage the tile in LDS in digit order
#pragma unroll
  for (int c = 0; c < kSortChunks; ++c) {
    const int64_t i = base + c * kWave + lane;
    if (i < n) {
      const uint32_t p = dstart[digit[c]] + cnt[w][digit[c]] + (uint32_t)rank[c];
      skey[p] = key[c];
      sval[p] = val[c];
    }
  }
  __syncthreads();
  // write out: consecutive threads hold consecutive positions of one digit run
  for (int p = threadIdx.x; p < tile_n; p += kSortThreads) {
    const uint64_t k = skey[p];
    const uint32_t v = sval[p];
    const int d = dig.of(k, v);
    const uint32_t dst = offs[(int64_t)d * ntiles + blockIdx.x] + (uint32_t)p - dstart[d];
    kout[dst] = k;
    vout[dst] = v;
  }
}

// State of the key passes (32-bit words): digit counts per pass, a tile
// counter per pass, then per pass and tile the posted word of each digit:
// flag (bits 30-31: 1 the tile's own count, 2 the inclusive prefix over
// tiles) and value (bits 0-29).
constexpr int kMaxPasses = 8;
constexpr int kStateCounts = 0;
constexpr int kStateTiles = kMaxPasses * kRadix;
constexpr int kStateHead = kStateTiles + 64;
constexpr uint32_t kPostOwn = 1u << 30, kPostPrefix = 2u << 30, kPostMask = (1u << 30) - 1u;
constexpr int kSpinLimit = 1 << 22;
constexpr int kLookWindow = 8;  // predecessors read together in the look-back

__device__ __forceinline__ uint32_t load_post(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_post(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Digit counts of passes [0, npass) (digit bit0 + 8 p) over all keys.
// (Four copies of the counters, taken by lane & 3, so that lanes with equal
// digits, common in the top digits, contend less.)
__global__ __launch_bounds__(kSortThreads) void k_digit_counts(const uint64_t *__restrict__ keys, int64_t n, int bit0,
                                                               int npass, uint32_t *__restrict__ state) {
  __shared__ uint32_t cnt[kMaxPasses][kRadix][4];
  for (int d = threadIdx.x; d < kMaxPasses * kRadix * 4; d += kSortThreads) (&cnt[0][0][0])[d] = 0;
  __syncthreads();
  const int cp = threadIdx.x & 3;
  for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kSortThreads) {
    const uint64_t k = keys[i];
    for (int p = 0; p < npass; ++p) atomicAdd(&cnt[p][(k >> (bit0 + 8 * p)) & 255u][cp], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < npass * kRadix; d += kSortThreads) {
    const uint32_t *c = &cnt[0][0][0] + 4 * d;
    const uint32_t t = c[0] + c[1] + c[2] + c[3];
    if (t) atomicAdd(&state[kStateCounts + d], t);
  }
}

// One key pass: rank, look back, scatter.
__global__ __launch_bounds__(kSortThreads) void k_onesweep(const uint64_t *__restrict__ kin,
                                                           const uint32_t *__restrict__ vin,
                                                           uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                           int64_t n, int bit, int pass, int64_t ntiles,
                                                           uint32_t *__restrict__ state, int32_t *err) {
  static_assert(kSortThreads == kRadix, "one thread per digit");
  __shared__ uint32_t cnt[kSortWaves][kRadix];
  __shared__ uint32_t dstart[kRadix];  // tile-local start of each digit; then its output index minus that
  __shared__ uint64_t skey[kSortTile];
  __shared__ uint32_t sval[kSortTile];
  __shared__ uint32_t wtot[2][kSortWaves];
  __shared__ int tile_sh;
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortThreads) (&cnt[0][0])[d] = 0;
  if (threadIdx.x == 0) tile_sh = (int)atomicAdd(&state[kStateTiles + pass], 1u);
  __syncthreads();
  const int64_t tile = tile_sh;
  uint32_t *post = state + kStateHead + ((int64_t)pass * ntiles + tile) * kRadix;
  const int64_t tile0 = tile * kSortTile;
  const int64_t base = tile0 + (int64_t)w * (kSortChunks * kWave);
  const int tile_n = (int)min((int64_t)kSortTile, n - tile0);
  uint64_t key[kSortChunks];
  uint32_t val[kSortChunks];
  int rank[kSortChunks];
  int digit[kSortChunks];
#pragma unroll
  for (int c = 0; c < kSortChunks; ++c) {
    int64_t i = base + c * kWave + lane;
    bool ok = i < n;
    key[c] = ok ? kin[i] : 0;
    val[c] = ok ? vin[i] : 0;
    int d = ok ? (int)((key[c] >> bit) & 255u) : 0;
    digit[c] = d;
    unsigned long long valid = __ballot(ok);
    unsigned long long peers = valid;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      unsigned long long m = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    if (!ok) peers = 0;
    // all peers read the running count before the lowest peer advances it
    uint32_t before = ok ? cnt[w][d] : 0;
    rank[c] = (int)before + rank_below(peers);
    __builtin_amdgcn_wave_barrier();
    if (ok && rank_below(peers) == 0) cnt[w][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // thread d: the tile's count of digit d (posted at once; within the digit
  // the waves in order), and the pass's count of d over all keys
  const int d = threadIdx.x;
  uint32_t own = 0;
  for (int k = 0; k < kSortWaves; ++k) {
    const uint32_t c = cnt[k][d];
    cnt[k][d] = own;
    own += c;
  }
  store_post(&post[d], (tile == 0 ? kPostPrefix : kPostOwn) | own);
  const uint32_t total = state[kStateCounts + pass * kRadix + d];
  // exclusive scans over the digits of both, across the four waves
  const uint32_t inc = (uint32_t)wave_inclusive_sum((int)own);
  const uint32_t tinc = (uint32_t)wave_inclusive_sum((int)total);
  if (lane == kWave - 1) {
    wtot[0][w] = inc;
    wtot[1][w] = tinc;
  }
  // look back: the keys of digit d in the tiles before this one; the posts
  // of kLookWindow predecessors are read together, then taken nearest first,
  // a post not yet made being read again until it is
  uint32_t prev = 0;
  if (tile > 0) {
    bool timed_out = false, done = false;
    const uint32_t *col = state + kStateHead + (int64_t)pass * ntiles * kRadix + d;
    for (int64_t t0 = tile - 1; t0 >= 0 && !done && !timed_out; t0 -= kLookWindow) {
      uint32_t v[kLookWindow];
#pragma unroll
      for (int u = 0; u < kLookWindow; ++u) v[u] = (t0 - u >= 0) ? load_post(col + (t0 - u) * kRadix) : kPostPrefix;
#pragma unroll
      for (int u = 0; u < kLookWindow; ++u) {
        if (done || timed_out) break;
        const uint32_t *q = col + (t0 - u) * kRadix;
        for (int spin = 0; (v[u] & ~kPostMask) == 0u; ++spin) {
          if (spin >= kSpinLimit) {
            timed_out = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          v[u] = load_post(q);
        }
        if (timed_out) break;
        prev += v[u] & kPostMask;
        done = (v[u] & ~kPostMask) == kPostPrefix;
      }
    }
    if (timed_out && err) atomicOr(err, (int32_t)kErrWait);
    store_post(&post[d], kPostPrefix | (prev + own));
  }
  __syncthreads();
  uint32_t lo = 0, tlo = 0;
  for (int k = 0; k < w; ++k) {
    lo += wtot[0][k];
    tlo += wtot[1][k];
  }
  const uint32_t start = lo + inc - own;            // tile-local start of digit d
  const uint32_t gstart = tlo + tinc - total;       // start of digit d in the output
  dstart[d] = start;
  __syncthreads();
  // stage the tile in LDS in digit order
#pragma unroll
  for (int c = 0; c < kSortChunks; ++c) {
    const int64_t i = base + c * kWave + lane;
    if (i < n) {
      const uint32_t p = dstart[digit[c]] + cnt[w][digit[c]] + (uint32_t)rank[c];
      skey[p] = key[c];
      sval[p] = val[c];
    }
  }
  __syncthreads();
  // output index of a staged position p of digit d: p + dstart[d] from here on
  dstart[d] = gstart + prev - start;
  __syncthreads();
  // write out: consecutive threads hold consecutive positions of one digit run
  for (int p = threadIdx.x; p < tile_n; p += kSortThreads) {
    const uint64_t k = skey[p];
    const uint32_t v = sval[p];
    const uint32_t dst = dstart[(int)((k >> bit) & 255u)] + (uint32_t)p;
    kout[dst] = k;
    vout[dst] = v;
  }
}

__global__ void k_iota(uint32_t *v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (uint32_t)i;
}

template <class Digit>
void one_pass(const uint64_t *kin, const uint32_t *vin, uint64_t *kout, uint32_t *vout, int64_t n, Digit dig,
              uint32_t *hist, void *scan_tmp, hipStream_t s) {
  int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  k_hist<Digit><<<(unsigned)ntiles, kSortThreads, 0, s>>>(kin, vin, n, dig, ntiles, hist);
  scan_exclusive_i32((const int32_t *)hist, (int32_t *)hist, ntiles * kRadix, nullptr, scan_tmp, s);
  k_scatter<Digit><<<(unsigned)ntiles, kSortThreads, 0, s>>>(kin, vin, kout, vout, n, dig, ntiles, hist);
}

}  // namespace

size_t radix_hist_bytes(int64_t n) {
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  const int64_t table = ntiles * kRadix + 1;                        // external-digit passes
  const int64_t state = kStateHead + (int64_t)kMaxPasses * ntiles * kRadix;  // key passes
  return (size_t)std::max(table, state) * sizeof(uint32_t);
}

size_t radix_scan_elems(int64_t n) {
  int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  return (size_t)(ntiles * kRadix);
}

int radix_sort_pairs(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit0, int bit1,
                     uint32_t *hist, void *scan_tmp, int32_t *err, hipStream_t s) {
  (void)scan_tmp;
  uint64_t *k[2] = {k0, k1};
  uint32_t *v[2] = {v0, v1};
  int cur = 0;
  if (n <= 1) return cur;
  const int npass = (bit1 - bit0 + 7) / 8;
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  fill_i32(reinterpret_cast<int32_t *>(hist), 0, kStateHead + (int64_t)npass * ntiles * kRadix, s);
  k_digit_counts<<<(unsigned)std::min<int64_t>(ntiles, 512), kSortThreads, 0, s>>>(k[cur], n, bit0, npass, hist);
  for (int p = 0; p < npass; ++p) {
    k_onesweep<<<(unsigned)ntiles, kSortThreads, 0, s>>>(k[cur], v[cur], k[cur ^ 1], v[cur ^ 1], n, bit0 + 8 * p, p,
                                                         ntiles, hist, err);
    cur ^= 1;
  }
  return cur;
}

int radix_pass_by_system(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int cur, int64_t n,
                         const int32_t *sys_in, int shift, uint32_t *hist, void *scan_tmp, hipStream_t s) {
  uint64_t *k[2] = {k0, k1};
  uint32_t *v[2] = {v0, v1};
  if (n <= 1) return cur;
  SysDigit dig{sys_in, shift};
  one_pass(k[cur], v[cur], k[cur ^ 1], v[cur ^ 1], n, dig, hist, scan_tmp, s);
  return cur ^ 1;
}

void iota_u32(uint32_t *v, int64_t n, hipStream_t s) {
  if (n > 0) k_iota<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(v, n);
}

}  // namespace bh
