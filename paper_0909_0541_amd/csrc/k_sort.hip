// Stable LSD radix sort of (u64 Morton key, u32 index) pairs, 8-bit digits.
//
// Per pass: per-tile digit histograms (LDS counters), one exclusive scan of
// the digit-major histogram table, then a scatter in which each wave ranks its
// keys stably with ballot-based peer masks and per-wave digit counters in LDS;
// the tile is staged in LDS in digit order so that the writes to HBM are runs
// of consecutive addresses.
// A tile is 4 waves x 16 chunks x 64 keys = 4096 keys; keys of wave w, chunk
// c, lane l sit at tile offset w*1024 + c*64 + l, so (w, c, l) order is input
// order and the sort is stable.
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
  int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  return (size_t)(ntiles * kRadix + 1) * sizeof(uint32_t);
}

size_t radix_scan_elems(int64_t n) {
  int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  return (size_t)(ntiles * kRadix);
}

int radix_sort_pairs(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit0, int bit1,
                     uint32_t *hist, void *scan_tmp, hipStream_t s) {
  uint64_t *k[2] = {k0, k1};
  uint32_t *v[2] = {v0, v1};
  int cur = 0;
  if (n <= 1) return cur;
  for (int bit = bit0; bit < bit1; bit += 8) {
    KeyDigit dig{bit};
    one_pass(k[cur], v[cur], k[cur ^ 1], v[cur ^ 1], n, dig, hist, scan_tmp, s);
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
