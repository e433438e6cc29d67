// Device-wide exclusive scan of int32 values and a fill kernel.
//
// Three launches: per-tile sums, one-block scan of the tile sums, per-tile
// rescan plus tile offset.  A tile is 256 threads x 16 items.  Up to
// kScanDirectTiles tiles the middle launch is left out: each tile adds up
// the sums of the tiles before it itself (at most 4 KiB of reads per tile).
#include "bh_device.h"

namespace bh {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int64_t kScanDirectTiles = 1024;

__device__ __forceinline__ int block_exclusive_sum(int v, int *lds_wave, int *total) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  int inc = wave_inclusive_sum(v);
  if (lane == kWave - 1) lds_wave[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
  for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
    int s = lds_wave[k];
    if (k < w) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int32_t *__restrict__ in, int64_t n,
                                                            int32_t *__restrict__ sums) {
  __shared__ int lds[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int v = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) v += in[i];
  }
  int tot;
  block_exclusive_sum(v, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_sums(int32_t *__restrict__ sums, int64_t nt, int32_t *total) {
  __shared__ int lds[1024 / kWave];
  // each thread owns a consecutive run of tile sums
  const int64_t per = (nt + blockDim.x - 1) / blockDim.x;
  const int64_t b = (int64_t)threadIdx.x * per;
  int v = 0;
  for (int64_t k = 0; k < per; ++k)
    if (b + k < nt) v += sums[b + k];
  int tot;
  int off = block_exclusive_sum(v, lds, &tot);
  for (int64_t k = 0; k < per; ++k)
    if (b + k < nt) {
      int s = sums[b + k];
      sums[b + k] = off;
      off += s;
    }
  if (threadIdx.x == 0 && total) *total = tot;
}

// Direct: sums[] holds each tile's own sum; the tile's offset is the sum of
// those before it, and the last tile writes the total.  Otherwise sums[]
// holds the offsets already.
template <bool Direct>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const int32_t *in, int32_t *out, int64_t n,
                                                            const int32_t *__restrict__ sums, int32_t *total) {
  __shared__ int lds[kScanThreads / kWave];
  int tile_off;
  if (Direct) {
    int p = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kScanThreads) p += sums[k];
    block_exclusive_sum(p, lds, &tile_off);
  } else {
    tile_off = sums[blockIdx.x];
  }
  // blocked layout: thread t owns items [t*16, t*16+16) of the tile
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    v[k] = (i < n) ? in[i] : 0;
    s += v[k];
  }
  int tot;
  int off = block_exclusive_sum(s, lds, &tot) + tile_off;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = off;
    off += v[k];
  }
  if (Direct && total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = tile_off + tot;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) {
  int64_t nt = (n + kScanTile - 1) / kScanTile;
  return (size_t)(nt + 1) * sizeof(int32_t);
}

void scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, void *tmp, hipStream_t s) {
  int64_t nt = (n + kScanTile - 1) / kScanTile;
  if (nt == 0) {
    if (total) k_fill_i32<<<1, 64, 0, s>>>(total, 0, 1);
    return;
  }
  int32_t *sums = (int32_t *)tmp;
  k_tile_sums<<<(unsigned)nt, kScanThreads, 0, s>>>(in, n, sums);
  if (nt <= kScanDirectTiles) {
    k_tile_scan<true><<<(unsigned)nt, kScanThreads, 0, s>>>(in, out, n, sums, total);
    return;
  }
  k_scan_sums<<<1, 1024, 0, s>>>(sums, nt, total);
  k_tile_scan<false><<<(unsigned)nt, kScanThreads, 0, s>>>(in, out, n, sums, nullptr);
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill_i32<<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
}

}  // namespace bh
