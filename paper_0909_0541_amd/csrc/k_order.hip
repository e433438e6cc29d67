// Longest-first processing order for the persistent force kernel.
//
// The kernel pulls work items from an atomic queue; when a few long items are
// pulled last, the grid idles while they finish.  Ordering the queue by cost,
// longest first, bounds that tail (list scheduling).  The order is a counting
// sort over integer cost bins (descending): cost bin = (far entries + 2 near
// entries) / lane partitions / 64, the passes one item makes over its lists.
// Each block ranks one tile of items per bin with LDS atomics and takes one
// run of positions per non-empty bin from the global cursors.  The order
// within a bin does not change any result: every item computes its own
// outputs.
#include <algorithm>

#include "bh_device.h"

namespace bh {

namespace {

constexpr int kBins = 1024;
constexpr int kTile = 2048;  // items ranked per block

__device__ __forceinline__ int item_key(const ForceArgs &f, int64_t it) {
  const int g = f.items[2 * it], iv = f.items[2 * it + 1];
  const int blk = iv & 255, segl = iv >> 8;
  const int gc = f.ginfo[3 * g + 1];
  const int m = min(gc - blk * kWave, kWave);  // full blocks of 64, then the remainder
  int R = 1;
  while (R < kWave && m * (2 * R) <= kWave) R *= 2;
  int64_t len;
  if (segl == 0) {
    len = (int64_t)f.glists[4 * g + 1] + 2 * (int64_t)f.glists[4 * g + 3];
  } else {
    const Segment &sg = f.segs[f.seg_order[f.gsegfirst[g] + segl - 1]];
    len = (int64_t)sg.fn + 2 * (int64_t)sg.nn;
  }
  return (int)min<int64_t>((len / R) >> 6, kBins - 1);
}

__global__ void k_order_clear(int32_t *hist) {
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) hist[b] = 0;
}

__global__ __launch_bounds__(256) void k_order_hist(ForceArgs f, int64_t cap, int32_t *__restrict__ hist) {
  __shared__ int32_t h[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t n = min<int64_t>(f.info->n_items, cap);
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  for (int64_t i = t0 + threadIdx.x; i < n && i < t0 + kTile; i += blockDim.x)
    atomicAdd(&h[kBins - 1 - item_key(f, i)], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Exclusive scan of the bins (one block of kBins threads), in place.
__global__ __launch_bounds__(kBins) void k_order_scan(int32_t *hist) {
  __shared__ int32_t w[kBins / kWave];
  const int t = threadIdx.x;
  const int v = hist[t];
  const int inc = wave_inclusive_sum(v);
  if (lane_id() == kWave - 1) w[t / kWave] = inc;
  __syncthreads();
  int off = 0;
  for (int k = 0; k < t / kWave; ++k) off += w[k];
  hist[t] = off + inc - v;
}

__global__ __launch_bounds__(256) void k_order_scatter(ForceArgs f, int64_t cap, int32_t *__restrict__ cursor,
                                                       int32_t *__restrict__ order) {
  constexpr int kPer = kTile / 256;
  __shared__ int32_t cnt[kBins], base[kBins];
  const int64_t n = min<int64_t>(f.info->n_items, cap);
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  if (t0 >= n) return;
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  int key[kPer], rank[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int64_t i = t0 + j * 256 + threadIdx.x;
    key[j] = -1;
    if (i < n) {
      key[j] = kBins - 1 - item_key(f, i);
      rank[j] = atomicAdd(&cnt[key[j]], 1);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) base[b] = cnt[b] ? atomicAdd(&cursor[b], cnt[b]) : 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; ++j)
    if (key[j] >= 0) order[base[key[j]] + rank[j]] = (int32_t)(t0 + j * 256 + threadIdx.x);
}

}  // namespace

size_t order_hist_bytes() { return sizeof(int32_t) * kBins; }

void item_order_device(const ForceArgs &f, int64_t cap, int32_t *hist, int32_t *order, hipStream_t s) {
  if (cap <= 0) return;
  const unsigned grid = (unsigned)((cap + kTile - 1) / kTile);
  k_order_clear<<<1, 256, 0, s>>>(hist);
  k_order_hist<<<grid, 256, 0, s>>>(f, cap, hist);
  k_order_scan<<<1, kBins, 0, s>>>(hist);
  k_order_scatter<<<grid, 256, 0, s>>>(f, cap, hist, order);
}

}  // namespace bh
