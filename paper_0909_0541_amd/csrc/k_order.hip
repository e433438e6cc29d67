// Longest-first processing order for the persistent force kernel.
//
// The kernel pulls work items from an atomic queue; when a few long items are
// pulled last, the grid idles while they finish.  Ordering the queue by cost,
// longest first, bounds that tail (list scheduling).  The order is a counting
// sort over integer cost bins (descending): cost bin = (far entries + 2 near
// entries) / lane partitions / 64, the passes one item makes over its lists.
// Each block ranks one tile of items per bin in LDS and takes one run of
// positions per non-empty bin from the global cursors.  The order within a
// bin does not change any result: every item computes its own outputs.
#include <algorithm>

#include "bh_device.h"

namespace bh {

namespace {

constexpr int kBins = 1024;
constexpr int kTile = 2048;  // items ranked per block

__device__ __forceinline__ int item_key(const int32_t *ginfo, const int32_t *glists, const int32_t *items,
                                        int64_t it) {
  const int g = items[2 * it];
  const int gc = ginfo[3 * g + 1];
  const int nb = (gc + kWave - 1) / kWave;
  const int blk = items[2 * it + 1];
  const int m = (int)((int64_t)gc * (blk + 1) / nb) - (int)((int64_t)gc * blk / nb);
  int R = 1;
  while (R < kWave && m * (2 * R) <= kWave) R *= 2;
  const int64_t cost = ((int64_t)glists[4 * g + 1] + 2 * (int64_t)glists[4 * g + 3]) / R;
  return (int)min<int64_t>(cost >> 6, kBins - 1);
}

__global__ void k_order_clear(int32_t *hist) {
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) hist[b] = 0;
}

__global__ __launch_bounds__(256) void k_order_hist(const int32_t *__restrict__ ginfo,
                                                    const int32_t *__restrict__ glists,
                                                    const int32_t *__restrict__ items,
                                                    const DevInfo *__restrict__ info, int64_t cap,
                                                    int32_t *__restrict__ hist) {
  __shared__ int32_t h[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t n = min<int64_t>(info->n_items, cap);
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  for (int64_t i = t0 + threadIdx.x; i < n && i < t0 + kTile; i += blockDim.x)
    atomicAdd(&h[kBins - 1 - item_key(ginfo, glists, items, i)], 1);
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

__global__ __launch_bounds__(256) void k_order_scatter(const int32_t *__restrict__ ginfo,
                                                       const int32_t *__restrict__ glists,
                                                       const int32_t *__restrict__ items,
                                                       const DevInfo *__restrict__ info, int64_t cap,
                                                       int32_t *__restrict__ cursor, int32_t *__restrict__ order) {
  __shared__ int32_t cnt[kBins], base[kBins];
  __shared__ int16_t key[kTile];
  const int64_t n = min<int64_t>(info->n_items, cap);
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  if (t0 >= n) return;
  const int tn = (int)min<int64_t>(kTile, n - t0);
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < tn; k += blockDim.x) {
    const int b = kBins - 1 - item_key(ginfo, glists, items, t0 + k);
    key[k] = (int16_t)b;
    atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) base[b] = cnt[b] ? atomicAdd(&cursor[b], cnt[b]) : 0;
  __syncthreads();
  // one thread per bin walks the tile in index order
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) {
    if (!cnt[b]) continue;
    int pos = base[b];
    for (int k = 0; k < tn; ++k)
      if (key[k] == b) order[pos++] = (int32_t)(t0 + k);
  }
}

}  // namespace

size_t order_hist_bytes() { return sizeof(int32_t) * kBins; }

void item_order_device(const int32_t *ginfo, const int32_t *glists, const int32_t *items, const DevInfo *info,
                       int64_t cap, int32_t *hist, int32_t *order, int num_cu, hipStream_t s) {
  (void)num_cu;
  if (cap <= 0) return;
  const unsigned grid = (unsigned)((cap + kTile - 1) / kTile);
  k_order_clear<<<1, 256, 0, s>>>(hist);
  k_order_hist<<<grid, 256, 0, s>>>(ginfo, glists, items, info, cap, hist);
  k_order_scan<<<1, kBins, 0, s>>>(hist);
  k_order_scatter<<<grid, 256, 0, s>>>(ginfo, glists, items, info, cap, hist, order);
}

}  // namespace bh
