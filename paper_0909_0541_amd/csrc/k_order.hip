// Longest-first processing orders for the persistent walk and force kernels.
//
// Both kernels pull work from an atomic queue; when a few long tasks are
// pulled last, the grid idles while they finish.  Ordering the queue by a
// cost estimate, longest first, bounds that tail (list scheduling).  The
// order is a counting sort over integer cost bins (descending); ties keep no
// particular order, which does not change any result: every task computes
// its own outputs independently.
//   walk:  cost bin = member count of the group (larger groups walk longer);
//   force: cost bin = (far entries + 2 near entries) / partitions / 64, the
//          passes one item makes over its lists.
#include <algorithm>

#include "bh_device.h"

namespace bh {

namespace {

constexpr int kBins = 1024;

__device__ __forceinline__ int walk_key(const int32_t *ginfo, int64_t g) {
  return min(ginfo[3 * g + 1], kBins - 1);
}

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

__device__ __forceinline__ int count_of(const DevInfo *info, int mode) {
  return mode == 0 ? info->n_groups : info->n_items;
}

__device__ __forceinline__ int key_of(int mode, const int32_t *ginfo, const int32_t *glists, const int32_t *items,
                                      int64_t i) {
  return mode == 0 ? walk_key(ginfo, i) : item_key(ginfo, glists, items, i);
}

__global__ void k_order_clear(int32_t *hist) {
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) hist[b] = 0;
}

__global__ void k_order_hist(int mode, const int32_t *__restrict__ ginfo, const int32_t *__restrict__ glists,
                             const int32_t *__restrict__ items, const DevInfo *__restrict__ info, int64_t cap,
                             int32_t *__restrict__ hist) {
  __shared__ int32_t h[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t n = count_of(info, mode);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n && i < cap;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[kBins - 1 - key_of(mode, ginfo, glists, items, i)], 1);
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

__global__ void k_order_scatter(int mode, const int32_t *__restrict__ ginfo, const int32_t *__restrict__ glists,
                                const int32_t *__restrict__ items, const DevInfo *__restrict__ info, int64_t cap,
                                int32_t *__restrict__ cursor, int32_t *__restrict__ order) {
  const int64_t n = count_of(info, mode);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n && i < cap;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int b = kBins - 1 - key_of(mode, ginfo, glists, items, i);
    order[atomicAdd(&cursor[b], 1)] = (int32_t)i;
  }
}

void order_device(int mode, const int32_t *ginfo, const int32_t *glists, const int32_t *items, const DevInfo *info,
                  int64_t cap, int32_t *hist, int32_t *order, int num_cu, hipStream_t s) {
  if (cap <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>((cap + 255) / 256, (int64_t)num_cu * 4);
  k_order_clear<<<1, 256, 0, s>>>(hist);
  k_order_hist<<<grid, 256, 0, s>>>(mode, ginfo, glists, items, info, cap, hist);
  k_order_scan<<<1, kBins, 0, s>>>(hist);
  k_order_scatter<<<grid, 256, 0, s>>>(mode, ginfo, glists, items, info, cap, hist, order);
}

}  // namespace

size_t order_hist_bytes() { return sizeof(int32_t) * kBins; }

void walk_order_device(const int32_t *ginfo, const DevInfo *info, int64_t cap, int32_t *hist, int32_t *order,
                       int num_cu, hipStream_t s) {
  order_device(0, ginfo, nullptr, nullptr, info, cap, hist, order, num_cu, s);
}

void item_order_device(const int32_t *ginfo, const int32_t *glists, const int32_t *items, const DevInfo *info,
                       int64_t cap, int32_t *hist, int32_t *order, int num_cu, hipStream_t s) {
  order_device(1, ginfo, glists, items, info, cap, hist, order, num_cu, s);
}

}  // namespace bh
