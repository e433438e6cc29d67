// Processing order of the persistent force kernel: eight queues, one per
// XCD, longest first, with the member blocks of a group next to each other.
//
// A group's member blocks (and the segments of a split group) all read the
// same interaction list.  When they run at the same time on the same XCD,
// the first block to reach a stretch of the list brings it into that XCD's
// L2 and the others find it there; spread over the chip, every block fetches
// the list from HBM again.  So every group is given to one XCD (the group
// index modulo 8: neighbouring groups have similar lists, so each XCD gets
// an even share of the work), and its items occupy consecutive places of
// that XCD's queue, where consecutive waves take them.  Within a queue the
// groups are ordered by cost, longest first, which bounds the tail of the
// launch (list scheduling); a wave whose queue is empty takes from the
// others.  The order is a counting sort of the groups over (XCD, cost bin),
// each group weighted by its item count; cost bin = list length / lane
// partitions of its first block / 128.  The order within a bin does not
// change any result: every item computes its own outputs.  The items are
// written straight into their queue places.
#include <algorithm>

#include "bh_device.h"

namespace bh {

namespace {

constexpr int kBins = 512;
constexpr int kXcd = 8;
constexpr int kKeys = kXcd * kBins;
constexpr int kTile = 2048;  // groups ranked per block

__device__ __forceinline__ int group_key(const ForceArgs &f, int g) {
  const int gc = f.ginfo[3 * g + 1];
  const int m = min(gc, kWave);  // the first block (full, or the whole small group)
  int R = 1;
  while (R < kWave && m * (2 * R) <= kWave) R *= 2;
  const int64_t len = (int64_t)max(f.glist[g], 0);
  const int bin = (int)min<int64_t>((len / R) >> 7, kBins - 1);
  return (g & (kXcd - 1)) * kBins + (kBins - 1 - bin);
}

__global__ void k_order_clear(int32_t *hist) {
  for (int b = threadIdx.x; b < kKeys; b += blockDim.x) hist[b] = 0;
}

// Work items of group g: ceil(count / 64) member blocks, times the segments
// of a split group.
__device__ __forceinline__ int group_items(const ForceArgs &f, const int32_t *__restrict__ gsplit,
                                           const int32_t *__restrict__ gnseg, int g) {
  const int nb = (f.ginfo[3 * g + 1] + kWave - 1) / kWave;
  return gsplit[g] ? nb * gnseg[g] : nb;
}

// Item counts per (XCD, bin) into hist (zero on entry), and the list
// statistics (interactions, entries, longest list), one atomic per wave.
__global__ __launch_bounds__(256) void k_order_hist(ForceArgs f, const int32_t *__restrict__ gsplit,
                                                    const int32_t *__restrict__ gnseg, int64_t cap,
                                                    int32_t *__restrict__ hist) {
  __shared__ int32_t h[kKeys];
  for (int b = threadIdx.x; b < kKeys; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t G = min<int64_t>(f.info->n_groups, cap);
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  unsigned long long inter = 0, entries = 0;
  int longest = 0;
  for (int64_t g = t0 + threadIdx.x; g < G && g < t0 + kTile; g += blockDim.x) {
    const int nb = group_items(f, gsplit, gnseg, (int)g);
    if (nb > 0) atomicAdd(&h[group_key(f, (int)g)], nb);
    const int c = f.ginfo[3 * g + 1], len = f.glist[g];
    inter += (unsigned long long)c * (unsigned long long)max(len - 1, 0);
    entries += (unsigned long long)max(len, 0);
    longest = max(longest, len);
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    inter += __shfl_xor(inter, d, kWave);
    entries += __shfl_xor(entries, d, kWave);
    longest = max(longest, __shfl_xor(longest, d, kWave));
  }
  if (lane_id() == 0 && (inter || entries || longest)) {
    atomicAdd(&f.info->interactions, inter);
    atomicAdd(&f.info->list_entries, entries);
    atomicMax(&f.info->max_list, longest);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kKeys; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Exclusive scan of the bins (one block of 1024 threads, kKeys / 1024 bins
// each) into the cursors; hist is left zero for the next call.  xstart[x] =
// first queue position of XCD x, xstart[8] the item count; mean_list (when
// set) = this call's mean list length, for the next walk's split cap.
__global__ __launch_bounds__(1024) void k_order_scan(int32_t *__restrict__ hist, int32_t *__restrict__ cursor,
                                                     int32_t *__restrict__ xstart, const DevInfo *__restrict__ info,
                                                     int32_t *__restrict__ mean_list) {
  constexpr int kPer = kKeys / 1024;
  __shared__ int32_t w[1024 / kWave];
  const int t = threadIdx.x;
  int v[kPer], s = 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    v[j] = hist[t * kPer + j];
    hist[t * kPer + j] = 0;
    s += v[j];
  }
  const int inc = wave_inclusive_sum(s);
  if (lane_id() == kWave - 1) w[t / kWave] = inc;
  __syncthreads();
  int off = 0;
  for (int k = 0; k < t / kWave; ++k) off += w[k];
  off += inc - s;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int b = t * kPer + j;
    if (b % kBins == 0) xstart[b / kBins] = off;
    cursor[b] = off;
    off += v[j];
  }
  if (t == 1023) xstart[kXcd] = off;
  if (t == 0 && mean_list) {
    const unsigned long long G = (unsigned long long)max(info->n_groups, 1);
    mean_list[0] = (int32_t)min(info->list_entries / G, (unsigned long long)(INT32_MAX / 64));
  }
}

// Each group takes a run of queue places from its bin's cursor and writes
// its items there: (group, member block + 256 x (segment + 1) for a split
// group), segments in order, blocks in order within a segment.
__global__ __launch_bounds__(256) void k_order_scatter(ForceArgs f, const int32_t *__restrict__ gsplit,
                                                       const int32_t *__restrict__ gnseg, int64_t cap,
                                                       int32_t *__restrict__ cursor, int32_t *__restrict__ items) {
  constexpr int kPer = kTile / 256;
  __shared__ int32_t cnt[kKeys], base[kKeys];
  const int64_t G = min<int64_t>(f.info->n_groups, cap);
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  if (t0 >= G) return;
  for (int b = threadIdx.x; b < kKeys; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  int key[kPer], rank[kPer], nbk[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int64_t g = t0 + j * 256 + threadIdx.x;
    key[j] = -1;
    nbk[j] = 0;
    if (g < G) {
      nbk[j] = group_items(f, gsplit, gnseg, (int)g);
      if (nbk[j] > 0) {
        key[j] = group_key(f, (int)g);
        rank[j] = atomicAdd(&cnt[key[j]], nbk[j]);
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kKeys; b += blockDim.x) base[b] = cnt[b] ? atomicAdd(&cursor[b], cnt[b]) : 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (key[j] < 0) continue;
    const int g = (int)(t0 + j * 256 + threadIdx.x);
    const int nb = (f.ginfo[3 * g + 1] + kWave - 1) / kWave;
    const int ns = gsplit[g] ? gnseg[g] : 0;
    int64_t p = base[key[j]] + rank[j];
    for (int sg = 0; sg < (ns ? ns : 1); ++sg)
      for (int b = 0; b < nb; ++b, ++p) {
        items[2 * p] = g;
        items[2 * p + 1] = b + (ns ? 256 * (sg + 1) : 0);
      }
  }
}

// Walk order of a learned-theta step.  The list walk takes the groups of
// each eighth of [0, G) on one XCD (Morton order keeps neighbouring walks on
// one L2), and a launch ends with the walks taken last: a long walk taken
// late holds the launch open while the other waves idle.  With the
// features at hand, the groups of each eighth are taken longest first by a
// predicted walk time: log2 t = sum_k w_k f_k + w_theta log2(theta) + w_0
// (t in microseconds under a full launch), the weights a least-squares fit
// to the measured walk time of every group of the clustered 2M and 4M
// boxes (correlation 0.79 and 0.83 with the measured times), binned in
// 1/32 octaves.  The order changes which wave walks which group and when,
// never a group's list.
constexpr float kWalkW[BH_MLP_FEATURES] = {0.1395f, 0.1570f, -0.0535f, -0.1039f, 0.0227f, -0.1509f,
                                           0.0256f, 0.2257f,  -0.0245f, 0.2982f,  0.1105f, 0.0308f};
constexpr float kWalkWTheta = -1.5131f, kWalkW0 = 0.4690f;

__device__ __forceinline__ int eighth_of(int64_t G, int g) {
  int x = 0;
#pragma unroll
  for (int k = 1; k < kXcd; ++k) x += (g >= (int)(G * k / kXcd)) ? 1 : 0;
  return x;
}

// (XCD, bin) key of group g: its eighth, then longest first.
__device__ __forceinline__ int walk_key(const float *__restrict__ feat, const float *__restrict__ theta, int64_t G,
                                        int g) {
  float p = kWalkW0;
#pragma unroll
  for (int k = 0; k < BH_MLP_FEATURES; ++k) p = fmaf(kWalkW[k], feat[(int64_t)BH_MLP_FEATURES * g + k], p);
  p = fmaf(kWalkWTheta, __log2f(theta[g]), p);
  p = fminf(fmaxf(p, 0.0f), 15.99f);  // (a NaN, from a theta <= 0 or a NaN feature, goes to bin 0)
  const int bin = (int)(p * 32.0f);
  return eighth_of(G, g) * kBins + (kBins - 1 - bin);
}

__global__ __launch_bounds__(256) void k_worder_hist(const float *__restrict__ feat, const float *__restrict__ theta,
                                                     const DevInfo *__restrict__ info, int64_t cap,
                                                     int32_t *__restrict__ hist) {
  __shared__ int32_t h[kKeys];
  const int64_t G = min<int64_t>(info->n_groups, cap);
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  if (t0 >= G) return;
  for (int b = threadIdx.x; b < kKeys; b += blockDim.x) h[b] = 0;
  __syncthreads();
  for (int64_t g = t0 + threadIdx.x; g < G && g < t0 + kTile; g += blockDim.x)
    atomicAdd(&h[walk_key(feat, theta, G, (int)g)], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < kKeys; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Each group takes a place from its key's cursor (the order within a key is
// that of the atomics, which changes no result).
__global__ __launch_bounds__(256) void k_worder_scatter(const float *__restrict__ feat,
                                                        const float *__restrict__ theta,
                                                        const DevInfo *__restrict__ info, int64_t cap,
                                                        int32_t *__restrict__ cursor, int32_t *__restrict__ order) {
  constexpr int kPer = kTile / 256;
  __shared__ int32_t cnt[kKeys], base[kKeys];
  const int64_t G = min<int64_t>(info->n_groups, cap);
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  if (t0 >= G) return;
  for (int b = threadIdx.x; b < kKeys; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  int key[kPer], rank[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int64_t g = t0 + j * 256 + threadIdx.x;
    key[j] = -1;
    if (g < G) {
      key[j] = walk_key(feat, theta, G, (int)g);
      rank[j] = atomicAdd(&cnt[key[j]], 1);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kKeys; b += blockDim.x) base[b] = cnt[b] ? atomicAdd(&cursor[b], cnt[b]) : 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (key[j] < 0) continue;
    const int64_t p = (int64_t)base[key[j]] + rank[j];
    if (p >= 0 && p < G) order[p] = (int)(t0 + j * 256 + threadIdx.x);
  }
}

}  // namespace

size_t order_hist_bytes() { return sizeof(int32_t) * (2 * kKeys + 16); }

void order_clear_device(int32_t *hist, hipStream_t s) { k_order_clear<<<1, 256, 0, s>>>(hist); }

void item_order_device(const ForceArgs &f, const int32_t *gsplit, const int32_t *gnseg, int64_t gcap, int32_t *hist,
                       int32_t *mean_list, int32_t *items, hipStream_t s) {
  if (gcap <= 0) return;
  const unsigned grid = (unsigned)((gcap + kTile - 1) / kTile);
  int32_t *cursor = hist + kKeys, *xstart = hist + 2 * kKeys;
  k_order_hist<<<grid, 256, 0, s>>>(f, gsplit, gnseg, gcap, hist);
  k_order_scan<<<1, 1024, 0, s>>>(hist, cursor, xstart, f.info, mean_list);
  k_order_scatter<<<grid, 256, 0, s>>>(f, gsplit, gnseg, gcap, cursor, items);
}

}  // namespace bh

namespace bh {

void walk_order_device(const float *feat, const float *theta, const DevInfo *info, int64_t cap, int32_t *hist,
                       int32_t *order, hipStream_t s) {
  if (cap <= 0) return;
  const unsigned grid = (unsigned)((cap + kTile - 1) / kTile);
  int32_t *cursor = hist + kKeys, *xstart = hist + 2 * kKeys;
  k_worder_hist<<<grid, 256, 0, s>>>(feat, theta, info, cap, hist);
  k_order_scan<<<1, 1024, 0, s>>>(hist, cursor, xstart, info, nullptr);
  k_worder_scatter<<<grid, 256, 0, s>>>(feat, theta, info, cap, cursor, order);
}

}  // namespace bh
