// Split groups: ordering their list segments, and reducing the partial sums
// of the force kernel.
//
// A group whose walk reached the visit cap has its list in segments, one per
// walk unit (k_walk_lists).  Segments are sorted by (group, key) -- the key is
// fixed by the walks, not by when they ran -- so that each group's segments
// are consecutive and in a fixed order.  The force kernel sums every segment
// separately for the group's members into FP64 partial rows; the reduction
// adds a member's rows in segment order, removes the self term as the
// unsplit path does, and writes the outputs in input order.
#include "bh_device.h"

namespace bh {

namespace {

// Sort keys: group in the high bits, segment key (< 2^25) below; unused
// positions sort last.
__global__ void k_seg_keys(const Segment *__restrict__ segs, const SplitCounters *__restrict__ ctr, int cap,
                           uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  const int n = min(ctr->segs, cap);
  keys[i] = (i < n) ? (((uint64_t)(uint32_t)segs[i].g << 25) | (uint64_t)(uint32_t)segs[i].key) : ~0ull;
  vals[i] = (uint32_t)i;
}

// Sorted position of each segment: the number of keys below its own (ties,
// which valid walks never make, broken by index, so that the result is a
// permutation).  Quadratic work, but in two launches: blocks of 256 keys
// against 256-key tiles of the others (a 2-D grid) add to the ranks, then
// the positions are written; for the thousands of segments of a step this
// is far cheaper than a radix sort's passes.
constexpr int kRankSortMax = 16384;
constexpr int kRankTile = 256;
__global__ __launch_bounds__(256) void k_seg_rank(const uint64_t *__restrict__ keys,
                                                  const SplitCounters *__restrict__ ctr, int cap,
                                                  int32_t *__restrict__ rank) {
  __shared__ uint64_t tile[kRankTile];
  const int n = min(ctr->segs, cap);
  const int i0 = blockIdx.x * 256, j0 = blockIdx.y * kRankTile;
  if (i0 >= n || j0 >= n) return;  // whole block
  const int i = i0 + threadIdx.x;
  if (j0 + (int)threadIdx.x < n) tile[threadIdx.x] = keys[j0 + threadIdx.x];
  __syncthreads();
  if (i >= n) return;
  const uint64_t ki = keys[i];
  const int m = min(kRankTile, n - j0);
  int r = 0;
  for (int j = 0; j < m; ++j) {
    const uint64_t kj = tile[j];
    r += (kj < ki || (kj == ki && j0 + j < i)) ? 1 : 0;
  }
  if (r) atomicAdd(&rank[i], r);
}

__global__ void k_seg_place(const int32_t *__restrict__ rank, const SplitCounters *__restrict__ ctr, int cap,
                            uint32_t *__restrict__ order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < min(ctr->segs, cap)) order[rank[i]] = (uint32_t)i;
}

// Per split group (at the first of its sorted segments): segment count and
// first position, list totals and statistics; rows of partial sums per
// sorted position.
__global__ void k_seg_finish(const Segment *__restrict__ segs, const uint32_t *__restrict__ order,
                             const SplitCounters *__restrict__ ctr, int cap, const int32_t *__restrict__ ginfo,
                             int32_t *__restrict__ gsegfirst, int32_t *__restrict__ gnseg,
                             int32_t *__restrict__ glist, double *__restrict__ gmass, int32_t *__restrict__ rows,
                             int32_t *__restrict__ sgroups, int32_t *__restrict__ nsg, DevInfo *__restrict__ info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  const int n = min(ctr->segs, cap);
  if (i >= n) {
    rows[i] = 0;
    return;
  }
  const int g = segs[order[i]].g;
  const int c = ginfo[3 * (int64_t)g + 1];
  rows[i] = c;
  if (i > 0 && segs[order[i - 1]].g == g) return;
  int j = i, len = 0;
  double mass = 0.0;
  while (j < n && segs[order[j]].g == g) {
    len += segs[order[j]].len;
    mass += segs[order[j]].mass;
    ++j;
  }
  gsegfirst[g] = i;
  gnseg[g] = j - i;
  glist[g] = len;
  gmass[g] = mass;
  sgroups[atomicAdd(nsg, 1)] = g;
}

// One block per split group, one thread per member.
__global__ __launch_bounds__(256) void k_split_reduce(const int32_t *__restrict__ sgroups,
                                                      const int32_t *__restrict__ nsg, int cap,
                                                      const int32_t *__restrict__ ginfo,
                                                      const int32_t *__restrict__ gsegfirst,
                                                      const int32_t *__restrict__ gnseg,
                                                      const int32_t *__restrict__ pbase,
                                                      const double *__restrict__ psum, const double *__restrict__ smass,
                                                      const int32_t *__restrict__ perm,
                                                      const SysParam *__restrict__ par, float *__restrict__ acc,
                                                      float *__restrict__ pot) {
  const int k = blockIdx.x;
  if (k >= min(*nsg, cap)) return;
  const int g = sgroups[k];
  const int gf = ginfo[3 * (int64_t)g], c = ginfo[3 * (int64_t)g + 1], gs = ginfo[3 * (int64_t)g + 2];
  const int p0 = gsegfirst[g], ns = gnseg[g];
  const double eps = par[gs].eps;
  const float eps2 = (float)(eps * eps);
  for (int u = threadIdx.x; u < c; u += blockDim.x) {
    double vx = 0.0, vy = 0.0, vz = 0.0, vp = 0.0;
    for (int p = p0; p < p0 + ns; ++p) {
      const double *q = psum + 4 * ((int64_t)pbase[p] + u);
      vx += q[0];
      vy += q[1];
      vz += q[2];
      vp += q[3];
    }
    const int i = gf + u;
    const float self_ri = __builtin_amdgcn_rsqf(__builtin_fmaf(0.0f, 0.0f, eps2));
    const double self = (double)((float)smass[i] * self_ri);
    const int o = perm[i];
    acc[3 * (int64_t)o] = (float)vx;
    acc[3 * (int64_t)o + 1] = (float)vy;
    acc[3 * (int64_t)o + 2] = (float)vz;
    pot[o] = (float)(self - vp);
  }
}

__global__ void k_zero_i32(int32_t *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void split_finish_device(SplitBuffers &S, const int32_t *ginfo, int32_t *glist, double *gmass, DevInfo *info,
                         hipStream_t s) {
  const int cap = S.seg_cap;
  k_seg_keys<<<blocks(cap), 256, 0, s>>>(S.segs, S.ctr, cap, S.keys[0], S.vals[0]);
  uint32_t *order;
  if (cap <= kRankSortMax) {
    order = S.vals[1];
    int32_t *rank = reinterpret_cast<int32_t *>(S.vals[0]);
    k_zero_i32<<<blocks(cap), 256, 0, s>>>(rank, cap);
    k_seg_rank<<<dim3(blocks(cap), (unsigned)((cap + kRankTile - 1) / kRankTile)), 256, 0, s>>>(S.keys[0], S.ctr, cap,
                                                                                              rank);
    k_seg_place<<<blocks(cap), 256, 0, s>>>(rank, S.ctr, cap, order);
  } else {
    const int cur = radix_sort_pairs(S.keys[0], S.keys[1], S.vals[0], S.vals[1], cap, 0, 64, S.hist, S.scan_tmp,
                                     &info->err, s);
    order = S.vals[cur];
  }
  S.order = order;
  k_zero_i32<<<1, 64, 0, s>>>(S.nsg, 1);
  k_seg_finish<<<blocks(cap), 256, 0, s>>>(S.segs, order, S.ctr, cap, ginfo, S.gsegfirst, S.gnseg, glist, gmass,
                                           S.rows, S.sgroups, S.nsg, info);
  scan_exclusive_i32(S.rows, S.pbase, cap, S.total_rows, S.scan_tmp, s);
}

void split_reduce_device(const SplitBuffers &S, const int32_t *ginfo, const double *smass, const int32_t *perm,
                         const SysParam *par, float *acc, float *pot, hipStream_t s) {
  if (S.seg_cap > 0)
    k_split_reduce<<<(unsigned)S.seg_cap, 256, 0, s>>>(S.sgroups, S.nsg, S.seg_cap, ginfo, S.gsegfirst, S.gnseg,
                                                       S.pbase, S.psum, smass, perm, par, acc, pot);
}

}  // namespace bh
