// Particle groups for the vectorised walk.
//
// A cell with more than n_crit particles is split further; the runs of its
// consecutive sub-cells (octant order) holding at most n_crit particles each
// are packed greedily into groups of at most n_crit particles; a system with
// at most n_crit particles is a single group.  Groups are contiguous Morton
// ranges; each gets its FP64 bounding box.
#include "bh_device.h"

namespace bh {

namespace {

__global__ void k_group_mark(const int8_t *__restrict__ level, const int32_t *__restrict__ ccount,
                             const int32_t *__restrict__ cfc, const int32_t *__restrict__ nchild,
                             const NodeRec *__restrict__ nodes, const SysInfo *__restrict__ sys, int nsys,
                             int64_t n, int n_crit, int32_t *__restrict__ gflag, int32_t *__restrict__ glen,
                             DevInfo *info) {
  int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jj < nsys) {
    const SysInfo &S = sys[jj];
    if (S.count > 0 && S.count <= n_crit) {
      gflag[S.first] = 1;
      glen[S.first] = S.count;
    }
  }
  if (jj >= n) return;
  const int j = (int)jj;
  if (level[j] < 0 || ccount[j] <= n_crit) return;
  const int c0 = nsys + cfc[j], nc = nchild[j];
  if ((int64_t)c0 + nc > nsys + info->n_slots) {
    atomicOr(&info->err, kErrBuild);
    return;
  }
  int run_first = -1, run_count = 0;
  for (int k = 0; k < nc; ++k) {
    const NodeRec &ch = nodes[c0 + k];
    const int cc = ch.count, cf = ch.first;
    if (cc > n_crit) {
      if (run_count > 0) {
        gflag[run_first] = 1;
        glen[run_first] = run_count;
      }
      run_count = 0;
      continue;
    }
    if (run_count > 0 && run_count + cc > n_crit) {
      gflag[run_first] = 1;
      glen[run_first] = run_count;
      run_count = 0;
    }
    if (run_count == 0) run_first = cf;
    run_count += cc;
  }
  if (run_count > 0) {
    gflag[run_first] = 1;
    glen[run_first] = run_count;
  }
}

__global__ void k_group_scatter(const int32_t *__restrict__ gflag, const int32_t *__restrict__ gidx,
                                const int32_t *__restrict__ glen, const SysInfo *__restrict__ sys, int nsys,
                                int64_t n, int32_t *__restrict__ ginfo) {
  int64_t ff = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ff >= n) return;
  const int f = (int)ff;
  if (!gflag[f]) return;
  const int g = gidx[f];
  ginfo[3 * (int64_t)g] = f;
  ginfo[3 * (int64_t)g + 1] = glen[f];
  ginfo[3 * (int64_t)g + 2] = system_of(sys, nsys, f);
}

// One wave per group: FP64 bounding box of the members.
__global__ __launch_bounds__(256) void k_group_box(const int32_t *__restrict__ ginfo, const double *__restrict__ spos,
                                                   const DevInfo *__restrict__ info, double *__restrict__ gbox) {
  const int lane = lane_id();
  const int G = info->n_groups;
  const int wpb = blockDim.x / kWave;
  for (int g = blockIdx.x * wpb + threadIdx.x / kWave; g < G; g += gridDim.x * wpb) {
    const int f = ginfo[3 * g], c = ginfo[3 * g + 1];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = lane; i < c; i += kWave) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double x = spos[3 * (int64_t)(f + i) + k];
        lo[k] = fmin(lo[k], x);
        hi[k] = fmax(hi[k], x);
      }
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        lo[k] = fmin(lo[k], shfl_xor_d(lo[k], d));
        hi[k] = fmax(hi[k], shfl_xor_d(hi[k], d));
      }
    if (lane < 3) {
      gbox[6 * (int64_t)g + lane] = lo[lane];
      gbox[6 * (int64_t)g + 3 + lane] = hi[lane];
    }
  }
}

__global__ void k_reset_force_counters(DevInfo *info) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    info->queue = 0;
    info->queue2 = 0;
    info->far_chunks = 0;
    info->near_chunks = 0;
    info->interactions = 0;
    info->list_entries = 0;
    info->max_list = 0;
    info->theta_fallback = 0;
    info->node_visits = 0;
    info->near_entries = 0;
    info->err &= ~kErrPool;
    for (int x = 0; x < 8; ++x) {
      info->xq[x * kLineInts] = 0;
      info->fq[x * kLineInts] = 0;
    }
  }
}

inline unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace



void make_groups_device(GroupBuffers &B, hipStream_t s) {
  const int64_t n = B.n;
  fill_i32(B.gflag, 0, n, s);
  const int64_t span = n > B.nsys ? n : B.nsys;
  if (span > 0)
    k_group_mark<<<blocks_for(span), 256, 0, s>>>(B.level, B.ccount, B.cfc, B.nchild, B.nodes, B.sys, B.nsys, n,
                                                   B.n_crit, B.gflag, B.glen, B.info);
  scan_exclusive_i32(B.gflag, B.gidx, n, &B.info->n_groups, B.scan_tmp, s);
  if (n > 0) {
    k_group_scatter<<<blocks_for(n), 256, 0, s>>>(B.gflag, B.gidx, B.glen, B.sys, B.nsys, n, B.ginfo);
    k_group_box<<<(unsigned)(B.num_cu * 8), 256, 0, s>>>(B.ginfo, B.spos, B.info, B.gbox);
  }
  k_reset_force_counters<<<1, 64, 0, s>>>(B.info);
}

void reset_force_counters(DevInfo *info, hipStream_t s) { k_reset_force_counters<<<1, 64, 0, s>>>(info); }
void reset_list_counters(DevInfo *info, hipStream_t s) { k_reset_force_counters<<<1, 64, 0, s>>>(info); }

}  // namespace bh
