// Per-particle tree walk: the paper's own GPU form (Fig. "treegpu", the
// threaded tree of Sec. 3.4), where each particle walks the tree by itself
// and sums its forces on the way, with no shared list.
//
// Threading: every node gets a "next" pointer, the node that follows its
// subtree in depth-first pre-order (its next sibling, or the next of its
// parent for a last child; -1 after a system's root), while "more" is the
// first child.  A cell's children occupy consecutive slots, so the next of a
// child that is not the last is the slot after it; the rest are resolved by
// pointer jumping (each round halves the remaining chains; the tree is at
// most 23 levels deep).
//
// Walk: one lane per particle, in Morton order so that the lanes of a wave
// walk nearby paths (the cache behaviour the paper measures).  The opening
// test is the group test with the group reduced to the particle (a point
// box): d^2 = |com - x_i|^2 (FP64) against (l/theta + s)^2 (Eq. 2/3), so the
// lists this walk sums are those of one-particle groups.  A lane's own
// particle is skipped.  Terms are summed in FP32 from the FP64 relative
// vector (x_j - x_i rounded once), folded into FP64 every kFold terms.
#include "bh_device.h"

namespace bh {

namespace {

constexpr int kJumpRounds = 6;  // 2^6 > 23 levels
constexpr int kFold = 64;       // FP32 terms between FP64 folds

// next[] encoding before resolution: >= 0 a slot, -1 the end, <= -2 "the
// next of slot -(x + 2)".
__global__ void k_pp_links(const NodeRec *__restrict__ nodes, int nslots, int nsys, int32_t *__restrict__ nxt) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nslots) return;
  if (v < nsys) nxt[v] = -1;  // a system's root: its walk ends after it
  const NodeRec &r = nodes[v];
  if (r.child < 0) return;
  const int c0 = r.child, c1 = r.child + r.nchild;
  for (int k = c0; k < c1; ++k) {
    if (k < 0 || k >= nslots) break;
    nxt[k] = (k + 1 < c1) ? k + 1 : -(v + 2);
  }
}

__global__ void k_pp_jump(int nslots, int32_t *__restrict__ nxt) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nslots) return;
  const int x = nxt[v];
  if (x <= -2) {
    const int p = -(x + 2);
    nxt[v] = (p >= 0 && p < nslots) ? nxt[p] : -1;
  }
}

struct Acc {
  float ax = 0.f, ay = 0.f, az = 0.f, pt = 0.f;
  double dx = 0.0, dy = 0.0, dz = 0.0, dp = 0.0;
  int since = 0;
};

__device__ __forceinline__ void fold(Acc &A) {
  A.dx += (double)A.ax;
  A.dy += (double)A.ay;
  A.dz += (double)A.az;
  A.dp += (double)A.pt;
  A.ax = A.ay = A.az = A.pt = 0.f;
  A.since = 0;
}

__global__ __launch_bounds__(kWave) void k_pp_forces(const NodeRec *__restrict__ nodes,
                                                     const int32_t *__restrict__ nxt, int nslots,
                                                     const SysInfo *__restrict__ sys, int nsys,
                                                     const SysParam *__restrict__ par,
                                                     const double *__restrict__ spos,
                                                     const int32_t *__restrict__ perm, int64_t n,
                                                     float *__restrict__ acc, float *__restrict__ pot,
                                                     DevInfo *__restrict__ info) {
  const int64_t i64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i64 < n;
  const int i = live ? (int)i64 : 0;
  // a lane's list, as the one-particle group would hold it: the entries taken
  // plus its own particle when the walk reaches it (not an interaction)
  unsigned long long entries = 0;
  int len = 0;
  if (live) {
    const int s = system_of(sys, nsys, i);
    const double x0 = spos[3 * (int64_t)i], x1 = spos[3 * (int64_t)i + 1], x2 = spos[3 * (int64_t)i + 2];
    const double eps = par[s].eps;
    const float eps2 = (float)(eps * eps);
    double theta = par[s].theta;
    // l / theta = (side / theta) * 2^-level exactly, as in the group walk
    const double side = sys[s].side;
    const double side_theta = side / theta;
    const int side_exp = ilogb(side);
    Acc A;
    int v = s;
    int guard = 2 * nslots + 4;
    while (v >= 0) {
      if (--guard < 0 || v >= nslots) {
        atomicOr(&info->err, kErrStack);
        break;
      }
      const NodeRec r = nodes[v];
      const int skip = nxt[v];  // loaded with the record, not after it
      bool take;
      int next;
      if (r.child < 0) {
        take = r.first != i;  // a particle; the lane's own is skipped
        if (!take) ++len;
        next = skip;
      } else {
        // squared distance from the centre of mass to the particle (the
        // group test with a point box)
        double d2 = 0.0;
        const double xs[3] = {x0, x1, x2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double ek = fmax(0.0, fmax(__dsub_rn(xs[k], r.com[k]), __dsub_rn(r.com[k], xs[k])));
          d2 = (k == 0) ? __dmul_rn(ek, ek) : __dadd_rn(d2, __dmul_rn(ek, ek));
        }
        double q = isfinite(r.l) ? ldexp(side_theta, ilogb(r.l) - side_exp) : r.l;
        q = __dadd_rn(q, r.s);
        take = d2 > __dmul_rn(q, q);
        next = take ? skip : r.child;
      }
      if (take) {
        const float dx = (float)__dsub_rn(r.com[0], x0), dy = (float)__dsub_rn(r.com[1], x1),
                    dz = (float)__dsub_rn(r.com[2], x2);
        float q = __builtin_fmaf(dx, dx, eps2);
        q = __builtin_fmaf(dy, dy, q);
        q = __builtin_fmaf(dz, dz, q);
        const float ri = __builtin_amdgcn_rsqf(q);
        const float mr = (float)r.m * ri;
        const float f = mr * (ri * ri);
        A.ax = __builtin_fmaf(f, dx, A.ax);
        A.ay = __builtin_fmaf(f, dy, A.ay);
        A.az = __builtin_fmaf(f, dz, A.az);
        A.pt += mr;
        ++len;
        if (++A.since == kFold) fold(A);
      }
      if (next <= -2) {  // an unresolved thread pointer: report, never walk on
        atomicOr(&info->err, kErrStack);
        break;
      }
      v = next;
    }
    fold(A);
    const int o = perm[i];
    acc[3 * (int64_t)o] = (float)A.dx;
    acc[3 * (int64_t)o + 1] = (float)A.dy;
    acc[3 * (int64_t)o + 2] = (float)A.dz;
    pot[o] = (float)(-A.dp);
  }
  // interactions: list length - 1 per particle (the own entry is not one)
  unsigned long long inter = live ? (unsigned long long)max(len - 1, 0) : 0ull;
  entries = live ? (unsigned long long)len : 0ull;
  int longest = live ? len : 0;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    inter += __shfl_xor(inter, d, kWave);
    entries += __shfl_xor(entries, d, kWave);
    longest = max(longest, __shfl_xor(longest, d, kWave));
  }
  if (lane_id() == 0 && entries) {
    atomicAdd(&info->interactions, inter);
    atomicAdd(&info->list_entries, entries);
    atomicMax(&info->max_list, longest);
  }
}

inline unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void particle_forces_device(const NodeRec *nodes, int nslots, int nsys, const SysInfo *sys, const SysParam *par,
                            const double *spos, const int32_t *perm, int64_t n, int32_t *nxt, float *acc,
                            float *pot, DevInfo *info, hipStream_t s) {
  if (nslots <= 0) return;
  k_pp_links<<<blocks_of(nslots, 256), 256, 0, s>>>(nodes, nslots, nsys, nxt);
  for (int r = 0; r < kJumpRounds; ++r) k_pp_jump<<<blocks_of(nslots, 256), 256, 0, s>>>(nslots, nxt);
  if (n > 0)
    k_pp_forces<<<blocks_of(n, kWave), kWave, 0, s>>>(nodes, nxt, nslots, sys, nsys, par, spos, perm, n, acc, pot,
                                                      info);
}

}  // namespace bh
