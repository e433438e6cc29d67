// Fused group walk + force sum (Fig. "treewalk" for a group, Eq. 1/2/3).
//
// One wavefront per group, persistent grid pulling groups from an atomic
// queue.  The wave walks the tree in batches of up to 64 nodes taken from a
// stack of slot ranges (a cell's children occupy consecutive slots) kept in
// LDS.  Each lane tests one node with the FP64 opening test
// d^2 > (l/theta + s)^2, d = distance from the cell's centre of mass to the
// group's bounding box.  Accepted cells and reached particles are appended to
// LDS lists as FP32 (x - c_g, m) with c_g the box centre; entries close to the
// box also keep the FP32 rounding residue of x - c_g (the near list), so that
// dx is exact to FP32 for close pairs however large the group.  Opened cells
// push their child range.  When a list is nearly full the whole wave sums
// Eq. (1) over it: lanes hold group members (K per lane, R lane partitions each
// taking every R-th entry, chosen per group to keep lanes busy); a lane
// computes dx, r^2 = |dx|^2 + eps^2 (FMA), v_rsq_f32, and accumulates m r^-3 dx
// and m r^-1.  Partial sums are folded into FP64 after every flush.  The
// member's own entry contributes 0 force and m_i/eps potential, removed at the
// end.
//
// Stack bound: a batch pops up to 64 nodes and pushes at most one range per
// node.  While the stack is high, the wave takes only the top range (at most 8
// cells), which is a depth-first walk: at most 8 ranges per level above the
// point where it started, at most 23 levels.  Batches of 64 are taken only
// while at least 64 + 8 * 24 free entries remain, so the stack never exceeds
// its capacity; an overflow check still guards every push, and an iteration
// budget (a tree visits each slot once) bounds the walk of every group.
#include "bh_device.h"

namespace bh {

namespace {

constexpr int kFar = 256;         // far-list entries staged per flush (FP32 x - c_g, m)
constexpr int kNear = 128;        // near-list entries per flush (hi and lo parts)
constexpr int kStack = 512;       // range stack entries
constexpr int kReserve = 8 * 24;  // growth bound of the stack in one-range mode
constexpr int kMaxK = 4;          // group members per lane
// An entry is "near" when its distance to the group's box is at most
// kNearFrac times the box half-diagonal R.  Near entries keep the FP32
// rounding residue of x - c_g, so dx is exact to FP32 for close pairs; a far
// entry has r >= kNearFrac R and |x - c_g| <= r + 2R, so its dx carries a
// relative rounding error of at most (1 + 3 / kNearFrac) 2^-24.
constexpr double kNearFrac = 0.1;

// The block is one wavefront: a barrier orders its LDS writes and reads.
__device__ __forceinline__ void wave_sync() { __syncthreads(); }

struct WalkArgs {
  const NodeRec *nodes;
  const int32_t *ginfo;
  const double *gbox;
  const double *spos;
  const double *smass;
  const int32_t *perm;
  const SysInfo *sys;
  const SysParam *par;
  const float *theta_group;
  float *acc;
  float *pot;
  int32_t *glist;
  double *gmass;
  DevInfo *info;
  int nsys;
};

struct Members {
  float x[kMaxK], y[kMaxK], z[kMaxK];     // FP32 x_i - c_g
  float lx[kMaxK], ly[kMaxK], lz[kMaxK];  // rounding residue of x_i - c_g
  float ax[kMaxK], ay[kMaxK], az[kMaxK], pt[kMaxK];
  double dx[kMaxK], dy[kMaxK], dz[kMaxK], dp[kMaxK];
};

// One term of Eq. (1): dx = x_j - x_i, r^2 = |dx|^2 + eps^2,
// acc += m r^-3 dx, pt += m r^-1 (the potential is -pt).
__device__ __forceinline__ void term(Members &M, int p, float dx, float dy, float dz, float m, float eps2) {
  float r2 = __builtin_fmaf(dx, dx, eps2);
  r2 = __builtin_fmaf(dy, dy, r2);
  r2 = __builtin_fmaf(dz, dz, r2);
  const float ri = __builtin_amdgcn_rsqf(r2);
  const float mr = m * ri;
  const float ri2 = ri * ri;
  const float mr3 = mr * ri2;
  M.ax[p] = __builtin_fmaf(mr3, dx, M.ax[p]);
  M.ay[p] = __builtin_fmaf(mr3, dy, M.ay[p]);
  M.az[p] = __builtin_fmaf(mr3, dz, M.az[p]);
  M.pt[p] += mr;
}

template <int K>
__device__ __forceinline__ void far_entry(Members &M, const float4 e, float eps2) {
#pragma unroll
  for (int p = 0; p < K; ++p) term(M, p, e.x - M.x[p], e.y - M.y[p], e.z - M.z[p], e.w, eps2);
}

template <int K>
__device__ __forceinline__ void near_entry(Members &M, const float4 h, const float4 l, float eps2) {
#pragma unroll
  for (int p = 0; p < K; ++p)
    term(M, p, (h.x - M.x[p]) + (l.x - M.lx[p]), (h.y - M.y[p]) + (l.y - M.ly[p]), (h.z - M.z[p]) + (l.z - M.lz[p]),
         h.w, eps2);
}

template <int K>
__device__ __forceinline__ void fold(Members &M) {
#pragma unroll
  for (int p = 0; p < K; ++p) {
    M.dx[p] += (double)M.ax[p];
    M.dy[p] += (double)M.ay[p];
    M.dz[p] += (double)M.az[p];
    M.dp[p] += (double)M.pt[p];
    M.ax[p] = M.ay[p] = M.az[p] = M.pt[p] = 0.0f;
  }
}

// Partition `part` of R sums entries part, part + R, part + 2R, ... < nent.
template <int K>
__device__ __forceinline__ void sum_far(Members &M, const float4 *__restrict__ tile, int nent, int R, int part,
                                        float eps2) {
  const int full = nent / R;
  int t = 0;
  for (; t + 1 < full; t += 2) {
    const float4 e0 = tile[t * R + part], e1 = tile[(t + 1) * R + part];
    far_entry<K>(M, e0, eps2);
    far_entry<K>(M, e1, eps2);
  }
  if (t < full) far_entry<K>(M, tile[t * R + part], eps2);
  if (part < nent - full * R) far_entry<K>(M, tile[full * R + part], eps2);
  fold<K>(M);
}

template <int K>
__device__ __forceinline__ void sum_near(Members &M, const float4 *__restrict__ hi, const float4 *__restrict__ lo,
                                         int nent, int R, int part, float eps2) {
  const int full = nent / R;
  int t = 0;
  for (; t + 1 < full; t += 2) {
    const int j0 = t * R + part, j1 = (t + 1) * R + part;
    const float4 h0 = hi[j0], l0 = lo[j0], h1 = hi[j1], l1 = lo[j1];
    near_entry<K>(M, h0, l0, eps2);
    near_entry<K>(M, h1, l1, eps2);
  }
  if (t < full) near_entry<K>(M, hi[t * R + part], lo[t * R + part], eps2);
  if (part < nent - full * R) near_entry<K>(M, hi[full * R + part], lo[full * R + part], eps2);
  fold<K>(M);
}

__device__ __forceinline__ void flush_far(int K, Members &M, const float4 *tile, int nent, int R, int part,
                                          float eps2) {
  switch (K) {
    case 1: sum_far<1>(M, tile, nent, R, part, eps2); break;
    case 2: sum_far<2>(M, tile, nent, R, part, eps2); break;
    case 3: sum_far<3>(M, tile, nent, R, part, eps2); break;
    default: sum_far<4>(M, tile, nent, R, part, eps2); break;
  }
}

__device__ __forceinline__ void flush_near(int K, Members &M, const float4 *hi, const float4 *lo, int nent, int R,
                                           int part, float eps2) {
  switch (K) {
    case 1: sum_near<1>(M, hi, lo, nent, R, part, eps2); break;
    case 2: sum_near<2>(M, hi, lo, nent, R, part, eps2); break;
    case 3: sum_near<3>(M, hi, lo, nent, R, part, eps2); break;
    default: sum_near<4>(M, hi, lo, nent, R, part, eps2); break;
  }
}

// Lane layout for a group of c members: R partitions of W = 64/R lanes, K
// members per lane, maximising the busy fraction c R / (64 K).
__device__ __forceinline__ void choose_layout(int c, int &K, int &R) {
  K = (c + kWave - 1) / kWave;
  R = 1;
  for (int r = 2; r <= kWave; r <<= 1) {
    const int W = kWave / r;
    const int k = (c + W - 1) / W;
    if (k > kMaxK) break;
    if (r * K > R * k) {
      R = r;
      K = k;
    }
  }
}

__global__ __launch_bounds__(kWave) void k_walk_force(WalkArgs a) {
  __shared__ int2 stk[kStack];
  __shared__ float4 tile[kFar];
  __shared__ float4 nhi[kNear], nlo[kNear];
  __shared__ int mark[kWave];
  const int lane = lane_id();
  const int G = a.info->n_groups;
  const int nslots = a.nsys + a.info->n_slots;

  for (;;) {
    // Every lane executes the atomic (lane 0 adds 1, the others 0) so that no
    // divergent branch precedes the broadcast: a divergent branch at the top
    // of this loop lets the compiler split the wave, with lanes re-entering
    // the loop without lane 0.
    const int t = atomicAdd(&a.info->queue, lane == 0 ? 1 : 0);
    const int g = __builtin_amdgcn_readfirstlane(t);  // all lanes active: lane 0's value
    if (g >= G) break;

    const int gf = a.ginfo[3 * g], gc = a.ginfo[3 * g + 1], gs = a.ginfo[3 * g + 2];
    double blo[3], bhi[3], cen[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      blo[k] = a.gbox[6 * (int64_t)g + k];
      bhi[k] = a.gbox[6 * (int64_t)g + 3 + k];
      cen[k] = __dmul_rn(__dadd_rn(blo[k], bhi[k]), 0.5);
    }
    const SysParam &S = a.par[gs];
    double theta = a.theta_group ? (double)a.theta_group[g] : S.theta;
    if (!(theta >= 0.0 && theta <= 1.0)) {
      if (lane == 0) atomicOr(&a.info->err, kErrTheta);
      theta = (theta > 1.0) ? 1.0 : 0.0;
    }
    const float eps2 = (float)(S.eps * S.eps);
    const double half_diag = 0.5 * sqrt(__dadd_rn(__dadd_rn(__dmul_rn(bhi[0] - blo[0], bhi[0] - blo[0]),
                                                            __dmul_rn(bhi[1] - blo[1], bhi[1] - blo[1])),
                                                   __dmul_rn(bhi[2] - blo[2], bhi[2] - blo[2])));
    const double near2 = (kNearFrac * half_diag) * (kNearFrac * half_diag);

    int K, R;
    choose_layout(gc, K, R);
    const int W = kWave / R;
    const int part = lane / W, u = lane % W;

    Members M;
#pragma unroll
    for (int p = 0; p < kMaxK; ++p) {
      const int i = u + W * p;
      double rx = 0.0, ry = 0.0, rz = 0.0;
      if (p < K && i < gc) {
        const double *q = a.spos + 3 * (int64_t)(gf + i);
        rx = __dsub_rn(q[0], cen[0]);
        ry = __dsub_rn(q[1], cen[1]);
        rz = __dsub_rn(q[2], cen[2]);
      }
      M.x[p] = (float)rx; M.y[p] = (float)ry; M.z[p] = (float)rz;
      M.lx[p] = (float)__dsub_rn(rx, (double)M.x[p]);
      M.ly[p] = (float)__dsub_rn(ry, (double)M.y[p]);
      M.lz[p] = (float)__dsub_rn(rz, (double)M.z[p]);
      M.ax[p] = M.ay[p] = M.az[p] = M.pt[p] = 0.0f;
      M.dx[p] = M.dy[p] = M.dz[p] = M.dp[p] = 0.0;
    }

    // ---- walk ----
    int sp = 1, tc = 0, nc = 0, nlist = 0;
    bool overflow = false;
    // every batch takes at least one node or pops an empty range, and a tree
    // visits each slot at most once: more iterations mean a corrupt tree
    int budget = 2 * nslots + 2;
    double lmass = 0.0;
    if (lane == 0) stk[0] = make_int2(gs, 1);
    wave_sync();
    while (sp > 0) {
      if (--budget < 0) {
        overflow = true;
        break;
      }
      const bool starved = sp > kStack - kWave - kReserve;
      const int nread = starved ? 1 : min(sp, kWave);
      int2 e = make_int2(0, 0);
      if (lane < nread) e = stk[sp - 1 - lane];
      const int cnt = (lane < nread) ? e.y : 0;
      const int pre = wave_inclusive_sum(cnt);
      const int total = __shfl(pre, nread - 1, kWave);
      const int B = min(starved ? 8 : kWave, total);
      const int start = pre - cnt;
      const int kfull = __popcll(__ballot(lane < nread && pre <= B));
      mark[lane] = -1;
      wave_sync();
      if (lane < nread && start < B) mark[start] = lane;
      wave_sync();
      const int ei = wave_inclusive_max(mark[lane]);
      const int e_start = __shfl(start, ei < 0 ? 0 : ei, kWave);
      const int e_first = __shfl(e.x, ei < 0 ? 0 : ei, kWave);
      int nsp = sp - kfull;
      if (kfull < nread) {
        const int pstart = __shfl(start, kfull, kWave);
        if (pstart < B && lane == kfull) stk[sp - 1 - kfull] = make_int2(e.x + (B - pstart), e.y - (B - pstart));
      }
      bool emit = false, push = false, near = false;
      float4 ent = make_float4(0.f, 0.f, 0.f, 0.f), lo4 = ent;
      int2 rng = make_int2(0, 0);
      const int node = e_first + (lane - e_start);
      if (__ballot(lane < B && (node < 0 || node >= nslots))) {
        overflow = true;  // corrupt range: report, never read out of bounds
        break;
      }
      if (lane < B) {
        const NodeRec r = a.nodes[node];
        // squared distance from the centre of mass to the group's box
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double below = __dsub_rn(blo[k], r.com[k]);
          const double above = __dsub_rn(r.com[k], bhi[k]);
          const double ek = fmax(0.0, fmax(below, above));
          d2 = (k == 0) ? __dmul_rn(ek, ek) : __dadd_rn(d2, __dmul_rn(ek, ek));
        }
        if (r.child < 0) {
          emit = true;  // a particle
        } else {
          // Eq. (2)/(3): far enough iff d^2 > (l/theta + s)^2
          double q = r.l / theta;
          q = __dadd_rn(q, r.s);
          const double seff = __dmul_rn(q, q);
          if (d2 > seff) emit = true;
          else push = true;
        }
        if (emit) {
          const double rx = __dsub_rn(r.com[0], cen[0]), ry = __dsub_rn(r.com[1], cen[1]),
                       rz = __dsub_rn(r.com[2], cen[2]);
          ent = make_float4((float)rx, (float)ry, (float)rz, (float)r.m);
          near = d2 <= near2;
          if (near)
            lo4 = make_float4((float)__dsub_rn(rx, (double)ent.x), (float)__dsub_rn(ry, (double)ent.y),
                              (float)__dsub_rn(rz, (double)ent.z), 0.0f);
          lmass += r.m;
        }
        if (push) rng = make_int2(r.child, r.nchild);
      }
      const unsigned long long em = __ballot(emit), pm = __ballot(push);
      const int npush = __popcll(pm);
      if (nsp + npush > kStack) {
        overflow = true;
        break;
      }
      const unsigned long long nm = __ballot(emit && near), fm = em & ~nm;
      if (emit && !near) tile[tc + rank_below(fm)] = ent;
      if (emit && near) {
        nhi[nc + rank_below(nm)] = ent;
        nlo[nc + rank_below(nm)] = lo4;
      }
      if (push) stk[nsp + rank_below(pm)] = rng;
      wave_sync();
      tc += __popcll(fm);
      nc += __popcll(nm);
      nlist += __popcll(em);
      sp = nsp + npush;
      if (tc > kFar - kWave) {
        flush_far(K, M, tile, tc, R, part, eps2);
        wave_sync();
        tc = 0;
      }
      if (nc > kNear - kWave) {
        flush_near(K, M, nhi, nlo, nc, R, part, eps2);
        wave_sync();
        nc = 0;
      }
    }
    if (overflow) {
      if (lane == 0) atomicOr(&a.info->err, kErrStack);
      continue;
    }
    // what is left of both lists
    if (tc > 0) flush_far(K, M, tile, tc, R, part, eps2);
    if (nc > 0) flush_near(K, M, nhi, nlo, nc, R, part, eps2);
    wave_sync();

    // ---- reduce partitions, remove the self term, write in input order ----
    const float self_ri = __builtin_amdgcn_rsqf(__builtin_fmaf(0.0f, 0.0f, eps2));
#pragma unroll
    for (int p = 0; p < kMaxK; ++p) {
      if (p >= K) break;
      double vx = M.dx[p], vy = M.dy[p], vz = M.dz[p], vp = M.dp[p];
      for (int b = W; b < kWave; b <<= 1) {
        vx += shfl_xor_d(vx, b);
        vy += shfl_xor_d(vy, b);
        vz += shfl_xor_d(vz, b);
        vp += shfl_xor_d(vp, b);
      }
      const int i = u + W * p;
      if (part == 0 && i < gc) {
        const float mi = (float)a.smass[gf + i];
        const double self = (double)(mi * self_ri);
        const int o = a.perm[gf + i];
        a.acc[3 * (int64_t)o] = (float)vx;
        a.acc[3 * (int64_t)o + 1] = (float)vy;
        a.acc[3 * (int64_t)o + 2] = (float)vz;
        a.pot[o] = (float)(self - vp);
      }
    }
    // list statistics
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) lmass += shfl_xor_d(lmass, d);
    if (lane == 0) {
      a.glist[g] = nlist;
      a.gmass[g] = lmass;
      atomicAdd(&a.info->interactions, (unsigned long long)gc * (unsigned long long)(nlist - 1));
      atomicAdd(&a.info->list_entries, (unsigned long long)nlist);
      atomicMax(&a.info->max_list, nlist);
    }
  }
}

}  // namespace



void walk_force_device(const WalkLaunch &L, hipStream_t s) {
  WalkArgs a{L.nodes, L.ginfo, L.gbox, L.spos, L.smass, L.perm, L.sys, L.par, L.theta_group,
             L.acc, L.pot, L.glist, L.gmass, L.info, L.nsys};
  k_walk_force<<<(unsigned)L.grid, kWave, 0, s>>>(a);
}

}  // namespace bh
