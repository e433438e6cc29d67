// Neighbour search and SPH density: the general treewalk of Sec. 3.3 (Fig.
// "general_treewalk") applied to a short-range interaction, as in smoothed
// particle hydrodynamics, the application the paper names.
//
// The neighbours of particle i are the particles j != i with |x_j - x_i| <
// h_i, its own search radius (the "gather" form).  The walk is the group form
// used for gravity: one wavefront per group, persistent grid pulling groups
// from an atomic queue, up to 64 nodes tested per iteration from a stack of
// slot ranges in LDS.  The distance test of the general walk prunes a cell
// whose particles all lie farther than the group's largest radius from the
// group's bounding box: every particle of a cell lies within
// (sqrt(3)/2) l + s of its centre of mass (l the cube side, s the distance of
// the centre of mass from the cube's centre).  A particle leaf within that
// radius of the box is a candidate; candidates collect in LDS and are
// tested against every member, one member per lane, in FP64 with the
// squared distance (dx^2 + dy^2) + dz^2 rounded as written, so the decision
// r^2 < h_i^2 is the same as a plain CPU evaluation.  A candidate's index,
// position and mass go to LDS from the node record its lane just read, so
// the member loop reads them as LDS broadcasts.  The pruning bounds
// carry margins far above FP64 rounding; they only skip work, the per-pair
// test decides.
//
// The SPH density sums m_j W(r_ij, h_i) over the neighbours, plus the
// particle's own m_i W(0, h_i), with the cubic spline kernel of Monaghan and
// Lattanzio with compact support h (the paper fixes no kernel).  Lists, when
// asked for, hold the input indices of the neighbours in walk order.
#include "bh_device.h"

namespace bh {

namespace {

constexpr int kNbStack = 512;                    // range stack entries
constexpr int kNbReserve = 8 * 24;               // growth bound in one-range mode
constexpr int kNbCand = 128;                     // candidate buffer
constexpr double kHalfSqrt3 = 0.86602540378443865;

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

__device__ __forceinline__ double sph_w(double r, double h) {
  const double q = r / h;
  const double sigma = 8.0 / (3.14159265358979323846 * h * h * h);
  if (q < 0.5) return sigma * (1.0 - 6.0 * q * q + 6.0 * q * q * q);
  if (q < 1.0) {
    const double u = 1.0 - q;
    return sigma * 2.0 * u * u * u;
  }
  return 0.0;
}

__global__ void k_nb_reset(DevInfo *info) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    info->queue = 0;
    info->nb_pairs = 0;
    info->nb_tests = 0;
  }
}

// Candidates staged in LDS: sorted index, position and mass (taken from the
// particle's node record by the lane that accepted it).
struct alignas(16) CandRec {
  double x, y, z, m;
};
struct Cand {
  CandRec c[kNbCand];
  int j[kNbCand];
};

// One member against one staged candidate.
__device__ __forceinline__ void test_pair(const NeighborArgs &a, const CandRec &q, int j, int i, bool live, double x0,
                                          double x1, double x2, double h, double h2, int64_t ob, int64_t lb, int &c,
                                          double &r) {
  const double dx = __dsub_rn(q.x, x0);
  const double dy = __dsub_rn(q.y, x1);
  const double dz = __dsub_rn(q.z, x2);
  const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  if (live && j != i && r2 < h2) {
    if (a.rho) r = __dadd_rn(r, __dmul_rn(q.m, sph_w(sqrt(r2), h)));
    if (a.nbr && c < lb) a.nbr[ob + c] = a.perm[j];
    ++c;
  }
}

// Tests the ncand staged candidates against every member block.
template <int kNbBlocks>
__device__ __forceinline__ void flush(const NeighborArgs &a, const Cand &cd, int ncand, int gf, int gc, int nb,
                                      int lane, const double (&hb)[kNbBlocks], int (&cb)[kNbBlocks],
                                      double (&rb)[kNbBlocks], const int64_t (&ob)[kNbBlocks],
                                      const int64_t (&lb)[kNbBlocks], unsigned long long &tests) {
#pragma unroll
  for (int b = 0; b < kNbBlocks; ++b) {
    if (b < nb) {
      const int i = gf + b * kWave + lane;
      const bool live = i < gf + gc;
      double x0 = 0.0, x1 = 0.0, x2 = 0.0;
      if (live) {
        x0 = a.spos[3 * (int64_t)i];
        x1 = a.spos[3 * (int64_t)i + 1];
        x2 = a.spos[3 * (int64_t)i + 2];
      }
      const double h = hb[b];
      const double h2 = __dmul_rn(h, h);
      int c = cb[b];
      double r = rb[b];
      for (int k = 0; k < ncand; ++k) test_pair(a, cd.c[k], cd.j[k], i, live, x0, x1, x2, h, h2, ob[b], lb[b], c, r);
      if (live) tests += (unsigned long long)ncand;
      cb[b] = c;
      rb[b] = r;
    }
  }
}

// kNbBlocks: member blocks of 64 held per lane (the largest group / 64),
// chosen by the host from the grouping so that small groups keep registers
// free.
template <int kNbBlocks>
__global__ __launch_bounds__(kWave) void k_neighbors(NeighborArgs a) {
  __shared__ int2 stk[kNbStack];
  __shared__ Cand cd;
  __shared__ int mark[kWave];
  const int lane = lane_id();
  const int G = a.info->n_groups;
  const int nslots = a.nsys + a.info->n_slots;
  unsigned long long pairs = 0, tests = 0;
  for (;;) {
    const int g = take_one(&a.info->queue, lane);
    if (g >= G) break;
    const int gf = a.ginfo[3 * g], gc = a.ginfo[3 * g + 1], gs = a.ginfo[3 * g + 2];
    const int nb = min((gc + kWave - 1) / kWave, kNbBlocks);
    if ((gc + kWave - 1) / kWave > kNbBlocks || gs < 0 || gs >= a.nsys) {
      if (lane == 0) atomicOr(&a.info->err, kErrStack);
      continue;
    }
    // members: radii, the group's largest, output offsets
    double hb[kNbBlocks], rb[kNbBlocks];
    int cb[kNbBlocks];
    int64_t ob[kNbBlocks], lb[kNbBlocks];
    double hmax = 0.0;
    bool bad = false;
#pragma unroll
    for (int b = 0; b < kNbBlocks; ++b) {
      const int i = gf + b * kWave + lane;
      const bool live = b < nb && i < gf + gc;
      const int o = live ? a.perm[i] : 0;
      hb[b] = live ? a.h[o] : 1.0;
      if (live && !(hb[b] > 0.0 && hb[b] < INFINITY)) bad = true;
      if (live) hmax = fmax(hmax, hb[b]);
      cb[b] = 0;
      rb[b] = 0.0;
      ob[b] = 0;
      lb[b] = 0;
      if (live && a.offsets) {
        ob[b] = a.offsets[o];
        lb[b] = a.offsets[o + 1] - ob[b];
      }
    }
    if (__ballot(bad)) {
      if (lane == 0) atomicOr(&a.info->err, kErrRadius);
      continue;
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) hmax = fmax(hmax, shfl_xor_d(hmax, d));
    // the group's box, widened by a margin above the rounding of the
    // distance sums, and the largest radius with a relative margin: a
    // neighbour of any member lies within rad of the box (a rounded box,
    // not the box grown into a cube)
    double elo[3], ehi[3], cpad = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double lo = a.gbox[6 * (int64_t)g + k], hi = a.gbox[6 * (int64_t)g + 3 + k];
      const double pad = 1e-15 * fmax(fabs(lo), fabs(hi)) + 1e-300;
      elo[k] = lo - pad;
      ehi[k] = hi + pad;
      cpad += pad;
    }
    const double rad = hmax * (1.0 + 1e-9) + cpad;

    int sp = 1, ncand = 0;
    if (lane == 0) stk[0] = make_int2(gs, 1);
    wave_sync();
    int budget = 4 * nslots + 4;
    while (sp > 0) {
      if (--budget < 0) {
        if (lane == 0) atomicOr(&a.info->err, kErrStack);
        break;
      }
      // take up to 64 nodes from the top ranges (one range while the stack
      // is high: then the walk is depth first and the stack stays bounded)
      const bool starved = sp > kNbStack - kWave - kNbReserve;
      const int nread = starved ? 1 : min(sp, kWave);
      int2 e = make_int2(0, 0);
      if (lane < nread) e = stk[sp - 1 - lane];
      const int cnt = (lane < nread) ? e.y : 0;
      const int pre = wave_inclusive_sum(cnt);
      const int total = __shfl(pre, nread - 1, kWave);
      const int take = min(starved ? 8 : kWave, total);
      const int start = pre - cnt;
      const int kfull = __popcll(__ballot(lane < nread && pre <= take));
      mark[lane] = -1;
      wave_sync();
      if (lane < nread && start < take) mark[start] = lane;
      wave_sync();
      const int ei = wave_inclusive_max(mark[lane]);
      const int e_start = __shfl(start, ei < 0 ? 0 : ei, kWave);
      const int e_first = __shfl(e.x, ei < 0 ? 0 : ei, kWave);
      if (kfull < nread) {
        const int pstart = __shfl(start, kfull, kWave);
        if (pstart < take && lane == kfull)
          stk[sp - 1 - kfull] = make_int2(e.x + (take - pstart), e.y - (take - pstart));
      }
      sp -= kfull;
      const int node = e_first + (lane - e_start);
      if (__ballot(lane < take && (node < 0 || node >= nslots))) {
        if (lane == 0) atomicOr(&a.info->err, kErrStack);
        break;
      }
      bool push = false, is_cand = false;
      int2 rng = make_int2(0, 0);
      int j = 0;
      double px = 0.0, py = 0.0, pz = 0.0, pm = 0.0;
      if (lane < take) {
        const NodeRec r = a.nodes[node];
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double ek = fmax(0.0, fmax(elo[k] - r.com[k], r.com[k] - ehi[k]));
          d2 += ek * ek;
        }
        if (r.child < 0) {
          is_cand = r.count > 0 && d2 <= rad * rad;  // a particle within rad of the box
          j = r.first;
          px = r.com[0];
          py = r.com[1];
          pz = r.com[2];
          pm = r.m;
        } else {
          // every particle of the cell lies within R of its centre of mass
          const double R = (kHalfSqrt3 * r.l + r.s) * (1.0 + 1e-9) + rad;
          push = !(d2 > R * R);
          rng = make_int2(r.child, r.nchild);
        }
      }
      const unsigned long long pmask = __ballot(push), cm = __ballot(is_cand);
      const int npush = __popcll(pmask), nc = __popcll(cm);
      wave_sync();
      if (sp + npush > kNbStack) {
        if (lane == 0) atomicOr(&a.info->err, kErrStack);
        break;
      }
      if (push) stk[sp + rank_below(pmask)] = rng;
      if (is_cand) {
        const int q = ncand + rank_below(cm);
        cd.j[q] = j;
        cd.c[q] = CandRec{px, py, pz, pm};
      }
      sp += npush;
      ncand += nc;
      wave_sync();
      if (ncand > kNbCand - kWave) {
        flush<kNbBlocks>(a, cd, ncand, gf, gc, nb, lane, hb, cb, rb, ob, lb, tests);
        ncand = 0;
        wave_sync();
      }
    }
    flush<kNbBlocks>(a, cd, ncand, gf, gc, nb, lane, hb, cb, rb, ob, lb, tests);
    wave_sync();
    // outputs in input order
    bool short_list = false;
#pragma unroll
    for (int b = 0; b < kNbBlocks; ++b) {
      const int i = gf + b * kWave + lane;
      if (b < nb && i < gf + gc) {
        const int o = a.perm[i];
        if (a.count) a.count[o] = cb[b];
        if (a.rho) a.rho[o] = __dadd_rn(__dmul_rn(a.smass[i], sph_w(0.0, hb[b])), rb[b]);
        if (a.offsets && (int64_t)cb[b] != lb[b]) short_list = true;
        pairs += (unsigned long long)cb[b];
      }
    }
    if (__ballot(short_list) && lane == 0) atomicOr(&a.info->err, kErrListSpace);
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    pairs += __shfl_xor(pairs, d, kWave);
    tests += __shfl_xor(tests, d, kWave);
  }
  if (lane == 0 && (pairs || tests)) {
    atomicAdd(&a.info->nb_pairs, pairs);
    atomicAdd(&a.info->nb_tests, tests);
  }
}

}  // namespace

int neighbors_blocks_per_cu(int n_crit) {
  int b = 0;
  hipError_t e;
  if (n_crit <= kWave) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_neighbors<1>, kWave, 0);
  else if (n_crit <= 2 * kWave) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_neighbors<2>, kWave, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_neighbors<BH_MAX_NCRIT / kWave>, kWave, 0);
  if (e != hipSuccess || b < 1) b = 8;
  return b;
}

void neighbors_device(const NeighborArgs &a, int n_crit, int grid, hipStream_t s) {
  k_nb_reset<<<1, 64, 0, s>>>(a.info);
  if (n_crit <= kWave) k_neighbors<1><<<(unsigned)grid, kWave, 0, s>>>(a);
  else if (n_crit <= 2 * kWave) k_neighbors<2><<<(unsigned)grid, kWave, 0, s>>>(a);
  else k_neighbors<BH_MAX_NCRIT / kWave><<<(unsigned)grid, kWave, 0, s>>>(a);
}

}  // namespace bh
