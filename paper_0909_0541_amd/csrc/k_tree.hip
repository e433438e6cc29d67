// Oct-tree construction from sorted Morton keys (Sec. 3.1, 3.5).
//
// Cells are identified without pointer chasing.  For neighbouring sorted keys
// i, i+1 of one system let delta_i be the number of leading octal digits they
// share (21 when equal, -1 across a system boundary).  A "split" at i with
// delta_i = l < 21 separates two sub-cells of the level-l cell holding i; the
// cell is owned by its first split (the last particle of its first sub-cell).
// A run of equal keys is a bucket owned by its first particle.  Every other
// prefix with a single non-empty sub-cell is a chain link, which is skipped:
// it holds the same particles as its only child and, for theta < 2/sqrt(3),
// its opening test never accepts it while rejecting the child.
//
// Per-position arrays (index = Morton position) describe the cell owned
// there.  Node records are then placed in slots: system roots first, the
// children of every cell in consecutive slots in octant order.  Moments are
// summed level by level from the deepest level up, each cell adding its
// children in slot order starting from zero, so the FP64 sums are exactly
// those of a recursive evaluation.
#include <algorithm>

#include "bh_device.h"

namespace bh {

namespace {

// ---------------------------------------------------------------------------
// root cube per system
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_bbox_partial(const double *__restrict__ pos, const SysInfo *__restrict__ sys,
                                                      int bps, double *__restrict__ part, DevInfo *info) {
  __shared__ double red[6][256];
  const int s = blockIdx.x / bps, b = blockIdx.x % bps;
  const int64_t first = sys[s].first, end = first + sys[s].count;
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = first + (int64_t)b * blockDim.x + threadIdx.x; i < end; i += (int64_t)bps * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double x = pos[3 * i + k];
      bad |= !isfinite(x);
      mn[k] = fmin(mn[k], x);
      mx[k] = fmax(mx[k], x);
    }
  }
  if (bad) atomicOr(&info->err, kErrNonFinitePos);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    red[k][threadIdx.x] = mn[k];
    red[3 + k][threadIdx.x] = mx[k];
  }
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * (int64_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_bbox_final(const double *__restrict__ part, int bps, SysInfo *sys) {
  __shared__ double red[6][256];
  const int s = blockIdx.x;
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < bps; b += blockDim.x)
    for (int k = 0; k < 3; ++k) {
      mn[k] = fmin(mn[k], part[6 * ((int64_t)s * bps + b) + k]);
      mx[k] = fmax(mx[k], part[6 * ((int64_t)s * bps + b) + 3 + k]);
    }
  for (int k = 0; k < 3; ++k) {
    red[k][threadIdx.x] = mn[k];
    red[3 + k][threadIdx.x] = mx[k];
  }
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double lo[3], ext = 0.0;
  for (int k = 0; k < 3; ++k) {
    lo[k] = red[k][0];
    const double e = red[3 + k][0] - red[k][0];
    if (e > ext) ext = e;
  }
  if (sys[s].count == 0 || !isfinite(ext)) {
    lo[0] = lo[1] = lo[2] = 0.0;
    ext = 0.0;
  }
  // corner at the per-axis minimum, side = largest extent widened by 2^-20
  const double side = (ext > 0.0) ? __dmul_rn(ext, 1.0 + 0x1p-20) : 1.0;
  for (int k = 0; k < 3; ++k) sys[s].lo[k] = lo[k];
  sys[s].side = side;
  sys[s].scale = 0x1p21 / side;
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------

__global__ void k_system_of_input(const SysInfo *__restrict__ sys, int nsys, int64_t n, int32_t *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = system_of(sys, nsys, (int)i);
}

__device__ __forceinline__ uint32_t quantise(double x, double lo, double scale) {
  double u = __dsub_rn(x, lo);
  u = __dmul_rn(u, scale);
  if (!(u >= 0.0)) return 0u;
  if (u >= (double)kQMax) return kQMax;
  return (uint32_t)u;  // truncation == floor for u >= 0
}

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// Peano-Hilbert order (the transposed-index construction of J. Skilling,
// 2004): from the top bit down, the lower bits of x are inverted where an
// axis has the current bit set, and exchanged between x and that axis where
// it has not; a Gray decode across the axes then gives the "transpose" of
// the index, whose bits interleaved level by level (x first) are the index.
// Consecutive indices are face-adjacent cells and every aligned cube is one
// contiguous index range, so the octal digits still name the octree's cells.
__device__ __forceinline__ void hilbert_transpose(uint32_t (&x)[3]) {
  for (int b = kKeyLevels - 1; b >= 1; --b) {
    const uint32_t bit = 1u << b, low = bit - 1u;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const bool set = (x[a] & bit) != 0u;
      const uint32_t sw = (x[0] ^ x[a]) & low;  // (0 for the x axis itself)
      x[0] ^= set ? low : sw;
      x[a] ^= set ? 0u : sw;
    }
  }
  x[1] ^= x[0];
  x[2] ^= x[1];
  uint32_t flip = 0u;
  for (int b = kKeyLevels - 1; b >= 1; --b)
    if (x[2] & (1u << b)) flip ^= (1u << b) - 1u;
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] ^= flip;
}

__global__ void k_keys(const double *__restrict__ pos, const double *__restrict__ mass, int64_t n,
                       const int32_t *__restrict__ sys_in, const SysInfo *__restrict__ sys, int curve,
                       uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, PosMass *__restrict__ pm,
                       DevInfo *info) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const SysInfo &S = sys[sys_in ? sys_in[i] : 0];
  const double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  uint32_t q[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) q[k] = quantise(x[k], S.lo[k], S.scale);
  if (curve) hilbert_transpose(q);
  // x bit is the most significant of each octal digit
  keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  vals[i] = (uint32_t)i;
  const double m = mass[i];
  PosMass r;
  r.x = x[0];
  r.y = x[1];
  r.z = x[2];
  r.m = m;
  pm[i] = r;
  if (!(m >= 0.0) || !isfinite(m)) atomicOr(&info->err, kErrBadMass);
}

// Sorted copies and the inverse permutation; the split depth delta_i of each
// pair of neighbouring keys (-1 across a system boundary or at the end); the
// octant masks cleared for the topology pass and the level counters for the
// level pass.
__global__ void k_gather(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                         const PosMass *__restrict__ pm, int64_t n,
                         const int32_t *__restrict__ sys_in, double *__restrict__ spos, double *__restrict__ smass,
                         int32_t *__restrict__ perm, int8_t *__restrict__ delta, int32_t *__restrict__ mask,
                         int32_t *__restrict__ lcount) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0)
    for (int l = 0; l < 72; ++l) lcount[l] = 0;  // counts, offsets, cursors
  if (i >= n) return;
  uint32_t j = vals[i];
  perm[i] = (int32_t)j;
  const PosMass r = pm[j];
  spos[3 * i] = r.x;
  spos[3 * i + 1] = r.y;
  spos[3 * i + 2] = r.z;
  smass[i] = r.m;
  int d = -1;
  if (i + 1 < n) {
    const bool same = sys_in ? (sys_in[j] == sys_in[vals[i + 1]]) : true;
    if (same) d = common_digits(keys[i], keys[i + 1]);
  }
  delta[i] = (int8_t)d;
  mask[i] = 0;
}

// ---------------------------------------------------------------------------
// topology
// ---------------------------------------------------------------------------

// owner[j]: the owning position of the cell split at j (its first split), or
// the first particle of the run of equal keys containing j; level[j]: level
// of the cell owned at j, -1 when j owns none; for an owned cell also its
// particle range (cfirst, ccount).
__global__ void k_owner(const uint64_t *__restrict__ keys, const int8_t *__restrict__ delta, int64_t n,
                        const SysInfo *__restrict__ sys, int nsys, int32_t *__restrict__ owner,
                        int8_t *__restrict__ level, int32_t *__restrict__ cfirst, int32_t *__restrict__ ccount) {
  int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= n) return;
  const int j = (int)jj;
  const int d = delta[j];
  int own = -1, lev = -1, a = 0, b = -1;
  if (d >= 0) {
    const int s = system_of(sys, nsys, j);
    const int lo = sys[s].first, hi = lo + sys[s].count;
    const uint64_t kj = keys[j];
    if (d < kKeyLevels) {
      const int sh = prefix_shift(d);
      a = gallop_first(keys, lo, j, kj >> sh, sh);
      const int sh1 = prefix_shift(d + 1);
      int e = gallop_past(keys, a, j + 1, keys[a] >> sh1, sh1);
      own = e - 1;
      if (own == j) {
        lev = d;
        b = gallop_past(keys, j, hi, kj >> sh, sh) - 1;
      }
    } else {
      own = gallop_first(keys, lo, j, kj, 0);
      if (j == lo || delta[j - 1] != kKeyLevels) {
        lev = kKeyLevels;
        a = j;
        b = gallop_past(keys, j, hi, kj, 0) - 1;
      }
    }
  }
  owner[j] = own;
  level[j] = (int8_t)lev;
  if (lev >= 0) {
    cfirst[j] = a;
    ccount[j] = b - a + 1;
  }
}

// bit into mask[P] for every active lane of the wave, with one atomic per
// run of neighbouring lanes that share P (neighbouring positions mostly
// share a parent; an OR is the same whatever the grouping).  Every lane of
// the wave must call it.
__device__ __forceinline__ void or_into_parent(int32_t *__restrict__ mask, int P, int bit, bool active) {
  const int lane = lane_id();
  const int key = active ? P : -1;
  // (every lane takes part in the shuffles: a lane left out of one gives 0)
  const int prev = __shfl_up(key, 1, kWave), next = __shfl_down(key, 1, kWave);
  const bool head = lane == 0 || prev != key;
  const int run = __popcll(__ballot(head) & ((2ull << lane) - 1ull));
  int v = active ? bit : 0;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int u = __shfl_up(v, d, kWave);
    const int r = __shfl_up(run, d, kWave);
    if (lane >= d && r == run) v |= u;
  }
  const bool tail = lane == kWave - 1 || next != key;
  if (active && tail && v) atomicOr(&mask[P], v);
}

// Parent and octant of every owned cell; octant masks of the parents.
__global__ void k_cells(const uint64_t *__restrict__ keys, const int8_t *__restrict__ delta,
                        const int32_t *__restrict__ owner, const int8_t *__restrict__ level, int64_t n,
                        const SysInfo *__restrict__ sys, int nsys, const int32_t *__restrict__ cfirst,
                        const int32_t *__restrict__ ccount, int32_t *__restrict__ cparent, int8_t *__restrict__ cdigit,
                        int32_t *__restrict__ mask, DevInfo *info) {
  const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = (int)jj;
  const int l = (jj < n) ? level[j] : -1;
  int P = -1, bit = 0;
  if (l >= 0) {
    const int s = system_of(sys, nsys, j);
    const int lo = sys[s].first;
    const int a = cfirst[j], b = a + ccount[j] - 1;
    const int dl = (a > lo) ? delta[a - 1] : -1;
    const int dr = delta[b];
    const int lp = max(dl, dr);
    if (lp < 0) {
      cparent[j] = -1 - s;
      cdigit[j] = 0;
    } else {
      const int sp = (dl == lp) ? a - 1 : b;
      P = owner[sp];
      const int dg = key_digit(keys[a], lp + 1);
      cparent[j] = P;
      cdigit[j] = (int8_t)dg;
      bit = 1 << dg;
    }
  }
  or_into_parent(mask, P, bit, P >= 0);
}

// Parent of every particle: a cell (octant mask updated), a bucket, or none
// (a system holding one particle).
__global__ void k_particle_parents(const uint64_t *__restrict__ keys, const int8_t *__restrict__ delta,
                                   const int32_t *__restrict__ owner, int64_t n, const SysInfo *__restrict__ sys,
                                   int nsys, int32_t *__restrict__ pparent, int8_t *__restrict__ pdigit,
                                   int32_t *__restrict__ mask) {
  const int64_t ii = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)ii;
  int P = -1, bit = 0;
  if (ii < n) {
    const int s = system_of(sys, nsys, i);
    const int lo = sys[s].first;
    const int dl = (i > lo) ? delta[i - 1] : -1;
    const int dr = delta[i];
    const int lp = max(dl, dr);
    if (lp < 0) {
      pparent[i] = -1 - s;
      pdigit[i] = 0;
    } else {
      const int sp = (dl == lp) ? i - 1 : i;
      P = owner[sp];
      pparent[i] = P;
      if (lp == kKeyLevels) {
        pdigit[i] = 0;  // bucket member: slot order is Morton order
      } else {
        const int dg = key_digit(keys[i], lp + 1);
        pdigit[i] = (int8_t)dg;
        bit = 1 << dg;
      }
    }
  }
  or_into_parent(mask, P, bit, bit != 0);
}

__global__ void k_nchild(const int8_t *__restrict__ level, const int32_t *__restrict__ mask,
                         const int32_t *__restrict__ ccount, int64_t n, int32_t *__restrict__ nchild) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int l = level[j];
  int c = 0;
  if (l >= 0) c = (l == kKeyLevels) ? ccount[j] : __popc(mask[j]);
  nchild[j] = c;
}

__device__ __forceinline__ int child_slot(int P, int dg, bool bucket_member, int i, const int32_t *__restrict__ cfc,
                                          const int32_t *__restrict__ mask, int nsys) {
  if (bucket_member) return nsys + cfc[P] + (i - P);
  return nsys + cfc[P] + __popc(mask[P] & ((1 << dg) - 1));
}

// Slots of the cells; particle leaf records and their raw sums.
__global__ void k_slots(const int8_t *__restrict__ level, const int32_t *__restrict__ cparent,
                        const int8_t *__restrict__ cdigit, const int32_t *__restrict__ pparent,
                        const int8_t *__restrict__ pdigit, const int32_t *__restrict__ cfc,
                        const int32_t *__restrict__ mask, const double *__restrict__ spos,
                        const double *__restrict__ smass, int64_t n, int nsys, int64_t cap,
                        int32_t *__restrict__ cslot, NodeRec *__restrict__ nodes, double *__restrict__ msum,
                        int8_t *__restrict__ meta, DevInfo *info) {
  int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= n) return;
  const int j = (int)jj;
  if (level[j] >= 0) {
    const int P = cparent[j];
    int cs = (P < 0) ? (-1 - P) : child_slot(P, cdigit[j], false, j, cfc, mask, nsys);
    if (cs < 0 || cs >= cap) {
      atomicOr(&info->err, kErrBuild);
      cs = 0;
    }
    cslot[j] = cs;
  }
  // particle j
  const int P = pparent[j];
  int slot;
  if (P < 0) slot = -1 - P;
  else slot = child_slot(P, pdigit[j], level[P] == kKeyLevels, j, cfc, mask, nsys);
  if (slot < 0 || slot >= cap) {
    atomicOr(&info->err, kErrBuild);
    return;
  }
  const double m = smass[j];
  NodeRec r;
  r.com[0] = spos[3 * (int64_t)j];
  r.com[1] = spos[3 * (int64_t)j + 1];
  r.com[2] = spos[3 * (int64_t)j + 2];
  r.m = m;
  r.l = 0.0;
  r.s = 0.0;
  r.child = -1;
  r.nchild = 0;
  r.first = j;
  r.count = 1;
  nodes[slot] = r;
  meta[slot] = (int8_t)(32 * kParticle + 31);
  msum[4 * (int64_t)slot] = m;
  msum[4 * (int64_t)slot + 1] = __dmul_rn(m, r.com[0]);
  msum[4 * (int64_t)slot + 2] = __dmul_rn(m, r.com[1]);
  msum[4 * (int64_t)slot + 3] = __dmul_rn(m, r.com[2]);
}

__global__ void k_empty_roots(const SysInfo *__restrict__ sys, int nsys, NodeRec *__restrict__ nodes,
                              double *__restrict__ msum, int8_t *__restrict__ meta) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys || sys[s].count != 0) return;
  NodeRec r;
  r.com[0] = r.com[1] = r.com[2] = 0.0;
  r.m = 0.0;
  r.l = 0.0;
  r.s = 0.0;
  r.child = -1;
  r.nchild = 0;
  r.first = sys[s].first;
  r.count = 0;
  nodes[s] = r;
  meta[s] = (int8_t)(32 * kEmpty + 31);
  for (int k = 0; k < 4; ++k) msum[4 * (int64_t)s + k] = 0.0;
}

// Cells grouped by level: counts, offsets, then a scatter (order within a
// level is irrelevant: every cell sums its own children in slot order).
// Lanes of a wave with the same level are found with ballots (peer masks), so
// that LDS and global counters see one atomic per wave and level.
__device__ __forceinline__ unsigned long long level_peers(int l) {
  unsigned long long peers = __ballot(l >= 0);
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const unsigned long long m = __ballot(l >= 0 && ((l >> b) & 1));
    peers &= ((l >> b) & 1) ? m : ~m;
  }
  return (l >= 0) ? peers : 0ull;
}

constexpr int kLevelTile = 16;  // positions per thread in the level kernels

// The moments pass's record of the cell owned at position j (level lev).
__device__ __forceinline__ CellRec cell_record(int j, int lev, const int8_t *__restrict__ level,
                                               const int32_t *__restrict__ cparent, const int32_t *__restrict__ cslot,
                                               const int32_t *__restrict__ cfc, const int32_t *__restrict__ nchild,
                                               const int32_t *__restrict__ cfirst, const int32_t *__restrict__ ccount,
                                               const double *__restrict__ spos, const SysInfo *__restrict__ sys,
                                               int nsys) {
  CellRec r;
  r.c0 = nsys + cfc[j];
  r.nc = nchild[j];
  r.slot = cslot[j];
  r.first = cfirst[j];
  r.count = ccount[j];
  // A bucket (level 21) is opened unless a chain of single-child cells sits
  // above it: the opening bound shrinks down a chain (theta < 2/sqrt(3)), so
  // the chain is accepted iff its deepest cell, at level 20, is; the bucket
  // then carries that cell's side and s.
  int geo = lev;
  bool always_open = false;
  if (lev == kKeyLevels) {
    const int P = cparent[j];
    const int lp = (P < 0) ? -1 : (int)level[P];
    if (lp < kKeyLevels - 1) geo = kKeyLevels - 1;
    else always_open = true;
  }
  // The cell's coordinates at level geo: the top geo bits of each quantised
  // coordinate of any of its members (a cell of either curve is one aligned
  // cube, a bucket one point), here the particle at the owning position,
  // which lies in the cell.
  const SysInfo &S = sys[system_of(sys, nsys, j)];
  uint32_t q[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) q[k] = quantise(spos[3 * (int64_t)j + k], S.lo[k], S.scale) >> (kKeyLevels - geo);
  r.cx = q[0];
  r.cy = q[1];
  r.cz_geo = q[2] | ((uint32_t)geo << 21) | (always_open ? (1u << 26) : 0u);
  return r;
}

__global__ __launch_bounds__(256) void k_level_count(const int8_t *__restrict__ level, int64_t n,
                                                     int32_t *__restrict__ lcount) {
  __shared__ int32_t c[kKeyLevels + 1];
  if (threadIdx.x <= kKeyLevels) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * kLevelTile;
  for (int q = 0; q < kLevelTile; ++q) {
    const int64_t j = base + (int64_t)q * blockDim.x + threadIdx.x;
    const int l = (j < n) ? level[j] : -1;
    const unsigned long long peers = level_peers(l);
    if (l >= 0 && rank_below(peers) == 0) atomicAdd(&c[l], (int)__popcll(peers));
  }
  __syncthreads();
  if (threadIdx.x <= kKeyLevels && c[threadIdx.x]) atomicAdd(&lcount[threadIdx.x], c[threadIdx.x]);
}

// Each block takes the level offsets from the counts (block 0 also stores
// them, the cell count and the deepest level); rank = level offset + block
// base (one global atomic per block and level on the zeroed cursors) + wave
// base (one LDS atomic per wave, level and round) + lanes below with that
// level.
__global__ __launch_bounds__(256) void k_level_scatter(const int8_t *__restrict__ level, int64_t n,
                                                       const int32_t *__restrict__ lcount, int32_t *__restrict__ loff,
                                                       int32_t *__restrict__ lcursor, const int32_t *__restrict__ cparent,
                                                       const int32_t *__restrict__ cslot, const int32_t *__restrict__ cfc,
                                                       const int32_t *__restrict__ nchild,
                                                       const int32_t *__restrict__ cfirst,
                                                       const int32_t *__restrict__ ccount,
                                                       const double *__restrict__ spos, const SysInfo *__restrict__ sys,
                                                       int nsys, CellRec *__restrict__ lcells, DevInfo *info) {
  __shared__ int32_t c[kKeyLevels + 1], base[kKeyLevels + 1], off[kKeyLevels + 2];
  if (threadIdx.x <= kKeyLevels) c[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    int32_t sum = 0, deepest = 0;
    for (int l = 0; l <= kKeyLevels; ++l) {
      off[l] = sum;
      sum += lcount[l];
      if (lcount[l]) deepest = l;
    }
    off[kKeyLevels + 1] = sum;
    if (blockIdx.x == 0) {
      for (int l = 0; l <= kKeyLevels + 1; ++l) loff[l] = off[l];
      info->n_cells = sum;
      info->max_level = deepest;
    }
  }
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x * kLevelTile;
  int l[kLevelTile], pos[kLevelTile];
  for (int q = 0; q < kLevelTile; ++q) {
    const int64_t j = b0 + (int64_t)q * blockDim.x + threadIdx.x;
    l[q] = (j < n) ? level[j] : -1;
    const unsigned long long peers = level_peers(l[q]);
    int wbase = 0;
    if (l[q] >= 0 && rank_below(peers) == 0) wbase = atomicAdd(&c[l[q]], (int)__popcll(peers));
    const int leader = (l[q] >= 0) ? (__ffsll((long long)peers) - 1) : 0;
    wbase = __shfl(wbase, leader, kWave);
    pos[q] = wbase + rank_below(peers);
  }
  __syncthreads();
  if (threadIdx.x <= kKeyLevels && c[threadIdx.x])
    base[threadIdx.x] = off[threadIdx.x] + atomicAdd(&lcursor[threadIdx.x], c[threadIdx.x]);
  __syncthreads();
  for (int q = 0; q < kLevelTile; ++q) {
    const int64_t j = b0 + (int64_t)q * blockDim.x + threadIdx.x;
    if (l[q] >= 0)
      lcells[base[l[q]] + pos[q]] = cell_record((int)j, l[q], level, cparent, cslot, cfc, nchild, cfirst, ccount, spos,
                                                sys, nsys);
  }
}

// Moments of the cells of one level from their children's raw sums.  A
// level's time is the latency of one cell's chain of reads: a cell reads its
// record (written in position order by the level scatter), then its
// children's sums, kMomChunk children at a time (indices clamped to the last
// child, the extra values unused), before it adds any of them.  The sums add
// the children in slot order starting from zero.
constexpr int kMomChunk = 4;

__global__ void k_moments(int lev, const CellRec *__restrict__ lcells, const int32_t *__restrict__ loff,
                          const SysInfo *__restrict__ sys, int nsys, int64_t cap, NodeRec *__restrict__ nodes,
                          double *__restrict__ msum, double *__restrict__ qmom, float4 *__restrict__ qpack,
                          int8_t *__restrict__ meta, DevInfo *info) {
  const int64_t end = loff[lev + 1];
  // the system's frame: loaded once when there is one system
  double slo[3] = {sys[0].lo[0], sys[0].lo[1], sys[0].lo[2]}, sside = sys[0].side;
  for (int64_t k = (int64_t)loff[lev] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < end;
       k += (int64_t)gridDim.x * blockDim.x) {
  const CellRec cr = lcells[k];
  const int c0 = cr.c0, nc = cr.nc, slot = cr.slot;
  if (c0 < 0 || nc < 0 || (int64_t)c0 + nc > cap || slot < 0 || slot >= cap) {
    atomicOr(&info->err, kErrBuild);
    continue;
  }
  if (nsys > 1) {
    const SysInfo &S = sys[system_of(sys, nsys, cr.first)];
    slo[0] = S.lo[0];
    slo[1] = S.lo[1];
    slo[2] = S.lo[2];
    sside = S.side;
  }
  double m = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
  for (int cb = 0; cb < nc; cb += kMomChunk) {
    double2 a[kMomChunk], b[kMomChunk];
#pragma unroll
    for (int u = 0; u < kMomChunk; ++u) {
      const double2 *q = reinterpret_cast<const double2 *>(msum + 4 * (int64_t)(c0 + min(cb + u, nc - 1)));
      a[u] = q[0];
      b[u] = q[1];
    }
#pragma unroll
    for (int u = 0; u < kMomChunk; ++u) {
      if (cb + u < nc) {
        m = __dadd_rn(m, a[u].x);
        mx = __dadd_rn(mx, a[u].y);
        my = __dadd_rn(my, b[u].x);
        mz = __dadd_rn(mz, b[u].y);
      }
    }
  }
  msum[4 * (int64_t)slot] = m;
  msum[4 * (int64_t)slot + 1] = mx;
  msum[4 * (int64_t)slot + 2] = my;
  msum[4 * (int64_t)slot + 3] = mz;
  const int geo = (int)((cr.cz_geo >> 21) & 31u);
  const bool always_open = (cr.cz_geo >> 26) & 1u;
  const double l = ldexp(sside, -geo);
  const uint32_t q[3] = {cr.cx, cr.cy, cr.cz_geo & 0x1fffffu};
  double c[3], com[3];
  const double mv[3] = {mx, my, mz};
  for (int k = 0; k < 3; ++k) {
    double h = (double)q[k] + 0.5;
    h = __dmul_rn(h, l);
    c[k] = __dadd_rn(slo[k], h);
    com[k] = (m > 0.0) ? mv[k] / m : c[k];
  }
  const double dx = __dsub_rn(c[0], com[0]), dy = __dsub_rn(c[1], com[1]), dz = __dsub_rn(c[2], com[2]);
  const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  NodeRec r;
  r.com[0] = com[0];
  r.com[1] = com[1];
  r.com[2] = com[2];
  r.m = m;
  r.l = always_open ? INFINITY : l;
  r.s = sqrt(d2);
  r.child = c0;
  r.nchild = nc;
  r.first = cr.first;
  r.count = cr.count;
  nodes[slot] = r;
  if (qmom) {
    // second moments about the centre of mass from the children's own, each
    // shifted to this centre (parallel axes); a particle's own are zero.  A
    // child's mass and centre of mass come from its raw sums (its kind from
    // meta), not from its 64-byte record; a massless child adds nothing.
    double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int ci = 0; ci < nc; ++ci) {
      const int cs = c0 + ci;
      const double *q = msum + 4 * (int64_t)cs;
      const double mc = q[0];
      if (!(mc > 0.0)) continue;
      const double ex = __dsub_rn(q[1] / mc, com[0]), ey = __dsub_rn(q[2] / mc, com[1]),
                   ez = __dsub_rn(q[3] / mc, com[2]);
      const double sh[6] = {mc * ex * ex, mc * ey * ey, mc * ez * ez, mc * ex * ey, mc * ex * ez, mc * ey * ez};
      const bool leaf = (meta[cs] >> 5) == kParticle;
#pragma unroll
      for (int k = 0; k < 6; ++k) S[k] = __dadd_rn(S[k], leaf ? sh[k] : __dadd_rn(qmom[6 * (int64_t)cs + k], sh[k]));
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) qmom[6 * (int64_t)slot + k] = S[k];
    // as the force sum reads them: 3 S and the trace T (and 1.5 T)
    const double T = S[0] + S[1] + S[2];
    qpack[2 * (int64_t)slot] = make_float4((float)(3.0 * S[0]), (float)(3.0 * S[1]), (float)(3.0 * S[2]),
                                           (float)(3.0 * S[3]));
    qpack[2 * (int64_t)slot + 1] = make_float4((float)(3.0 * S[4]), (float)(3.0 * S[5]), (float)T, (float)(1.5 * T));
  }
  meta[slot] = (int8_t)(lev == kKeyLevels ? 32 * kBucket + lev : lev);
  }
}

inline unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------------------
// host-side driver of the build
// ---------------------------------------------------------------------------



int bbox_blocks_per_system(int nsys) {
  int bps = 1024 / (nsys > 0 ? nsys : 1);
  return bps < 4 ? 4 : bps;
}

void build_tree_device(TreeBuffers &B, hipStream_t s) {
  const int64_t n = B.n;
  const int nsys = B.nsys;
  const int bps = bbox_blocks_per_system(nsys);
  k_bbox_partial<<<(unsigned)(nsys * bps), 256, 0, s>>>(B.pos, B.sys, bps, B.bbox_part, B.info);
  k_bbox_final<<<(unsigned)nsys, 256, 0, s>>>(B.bbox_part, bps, B.sys);
  if (n == 0) {
    B.sorted_keys = B.keys[0];
    k_empty_roots<<<blocks_for(nsys), 256, 0, s>>>(B.sys, nsys, B.nodes, B.msum, B.meta);
    return;
  }
  if (nsys > 1) k_system_of_input<<<blocks_for(n), 256, 0, s>>>(B.sys, nsys, n, B.sys_in);
  k_keys<<<blocks_for(n), 256, 0, s>>>(B.pos, B.mass, n, nsys > 1 ? B.sys_in : nullptr, B.sys, B.curve, B.keys[0],
                                        B.vals[0], B.pm, B.info);
  int cur = radix_sort_pairs(B.keys[0], B.keys[1], B.vals[0], B.vals[1], n, 0, 64, B.hist, B.scan_tmp,
                             &B.info->err, s);
  if (nsys > 1) {
    for (int shift = 0; (nsys - 1) >> shift; shift += 8)
      cur = radix_pass_by_system(B.keys[0], B.keys[1], B.vals[0], B.vals[1], cur, n, B.sys_in, shift, B.hist,
                                 B.scan_tmp, s);
  }
  const uint64_t *keys = B.keys[cur];
  B.sorted_keys = B.keys[cur];
  k_gather<<<blocks_for(n), 256, 0, s>>>(keys, B.vals[cur], B.pm, n, nsys > 1 ? B.sys_in : nullptr, B.spos,
                                          B.smass, B.perm, B.delta, B.mask, B.lcount);
  k_owner<<<blocks_for(n), 256, 0, s>>>(keys, B.delta, n, B.sys, nsys, B.owner, B.level, B.cfirst, B.ccount);
  k_cells<<<blocks_for(n), 256, 0, s>>>(keys, B.delta, B.owner, B.level, n, B.sys, nsys, B.cfirst, B.ccount,
                                         B.cparent, B.cdigit, B.mask, B.info);
  k_particle_parents<<<blocks_for(n), 256, 0, s>>>(keys, B.delta, B.owner, n, B.sys, nsys, B.pparent, B.pdigit,
                                                    B.mask);
  k_nchild<<<blocks_for(n), 256, 0, s>>>(B.level, B.mask, B.ccount, n, B.nchild);
  scan_exclusive_i32(B.nchild, B.cfc, n, &B.info->n_slots, B.scan_tmp, s);
  k_slots<<<blocks_for(n), 256, 0, s>>>(B.level, B.cparent, B.cdigit, B.pparent, B.pdigit, B.cfc, B.mask, B.spos,
                                         B.smass, n, nsys, B.slot_cap, B.cslot, B.nodes, B.msum, B.meta, B.info);
  if (B.any_empty) k_empty_roots<<<blocks_for(nsys), 256, 0, s>>>(B.sys, nsys, B.nodes, B.msum, B.meta);
  k_level_count<<<blocks_for(n, 256 * kLevelTile), 256, 0, s>>>(B.level, n, B.lcount);
  k_level_scatter<<<blocks_for(n, 256 * kLevelTile), 256, 0, s>>>(B.level, n, B.lcount, B.loff, B.lcursor,
                                                                   B.cparent, B.cslot, B.cfc, B.nchild, B.cfirst,
                                                                   B.ccount, B.spos, B.sys, nsys, B.lcells, B.info);
  const unsigned mgrid = (unsigned)std::min<int64_t>(blocks_for(n), 512);
  for (int lev = kKeyLevels; lev >= 0; --lev)
    k_moments<<<mgrid, 256, 0, s>>>(lev, B.lcells, B.loff, B.sys, nsys, B.slot_cap, B.nodes, B.msum, B.qmom, B.qpack,
                                    B.meta, B.info);
}

}  // namespace bh
