// Force sum over the interaction lists (Eq. 1, FP32 with group-relative
// coordinates, partial sums folded into FP64).
//
// Work items are (group, block of 64 members, or the group's remainder); a
// persistent grid of single-wave workgroups pulls items from eight atomic
// queues, one per XCD, which hold the items of each group next to each other
// (so that the blocks of a group read its list through the same L2).
// A block of m members uses R lane partitions of W = 64/R >= m lanes, one
// member per lane;
// partition `part` takes list entries part, part + R, ...  With R = 1 every
// lane reads the same entry, so entries are fetched with scalar loads and used
// as scalar operands.  Per term a lane computes dx = x_j - x_i (near entries:
// from the FP32 value and its rounding residue), r^2 = |dx|^2 + eps^2 (FMA),
// v_rsq_f32, and accumulates m r^-3 dx and m r^-1, the terms of a block of
// entries written stage by stage so that dependent instructions issue far
// apart.  After each list chunk the FP32 partial sums are folded into FP64.  A
// member's own entry is in the near list with dx = 0 exactly: it adds 0 force
// and m_i/eps potential, removed at the end.
//
// Quadrupole sums (a template variant): a cell entry also adds the
// second-order term of the softened potential of its particles about their
// centre of mass, from the cell's second moments S (FP32, packed as 3 S and
// the trace, read by node slot: far entries carry the slot in a parallel
// array, near entries in the .w of their residue).  With u = dx, R^-1 as above and T = tr S:
//   potential  -3 (u.S.u) / (2 R^5) + T / (2 R^3)
//   force      -3 S u / R^5 + (15 (u.S.u) / (2 R^7) - 3 T / (2 R^5)) u.
#include "bh_device.h"

namespace bh {

namespace {

struct Member {
  float x, y, z;     // FP32 x_i - c_g
  float lx, ly, lz;  // rounding residue of x_i - c_g
  float ax, ay, az, pt;
  double dx, dy, dz, dp;
};

// The quadrupole term of one cell entry at relative position (dx, dy, dz),
// with R^2 = |u|^2 + eps^2 and ri = 1/R; a = 3 (xx, yy, zz, xy), b = (3 xz,
// 3 yz, T, 1.5 T).  With S3 = 3 S and w = u.S3.u the terms above read
//   force       r5 (2.5 w ri^2 - 1.5 T) u - r5 S3 u
//   -potential  0.5 r5 (w - T R^2),        r5 = ri^5.
__device__ __forceinline__ void quad_term(Member &M, const float4 a, const float4 b, float dx, float dy, float dz,
                                          float R2, float ri) {
  const float sx = __builtin_fmaf(a.x, dx, __builtin_fmaf(a.w, dy, b.x * dz));
  const float sy = __builtin_fmaf(a.w, dx, __builtin_fmaf(a.y, dy, b.y * dz));
  const float sz = __builtin_fmaf(b.x, dx, __builtin_fmaf(b.y, dy, a.z * dz));
  const float w = __builtin_fmaf(dx, sx, __builtin_fmaf(dy, sy, dz * sz));
  const float ri2 = ri * ri;
  const float r5 = ri2 * ri2 * ri;
  const float c = r5 * __builtin_fmaf(2.5f * w, ri2, -b.w);
  M.ax = __builtin_fmaf(-r5, sx, __builtin_fmaf(c, dx, M.ax));
  M.ay = __builtin_fmaf(-r5, sy, __builtin_fmaf(c, dy, M.ay));
  M.az = __builtin_fmaf(-r5, sz, __builtin_fmaf(c, dz, M.az));
  M.pt = __builtin_fmaf(0.5f * r5, __builtin_fmaf(-b.z, R2, w), M.pt);
}

// U entries (value e, rounding residue l when NEAR) against this lane's
// member, written stage by stage across the U independent terms.  With QUAD,
// sl[u] is the node slot of a far entry (near entries: l[u].w), -1 for a
// particle.
template <int U, bool NEAR, bool QUAD = false>
__device__ __forceinline__ void terms(Member &M, const float4 (&e)[U], const float4 (&l)[U], float eps2,
                                      const int (&sl)[U], const float4 *__restrict__ qpack) {
  float dx[U], dy[U], dz[U], q[U], mr[U], ri[U], R2[U];
  // the moments are fetched first (a particle's slot is clamped to 0 and its
  // values unused), so that the monopole terms hide their latency
  float4 qa[U], qb[U];
  int slot[U];
  if (QUAD) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      slot[u] = NEAR ? __float_as_int(l[u].w) : sl[u];
      const int64_t at = 2 * (int64_t)max(slot[u], 0);
      qa[u] = qpack[at];
      qb[u] = qpack[at + 1];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    dx[u] = e[u].x - M.x;
    dy[u] = e[u].y - M.y;
    dz[u] = e[u].z - M.z;
  }
  if (NEAR) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      dx[u] += l[u].x - M.lx;
      dy[u] += l[u].y - M.ly;
      dz[u] += l[u].z - M.lz;
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) q[u] = __builtin_fmaf(dx[u], dx[u], eps2);
#pragma unroll
  for (int u = 0; u < U; ++u) q[u] = __builtin_fmaf(dy[u], dy[u], q[u]);
#pragma unroll
  for (int u = 0; u < U; ++u) q[u] = __builtin_fmaf(dz[u], dz[u], q[u]);
  if (QUAD) {
#pragma unroll
    for (int u = 0; u < U; ++u) R2[u] = q[u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) q[u] = __builtin_amdgcn_rsqf(q[u]);  // 1/r
  if (QUAD) {
#pragma unroll
    for (int u = 0; u < U; ++u) ri[u] = q[u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    mr[u] = e[u].w * q[u];
    q[u] = q[u] * q[u];  // 1/r^2
  }
#pragma unroll
  for (int u = 0; u < U; ++u) q[u] = mr[u] * q[u];  // m/r^3
#pragma unroll
  for (int u = 0; u < U; ++u) {
    M.ax = __builtin_fmaf(q[u], dx[u], M.ax);
    M.ay = __builtin_fmaf(q[u], dy[u], M.ay);
    M.az = __builtin_fmaf(q[u], dz[u], M.az);
    M.pt += mr[u];
  }
  if (QUAD) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (slot[u] >= 0) quad_term(M, qa[u], qb[u], dx[u], dy[u], dz[u], R2[u], ri[u]);
  }
}

__device__ __forceinline__ void fold(Member &M) {
  M.dx += (double)M.ax;
  M.dy += (double)M.ay;
  M.dz += (double)M.az;
  M.dp += (double)M.pt;
  M.ax = M.ay = M.az = M.pt = 0.0f;
}

constexpr int kU = 8;      // entries per block of terms
constexpr int kUQuad = 4;  // the same for the quadrupole sums (register pressure)

// One chunk with R lane partitions: partition `part` takes entries part,
// part + R, ...; R is a compile-time constant so that the four entries of a
// block are loaded at constant offsets from one running pointer.  hs: the
// node slots of far entries (QUAD only).
template <bool NEAR, int R, bool QUAD>
__device__ __forceinline__ void chunk_part(Member &M, const float4 *__restrict__ h, const float4 *__restrict__ l,
                                           const int *__restrict__ hs, const float4 *__restrict__ qpack, int n,
                                           int part, float eps2) {
  constexpr int B = QUAD ? 2 : 4;  // entries per block (register pressure of the quadrupole terms)
  const int mine = (n - part + R - 1) / R;
  const float4 *ph = h + part;
  const float4 *pl = l + part;
  const int *ps = QUAD && !NEAR ? hs + part : nullptr;
  int t = 0;
  for (; t + B <= mine; t += B, ph += B * R, pl += B * R) {
    float4 e4[B], r4[B];
    int s4[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      e4[u] = ph[u * R];
      r4[u] = NEAR ? pl[u * R] : e4[u];
      s4[u] = (QUAD && !NEAR) ? ps[u * R] : -1;
    }
    if (QUAD && !NEAR) ps += B * R;
    terms<B, NEAR, QUAD>(M, e4, r4, eps2, s4, qpack);
  }
  for (; t < mine; ++t, ph += R, pl += R) {
    const float4 e1[1] = {ph[0]}, r1[1] = {NEAR ? pl[0] : ph[0]};
    int s1[1] = {-1};
    if (QUAD && !NEAR) {
      s1[0] = ps[0];
      ps += R;
    }
    terms<1, NEAR, QUAD>(M, e1, r1, eps2, s1, qpack);
  }
}

// n entries of one chunk: values at h[0..n), residues at l[0..n) when NEAR,
// node slots at hs[0..n) for far entries with QUAD.
template <bool NEAR, bool QUAD = false>
__device__ __forceinline__ void chunk_sum(Member &M, const float4 *__restrict__ h, const float4 *__restrict__ l,
                                          int n, int R, int part, float eps2, const int *__restrict__ hs = nullptr,
                                          const float4 *__restrict__ qpack = nullptr) {
  constexpr bool FS = QUAD && !NEAR;  // far slots to load
  constexpr int KU = QUAD ? kUQuad : kU;  // entries per block
  float4 e[KU], r[KU];
  int sl[KU];
#pragma unroll
  for (int u = 0; u < KU; ++u) sl[u] = -1;
  if (R == 1) {
    // every lane takes the same entries: scalar loads, scalar operands; the
    // next block is fetched while the current one is summed
    int t = 0;
    if (n >= KU) {
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        e[u] = h[u];
        r[u] = NEAR ? l[u] : e[u];
        if (FS) sl[u] = hs[u];
      }
      for (t = KU; t + KU <= n; t += KU) {
        float4 ne[KU], nr[KU];
        int ns[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          ne[u] = h[t + u];
          nr[u] = NEAR ? l[t + u] : ne[u];
          ns[u] = FS ? hs[t + u] : -1;
        }
        terms<KU, NEAR, QUAD>(M, e, r, eps2, sl, qpack);
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          e[u] = ne[u];
          r[u] = nr[u];
          sl[u] = ns[u];
        }
      }
      terms<KU, NEAR, QUAD>(M, e, r, eps2, sl, qpack);
    }
    for (; t < n; ++t) {
      const float4 e1[1] = {h[t]}, r1[1] = {NEAR ? l[t] : h[t]};
      const int s1[1] = {FS ? hs[t] : -1};
      terms<1, NEAR, QUAD>(M, e1, r1, eps2, s1, qpack);
    }
  } else {
    switch (R) {
      case 2: chunk_part<NEAR, 2, QUAD>(M, h, l, hs, qpack, n, part, eps2); break;
      case 4: chunk_part<NEAR, 4, QUAD>(M, h, l, hs, qpack, n, part, eps2); break;
      case 8: chunk_part<NEAR, 8, QUAD>(M, h, l, hs, qpack, n, part, eps2); break;
      case 16: chunk_part<NEAR, 16, QUAD>(M, h, l, hs, qpack, n, part, eps2); break;
      case 32: chunk_part<NEAR, 32, QUAD>(M, h, l, hs, qpack, n, part, eps2); break;
      default: chunk_part<NEAR, 64, QUAD>(M, h, l, hs, qpack, n, part, eps2); break;
    }
  }
  fold(M);
}

// The list data is read-only here; as separate restrict arguments the
// compiler can fetch wave-uniform entries with scalar loads.  QUAD: the
// quadrupole variant (far_slot and qpack set).
template <bool QUAD>
__global__ __launch_bounds__(kWave) void k_force_lists(ForceArgs a, const float4 *__restrict__ far_pool,
                                                       const int32_t *__restrict__ far_next,
                                                       const float4 *__restrict__ near_pool,
                                                       const int32_t *__restrict__ near_next,
                                                       const int32_t *__restrict__ glists,
                                                       const int32_t *__restrict__ items,
                                                       const int32_t *__restrict__ far_slot,
                                                       const float4 *__restrict__ qpack) {
  const int lane = lane_id();
  // workgroups are dealt to the XCDs round robin: this wave's XCD queue
  // first, then the others
  const int xcd = blockIdx.x & 7;
  int tried = 0;
  for (;;) {
    int it = -1;
    while (tried < 8) {
      // (a provably uniform queue index keeps the take a single atomic)
      const int x = __builtin_amdgcn_readfirstlane((xcd + tried) & 7);
      const int s0 = a.xstart[x], s1 = a.xstart[x + 1];
      const int q = take_one(&a.info->fq[x * kLineInts], lane);
      if (s0 + q < s1) {
        it = s0 + q;
        break;
      }
      ++tried;
    }
    if (it < 0) break;
    const int g = items[2 * it], iv = items[2 * it + 1];
    const int blk = iv & 255, segl = iv >> 8;
    const int gf = a.ginfo[3 * g], gc = a.ginfo[3 * g + 1], gs = a.ginfo[3 * g + 2];
    int fh, fn, nh, nn, prow = -1;
    if (segl == 0) {
      fh = glists[4 * g];
      fn = glists[4 * g + 1];
      nh = glists[4 * g + 2];
      nn = glists[4 * g + 3];
    } else {
      // one segment of a split group: partial sums go to its rows
      const int p = a.gsegfirst[g] + segl - 1;
      const Segment sg = a.segs[a.seg_order[p]];
      fh = sg.fh;
      fn = sg.fn;
      nh = sg.nh;
      nn = sg.nn;
      prow = a.pbase[p];
    }
    if ((fn > 0 && fh < 0) || (nn > 0 && nh < 0)) continue;  // incomplete list (reported by the walk)
    // members [b0, b1) of the group: full blocks of 64, then the remainder,
    // which takes several lane partitions when it is small
    const int b0 = blk * kWave, b1 = min(gc, b0 + kWave);
    const int m = b1 - b0;
    int R = 1;
    while (R < kWave && m * (2 * R) <= kWave) R *= 2;
    const int W = kWave / R;
    const int part = lane / W, u = lane % W;

    double cen[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      cen[k] = __dmul_rn(__dadd_rn(a.gbox[6 * (int64_t)g + k], a.gbox[6 * (int64_t)g + 3 + k]), 0.5);
    const double eps = a.par[gs].eps;
    const float eps2 = (float)(eps * eps);

    Member M;
    {
      double rx = 0.0, ry = 0.0, rz = 0.0;
      if (u < m) {
        const double *q = a.spos + 3 * (int64_t)(gf + b0 + u);
        rx = __dsub_rn(q[0], cen[0]);
        ry = __dsub_rn(q[1], cen[1]);
        rz = __dsub_rn(q[2], cen[2]);
      }
      M.x = (float)rx;
      M.y = (float)ry;
      M.z = (float)rz;
      M.lx = (float)__dsub_rn(rx, (double)M.x);
      M.ly = (float)__dsub_rn(ry, (double)M.y);
      M.lz = (float)__dsub_rn(rz, (double)M.z);
      M.ax = M.ay = M.az = M.pt = 0.0f;
      M.dx = M.dy = M.dz = M.dp = 0.0;
    }

    int ch = fh;
    for (int left = fn; left > 0;) {
      const int n = min(left, a.far_tile);
      const float4 *base = far_pool + (int64_t)ch * a.far_tile;
      chunk_sum<false, QUAD>(M, base, base, n, R, part, eps2, QUAD ? far_slot + (int64_t)ch * a.far_tile : nullptr,
                             qpack);
      left -= n;
      if (left > 0) ch = far_next[ch];
    }
    ch = nh;
    for (int left = nn; left > 0;) {
      const int n = min(left, a.near_tile);
      const float4 *base = near_pool + (int64_t)ch * (2 * a.near_tile);
      chunk_sum<true, QUAD>(M, base, base + a.near_tile, n, R, part, eps2, nullptr, qpack);
      left -= n;
      if (left > 0) ch = near_next[ch];
    }

    // reduce partitions, remove the self term, write in input order
    double vx = M.dx, vy = M.dy, vz = M.dz, vp = M.dp;
    for (int b = W; b < kWave; b <<= 1) {
      vx += shfl_xor_d(vx, b);
      vy += shfl_xor_d(vy, b);
      vz += shfl_xor_d(vz, b);
      vp += shfl_xor_d(vp, b);
    }
    if (prow >= 0) {
      if (part == 0 && u < m) {
        double *q = a.psum + 4 * ((int64_t)prow + b0 + u);
        q[0] = vx;
        q[1] = vy;
        q[2] = vz;
        q[3] = vp;
      }
    } else if (part == 0 && u < m) {
      const int i = gf + b0 + u;
      const float self_ri = __builtin_amdgcn_rsqf(__builtin_fmaf(0.0f, 0.0f, eps2));
      const double self = (double)((float)a.smass[i] * self_ri);
      const int o = a.perm[i];
      a.acc[3 * (int64_t)o] = (float)vx;
      a.acc[3 * (int64_t)o + 1] = (float)vy;
      a.acc[3 * (int64_t)o + 2] = (float)vz;
      a.pot[o] = (float)(self - vp);
    }
  }
}

}  // namespace

int force_lists_blocks_per_cu(bool quad) {
  int b = 0;
  const hipError_t e = quad ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_force_lists<true>, kWave, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_force_lists<false>, kWave, 0);
  if (e != hipSuccess || b < 1) b = 8;
  return b;
}

void force_lists_device(const ForceArgs &a, int grid, hipStream_t s) {
  if (a.far_slot && a.qpack)
    k_force_lists<true><<<(unsigned)grid, kWave, 0, s>>>(a, a.far_pool, a.far_next, a.near_pool, a.near_next,
                                                         a.glists, a.items, a.far_slot, a.qpack);
  else
    k_force_lists<false><<<(unsigned)grid, kWave, 0, s>>>(a, a.far_pool, a.far_next, a.near_pool, a.near_next,
                                                          a.glists, a.items, nullptr, nullptr);
}

}  // namespace bh
