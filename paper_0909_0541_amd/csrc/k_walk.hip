// Group walk that builds the interaction lists (Fig. "treewalk" for a group,
// Eq. 2/3; the interaction-list method of Sec. 3.2).
//
// One wavefront per group, persistent grid pulling groups from atomic
// queues.  The wave walks the tree in batches of up to 64 nodes taken from a
// stack of slot ranges (a cell's children occupy consecutive slots) kept in
// LDS.  Each lane tests one node with the FP64 opening test
// d^2 > (l/theta + s)^2, d = distance from the cell's centre of mass to the
// group's bounding box.  Accepted cells and reached particles are written to
// the group's lists in HBM as FP32 (x - c_g, m), c_g the box centre: the far
// list, and the near list for entries within kNearFrac * R of the box (R the
// box half-diagonal), which also keeps the FP32 rounding residue of x - c_g so
// that the force kernel can form dx exactly to FP32 for close pairs however
// large the group.  Opened cells push their child range.  Lists live in
// chunks taken from device pools with an atomic counter and linked per group;
// when a pool runs out the walk keeps counting, marks the group incomplete
// and the host grows the pool and walks again.
//
// Stack bound: a batch pops up to 64 nodes and pushes at most one range per
// node.  While the stack is high, the wave takes only the top range (at most 8
// cells) after the previous batch has pushed, which is a depth-first walk: at
// most 8 ranges per level above the point where it started, at most 23
// levels.  Batches of 64 are taken (ahead of the pushes of the batch in
// flight) only while at least 2 * 64 + 8 * 24 free entries remain, so the
// stack never exceeds its capacity; an overflow check still guards every
// push, and an iteration budget (a tree visits each slot once, and a batch
// is handled in two iterations) bounds the walk of every group.
#include "bh_device.h"

namespace bh {

namespace {

constexpr int kStack = 1024;      // range stack entries
constexpr int kReserve = 8 * 24;  // growth bound of the stack in one-range mode

// The block is one wavefront: a barrier orders its LDS writes and reads.
__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// Wave-uniform writer of one chunked list.
struct ChunkList {
  int head = -1;   // first chunk
  int cur = -1;    // chunk receiving entries
  int prev = -1;   // the chunk before it
  int count = 0;   // entries written
  int cap = 0;     // entries that fit in the chunks taken so far
};

// Make room for n more entries (n <= chunk size); returns false when the pool
// is exhausted (the list is then incomplete but keeps being counted).
__device__ __forceinline__ bool reserve(ChunkList &L, int n, int chunk, int *counter, int pool_chunks,
                                        int32_t *__restrict__ next, int lane, bool ok) {
  if (L.count + n <= L.cap) return ok;
  const int c = take_one(counter, lane);
  L.cap += chunk;
  if (!ok || c >= pool_chunks) return false;
  if (L.cur >= 0) {
    if (lane == 0) next[L.cur] = c;
  } else {
    L.head = c;
  }
  L.prev = L.cur;
  L.cur = c;
  return true;
}

// Chunk holding list position pos (the current one or the one before).
__device__ __forceinline__ int chunk_of(const ChunkList &L, int pos, int chunk) {
  return (pos / chunk == L.cap / chunk - 1) ? L.cur : L.prev;
}

__global__ __launch_bounds__(kWave) void k_walk_lists(WalkListArgs a) {
  __shared__ int2 stk[kStack];
  __shared__ int mark[kWave];
  const int lane = lane_id();
  const int G = a.info->n_groups;
  const int nslots = a.nsys + a.info->n_slots;

  // Groups are taken in Morton order from eight contiguous eighths, one per
  // XCD (workgroups go to the XCDs round robin), so that the waves sharing an
  // L2 walk neighbouring groups and read mostly the same nodes; a wave whose
  // eighth is done takes from the others.
  const int xcd = blockIdx.x & 7;
  int tried = 0;
  for (;;) {
    int g = -1;
    while (tried < 8) {
      const int x = (xcd + tried) & 7;
      const int s0 = (int)((int64_t)G * x / 8), s1 = (int)((int64_t)G * (x + 1) / 8);
      const int t = take_one(&a.info->xq[x], lane);
      if (s0 + t < s1) {
        g = s0 + t;
        break;
      }
      ++tried;
    }
    if (g < 0) break;

    const int gc = a.ginfo[3 * g + 1], gs = a.ginfo[3 * g + 2];
    double blo[3], bhi[3], cen[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      blo[k] = a.gbox[6 * (int64_t)g + k];
      bhi[k] = a.gbox[6 * (int64_t)g + 3 + k];
      cen[k] = __dmul_rn(__dadd_rn(blo[k], bhi[k]), 0.5);
    }
    double theta = a.theta_group ? (double)a.theta_group[g] : a.par[gs].theta;
    if (!(theta >= 0.0 && theta <= 1.0)) {
      if (lane == 0) atomicOr(&a.info->err, kErrTheta);
      theta = (theta > 1.0) ? 1.0 : 0.0;
    }
    // A cell's side is the root side times 2^-level exactly, so l / theta =
    // (side / theta) * 2^-level exactly: one division per group.
    const double side = a.sys[gs].side;
    const double side_theta = side / theta;
    const int side_exp = ilogb(side);
    double hd2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double e = __dsub_rn(bhi[k], blo[k]);
      hd2 = __dadd_rn(hd2, __dmul_rn(e, e));
    }
    // (kNearFrac * R)^2 with R^2 = |hi - lo|^2 / 4
    const double near2 = __dmul_rn(hd2, 0.25 * kNearFrac * kNearFrac);

    ChunkList F, N;
    bool fok = true, nok = true, corrupt = false;
    int sp = 1, nlist = 0;
    int budget = 4 * nslots + 4;
    double lmass = 0.0;
    if (lane == 0) stk[0] = make_int2(gs, 1);
    wave_sync();
    // Software pipeline: the records of the next batch are loaded while the
    // current batch is tested, so that one batch's memory latency hides
    // behind the other's work.  The next batch is taken from the stack before
    // the current batch pushes its children, except when the stack is high:
    // then the walk is the plain depth-first one of the stack bound above.
    int bcur = 0;
    NodeRec rcur;
    for (;;) {
      if (--budget < 0) {
        corrupt = true;
        break;
      }
      int bnext = 0, node = 0;
      const bool starved = sp > kStack - 2 * kWave - kReserve;
      if (sp > 0 && (bcur == 0 || !starved)) {
        const int nread = starved ? 1 : min(sp, kWave);
        int2 e = make_int2(0, 0);
        if (lane < nread) e = stk[sp - 1 - lane];
        const int cnt = (lane < nread) ? e.y : 0;
        const int pre = wave_inclusive_sum(cnt);
        const int total = __shfl(pre, nread - 1, kWave);
        bnext = min(starved ? 8 : kWave, total);
        const int start = pre - cnt;
        const int kfull = __popcll(__ballot(lane < nread && pre <= bnext));
        mark[lane] = -1;
        wave_sync();
        if (lane < nread && start < bnext) mark[start] = lane;
        wave_sync();
        const int ei = wave_inclusive_max(mark[lane]);
        const int e_start = __shfl(start, ei < 0 ? 0 : ei, kWave);
        const int e_first = __shfl(e.x, ei < 0 ? 0 : ei, kWave);
        const int nsp = sp - kfull;
        if (kfull < nread) {
          const int pstart = __shfl(start, kfull, kWave);
          if (pstart < bnext && lane == kfull)
            stk[sp - 1 - kfull] = make_int2(e.x + (bnext - pstart), e.y - (bnext - pstart));
        }
        sp = nsp;  // the partly taken range (if any) stays on the stack
        node = e_first + (lane - e_start);
        if (__ballot(lane < bnext && (node < 0 || node >= nslots))) {
          corrupt = true;  // corrupt range: report, never read out of bounds
          break;
        }
      }
      NodeRec rnext;
      if (lane < bnext) rnext = a.nodes[node];
      if (bcur > 0) {
        bool emit = false, push = false, near = false;
        float4 hi4 = make_float4(0.f, 0.f, 0.f, 0.f), lo4 = hi4;
        int2 rng = make_int2(0, 0);
        if (lane < bcur) {
          const NodeRec &r = rcur;
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
            double q = isfinite(r.l) ? ldexp(side_theta, ilogb(r.l) - side_exp) : r.l;
            q = __dadd_rn(q, r.s);
            const double seff = __dmul_rn(q, q);
            if (d2 > seff) emit = true;
            else push = true;
          }
          if (emit) {
            const double rx = __dsub_rn(r.com[0], cen[0]), ry = __dsub_rn(r.com[1], cen[1]),
                         rz = __dsub_rn(r.com[2], cen[2]);
            hi4 = make_float4((float)rx, (float)ry, (float)rz, (float)r.m);
            near = d2 <= near2;
            if (near)
              lo4 = make_float4((float)__dsub_rn(rx, (double)hi4.x), (float)__dsub_rn(ry, (double)hi4.y),
                                (float)__dsub_rn(rz, (double)hi4.z), 0.0f);
            lmass += r.m;
          }
          if (push) rng = make_int2(r.child, r.nchild);
        }
        const unsigned long long em = __ballot(emit), pm = __ballot(push);
        const unsigned long long nm = __ballot(emit && near), fm = em & ~nm;
        const int npush = __popcll(pm);
        if (sp + npush > kStack) {
          corrupt = true;
          break;
        }
        if (push) stk[sp + rank_below(pm)] = rng;
        const int nf = __popcll(fm), nn = __popcll(nm);
        if (nf > 0) {
          fok = reserve(F, nf, kFarChunk, &a.info->far_chunks, a.far_cap, a.far_next, lane, fok);
          if (fok && emit && !near) {
            const int pos = F.count + rank_below(fm);
            a.far_pool[(int64_t)chunk_of(F, pos, kFarChunk) * kFarChunk + pos % kFarChunk] = hi4;
          }
          F.count += nf;
        }
        if (nn > 0) {
          nok = reserve(N, nn, kNearChunk, &a.info->near_chunks, a.near_cap, a.near_next, lane, nok);
          if (nok && emit && near) {
            const int pos = N.count + rank_below(nm);
            float4 *base = a.near_pool + (int64_t)chunk_of(N, pos, kNearChunk) * (2 * kNearChunk);
            base[pos % kNearChunk] = hi4;
            base[kNearChunk + pos % kNearChunk] = lo4;
          }
          N.count += nn;
        }
        nlist += nf + nn;
        sp += npush;
      }
      wave_sync();
      bcur = bnext;
      rcur = rnext;
      if (bcur == 0 && sp == 0) break;
    }
    if (corrupt) {
      if (lane == 0) {
        atomicOr(&a.info->err, kErrStack);
        int32_t *q = a.glists + 4 * (int64_t)g;
        q[0] = -1;
        q[1] = 0;
        q[2] = -1;
        q[3] = 0;
      }
      continue;
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) lmass += shfl_xor_d(lmass, d);
    if (lane == 0) {
      int32_t *q = a.glists + 4 * (int64_t)g;
      q[0] = fok ? F.head : -1;
      q[1] = F.count;
      q[2] = nok ? N.head : -1;
      q[3] = N.count;
      if (!fok || !nok) atomicOr(&a.info->err, kErrPool);
      a.glist[g] = nlist;
      a.gmass[g] = lmass;
      atomicAdd(&a.info->interactions, (unsigned long long)gc * (unsigned long long)(nlist - 1));
      atomicAdd(&a.info->list_entries, (unsigned long long)nlist);
      atomicMax(&a.info->max_list, nlist);
    }
  }
}

__global__ void k_reset_queue(DevInfo *info) { info->queue = 0; }

// Probe walk of the learned-theta features: the group walk at theta = 1 (the
// traversal of k_walk_lists) with two shortcuts, summing over the entries
// instead of writing them.  A node that holds only members of the group is
// taken whole as inside mass, and a cell smaller than the box half-diagonal
// R is taken whole (as a monopole) without the opening test.  Sums: the field
// and its scale at the box centre from the entries whose centre of mass lies
// outside the box, the count of single particles among them, the number of
// entries and the mass inside the box.  Writes features f6..f10.
__global__ __launch_bounds__(kWave) void k_probe(ProbeArgs a) {
  __shared__ int2 stk[kStack];
  __shared__ int mark[kWave];
  const int lane = lane_id();
  const int G = a.info->n_groups;
  const int nslots = a.nsys + a.info->n_slots;
  for (;;) {
    const int g = take_one(&a.info->queue, lane);
    if (g >= G) break;
    const int gf = a.ginfo[3 * g], gc = a.ginfo[3 * g + 1], gs = a.ginfo[3 * g + 2];
    double blo[3], bhi[3], cen[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      blo[k] = a.gbox[6 * (int64_t)g + k];
      bhi[k] = a.gbox[6 * (int64_t)g + 3 + k];
      cen[k] = __dmul_rn(__dadd_rn(blo[k], bhi[k]), 0.5);
    }
    const double eps = a.eps[gs];
    const double eps2 = __dmul_rn(eps, eps);
    double hd2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double e = __dsub_rn(bhi[k], blo[k]);
      hd2 = __dadd_rn(hd2, __dmul_rn(e, e));
    }
    const double lmin = sqrt(hd2) / 2.0;  // cells smaller than the box half-diagonal are not opened
    double ax = 0.0, ay = 0.0, az = 0.0, S = 0.0, m_in = 0.0;
    int n_part = 0, nlist = 0;
    bool corrupt = false;
    int sp = 1;
    int budget = 2 * nslots + 2;
    if (lane == 0) stk[0] = make_int2(gs, 1);
    wave_sync();
    while (sp > 0) {
      if (--budget < 0) {
        corrupt = true;
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
      const int nsp = sp - kfull;
      if (kfull < nread) {
        const int pstart = __shfl(start, kfull, kWave);
        if (pstart < B && lane == kfull) stk[sp - 1 - kfull] = make_int2(e.x + (B - pstart), e.y - (B - pstart));
      }
      const int node = e_first + (lane - e_start);
      if (__ballot(lane < B && (node < 0 || node >= nslots))) {
        corrupt = true;
        break;
      }
      bool push = false, emit = false;
      int2 rng = make_int2(0, 0);
      if (lane < B) {
        const NodeRec r = a.nodes[node];
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double below = __dsub_rn(blo[k], r.com[k]);
          const double above = __dsub_rn(r.com[k], bhi[k]);
          const double ek = fmax(0.0, fmax(below, above));
          d2 = (k == 0) ? __dmul_rn(ek, ek) : __dadd_rn(d2, __dmul_rn(ek, ek));
        }
        // a node holding only members counts as inside and is not opened
        const bool member = r.first >= gf && r.first + r.count <= gf + gc;
        if (member || r.child < 0 || r.l < lmin) {
          emit = true;
        } else {
          const double q = __dadd_rn(r.l, r.s);  // l / theta + s at theta = 1
          if (d2 > __dmul_rn(q, q)) emit = true;
          else push = true;
        }
        if (emit) {
          if (member || d2 == 0.0) {
            m_in = __dadd_rn(m_in, r.m);
          } else {
            const double dx = __dsub_rn(r.com[0], cen[0]), dy = __dsub_rn(r.com[1], cen[1]),
                         dz = __dsub_rn(r.com[2], cen[2]);
            const double r2 =
                __dadd_rn(__dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)), eps2);
            const double w = r.m / __dmul_rn(r2, sqrt(r2));
            ax = __dadd_rn(ax, __dmul_rn(w, dx));
            ay = __dadd_rn(ay, __dmul_rn(w, dy));
            az = __dadd_rn(az, __dmul_rn(w, dz));
            S = __dadd_rn(S, r.m / r2);
            if (r.child < 0) ++n_part;
          }
        }
        if (push) rng = make_int2(r.child, r.nchild);
      }
      const unsigned long long pm = __ballot(push);
      const int npush = __popcll(pm);
      if (nsp + npush > kStack) {
        corrupt = true;
        break;
      }
      if (push) stk[nsp + rank_below(pm)] = rng;
      nlist += __popcll(__ballot(emit));
      wave_sync();
      sp = nsp + npush;
    }
    if (corrupt) {
      if (lane == 0) atomicOr(&a.info->err, kErrStack);
      continue;
    }
    double mg = 0.0;
    for (int i = gf + lane; i < gf + gc; i += kWave) mg = __dadd_rn(mg, a.smass[i]);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      ax += shfl_xor_d(ax, d);
      ay += shfl_xor_d(ay, d);
      az += shfl_xor_d(az, d);
      S += shfl_xor_d(S, d);
      m_in += shfl_xor_d(m_in, d);
      mg += shfl_xor_d(mg, d);
      n_part += __shfl_xor(n_part, d, kWave);
    }
    if (lane == 0) {
      const double tiny = 0x1p-100;
      float *f = a.feat + 12 * (int64_t)g;
      f[6] = (float)log2(__dadd_rn(sqrt(__dadd_rn(__dadd_rn(__dmul_rn(ax, ax), __dmul_rn(ay, ay)), __dmul_rn(az, az))),
                                   tiny));
      f[7] = (float)log2(__dadd_rn(S, tiny));
      f[8] = (float)log2(1.0 + (double)n_part);
      f[9] = (float)log2((double)nlist);
      f[10] = (float)log2(m_in / mg);
    }
  }
}

}  // namespace

int walk_lists_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_walk_lists, kWave, 0) != hipSuccess || b < 1) b = 8;
  return b;
}

void walk_lists_device(const WalkListArgs &a, int grid, hipStream_t s) {
  k_walk_lists<<<(unsigned)grid, kWave, 0, s>>>(a);
}

int probe_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_probe, kWave, 0) != hipSuccess || b < 1) b = 8;
  return b;
}

void probe_device(const ProbeArgs &a, int grid, hipStream_t s) {
  k_reset_queue<<<1, 1, 0, s>>>(a.info);
  k_probe<<<(unsigned)grid, kWave, 0, s>>>(a);
}

}  // namespace bh
