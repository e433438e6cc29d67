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
// flight) only while at least 3 * 64 + 8 * 24 free entries remain (one batch
// more for a hand-over, below), so the stack never exceeds its capacity; an
// overflow check still guards every push, and an iteration budget (a tree
// visits each slot once, and a batch is handled in two iterations) bounds
// the walk of every group.
//
// Split walks: a walk that has tested visit_cap nodes deals the nodes left on
// its stack to up to 16 tasks and ends its own segment of the group's list;
// tasks run in the same launch (tasks first, then groups), hand over again
// up to kSplitDepth levels, and are keyed so that the order in which
// segments are summed does not depend on when or where they ran.
#include "bh_device.h"

namespace bh {

namespace {

constexpr int kStack = 1024;      // range stack entries
constexpr int kReserve = 8 * 24;  // growth bound of the stack in one-range mode
constexpr int kTaskStack = 512;   // largest first stack of a task
constexpr int kWaiters = 256;     // waves that wait for tasks once the groups are taken
constexpr int kProbeStack = 512;  // range stack of the probe walk (its theta = 1 lists are short)

__device__ __forceinline__ double norm3(double a, double b, double c) {
  return sqrt(__dadd_rn(__dadd_rn(__dmul_rn(a, a), __dmul_rn(b, b)), __dmul_rn(c, c)));
}

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

// The list chunks of one wave: taken from the pool kChunkRun at a time (one
// atomic on the shared counter per run) and handed out in order; the rest of a
// run carries over from unit to unit.  The next run is requested while the
// list is within two batches of needing a chunk and the current run is used
// up, together with a batch's node loads, and its number is read at the top
// of the next iteration, so the atomic's round trip overlaps a batch.
struct ChunkSource {
  int next = 0, end = 0;  // chunks [next, end) of the current run
  int spare = -1;         // a run that has arrived
  int req = 0;            // a requested run (VGPR, read once arrived)
  bool pend = false;
};

__device__ __forceinline__ int take_chunk(ChunkSource &S, int *counter, int lane) {
  if (S.next >= S.end) {
    const int run = (S.spare >= 0) ? S.spare : take_one(counter, lane);
    S.spare = -1;
    S.next = run * kChunkRun;
    S.end = S.next + kChunkRun;
  }
  return S.next++;
}

// Make room for n more entries (n <= chunk size); returns false when the pool
// is exhausted (the list is then incomplete but keeps being counted).
__device__ __forceinline__ bool reserve(ChunkList &L, int n, int chunk, ChunkSource &S, int *counter,
                                        int pool_chunks, int32_t *__restrict__ next, int lane, bool ok) {
  if (L.count + n <= L.cap) return ok;
  const int c = take_chunk(S, counter, lane);
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
  return (pos >= L.cap - chunk) ? L.cur : L.prev;  // cap is a multiple of chunk, pos < cap
}

// Task slots: rcount -1 until published, then the task's range count, or 0
// for a slot that a hand-over reserved but could not fill (a pool ran out).
// Wait for slot t: returns its rcount, or -1 when it is still unpublished and
// no unit is left that could publish it.  The polls are relaxed loads (an
// acquiring load would invalidate the L2 that the walking waves read their
// nodes from, on every poll); one acquire fence follows what was seen.
__device__ __forceinline__ int wait_slot(const WalkListArgs &a, int t, int lane) {
  const long long t0 = wall_clock64();
  int r = -1;
  for (int poll = 0;; ++poll) {
    const int rc = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&a.tasks[t].rcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (rc >= 0) {
      r = rc;
      break;
    }
    // every unit publishes its tasks before it leaves the count of pending
    // units (read every fourth poll: all waiting waves read this one word)
    const int p = (poll & 3) ? 1 : __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&a.ctr->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (p <= 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      r = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(&a.tasks[t].rcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      break;
    }
    if (wall_clock64() - t0 > a.wait_ticks) {
      if (lane == 0) atomicOr(&a.info->err, kErrWait);
      break;
    }
    __builtin_amdgcn_s_sleep(60);
  }
  if (r > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the task's fields and ranges
  return r;
}

// The next unit of a wave: its group, with task >= 0 when it is a task; a
// negative group when the wave has no more work.  A wave looks for tasks
// once the group queues are empty (a look at the shared task counters before
// every group would make every unit wait on a line that the units' own
// counter keeps busy): a task continues a long walk, and the tasks run in
// the tail of the launch, where the waves left have nothing else to do.  A
// wave that sees a reserved slot no wave has claimed takes a ticket (the
// next slot number); a ticket whose slot is not yet published is looked at
// again at the end of each unit.  When no group is left, the wave waits for
// its ticket's slot (taking a ticket if it has none): the waiting waves form
// a queue in slot order.  Groups are taken in
// Morton order from eight contiguous eighths, one per XCD (workgroups go to
// the XCDs round robin), so that the waves sharing an L2 walk neighbouring
// groups and read mostly the same nodes; a wave whose eighth is done takes
// from the others.  With an order (learned theta), the q-th group taken from
// an eighth is the q-th of that eighth in the order: longest predicted walk
// first, so that the walks taken last are short ones.
template <bool SPLIT>
__device__ __forceinline__ int next_unit(const WalkListArgs &a, int G, int xcd, int &tried, int &ticket, bool &waiter,
                                         int &task, int lane) {
  task = -1;
  int g = -1;
  for (;;) {
    int rc = -1;
    if (SPLIT && a.visit_cap > 0) {
      if (ticket < 0 && tried >= 8) {
        const int head = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&a.ctr->queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const int res = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&a.ctr->tasks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (head < min(res, a.task_cap)) ticket = take_one(&a.ctr->queue, lane);
      }
      if (ticket >= 0 && ticket < a.task_cap)
        rc = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&a.tasks[ticket].rcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    if (rc < 0) {  // no published task at hand: a group
      while (tried < 8) {
        const int x = __builtin_amdgcn_readfirstlane((xcd + tried) & 7);
        const int s0 = (int)((int64_t)G * x / 8), s1 = (int)((int64_t)G * (x + 1) / 8);
        const int q = take_one(&a.info->xq[x * kLineInts], lane);
        if (s0 + q < s1) {
          g = s0 + q;
          if (a.order) {
            // the eighth's groups in the given order (a value outside the
            // eighth is reported and the Morton place taken instead)
            const int o = __builtin_amdgcn_readfirstlane(a.order[s0 + q]);
            if (o >= s0 && o < s1) g = o;
            else if (lane == 0) atomicOr(&a.info->err, kErrStack);
          }
          break;
        }
        ++tried;
      }
      if (g >= 0 || !SPLIT || a.visit_cap <= 0) break;
      if (ticket < 0) {
        // a bounded number of waves wait for tasks; the others leave (a
        // wave that holds no ticket owes no slot), which keeps the polling
        // of the waiting waves from slowing the last walks
        if (!waiter) {
          if (take_one(&a.ctr->waiters, lane) >= kWaiters) break;
          waiter = true;
        }
        ticket = take_one(&a.ctr->queue, lane);
      }
      if (ticket >= a.task_cap) break;  // no slot beyond the capacity is ever written
      rc = wait_slot(a, ticket, lane);
      if (rc < 0) break;
    } else if (rc > 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the task's fields and ranges
    }
    const int t = ticket;
    ticket = -1;
    if (rc > 0) {
      g = __builtin_amdgcn_readfirstlane(a.tasks[t].g);
      if (g >= 0 && g < G) {
        task = t;
      } else {  // corrupt: report, retire the unit, stop this wave
        if (lane == 0) atomicOr(&a.info->err, kErrStack);
        atomicAdd(&a.ctr->pending, lane == 0 ? -1 : 0);
        g = -1;
      }
      break;
    }
    // rc == 0: a slot released empty; look again
  }
  return g;
}

// Hand-over depth of a task from its key (key = 17 K + j + 1, K the parent's).
__device__ __forceinline__ int key_depth(int key) {
  int d = 0;
  for (int k = key; k > 0 && d < 8; k = (k - 1) / (kDonateTasks + 1)) ++d;
  return d;
}

// One unit of walk per pass of the outer loop: a group's whole walk, or a
// task handed over by a walk that reached the visit cap.  Units take chunks
// for their own list (the group's list unless the walk splits, else a
// segment).
// Four waves per SIMD: the split variant needs 128 VGPRs (a few spilled),
// and four hide more of the node reads' latency than three (measured 5 %
// (2M particles) to 10 % (8M) shorter walks).  SPLIT = false compiles the
// walk without split walks (no tasks, no hand-over): 106 VGPRs and 2 scalar
// registers spilled to vector lanes, 5 % faster than the split variant; at
// five waves per SIMD (96 VGPRs, a few spilled) it is 1-2 % slower.  The
// batch size is read as a wave-uniform value, which keeps the batch
// bookkeeping in scalar registers (it took 16 more VGPRs and 17 more scalar
// spills, and 11-13 % more time, when the compiler had to treat it as
// per-lane).  SLOTS: the far entries' node slots are recorded (the
// quadrupole sums); without them the pool pointer and its test leave the
// loop.
template <bool SPLIT, bool SLOTS>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_walk_lists(WalkListArgs a) {
  __shared__ int2 stk[kStack];
  __shared__ int mark[kWave];
  const int lane = lane_id();
  const int G = a.info->n_groups;
  const int nslots = a.nsys + a.info->n_slots;
  // the automatic cap also stays above a multiple of the last mean list
  int visit_cap = SPLIT ? a.visit_cap : 0;
  if (SPLIT && visit_cap > 0 && a.mean_list)
    visit_cap = max(visit_cap, kSplitMeanFactor * min(__builtin_amdgcn_readfirstlane(a.mean_list[0]), INT32_MAX / 64));

  const int xcd = blockIdx.x & 7;
  int tried = 0, ticket = -1;
  bool waiter = false;
  ChunkSource fsrc, nsrc;  // this wave's far and near list chunks
  for (;;) {
    int task;
    const int g = next_unit<SPLIT>(a, G, xcd, tried, ticket, waiter, task, lane);
    if (g < 0) break;
    const bool is_task = task >= 0;

    const int gc = a.ginfo[3 * g + 1], gs = a.ginfo[3 * g + 2];
    double blo[3], bhi[3], cen[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      blo[k] = a.gbox[6 * (int64_t)g + k];
      bhi[k] = a.gbox[6 * (int64_t)g + 3 + k];
      cen[k] = __dmul_rn(__dadd_rn(blo[k], bhi[k]), 0.5);
    }
    double theta = a.theta_group ? (double)a.theta_group[g] : a.par[gs].theta;
    if (isnan(theta)) {
      // no usable per-group value (e.g. a network whose output is not a
      // number): this group walks with the call's theta
      theta = a.par[gs].theta;
      if (lane == 0 && !is_task) atomicAdd(&a.info->theta_fallback, 1);
    }
    if (!(theta >= 0.0 && theta <= 1.0)) {
      if (lane == 0 && !is_task) atomicOr(&a.info->err, kErrTheta);
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
    bool fok = true, nok = true, corrupt = false, handed = false;
    int sp, nlist = 0, key = 0;
    int budget = 4 * nslots + 4;
    double lmass = 0.0;
    if (!is_task) {
      if (lane == 0) stk[0] = make_int2(gs, 1);
      sp = 1;
    } else {
      const WalkTask tk = a.tasks[task];
      sp = tk.rcount;
      key = tk.key;
      if (tk.roff < 0 || tk.rcount < 1 || tk.rcount > kStack || tk.roff + tk.rcount > a.range_cap) {
        corrupt = true;
        sp = 0;
      } else {
        for (int k = lane; k < sp; k += kWave) stk[k] = a.ranges[tk.roff + k];
      }
    }
    // units at the deepest level walk to the end
    int cap = (SPLIT && visit_cap > 0 && key_depth(key) < kSplitDepth) ? visit_cap : 0;
    wave_sync();
    int visits = 0;
    // Software pipeline: the records of the next batch are loaded while the
    // current batch is tested, so that one batch's memory latency hides
    // behind the other's work.  The next batch is taken from the stack before
    // the current batch pushes its children, except when the stack is high:
    // then the walk is the plain depth-first one of the stack bound above.
    int bcur = 0, ncur = 0;
    NodeRec rcur;
    for (;;) {
      if (--budget < 0) {
        corrupt = true;
        break;
      }
      if (fsrc.pend) {
        fsrc.spare = __builtin_amdgcn_readfirstlane(fsrc.req);
        fsrc.pend = false;
      }
      if (nsrc.pend) {
        nsrc.spare = __builtin_amdgcn_readfirstlane(nsrc.req);
        nsrc.pend = false;
      }
      int bnext = 0, node = 0;
      const bool starved = sp > kStack - 3 * kWave - kReserve;
      if (sp > 0 && (bcur == 0 || !starved)) {
        const int nread = starved ? 1 : min(sp, kWave);
        int2 e = make_int2(0, 0);
        if (lane < nread) e = stk[sp - 1 - lane];
        const int cnt = (lane < nread) ? e.y : 0;
        const int pre = wave_inclusive_sum(cnt);
        const int total = __builtin_amdgcn_readfirstlane(__shfl(pre, nread - 1, kWave));
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
          const int pstart = __builtin_amdgcn_readfirstlane(__shfl(start, kfull, kWave));
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
      if (fsrc.spare < 0 && fsrc.next >= fsrc.end && F.cap - F.count < 2 * kWave) {
        fsrc.req = atomicAdd(&a.info->far_chunks, lane == 0 ? 1 : 0);
        fsrc.pend = true;
      }
      if (nsrc.spare < 0 && nsrc.next >= nsrc.end && N.cap - N.count < 2 * kWave) {
        nsrc.req = atomicAdd(&a.info->near_chunks, lane == 0 ? 1 : 0);
        nsrc.pend = true;
      }
      if (bcur > 0) {
        visits += bcur;
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
            // (a near entry's residue carries in .w the node slot of a cell, -1
            // for a particle, for the quadrupole sums)
            if (near)
              lo4 = make_float4((float)__dsub_rn(rx, (double)hi4.x), (float)__dsub_rn(ry, (double)hi4.y),
                                (float)__dsub_rn(rz, (double)hi4.z), __int_as_float(r.child < 0 ? -1 : ncur));
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
          fok = reserve(F, nf, a.far_tile, fsrc, &a.info->far_chunks, a.far_cap, a.far_next, lane, fok);
          if (fok && emit && !near) {
            const int pos = F.count + rank_below(fm);
            const int64_t at = (int64_t)chunk_of(F, pos, a.far_tile) * a.far_tile + (pos & (a.far_tile - 1));
            a.far_pool[at] = hi4;
            if (SLOTS) a.far_slot[at] = rcur.child < 0 ? -1 : ncur;
          }
          F.count += nf;
        }
        if (nn > 0) {
          nok = reserve(N, nn, a.near_tile, nsrc, &a.info->near_chunks, a.near_cap, a.near_next, lane, nok);
          if (nok && emit && near) {
            const int pos = N.count + rank_below(nm);
            float4 *base = a.near_pool + (int64_t)chunk_of(N, pos, a.near_tile) * (2 * a.near_tile);
            base[pos & (a.near_tile - 1)] = hi4;
            base[a.near_tile + (pos & (a.near_tile - 1))] = lo4;
          }
          N.count += nn;
        }
        nlist += nf + nn;
        sp += npush;
      }
      wave_sync();
      bcur = bnext;
      rcur = rnext;
      ncur = node;
      if (bcur == 0 && sp == 0) break;
      // Visit cap reached: hand the rest (the popped batch as runs of
      // consecutive nodes, then the stack) to new tasks.
      if (SPLIT && cap > 0 && visits >= cap) {
        if (bcur > 0) {
          const int prev = __shfl_up(ncur, 1, kWave);
          const bool head = lane < bcur && (lane == 0 || ncur != prev + 1);
          const unsigned long long hm = __ballot(head);
          const int runs = __popcll(hm);
          if (sp + runs > kStack) {
            corrupt = true;
            break;
          }
          if (head) {
            // run length: up to the next head (or the end of the batch)
            const unsigned long long later = hm & ~((2ull << lane) - 1ull);
            const int end = later ? (__ffsll((long long)later) - 1) : bcur;
            stk[sp + rank_below(hm)] = make_int2(ncur, end - lane);
          }
          sp += runs;
          bcur = 0;
          wave_sync();
        }
        // The stack's nodes (bottom first) are dealt to the tasks round robin,
        // one node per range: the ranges at the bottom were pushed first and
        // hold the largest subtrees, and dealing spreads them over the tasks.
        int T = 0;
        for (int k0 = 0; k0 < sp; k0 += kWave) {
          const int c = (k0 + lane < sp) ? stk[k0 + lane].y : 0;
          T += __shfl(wave_inclusive_sum(c), kWave - 1, kWave);
        }
        T = __builtin_amdgcn_readfirstlane(T);
        const int nt = min(kDonateTasks, T);
        // (a task's first stack must leave the room of the stack bound above;
        // a larger stack, possible only under cells with very many
        // coincident particles, is walked on by this unit)
        const bool fits = T <= kDonateTasks * kTaskStack;
        const int off = __builtin_amdgcn_readfirstlane(atomicAdd(&a.ctr->ranges, (lane == 0 && fits) ? T : 0));
        const int toff = __builtin_amdgcn_readfirstlane(atomicAdd(&a.ctr->tasks, (lane == 0 && fits) ? nt : 0));
        if (!fits) {
          cap = 0;
        } else if (off + T > a.range_cap || toff + nt > a.task_cap) {
          // no room: report (the host grows the pools and walks again), walk
          // on as one unit, and release the reserved slots empty
          if (lane == 0) atomicOr(&a.info->err, kErrPool);
          if (lane < nt && toff + lane < a.task_cap)
            __hip_atomic_store(&a.tasks[toff + lane].rcount, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          cap = 0;
        } else {
          // count the new units before any of them can run and finish
          const int pend = atomicAdd(&a.ctr->pending, lane == 0 ? nt : 0);
          if (__builtin_amdgcn_readfirstlane(pend) < 0 && lane == 0) atomicOr(&a.info->err, kErrStack);
          // node q goes to task q % nt, as its (q / nt)-th range; task j's
          // ranges start at j * (T / nt) + min(j, T % nt)
          const int per = T / nt, extra = T % nt;
          int q0 = 0;
          for (int k0 = 0; k0 < sp; k0 += kWave) {
            const int2 e = (k0 + lane < sp) ? stk[k0 + lane] : make_int2(0, 0);
            const int inc = wave_inclusive_sum(e.y);
            for (int u = 0; u < e.y; ++u) {
              const int q = q0 + inc - e.y + u, j = q % nt;
              a.ranges[off + j * per + min(j, extra) + q / nt] = make_int2(e.x + u, 1);
            }
            q0 += __shfl(inc, kWave - 1, kWave);
          }
          const int cnt = (lane < nt) ? per + (lane < extra ? 1 : 0) : 0;
          if (lane < nt) {
            WalkTask *tk = a.tasks + toff + lane;
            tk->g = g;
            tk->roff = off + lane * per + min(lane, extra);
            tk->key = key * (kDonateTasks + 1) + lane + 1;
          }
          // publish: every lane's ranges and task fields before any rcount
          wave_sync();
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (lane < nt)
            __hip_atomic_store(&a.tasks[toff + lane].rcount, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          handed = true;
          sp = 0;
          break;
        }
      }
    }
    if (lane == 0) {
      atomicAdd(&a.info->node_visits, (unsigned long long)visits);
      atomicAdd(&a.info->near_entries, (unsigned long long)N.count);
    }
    if (!corrupt) {
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) lmass += shfl_xor_d(lmass, d);
      if (!fok || !nok) {
        if (lane == 0) atomicOr(&a.info->err, kErrPool);
      }
    }
    if (corrupt) {
      if (lane == 0) {
        atomicOr(&a.info->err, kErrStack);
        if (!is_task) {
          int32_t *q = a.glists + 4 * (int64_t)g;
          q[0] = -1;
          q[1] = 0;
          q[2] = -1;
          q[3] = 0;
          a.gsplit[g] = 0;
          a.glist[g] = 0;
        }
      }
    } else if (!is_task && !handed) {
      if (lane == 0) {
        int32_t *q = a.glists + 4 * (int64_t)g;
        q[0] = fok ? F.head : -1;
        q[1] = F.count;
        q[2] = nok ? N.head : -1;
        q[3] = N.count;
        a.gsplit[g] = 0;
        a.glist[g] = nlist;  // statistics are summed from these after the walk
        a.gmass[g] = lmass;
      }
    } else {
      // a segment of a split group: its list so far; totals come later
      const int sidx = __builtin_amdgcn_readfirstlane(atomicAdd(&a.ctr->segs, lane == 0 ? 1 : 0));
      if (lane == 0) {
        if (!is_task) {
          int32_t *q = a.glists + 4 * (int64_t)g;
          q[0] = -1;
          q[1] = 0;
          q[2] = -1;
          q[3] = 0;
          a.gsplit[g] = 1;
          atomicAdd(&a.ctr->n_split, 1);
        }
        atomicMax(&a.ctr->depth, key_depth(key) + (handed ? 1 : 0));
        if (sidx < a.seg_cap) {
          Segment sg;
          sg.g = g;
          sg.key = key;
          sg.fh = fok ? F.head : -1;
          sg.fn = F.count;
          sg.nh = nok ? N.head : -1;
          sg.nn = N.count;
          sg.len = nlist;
          sg.pad = 0;
          sg.mass = lmass;
          a.segs[sidx] = sg;
        } else {
          atomicOr(&a.info->err, kErrPool);
        }
      }
    }
    // this unit is done; a unit that published tasks orders them before
    // its decrement (the others published nothing that waiters read)
    if (SPLIT && a.visit_cap > 0) {
      if (handed) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      atomicAdd(&a.ctr->pending, lane == 0 ? -1 : 0);
    }
  }
}

// Counters of the split walk, and every task slot unpublished (rcount -1).
__global__ void k_split_reset(SplitCounters *ctr, const DevInfo *info, WalkTask *tasks, int task_cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctr->tasks = 0;
    ctr->queue = 0;
    ctr->ranges = 0;
    ctr->segs = 0;
    ctr->n_split = 0;
    ctr->pending = info->n_groups;
    ctr->depth = 0;
    ctr->waiters = 0;
  }
  if (i < task_cap) tasks[i].rcount = -1;
}

__global__ void k_reset_queue(DevInfo *info) {
  info->queue = 0;
  for (int x = 0; x < 8; ++x) info->xq[x * kLineInts] = 0;
}

// Probe walk of the learned-theta features: the group walk at theta = 1 (the
// traversal of k_walk_lists) with two shortcuts, summing over the entries
// instead of writing them.  A node that holds only members of the group is
// taken whole as inside mass, and a cell smaller than the box half-diagonal
// R is taken whole (as a monopole) without the opening test.  Sums: the field
// and its scale at the box centre from the entries whose centre of mass lies
// outside the box, the count of single particles among them, the number of
// entries and the mass inside the box.  Writes features f6..f10, and the
// group's own features f0..f5 and f11 (members' mass and centre of mass, the
// smallest split cell holding more than the group and the one above it).
// Seven waves per SIMD (at most 72 VGPRs, no spills) hide more of the node
// reads' latency than the five the compiler would choose: measured 22 % (2M)
// and 31 % (4M) shorter feature stages.
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(7, 7))) void k_probe(ProbeArgs a) {
  __shared__ int2 stk[kProbeStack];
  __shared__ int mark[kWave];
  const int lane = lane_id();
  const int G = a.info->n_groups;
  const int nslots = a.nsys + a.info->n_slots;
  // groups in Morton order from eight contiguous eighths, one per XCD (as the
  // list walk takes them), so that the waves sharing an L2 read mostly the
  // same nodes; a wave whose eighth is done takes from the others
  const int xcd = blockIdx.x & 7;
  int tried = 0;
  for (;;) {
    int g = -1;
    while (tried < 8) {
      const int x = __builtin_amdgcn_readfirstlane((xcd + tried) & 7);
      const int s0 = (int)((int64_t)G * x / 8), s1 = (int)((int64_t)G * (x + 1) / 8);
      const int q = take_one(&a.info->xq[x * kLineInts], lane);
      if (s0 + q < s1) {
        g = s0 + q;
        break;
      }
      ++tried;
    }
    if (g < 0) break;
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
      const bool starved = sp > kProbeStack - kWave - kReserve;
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
      if (nsp + npush > kProbeStack) {
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
    // the members' mass and mass moments
    double mg = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    for (int i = gf + lane; i < gf + gc; i += kWave) {
      const double m = a.smass[i];
      const double *x = a.spos + 3 * (int64_t)i;
      mg = __dadd_rn(mg, m);
      mx = __dadd_rn(mx, __dmul_rn(m, x[0]));
      my = __dadd_rn(my, __dmul_rn(m, x[1]));
      mz = __dadd_rn(mz, __dmul_rn(m, x[2]));
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      ax += shfl_xor_d(ax, d);
      ay += shfl_xor_d(ay, d);
      az += shfl_xor_d(az, d);
      S += shfl_xor_d(S, d);
      m_in += shfl_xor_d(m_in, d);
      mg += shfl_xor_d(mg, d);
      mx += shfl_xor_d(mx, d);
      my += shfl_xor_d(my, d);
      mz += shfl_xor_d(mz, d);
      n_part += __shfl_xor(n_part, d, kWave);
    }
    if (lane == 0) {
      const double tiny = 0x1p-100;
      float *f = a.feat + 12 * (int64_t)g;
      f[6] = (float)log2(__dadd_rn(norm3(ax, ay, az), tiny));
      f[7] = (float)log2(__dadd_rn(S, tiny));
      f[8] = (float)log2(1.0 + (double)n_part);
      f[9] = (float)log2((double)nlist);
      f[10] = (float)log2(m_in / mg);
      // the group's own features
      const double R = sqrt(hd2) / 2.0;
      const double re = __dadd_rn(R, eps);
      f[0] = (float)log2((double)gc);
      f[1] = (float)log2(__dadd_rn(1.0, R / eps));
      f[2] = (float)(norm3(__dsub_rn(mx / mg, cen[0]), __dsub_rn(my / mg, cen[1]), __dsub_rn(mz / mg, cen[2])) / re);
      // A1: the smallest split cell (not a bucket) holding more than c
      // particles (the cells of this tree are split cells: single-child
      // chains are not kept), A2 the next one above it
      float f3 = 0.0f, f4 = 0.0f, f5 = 0.0f, f11 = 0.0f;
      int p = a.pparent[gf];
      for (int it = 0; p >= 0 && (a.level[p] == kKeyLevels || a.ccount[p] <= gc); ++it) {
        if (it > 2 * kKeyLevels + 2) {
          atomicOr(&a.info->err, kErrBuild);
          p = -1;
          break;
        }
        p = a.cparent[p];
      }
      if (p >= 0) {
        const int q = a.cparent[p];
        const NodeRec r1 = a.nodes[a.cslot[p]];
        const NodeRec r2 = a.nodes[a.cslot[q >= 0 ? q : p]];
        f3 = (float)log2(r1.l / re);
        f4 = (float)log2(r1.m / mg);
        f5 = (float)(norm3(__dsub_rn(r1.com[0], cen[0]), __dsub_rn(r1.com[1], cen[1]), __dsub_rn(r1.com[2], cen[2])) /
                     r1.l);
        f11 = (float)log2(r2.m / mg);
      }
      f[3] = f3;
      f[4] = f4;
      f[5] = f5;
      f[11] = f11;
    }
  }
}

}  // namespace

int walk_lists_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_walk_lists<true, true>, kWave, 0) != hipSuccess || b < 1)
    b = 8;
  return b;
}

void walk_lists_device(const WalkListArgs &a, int grid, hipStream_t s) {
  const bool slots = a.far_slot != nullptr;
  if (a.visit_cap > 0) {
    if (slots)
      k_walk_lists<true, true><<<(unsigned)grid, kWave, 0, s>>>(a);
    else
      k_walk_lists<true, false><<<(unsigned)grid, kWave, 0, s>>>(a);
  } else {
    if (slots)
      k_walk_lists<false, true><<<(unsigned)grid, kWave, 0, s>>>(a);
    else
      k_walk_lists<false, false><<<(unsigned)grid, kWave, 0, s>>>(a);
  }
}

void split_reset(SplitCounters *ctr, const DevInfo *info, WalkTask *tasks, int task_cap, hipStream_t s) {
  k_split_reset<<<(unsigned)((task_cap + 255) / 256), 256, 0, s>>>(ctr, info, tasks, task_cap);
}

int probe_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_probe, kWave, 0) != hipSuccess || b < 1) b = 8;
  return b;
}

void probe_device(const ProbeArgs &a, int grid, bool reset, hipStream_t s) {
  if (reset) k_reset_queue<<<1, 1, 0, s>>>(a.info);
  k_probe<<<(unsigned)grid, kWave, 0, s>>>(a);
}

}  // namespace bh
