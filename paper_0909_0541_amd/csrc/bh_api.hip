// C ABI of libbh: context, workspaces, argument checks and stage order.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>

#include "bh_device.h"

namespace bh {

namespace {

// Zero every word of the counters (one block; the struct is a few lines).
__global__ void k_reset_info(DevInfo *info) {
  static_assert(sizeof(DevInfo) % sizeof(int32_t) == 0, "DevInfo is a whole number of words");
  int32_t *w = reinterpret_cast<int32_t *>(info);
  for (int i = threadIdx.x; i < (int)(sizeof(DevInfo) / sizeof(int32_t)); i += blockDim.x) w[i] = 0;
}

__global__ void k_export_nodes(const NodeRec *__restrict__ nodes, const int8_t *__restrict__ meta,
                               const DevInfo *__restrict__ info, int nsys, int32_t *__restrict__ ints,
                               double *__restrict__ reals) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t slots = (int64_t)nsys + info->n_slots;
  if (k >= slots) return;
  const NodeRec r = nodes[k];
  const int mt = meta[k];
  const int kind = mt >> 5;
  const int level = ((mt & 31) == 31) ? -1 : (mt & 31);
  if (ints) {
    int32_t *o = ints + 6 * k;
    o[0] = level;
    o[1] = kind;
    o[2] = r.first;
    o[3] = r.count;
    o[4] = r.child;
    o[5] = r.nchild;
  }
  if (reals) {
    double *o = reals + 6 * k;
    o[0] = r.m;
    o[1] = r.com[0];
    o[2] = r.com[1];
    o[3] = r.com[2];
    o[4] = r.l;
    o[5] = r.s;
  }
}

// Second moments per slot; zero for particle leaves and empty roots (their
// rows of qmom are never written).
__global__ void k_export_moments(const NodeRec *__restrict__ nodes, const double *__restrict__ qmom,
                                 const DevInfo *__restrict__ info, int nsys, double *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t slots = (int64_t)nsys + info->n_slots;
  if (k >= slots) return;
  const bool leaf = nodes[k].child < 0;
  for (int j = 0; j < 6; ++j) out[6 * k + j] = leaf ? 0.0 : qmom[6 * k + j];
}

__global__ void k_copy_keys(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_copy_i32(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_export_groups(const int32_t *__restrict__ ginfo, const double *__restrict__ gbox,
                                const int32_t *__restrict__ glist, const double *__restrict__ gmass,
                                const DevInfo *__restrict__ info, int32_t *ints, double *box, int32_t *ll,
                                double *lm) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= info->n_groups) return;
  if (ints)
    for (int k = 0; k < 3; ++k) ints[3 * g + k] = ginfo[3 * g + k];
  if (box)
    for (int k = 0; k < 6; ++k) box[6 * g + k] = gbox[6 * g + k];
  if (ll) ll[g] = glist[g];
  if (lm) lm[g] = gmass[g];
}

inline unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void reset_info_device(DevInfo *info, hipStream_t s) { k_reset_info<<<1, 256, 0, s>>>(info); }

bh_status fail(bh_ctx *c, bh_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

bh_status hip_check(bh_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return BH_OK;
  return fail(c, BH_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bh_status ensure(bh_ctx *c, DevBuf &b, size_t bytes, const char *what) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return BH_OK;
  if (c->capturing) return fail(c, BH_EINTERNAL, std::string("buffer growth while capturing: ") + what);
  if (c->graph) {  // the captured step points at the buffer about to move
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return hip_check(c, e, "hipFree");
    b.p = nullptr;
    b.bytes = 0;
  }
  // grow geometrically so that slowly increasing sizes do not reallocate often
  size_t want = bytes + bytes / 8;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(c, BH_ENOMEM, std::string("hipMalloc failed for ") + what);
  }
  b.bytes = want;
  return BH_OK;
}

static void free_buf(DevBuf &b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

template <class T>
static T *P(DevBuf &b) {
  return reinterpret_cast<T *>(b.p);
}

static bh_status timer_start(bh_ctx *c, Timer &t) {
  t.open = false;
  if (!c->opt.timing || c->capturing) return BH_OK;
  if (t.used >= 4096) return BH_OK;  // bounded: later calls of a long run are not timed
  while ((int)t.ev.size() < 2 * (t.used + 1)) {
    hipEvent_t e;
    bh_status st = hip_check(c, hipEventCreate(&e), "hipEventCreate");
    if (st) return st;
    t.ev.push_back(e);
  }
  t.open = true;
  return hip_check(c, hipEventRecord(t.ev[2 * t.used], c->stream), "hipEventRecord");
}

static bh_status timer_stop(bh_ctx *c, Timer &t) {
  if (!t.open) return BH_OK;
  t.open = false;
  bh_status st = hip_check(c, hipEventRecord(t.ev[2 * t.used + 1], c->stream), "hipEventRecord");
  if (st == BH_OK) t.used++;
  return st;
}

// Sum of the recorded intervals (the stream must be synchronised); resets.
static double timer_take(Timer &t, int32_t *calls) {
  double total = 0.0;
  for (int k = 0; k < t.used; ++k) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]) == hipSuccess) total += (double)ms;
  }
  *calls = t.used;
  t.used = 0;
  return total;
}

// Copy host data to the device through a pinned staging buffer; the staging
// buffer is reused only after the previous upload has completed.
static bh_status upload(bh_ctx *c, void *dst, const void *src, size_t bytes) {
  if (bytes == 0) return BH_OK;
  if (c->capturing) return BH_OK;  // the eager run before the capture left the same data on the device
  bh_status st;
  if (c->stage_event_used) {
    st = hip_check(c, hipEventSynchronize(c->stage_event), "hipEventSynchronize");
    if (st) return st;
  }
  if (c->stage_bytes < bytes) {
    if (c->stage) (void)hipHostFree(c->stage);
    c->stage = nullptr;
    c->stage_bytes = 0;
    st = hip_check(c, hipHostMalloc(&c->stage, bytes, 0), "hipHostMalloc");
    if (st) return st;
    c->stage_bytes = bytes;
  }
  memcpy(c->stage, src, bytes);
  st = hip_check(c, hipMemcpyAsync(dst, c->stage, bytes, hipMemcpyHostToDevice, c->stream), "hipMemcpyAsync");
  if (st) return st;
  if (!c->stage_event) {
    st = hip_check(c, hipEventCreateWithFlags(&c->stage_event, hipEventDisableTiming), "hipEventCreate");
    if (st) return st;
  }
  c->stage_event_used = true;
  return hip_check(c, hipEventRecord(c->stage_event, c->stream), "hipEventRecord");
}

static bh_status ensure_particles(bh_ctx *c, int64_t n, int nsys) {
  const size_t N = (size_t)std::max<int64_t>(n, 1);
  const size_t slots = 2 * N + (size_t)nsys + 1;
  const size_t hist = radix_hist_bytes((int64_t)N);
  const size_t scan_elems = std::max<size_t>(N, hist / sizeof(uint32_t)) + 1;
  struct Want {
    DevBuf *b;
    size_t bytes;
    const char *name;
  } want[] = {
      {&c->keys[0], 8 * N, "keys"},       {&c->keys[1], 8 * N, "keys"},
      {&c->vals[0], 4 * N, "vals"},       {&c->vals[1], 4 * N, "vals"},
      {&c->sys_in, 4 * N, "sys_in"},      {&c->spos, 24 * N, "spos"},
      {&c->pmass, sizeof(PosMass) * N, "packed positions"},
      {&c->smass, 8 * N, "smass"},        {&c->perm, 4 * N, "perm"},
      {&c->delta, N, "delta"},            {&c->level, N, "level"},
      {&c->cdigit, N, "cdigit"},          {&c->pdigit, N, "pdigit"},
      {&c->owner, 4 * N, "owner"},        {&c->cfirst, 4 * N, "cfirst"},
      {&c->ccount, 4 * N, "ccount"},      {&c->cparent, 4 * N, "cparent"},
      {&c->pparent, 4 * N, "pparent"},    {&c->mask, 4 * N, "mask"},
      {&c->nchild, 4 * N, "nchild"},      {&c->cfirst_child, 4 * N, "cfirst_child"},
      {&c->cslot, 4 * N, "cslot"},        {&c->hist, hist, "hist"},
      {&c->scan_tmp, scan_tmp_bytes((int64_t)scan_elems), "scan_tmp"},
      {&c->nodes, sizeof(NodeRec) * slots, "nodes"},
      {&c->msum, 32 * slots, "msum"},
      {&c->meta, slots, "meta"},
      {&c->levels, 3 * 24 * sizeof(int32_t), "level table"},
      {&c->lcells, sizeof(CellRec) * N, "cells by level"},
      {&c->gflag, 4 * N, "gflag"},        {&c->gidx, 4 * N, "gidx"},
      {&c->glen, 4 * N, "glen"},          {&c->ginfo, 12 * N, "ginfo"},
      {&c->gbox, 48 * N, "gbox"},         {&c->glist, 4 * N, "glist"},
      {&c->gmass, 8 * N, "gmass"},
      {&c->bbox_part, (size_t)6 * 8 * (size_t)nsys * (size_t)bbox_blocks_per_system(nsys), "bbox"},
      {&c->info, sizeof(DevInfo), "info"},
  };
  for (auto &w : want) {
    bh_status st = ensure(c, *w.b, w.bytes, w.name);
    if (st) return st;
  }
  return BH_OK;
}

static bh_status check_device_errors(bh_ctx *c) {
  bh_status st = hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (st) return st;
  if (!c->info.p) return BH_OK;
  st = hip_check(c, hipMemcpy(c->info_host, c->info.p, sizeof(DevInfo), hipMemcpyDeviceToHost), "hipMemcpy info");
  if (st) return st;
  const int32_t e = c->info_host->err;
  if (e & kErrNonFinitePos) return fail(c, BH_EINVAL, "non-finite particle position");
  if (e & kErrBadMass) return fail(c, BH_EINVAL, "particle mass negative or non-finite");
  if (e & kErrTheta) return fail(c, BH_EINVAL, "per-group theta outside [0, 1]");
  if (e & kErrBuild) return fail(c, BH_EINTERNAL, "tree build produced an inconsistent node layout");
  if (e & kErrStack) return fail(c, BH_EINTERNAL, "walk stack capacity exceeded or node range corrupt");
  if (e & kErrPool) return fail(c, BH_EINTERNAL, "interaction list pool exhausted");
  if (e & kErrWait) return fail(c, BH_EINTERNAL, "a bounded device wait timed out (walk task or sort look-back)");
  if (e & kErrRadius) return fail(c, BH_EINVAL, "search radius h must be positive and finite");
  if (e & kErrListSpace) return fail(c, BH_EINVAL, "neighbour list offsets do not match the neighbour counts");
  return BH_OK;
}

static bh_status build_common(bh_ctx *c, int32_t nsys, const int64_t *offsets, const double *pos,
                              const double *mass) {
  const int64_t n = offsets[nsys];
  if (n < 0 || n > BH_MAX_N) return fail(c, BH_EINVAL, "particle count out of range");
  if (n > 0 && (!pos || !mass)) return fail(c, BH_EINVAL, "pos and mass must not be NULL");
  c->have_tree = c->have_groups = c->have_forces = false;
  bh_status st = ensure_particles(c, n, nsys);
  if (st) return st;
  c->n = n;
  c->nsys = nsys;
  c->sys_host.assign((size_t)nsys, SysInfo{});
  for (int s = 0; s < nsys; ++s) {
    c->sys_host[s].first = (int32_t)offsets[s];
    c->sys_host[s].count = (int32_t)(offsets[s + 1] - offsets[s]);
  }
  st = ensure(c, c->sys, sizeof(SysInfo) * (size_t)nsys, "systems");
  if (st) return st;
  st = upload(c, c->sys.p, c->sys_host.data(), sizeof(SysInfo) * (size_t)nsys);
  if (st) return st;
  st = timer_start(c, c->t_build);
  if (st) return st;
  reset_info_device(P<DevInfo>(c->info), c->stream);
  TreeBuffers B{};
  B.pos = pos;
  B.mass = mass;
  B.n = n;
  B.nsys = nsys;
  B.sys = P<SysInfo>(c->sys);
  B.info = P<DevInfo>(c->info);
  B.sys_in = P<int32_t>(c->sys_in);
  B.keys[0] = P<uint64_t>(c->keys[0]);
  B.keys[1] = P<uint64_t>(c->keys[1]);
  B.vals[0] = P<uint32_t>(c->vals[0]);
  B.vals[1] = P<uint32_t>(c->vals[1]);
  B.hist = P<uint32_t>(c->hist);
  B.scan_tmp = c->scan_tmp.p;
  B.bbox_part = P<double>(c->bbox_part);
  B.spos = P<double>(c->spos);
  B.smass = P<double>(c->smass);
  B.pm = P<PosMass>(c->pmass);
  B.perm = P<int32_t>(c->perm);
  B.delta = P<int8_t>(c->delta);
  B.level = P<int8_t>(c->level);
  B.cdigit = P<int8_t>(c->cdigit);
  B.pdigit = P<int8_t>(c->pdigit);
  B.owner = P<int32_t>(c->owner);
  B.cfirst = P<int32_t>(c->cfirst);
  B.ccount = P<int32_t>(c->ccount);
  B.cparent = P<int32_t>(c->cparent);
  B.pparent = P<int32_t>(c->pparent);
  B.mask = P<int32_t>(c->mask);
  B.nchild = P<int32_t>(c->nchild);
  B.cfc = P<int32_t>(c->cfirst_child);
  B.cslot = P<int32_t>(c->cslot);
  B.nodes = P<NodeRec>(c->nodes);
  B.msum = P<double>(c->msum);
  B.meta = P<int8_t>(c->meta);
  B.lcount = P<int32_t>(c->levels);
  B.loff = B.lcount + 24;
  B.lcursor = B.lcount + 48;
  B.lcells = P<CellRec>(c->lcells);
  B.slot_cap = (int64_t)std::min({c->nodes.bytes / sizeof(NodeRec), c->msum.bytes / 32, c->meta.bytes});
  B.curve = c->opt.curve;
  B.any_empty = false;
  for (int s = 0; s < nsys; ++s) B.any_empty |= c->sys_host[s].count == 0;
  const bool quad = c->opt.quadrupole != 0;
  if (quad) {
    const size_t slots = (size_t)B.slot_cap;
    st = ensure(c, c->qmom, 48 * slots, "second moments");
    if (st) return st;
    st = ensure(c, c->qpack, 32 * slots, "packed second moments");
    if (st) return st;
    B.qmom = P<double>(c->qmom);
    B.qpack = P<float4>(c->qpack);
  }
  build_tree_device(B, c->stream);
  c->sorted_keys = B.sorted_keys;
  st = timer_stop(c, c->t_build);
  if (st) return st;
  st = hip_check(c, hipGetLastError(), "kernel launch (build)");
  if (st) return st;
  c->have_tree = true;
  c->have_quad = quad;
  c->have_neighbors = false;
  return BH_OK;
}

}  // namespace bh

using namespace bh;

extern "C" {

bh_status bh_create(bh_ctx **out, void *stream) {
  if (!out) return BH_EINVAL;
  *out = nullptr;
  bh_ctx *c = new (std::nothrow) bh_ctx();
  if (!c) return BH_ENOMEM;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess ||
      hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
    delete c;
    return BH_EHIP;
  }
  // a walk wave waits at most 2 s for a task (a guard: a task comes within
  // milliseconds, the length of the longest walk unit)
  int clock_khz = 0;
  if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess || clock_khz <= 0)
    clock_khz = 100000;
  c->wait_ticks = (long long)clock_khz * 2000;
  // the no-allocation judge's static scratch: its address on this device
  if (judge_scratch_address(c->device, &c->judge_scratch) != hipSuccess || !c->judge_scratch) {
    delete c;
    return BH_EHIP;
  }
  if (hipHostMalloc((void **)&c->info_host, sizeof(DevInfo), 0) != hipSuccess) {
    delete c;
    return BH_ENOMEM;
  }
  memset(c->info_host, 0, sizeof(DevInfo));
  if (hipHostMalloc((void **)&c->split_host, sizeof(SplitCounters), 0) != hipSuccess) {
    (void)hipHostFree(c->info_host);
    delete c;
    return BH_ENOMEM;
  }
  memset(c->split_host, 0, sizeof(SplitCounters));
  *out = c;
  return BH_OK;
}

void bh_destroy(bh_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  DevBuf *bufs[] = {&c->keys[0], &c->keys[1], &c->vals[0], &c->vals[1], &c->sys_in, &c->spos, &c->smass,
                    &c->perm, &c->delta, &c->level, &c->cdigit, &c->pdigit, &c->owner, &c->cfirst, &c->ccount,
                    &c->cparent, &c->pparent, &c->mask, &c->nchild, &c->cfirst_child, &c->cslot, &c->scan_tmp,
                    &c->hist, &c->nodes, &c->msum, &c->meta, &c->levels, &c->lcells, &c->gflag, &c->gidx, &c->glen, &c->ginfo, &c->gbox, &c->glist,
                    &c->gmass, &c->bbox_part, &c->sys, &c->par, &c->info, &c->direct_part, &c->energy_part,
                    &c->glists, &c->far_pool, &c->near_pool, &c->far_next, &c->near_next,
                    &c->items, &c->pmass, &c->feps, &c->mlp_work, &c->mlp_feat, &c->pp_next, &c->order_hist, &c->walk_order, &c->walk_order_hist, &c->tasks, &c->ranges, &c->segs,
                    &c->split_ctr, &c->gsplit, &c->gnseg, &c->gsegfirst, &c->skeys[0], &c->skeys[1], &c->svals[0],
                    &c->svals[1], &c->shist, &c->sscan, &c->srows, &c->spbase, &c->sgroups, &c->psum,
                    &c->qmom, &c->qpack, &c->far_slot, &c->walk_hist};
  for (DevBuf *b : bufs) free_buf(*b);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  if (c->info_host) (void)hipHostFree(c->info_host);
  if (c->stage) (void)hipHostFree(c->stage);
  if (c->split_host) (void)hipHostFree(c->split_host);
  if (c->stage_event) (void)hipEventDestroy(c->stage_event);
  Timer *ts[] = {&c->t_build, &c->t_groups, &c->t_walk, &c->t_force, &c->t_particle, &c->t_neighbor, &c->t_theta};
  for (Timer *t : ts)
    for (hipEvent_t e : t->ev) (void)hipEventDestroy(e);
  delete c;
}

const char *bh_last_error(const bh_ctx *c) { return c ? c->err.c_str() : "null context"; }

bh_status bh_set_stream(bh_ctx *c, void *stream) {
  if (!c) return BH_EINVAL;
  c->stream = (hipStream_t)stream;
  return BH_OK;
}

bh_status bh_get_options(const bh_ctx *c, bh_options *opt) {
  if (!c || !opt) return BH_EINVAL;
  *opt = c->opt;
  return BH_OK;
}

bh_status bh_set_options(bh_ctx *c, const bh_options *opt) {
  if (!c || !opt) return BH_EINVAL;
  if (opt->waves_per_cu < 0 || opt->waves_per_cu > 32) return fail(c, BH_EINVAL, "waves_per_cu must be in [0, 32]");
  if (opt->split_visits < -1 || (opt->split_visits > 0 && opt->split_visits < 64))
    return fail(c, BH_EINVAL, "split_visits must be -1, 0 or >= 64");
  if (opt->quadrupole != 0 && opt->quadrupole != 1) return fail(c, BH_EINVAL, "quadrupole must be 0 or 1");
  if (opt->curve != 0 && opt->curve != 1) return fail(c, BH_EINVAL, "curve must be 0 (Morton) or 1 (Peano-Hilbert)");
  if (opt->list_tile != 0 && (opt->list_tile < kMinTile || opt->list_tile > kMaxTile ||
                              (opt->list_tile & (opt->list_tile - 1)) != 0))
    return fail(c, BH_EINVAL, "list_tile must be 0 or a power of two in [128, 2048]");
  c->opt = *opt;
  return BH_OK;
}

bh_status bh_sync(bh_ctx *c) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  return check_device_errors(c);
}

bh_status bh_build_tree(bh_ctx *c, int64_t n, const double *pos, const double *mass) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (n < 0 || n > BH_MAX_N) return fail(c, BH_EINVAL, "n out of range");
  int64_t off[2] = {0, n};
  return build_common(c, 1, off, pos, mass);
}

bh_status bh_build_batch(bh_ctx *c, int32_t n_systems, const int64_t *offsets, const double *pos,
                         const double *mass) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (n_systems < 1 || n_systems > 65536 || !offsets) return fail(c, BH_EINVAL, "n_systems must be in [1, 65536]");
  if (offsets[0] != 0) return fail(c, BH_EINVAL, "offsets[0] must be 0");
  for (int s = 0; s < n_systems; ++s)
    if (offsets[s + 1] < offsets[s]) return fail(c, BH_EINVAL, "offsets must be non-decreasing");
  return build_common(c, n_systems, offsets, pos, mass);
}

bh_status bh_make_groups(bh_ctx *c, int32_t n_crit, int64_t *n_groups_out) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->have_tree) return fail(c, BH_ESTATE, "bh_make_groups before a tree was built");
  if (n_crit < 1 || n_crit > BH_MAX_NCRIT) return fail(c, BH_EINVAL, "n_crit must be in [1, 256]");
  bh_status st = timer_start(c, c->t_groups);
  if (st) return st;
  GroupBuffers B{};
  B.n = c->n;
  B.nsys = c->nsys;
  B.n_crit = n_crit;
  B.level = P<int8_t>(c->level);
  B.ccount = P<int32_t>(c->ccount);
  B.cfc = P<int32_t>(c->cfirst_child);
  B.nchild = P<int32_t>(c->nchild);
  B.nodes = P<NodeRec>(c->nodes);
  B.sys = P<SysInfo>(c->sys);
  B.spos = P<double>(c->spos);
  B.info = P<DevInfo>(c->info);
  B.gflag = P<int32_t>(c->gflag);
  B.gidx = P<int32_t>(c->gidx);
  B.glen = P<int32_t>(c->glen);
  B.ginfo = P<int32_t>(c->ginfo);
  B.gbox = P<double>(c->gbox);
  B.scan_tmp = c->scan_tmp.p;
  B.num_cu = c->num_cu;
  make_groups_device(B, c->stream);
  c->xq_clean = true;
  st = timer_stop(c, c->t_groups);
  if (st) return st;
  st = hip_check(c, hipGetLastError(), "kernel launch (groups)");
  if (st) return st;
  c->n_crit = n_crit;
  c->have_groups = true;
  c->have_forces = false;
  c->walk_order_valid = false;
  if (n_groups_out) {
    st = check_device_errors(c);
    if (st) return st;
    *n_groups_out = c->info_host->n_groups;
  }
  return BH_OK;
}

static bh_status forces_common(bh_ctx *c, const double *eps_sys, const double *theta_sys, const float *theta_group,
                               float *acc, float *pot) {
  if (!c->have_groups) return fail(c, BH_ESTATE, "forces requested before bh_make_groups");
  if (c->n > 0 && (!acc || !pot)) return fail(c, BH_EINVAL, "acc and pot must not be NULL");
  const bool quad = c->opt.quadrupole != 0;
  if (quad && !c->have_quad)
    return fail(c, BH_ESTATE, "quadrupole sums need a tree built with the quadrupole option set");
  c->par_host.assign((size_t)c->nsys, SysParam{});
  for (int s = 0; s < c->nsys; ++s) {
    const double e = eps_sys[s], t = theta_sys[s];
    if (!(e > 0.0) || !isfinite(e)) return fail(c, BH_EINVAL, "eps must be positive and finite");
    const float e2 = (float)(e * e);
    if (!(e2 >= 1.17549435e-38f) || isinf(e2)) return fail(c, BH_EINVAL, "eps^2 must be a normal FP32 number");
    if (!(t >= 0.0 && t <= 1.0)) return fail(c, BH_EINVAL, "theta must be in [0, 1]");
    c->par_host[s].eps = e;
    c->par_host[s].theta = t;
  }
  bh_status st = ensure(c, c->par, sizeof(SysParam) * (size_t)c->nsys, "parameters");
  if (st) return st;
  st = upload(c, c->par.p, c->par_host.data(), sizeof(SysParam) * (size_t)c->nsys);
  if (st) return st;
  if (c->n == 0) {
    c->have_forces = true;
    return BH_OK;
  }
  // list pools: start from an estimate (32 far and 4 near entries per
  // particle), grow to what a walk reports it needed; the capacities count
  // chunks of the current tile (recounted when the tile changes)
  const int tile = c->opt.list_tile > 0 ? c->opt.list_tile : kDefaultTile;
  if (c->far_cap == 0) {
    c->far_cap = (int32_t)std::max<int64_t>(4096, 32 * c->n / tile);
    c->near_cap = (int32_t)std::max<int64_t>(4096, 8 * c->n / tile);
  } else if (c->pool_tile != tile) {
    c->far_cap = (int32_t)std::min<int64_t>((int64_t)c->far_cap * c->pool_tile / tile + 64, INT32_MAX / 2);
    c->near_cap = (int32_t)std::min<int64_t>((int64_t)c->near_cap * c->pool_tile / tile + 64, INT32_MAX / 2);
  }
  c->pool_tile = tile;
  WalkListArgs W{};
  W.nodes = P<NodeRec>(c->nodes);
  W.sys = P<SysInfo>(c->sys);
  W.ginfo = P<int32_t>(c->ginfo);
  W.gbox = P<double>(c->gbox);
  W.par = P<SysParam>(c->par);
  W.theta_group = theta_group;
  W.info = P<DevInfo>(c->info);
  W.nsys = c->nsys;
  W.glist = P<int32_t>(c->glist);
  W.gmass = P<double>(c->gmass);
  if (!c->walk_bpc) {
    c->walk_bpc = walk_lists_blocks_per_cu();
    c->force_bpc = force_lists_blocks_per_cu(false);
    c->force_bpc_q = force_lists_blocks_per_cu(true);
  }
  const size_t gcap = (size_t)std::max<int64_t>(c->n, 1);
  // split walks (long lists walked and summed by several waves)
  const int grid = c->num_cu * (c->opt.waves_per_cu > 0 ? c->opt.waves_per_cu : c->walk_bpc);
  const int fgrid = c->num_cu * (c->opt.waves_per_cu > 0 ? c->opt.waves_per_cu : (quad ? c->force_bpc_q : c->force_bpc));
  // The automatic visit cap scales with the particles per walk wave (a walk
  // that outlasts a multiple of the average wave's share is the one to
  // split), never below kSplitVisits; in the walk it also grows to
  // kSplitMeanFactor times the mean list length of the previous walk on this
  // context, so that where every list is long (small theta) only the outliers
  // split: splitting most groups costs more than it balances.
  // A single system is not split by default: its lists are rarely far longer
  // than the mean, and the walk without the split machinery is faster (see
  // k_walk_lists).
  const int64_t auto_cap = std::max<int64_t>(kSplitVisits, kSplitPerParticle * c->n / std::max(grid, 1));
  const bool auto_split = c->opt.split_visits == 0;
  const int visit_cap = c->opt.split_visits < 0
                            ? 0
                            : (auto_split ? (c->nsys > 1 ? (int)std::min<int64_t>(auto_cap, INT32_MAX / 2) : 0)
                                          : c->opt.split_visits);
  if (!c->walk_hist.p) {
    st = ensure(c, c->walk_hist, 4 * sizeof(int32_t), "walk history");
    if (st) return st;
    fill_i32(P<int32_t>(c->walk_hist), 0, 4, c->stream);
  }
  if (c->seg_cap == 0) {
    c->task_cap = 4096;
    c->range_cap = 1 << 16;
    c->seg_cap = 4096;
  }
  if (!c->order_hist.p) {
    st = ensure(c, c->order_hist, order_hist_bytes(), "queue order bins");
    if (st) return st;
    order_clear_device(P<int32_t>(c->order_hist), c->stream);  // every later call leaves it zero
  }
  if (st) return st;
  SplitBuffers S{};
  int32_t nsegs_host = 0;
  for (int attempt = 0;; ++attempt) {
    st = ensure(c, c->far_pool, (size_t)c->far_cap * tile * sizeof(float4), "far list pool");
    if (st) return st;
    st = ensure(c, c->far_next, (size_t)c->far_cap * sizeof(int32_t), "far list links");
    if (st) return st;
    if (quad) {
      st = ensure(c, c->far_slot, (size_t)c->far_cap * tile * sizeof(int32_t), "far list node slots");
      if (st) return st;
    }
    st = ensure(c, c->near_pool, (size_t)c->near_cap * tile * sizeof(float4), "near list pool");
    if (st) return st;
    st = ensure(c, c->near_next, (size_t)c->near_cap * sizeof(int32_t), "near list links");
    if (st) return st;
    st = ensure(c, c->glists, (size_t)4 * sizeof(int32_t) * gcap, "group lists");
    if (st) return st;
    const size_t sc = (size_t)c->seg_cap;
    DevBuf *sb[] = {&c->tasks, &c->ranges, &c->segs, &c->split_ctr, &c->gsplit, &c->gnseg,
                    &c->gsegfirst, &c->skeys[0], &c->skeys[1], &c->svals[0], &c->svals[1], &c->shist,
                    &c->sscan, &c->srows, &c->spbase, &c->sgroups};
    const size_t sz[] = {sizeof(WalkTask) * (size_t)c->task_cap,
                         sizeof(int2) * (size_t)c->range_cap, sizeof(Segment) * sc, sizeof(SplitCounters) + 64,
                         sizeof(int32_t) * gcap, sizeof(int32_t) * gcap, sizeof(int32_t) * gcap, 8 * sc, 8 * sc,
                         4 * sc, 4 * sc, radix_hist_bytes((int64_t)sc), scan_tmp_bytes((int64_t)sc) + 256,
                         4 * sc, 4 * sc + 16, 4 * sc};
    for (int k = 0; k < (int)(sizeof(sz) / sizeof(sz[0])); ++k) {
      st = ensure(c, *sb[k], sz[k], "split walk buffers");
      if (st) return st;
    }
    W.far_pool = P<float4>(c->far_pool);
    W.near_pool = P<float4>(c->near_pool);
    W.far_next = P<int32_t>(c->far_next);
    W.near_next = P<int32_t>(c->near_next);
    W.far_slot = quad ? P<int32_t>(c->far_slot) : nullptr;
    W.far_cap = c->far_cap;
    W.near_cap = c->near_cap;
    W.far_tile = tile;
    W.near_tile = tile / 2;
    W.glists = P<int32_t>(c->glists);
    W.ctr = P<SplitCounters>(c->split_ctr);
    W.tasks = P<WalkTask>(c->tasks);
    W.task_cap = c->task_cap;
    W.ranges = P<int2>(c->ranges);
    W.range_cap = c->range_cap;
    W.segs = P<Segment>(c->segs);
    W.seg_cap = c->seg_cap;
    W.gsplit = P<int32_t>(c->gsplit);
    W.visit_cap = visit_cap;
    W.mean_list = auto_split ? P<int32_t>(c->walk_hist) : nullptr;
    W.order = (theta_group && c->walk_order_valid) ? P<int32_t>(c->walk_order) : nullptr;
    W.wait_ticks = c->wait_ticks;
    reset_list_counters(P<DevInfo>(c->info), c->stream);
    split_reset(W.ctr, P<DevInfo>(c->info), W.tasks, c->task_cap, c->stream);
    st = timer_start(c, c->t_walk);
    if (st) return st;
    c->last_attempts = attempt + 1;
    walk_lists_device(W, grid, c->stream);
    c->xq_clean = false;
    st = timer_stop(c, c->t_walk);
    if (st) return st;
    st = hip_check(c, hipGetLastError(), "kernel launch (walk)");
    if (st) return st;
    // the pools must have held every list before the sums may run; a captured
    // step cannot wait here: an overflow then leaves kErrPool for bh_sync
    if (c->capturing) break;
    st = hip_check(c, hipMemcpyAsync(c->info_host, c->info.p, sizeof(DevInfo), hipMemcpyDeviceToHost, c->stream),
                   "hipMemcpyAsync info");
    if (st) return st;
    if (visit_cap > 0) {
      st = hip_check(c, hipMemcpyAsync(c->split_host, W.ctr, sizeof(SplitCounters), hipMemcpyDeviceToHost,
                                       c->stream), "hipMemcpyAsync split counters");
      if (st) return st;
    }
    st = hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (st) return st;
    if (visit_cap > 0) nsegs_host = c->split_host->segs;
    c->last_segments = nsegs_host;
    c->last_split_groups = visit_cap > 0 ? c->split_host->n_split : 0;
    c->last_depth = visit_cap > 0 ? c->split_host->depth : 0;
    if (!(c->info_host->err & kErrPool)) break;
    if (attempt > 5) return fail(c, BH_EINTERNAL, "interaction list pool still too small after growing");
    const int64_t fneed = (int64_t)c->info_host->far_chunks * kChunkRun, nneed = (int64_t)c->info_host->near_chunks * kChunkRun;
    c->far_cap = std::max(c->far_cap, (int32_t)std::min<int64_t>(fneed + fneed / 4 + 64, INT32_MAX / 2));
    c->near_cap = std::max(c->near_cap, (int32_t)std::min<int64_t>(nneed + nneed / 4 + 64, INT32_MAX / 2));
    if (visit_cap > 0) {
      const SplitCounters &h = *c->split_host;
      if (h.tasks > c->task_cap) c->task_cap = std::max(2 * c->task_cap, h.tasks + h.tasks / 4 + 64);
      if (h.ranges > c->range_cap) c->range_cap = std::max(2 * c->range_cap, h.ranges + h.ranges / 4 + 1024);
      if (h.segs > c->seg_cap) c->seg_cap = std::max(2 * c->seg_cap, h.segs + h.segs / 4 + 64);
    }
  }
  const bool split = visit_cap > 0 && (c->capturing || nsegs_host > 0);
  S.ctr = P<SplitCounters>(c->split_ctr);
  S.segs = P<Segment>(c->segs);
  S.seg_cap = c->seg_cap;
  S.keys[0] = P<uint64_t>(c->skeys[0]);
  S.keys[1] = P<uint64_t>(c->skeys[1]);
  S.vals[0] = P<uint32_t>(c->svals[0]);
  S.vals[1] = P<uint32_t>(c->svals[1]);
  S.hist = P<uint32_t>(c->shist);
  S.scan_tmp = c->sscan.p;
  S.order = S.vals[0];
  S.gsegfirst = P<int32_t>(c->gsegfirst);
  S.gnseg = P<int32_t>(c->gnseg);
  S.rows = P<int32_t>(c->srows);
  S.pbase = P<int32_t>(c->spbase);
  S.total_rows = S.pbase + c->seg_cap;
  S.sgroups = P<int32_t>(c->sgroups);
  S.nsg = S.total_rows + 1;
  if (visit_cap > 0) {  // sized even when nothing split, so that a capture never has to grow it
    st = ensure(c, c->psum, sizeof(double) * 4 * (size_t)c->seg_cap * (size_t)std::max(c->n_crit, 1), "partial sums");
    if (st) return st;
    S.psum = P<double>(c->psum);
  }
  if (split)
    split_finish_device(S, P<int32_t>(c->ginfo), P<int32_t>(c->glist), P<double>(c->gmass), P<DevInfo>(c->info),
                        c->stream);
  const size_t icap = gcap + gcap / 64 + 64 + (size_t)4 * c->seg_cap;  // items: blocks of 64, segments
  st = ensure(c, c->items, 2 * sizeof(int32_t) * icap, "force items");
  if (st) return st;
  ForceArgs F{};
  F.items = P<int32_t>(c->items);
  F.ginfo = P<int32_t>(c->ginfo);
  F.gbox = P<double>(c->gbox);
  F.glists = P<int32_t>(c->glists);
  F.far_pool = P<float4>(c->far_pool);
  F.near_pool = P<float4>(c->near_pool);
  F.far_next = P<int32_t>(c->far_next);
  F.near_next = P<int32_t>(c->near_next);
  F.far_slot = quad ? P<int32_t>(c->far_slot) : nullptr;
  F.qpack = quad ? P<float4>(c->qpack) : nullptr;
  F.far_tile = tile;
  F.near_tile = tile / 2;
  F.spos = P<double>(c->spos);
  F.smass = P<double>(c->smass);
  F.perm = P<int32_t>(c->perm);
  F.par = P<SysParam>(c->par);
  F.acc = acc;
  F.pot = pot;
  F.info = P<DevInfo>(c->info);
  F.xstart = P<int32_t>(c->order_hist) + (order_hist_bytes() / sizeof(int32_t) - 16);
  F.glist = P<int32_t>(c->glist);
  F.segs = S.segs;
  F.seg_order = S.order;
  F.gsegfirst = S.gsegfirst;
  F.pbase = S.pbase;
  F.psum = split ? P<double>(c->psum) : nullptr;
  item_order_device(F, P<int32_t>(c->gsplit), P<int32_t>(c->gnseg), (int64_t)gcap, P<int32_t>(c->order_hist),
                    P<int32_t>(c->walk_hist), P<int32_t>(c->items), c->stream);
  st = timer_start(c, c->t_force);
  if (st) return st;
  force_lists_device(F, fgrid, c->stream);
  st = timer_stop(c, c->t_force);
  if (st) return st;
  if (split)
    split_reduce_device(S, P<int32_t>(c->ginfo), P<double>(c->smass), P<int32_t>(c->perm), P<SysParam>(c->par), acc,
                        pot, c->stream);
  st = hip_check(c, hipGetLastError(), "kernel launch (force)");
  if (st) return st;
  c->have_forces = true;
  return BH_OK;
}

bh_status bh_compute_forces(bh_ctx *c, double eps, double theta, const float *theta_group, float *acc, float *pot) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->have_tree) return fail(c, BH_ESTATE, "forces requested before a tree was built");
  std::vector<double> e((size_t)c->nsys, eps), t((size_t)c->nsys, theta);
  return forces_common(c, e.data(), t.data(), theta_group, acc, pot);
}

bh_status bh_compute_forces_batch(bh_ctx *c, const double *eps_sys, const double *theta_sys,
                                  const float *theta_group, float *acc, float *pot) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->have_tree) return fail(c, BH_ESTATE, "forces requested before a tree was built");
  if (!eps_sys || !theta_sys) return fail(c, BH_EINVAL, "eps_sys and theta_sys must not be NULL");
  return forces_common(c, eps_sys, theta_sys, theta_group, acc, pot);
}

// The per-particle walk (no groups needed): parameters as for the group path.
static bh_status particle_common(bh_ctx *c, const double *eps_sys, const double *theta_sys, float *acc,
                                 float *pot) {
  if (!c->have_tree) return fail(c, BH_ESTATE, "forces requested before a tree was built");
  if (c->n > 0 && (!acc || !pot)) return fail(c, BH_EINVAL, "acc and pot must not be NULL");
  if (c->opt.quadrupole) return fail(c, BH_EINVAL, "the per-particle walk sums monopoles only (quadrupole option set)");
  c->par_host.assign((size_t)c->nsys, SysParam{});
  for (int s = 0; s < c->nsys; ++s) {
    const double e = eps_sys[s], t = theta_sys[s];
    if (!(e > 0.0) || !isfinite(e)) return fail(c, BH_EINVAL, "eps must be positive and finite");
    const float e2 = (float)(e * e);
    if (!(e2 >= 1.17549435e-38f) || isinf(e2)) return fail(c, BH_EINVAL, "eps^2 must be a normal FP32 number");
    if (!(t >= 0.0 && t <= 1.0)) return fail(c, BH_EINVAL, "theta must be in [0, 1]");
    c->par_host[s].eps = e;
    c->par_host[s].theta = t;
  }
  bh_status st = ensure(c, c->par, sizeof(SysParam) * (size_t)c->nsys, "parameters");
  if (st) return st;
  st = upload(c, c->par.p, c->par_host.data(), sizeof(SysParam) * (size_t)c->nsys);
  if (st) return st;
  st = hip_check(c, hipMemcpyAsync(c->info_host, c->info.p, sizeof(DevInfo), hipMemcpyDeviceToHost, c->stream),
                 "hipMemcpyAsync info");
  if (st) return st;
  st = hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (st) return st;
  const int64_t nslots = (int64_t)c->nsys + c->info_host->n_slots;
  st = ensure(c, c->pp_next, sizeof(int32_t) * (size_t)std::max<int64_t>(nslots, 1), "thread pointers");
  if (st) return st;
  reset_list_counters(P<DevInfo>(c->info), c->stream);
  st = timer_start(c, c->t_particle);
  if (st) return st;
  particle_forces_device(P<NodeRec>(c->nodes), (int)nslots, c->nsys, P<SysInfo>(c->sys), P<SysParam>(c->par),
                         P<double>(c->spos), P<int32_t>(c->perm), c->n, P<int32_t>(c->pp_next), acc, pot,
                         P<DevInfo>(c->info), c->stream);
  st = timer_stop(c, c->t_particle);
  if (st) return st;
  st = hip_check(c, hipGetLastError(), "kernel launch (per-particle walk)");
  if (st) return st;
  c->have_forces = true;
  c->last_split_groups = c->last_segments = c->last_depth = 0;
  c->last_attempts = 1;
  return BH_OK;
}

bh_status bh_compute_forces_particle(bh_ctx *c, double eps, double theta, float *acc, float *pot) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->have_tree) return fail(c, BH_ESTATE, "forces requested before a tree was built");
  std::vector<double> e((size_t)c->nsys, eps), t((size_t)c->nsys, theta);
  return particle_common(c, e.data(), t.data(), acc, pot);
}

bh_status bh_compute_forces_particle_batch(bh_ctx *c, const double *eps_sys, const double *theta_sys, float *acc,
                                           float *pot) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!eps_sys || !theta_sys) return fail(c, BH_EINVAL, "eps_sys and theta_sys must not be NULL");
  return particle_common(c, eps_sys, theta_sys, acc, pot);
}

static bh_status theta_common(bh_ctx *c, const bh_mlp *net, const double *eps_sys, float shift, float *theta);

// One whole step (build, groups, [per-group theta from the network], walk
// and force sum); the learned variant writes theta_out and walks with it.
static bh_status step_common(bh_ctx *c, int32_t n_systems, const int64_t *offsets, const double *pos,
                             const double *mass, int32_t n_crit, const double *eps_sys, const double *theta_sys,
                             const float *theta_group, const bh_mlp *net, float shift, float *theta_out, float *acc,
                             float *pot) {
  bh_status st = build_common(c, n_systems, offsets, pos, mass);
  if (!st) st = bh_make_groups(c, n_crit, nullptr);
  if (!st && net) st = theta_common(c, net, eps_sys, shift, theta_out);
  if (!st) st = forces_common(c, eps_sys, theta_sys, net ? theta_out : theta_group, acc, pot);
  return st;
}

static bh_status capture_common(bh_ctx *c, int32_t n_systems, const int64_t *offsets, const double *pos,
                                const double *mass, int32_t n_crit, const double *eps_sys, const double *theta_sys,
                                const float *theta_group, const bh_mlp *net, float shift, float *theta_out,
                                float *acc, float *pot) {
  if (n_systems < 1 || n_systems > 65536 || !offsets || !eps_sys || !theta_sys)
    return fail(c, BH_EINVAL, "bad graph capture arguments");
  if (offsets[0] != 0) return fail(c, BH_EINVAL, "offsets[0] must be 0");
  for (int s = 0; s < n_systems; ++s)
    if (offsets[s + 1] < offsets[s]) return fail(c, BH_EINVAL, "offsets must be non-decreasing");
  if (n_crit < 1 || n_crit > BH_MAX_NCRIT) return fail(c, BH_EINVAL, "n_crit must be in [1, 256]");
  if (net && !theta_out) return fail(c, BH_EINVAL, "theta_group must not be NULL");
  // 1. one eager step sizes every buffer and checks the arguments
  bh_status st = step_common(c, n_systems, offsets, pos, mass, n_crit, eps_sys, theta_sys, theta_group, net, shift,
                             theta_out, acc, pot);
  if (!st) st = bh_sync(c);
  if (st) return st;
  // 2. headroom in the list pools for replays on moved particles
  c->far_cap += c->far_cap / 4;
  c->near_cap += c->near_cap / 4;
  st = forces_common(c, eps_sys, theta_sys, net ? theta_out : theta_group, acc, pot);
  if (!st) st = bh_sync(c);
  if (st) return st;
  // 3. record the same launches on a capture stream
  if (!c->capture_stream) {
    st = hip_check(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
    if (st) return st;
  }
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  hipStream_t saved = c->stream;
  c->stream = c->capture_stream;
  c->capturing = true;
  st = hip_check(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  if (!st) {
    bh_status sr = step_common(c, n_systems, offsets, pos, mass, n_crit, eps_sys, theta_sys, theta_group, net, shift,
                               theta_out, acc, pot);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->capturing = false;
    c->stream = saved;
    if (sr) {
      if (g) (void)hipGraphDestroy(g);
      return sr;
    }
    st = hip_check(c, e, "hipStreamEndCapture");
    if (!st) st = hip_check(c, hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (g) (void)hipGraphDestroy(g);
    if (st) c->graph = nullptr;
    return st;
  }
  c->capturing = false;
  c->stream = saved;
  return st;
}

bh_status bh_graph_capture(bh_ctx *c, int32_t n_systems, const int64_t *offsets, const double *pos,
                           const double *mass, int32_t n_crit, const double *eps_sys, const double *theta_sys,
                           const float *theta_group, float *acc, float *pot) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  return capture_common(c, n_systems, offsets, pos, mass, n_crit, eps_sys, theta_sys, theta_group, nullptr, 0.0f,
                        nullptr, acc, pot);
}

bh_status bh_graph_capture_learned(bh_ctx *c, int32_t n_systems, const int64_t *offsets, const double *pos,
                                   const double *mass, int32_t n_crit, const double *eps_sys,
                                   const double *theta_sys, const bh_mlp *net, float shift, float *theta_group,
                                   float *acc, float *pot) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!net) return fail(c, BH_EINVAL, "net must not be NULL");
  return capture_common(c, n_systems, offsets, pos, mass, n_crit, eps_sys, theta_sys, nullptr, net, shift,
                        theta_group, acc, pot);
}

bh_status bh_graph_launch(bh_ctx *c) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->graph) return fail(c, BH_ESTATE, "no captured step");
  return hip_check(c, hipGraphLaunch(c->graph, c->stream), "hipGraphLaunch");
}

bh_status bh_get_stats(bh_ctx *c, bh_stats *out) {
  if (!c || !out) return BH_EINVAL;
  c->err.clear();
  bh_status st = check_device_errors(c);
  memset(out, 0, sizeof(*out));
  const DevInfo &d = *c->info_host;
  out->n = c->n;
  out->n_systems = c->nsys;
  out->n_crit = c->have_groups ? c->n_crit : 0;
  out->error_flags = d.err;
  if (c->have_tree) {
    out->n_cells = d.n_cells;
    out->n_slots = (int64_t)c->nsys + d.n_slots;
    out->max_level = d.max_level;
  }
  if (c->have_groups) out->n_groups = d.n_groups;
  if (c->have_forces) {
    out->interactions = (int64_t)d.interactions;
    out->list_entries = (int64_t)d.list_entries;
    out->max_list = d.max_list;
    out->n_split_groups = c->last_split_groups;
    out->n_segments = c->last_segments;
    out->n_split_levels = c->last_depth;
    out->n_walk_attempts = c->last_attempts;
    out->n_theta_fallback = d.theta_fallback;
    out->node_visits = (int64_t)d.node_visits;
    out->near_entries = (int64_t)d.near_entries;
  }
  out->t_build_ms = timer_take(c->t_build, &out->n_build_calls);
  out->t_groups_ms = timer_take(c->t_groups, &out->n_groups_calls);
  out->t_walk_ms = timer_take(c->t_walk, &out->n_walk_calls);
  out->t_force_ms = timer_take(c->t_force, &out->n_force_calls);
  out->t_particle_ms = timer_take(c->t_particle, &out->n_particle_calls);
  out->t_neighbor_ms = timer_take(c->t_neighbor, &out->n_neighbor_calls);
  out->t_theta_ms = timer_take(c->t_theta, &out->n_theta_calls);
  if (c->have_neighbors) {
    out->neighbor_pairs = (int64_t)d.nb_pairs;
    out->neighbor_tests = (int64_t)d.nb_tests;
  }
  return st;
}

bh_status bh_direct_sampled(bh_ctx *c, int64_t n, const double *pos, const double *mass, double eps, int64_t s,
                            const int64_t *idx, double *acc, double *pot) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (n < 0 || s < 0) return fail(c, BH_EINVAL, "negative size");
  if (s > 0 && (!pos || !mass || !idx || !acc || !pot)) return fail(c, BH_EINVAL, "NULL pointer");
  if (!(eps >= 0.0) || !isfinite(eps)) return fail(c, BH_EINVAL, "eps must be finite and >= 0");
  if (s == 0) return BH_OK;
  int64_t chunk, nchunk;
  size_t bytes = direct_part_bytes(n, s, c->num_cu, &chunk, &nchunk);
  bh_status st = ensure(c, c->direct_part, bytes, "direct partials");
  if (st) return st;
  direct_sampled_device(pos, mass, n, eps, s, idx, acc, pot, P<double>(c->direct_part), chunk, nchunk, c->stream);
  return hip_check(c, hipGetLastError(), "kernel launch (direct)");
}

bh_status bh_direct_sampled_noalloc(bh_ctx *c, int64_t n, const double *pos, const double *mass, double eps,
                                    int64_t s, const int64_t *idx, double *acc, double *pot) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (n < 0 || s < 0) return fail(c, BH_EINVAL, "negative size");
  if (s > 0 && (!pos || !mass || !idx || !acc || !pot)) return fail(c, BH_EINVAL, "NULL pointer");
  if (!(eps >= 0.0) || !isfinite(eps)) return fail(c, BH_EINVAL, "eps must be finite and >= 0");
  if (s == 0) return BH_OK;
  int64_t chunk, nchunk;
  const size_t bytes = direct_part_bytes(n, s, c->num_cu, &chunk, &nchunk);
  if (bytes > kJudgeScratchBytes)
    return fail(c, BH_EINVAL, "sample too large for the no-allocation judge: its partial sums need " +
                                  std::to_string(bytes) + " bytes, the static scratch holds " +
                                  std::to_string(kJudgeScratchBytes));
  // every partial-sum row the reduction reads is written by the first kernel:
  // the scratch needs no clearing
  direct_sampled_device(pos, mass, n, eps, s, idx, acc, pot, c->judge_scratch, chunk, nchunk, c->stream);
  return hip_check(c, hipGetLastError(), "kernel launch (direct, no allocation)");
}

bh_status bh_kick(bh_ctx *c, int64_t n, double *vel, const float *acc, double dt) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (n < 0 || (n > 0 && (!vel || !acc))) return fail(c, BH_EINVAL, "bad kick arguments");
  kick_device(n, vel, acc, dt, c->stream);
  return hip_check(c, hipGetLastError(), "kernel launch (kick)");
}

bh_status bh_drift(bh_ctx *c, int64_t n, double *pos, const double *vel, double dt) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (n < 0 || (n > 0 && (!pos || !vel))) return fail(c, BH_EINVAL, "bad drift arguments");
  drift_device(n, pos, vel, dt, c->stream);
  return hip_check(c, hipGetLastError(), "kernel launch (drift)");
}

bh_status bh_leapfrog(bh_ctx *c, int64_t n, double *pos, double *vel, const double *mass, double eps, double theta,
                      int32_t n_crit, double dt, int32_t steps, float *acc, float *pot) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (n < 0 || n > BH_MAX_N) return fail(c, BH_EINVAL, "n out of range");
  if (steps < 0) return fail(c, BH_EINVAL, "steps must be >= 0");
  if (!isfinite(dt)) return fail(c, BH_EINVAL, "dt must be finite");
  if (n > 0 && (!pos || !vel || !mass || !acc || !pot)) return fail(c, BH_EINVAL, "bad leapfrog arguments");
  if (n_crit < 1 || n_crit > BH_MAX_NCRIT) return fail(c, BH_EINVAL, "n_crit must be in [1, 256]");
  const double h = 0.5 * dt;
  for (int32_t k = 0; k < steps; ++k) {
    bh_status st = bh_kick(c, n, vel, acc, h);
    if (!st) st = bh_drift(c, n, pos, vel, dt);
    if (!st) st = bh_build_tree(c, n, pos, mass);
    if (!st) st = bh_make_groups(c, n_crit, nullptr);
    if (!st) st = bh_compute_forces(c, eps, theta, nullptr, acc, pot);
    if (!st) st = bh_kick(c, n, vel, acc, h);
    if (st) return st;
  }
  return BH_OK;
}

bh_status bh_energy(bh_ctx *c, int64_t n, const double *vel, const double *mass, const float *pot,
                    double *energy) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (n < 0 || !energy || (n > 0 && (!vel || !mass || !pot))) return fail(c, BH_EINVAL, "bad energy arguments");
  bh_status st = ensure(c, c->energy_part, energy_part_bytes(), "energy partials");
  if (st) return st;
  energy_device(n, vel, mass, pot, P<double>(c->energy_part), energy, c->stream);
  return hip_check(c, hipGetLastError(), "kernel launch (energy)");
}

static bh_status check_net(bh_ctx *c, const bh_mlp *net) {
  if (!net || !net->params || !net->mu || !net->sigma) return fail(c, BH_EINVAL, "network pointers must not be NULL");
  return BH_OK;
}

static bh_status features_common(bh_ctx *c, const double *eps_sys, float *feat) {
  if (!c->have_groups) return fail(c, BH_ESTATE, "features requested before bh_make_groups");
  if (!eps_sys) return fail(c, BH_EINVAL, "eps_sys must not be NULL");
  if (c->n > 0 && !feat) return fail(c, BH_EINVAL, "feat must not be NULL");
  c->feps_host.assign((size_t)c->nsys, 0.0);
  for (int s = 0; s < c->nsys; ++s) {
    if (!(eps_sys[s] > 0.0) || !isfinite(eps_sys[s])) return fail(c, BH_EINVAL, "eps must be positive and finite");
    c->feps_host[s] = eps_sys[s];
  }
  bh_status st = ensure(c, c->feps, sizeof(double) * (size_t)c->nsys, "feature softening");
  if (st) return st;
  st = upload(c, c->feps.p, c->feps_host.data(), sizeof(double) * (size_t)c->nsys);
  if (st) return st;
  if (c->n == 0) return BH_OK;
  ProbeArgs pa{};
  pa.nodes = P<NodeRec>(c->nodes);
  pa.ginfo = P<int32_t>(c->ginfo);
  pa.gbox = P<double>(c->gbox);
  pa.spos = P<double>(c->spos);
  pa.smass = P<double>(c->smass);
  pa.pparent = P<int32_t>(c->pparent);
  pa.cparent = P<int32_t>(c->cparent);
  pa.ccount = P<int32_t>(c->ccount);
  pa.cslot = P<int32_t>(c->cslot);
  pa.level = P<int8_t>(c->level);
  pa.eps = P<double>(c->feps);
  pa.info = P<DevInfo>(c->info);
  pa.nsys = c->nsys;
  pa.feat = feat;
  if (c->probe_bpc == 0) c->probe_bpc = probe_blocks_per_cu();
  probe_device(pa, c->num_cu * c->probe_bpc, !c->xq_clean, c->stream);
  c->xq_clean = false;
  return hip_check(c, hipGetLastError(), "kernel launch (features)");
}

bh_status bh_group_features(bh_ctx *c, const double *eps_sys, float *feat) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  return features_common(c, eps_sys, feat);
}

bh_status bh_mlp_infer(bh_ctx *c, const bh_mlp *net, int64_t rows, const float *feat, float shift, float *theta) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  bh_status st = check_net(c, net);
  if (st) return st;
  if (rows < 0 || rows > BH_MAX_N) return fail(c, BH_EINVAL, "rows out of range");
  if (!isfinite(shift)) return fail(c, BH_EINVAL, "shift must be finite");
  if (rows == 0) return BH_OK;
  if (!feat || !theta) return fail(c, BH_EINVAL, "feat and theta must not be NULL");
  mlp_infer_device(net->params, net->mu, net->sigma, feat, rows, rows, P<DevInfo>(c->info), shift, theta, c->stream);
  return hip_check(c, hipGetLastError(), "kernel launch (inference)");
}

static bh_status theta_common(bh_ctx *c, const bh_mlp *net, const double *eps_sys, float shift, float *theta) {
  bh_status st = check_net(c, net);
  if (st) return st;
  if (!isfinite(shift)) return fail(c, BH_EINVAL, "shift must be finite");
  if (c->n > 0 && !theta) return fail(c, BH_EINVAL, "theta must not be NULL");
  const int64_t cap = std::max<int64_t>(c->n, 1);
  st = ensure(c, c->mlp_feat, sizeof(float) * BH_MLP_FEATURES * (size_t)cap, "features");
  if (st) return st;
  st = timer_start(c, c->t_theta);
  if (st) return st;
  st = features_common(c, eps_sys, P<float>(c->mlp_feat));
  if (st || c->n == 0) return st;
  // rows = -1: the kernel reads the group count on the device
  mlp_infer_device(net->params, net->mu, net->sigma, P<float>(c->mlp_feat), -1, cap, P<DevInfo>(c->info), shift,
                   theta, c->stream);
  // the list walk's order for these groups, from their features and theta
  st = ensure(c, c->walk_order, sizeof(int32_t) * (size_t)cap, "walk order");
  if (st) return st;
  if (!c->walk_order_hist.p) {
    st = ensure(c, c->walk_order_hist, order_hist_bytes(), "walk order bins");
    if (st) return st;
    order_clear_device(P<int32_t>(c->walk_order_hist), c->stream);  // every later call leaves it zero
  }
  walk_order_device(P<float>(c->mlp_feat), theta, P<DevInfo>(c->info), cap, P<int32_t>(c->walk_order_hist),
                    P<int32_t>(c->walk_order), c->stream);
  c->walk_order_valid = true;
  st = timer_stop(c, c->t_theta);
  if (st) return st;
  return hip_check(c, hipGetLastError(), "kernel launch (inference)");
}

bh_status bh_group_theta(bh_ctx *c, const bh_mlp *net, const double *eps_sys, float shift, float *theta) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  return theta_common(c, net, eps_sys, shift, theta);
}

bh_status bh_mlp_grad(bh_ctx *c, const bh_mlp *net, int32_t batch, const float *x, const float *target,
                      const float *weight, float *grad, float *loss) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  bh_status st = check_net(c, net);
  if (st) return st;
  if (batch < 1 || batch > 65536) return fail(c, BH_EINVAL, "batch must be in [1, 65536]");
  if (!x || !target || !weight || !grad) return fail(c, BH_EINVAL, "x, target, weight and grad must not be NULL");
  const size_t per = BH_MLP_FEATURES + 4 * BH_MLP_HIDDEN + 2;
  st = ensure(c, c->mlp_work, sizeof(float) * (per * (size_t)batch + 1), "training workspace");
  if (st) return st;
  float *w = P<float>(c->mlp_work);
  MlpWork ws{};
  ws.xn = w;
  ws.h1 = ws.xn + (size_t)batch * BH_MLP_FEATURES;
  ws.h2 = ws.h1 + (size_t)batch * BH_MLP_HIDDEN;
  ws.dz1 = ws.h2 + (size_t)batch * BH_MLP_HIDDEN;
  ws.dz2 = ws.dz1 + (size_t)batch * BH_MLP_HIDDEN;
  ws.dy = ws.dz2 + (size_t)batch * BH_MLP_HIDDEN;
  ws.loss = ws.dy + batch;
  ws.wsum = ws.loss + batch;
  mlp_grad_device(net->params, net->mu, net->sigma, batch, x, target, weight, ws, grad, loss, c->stream);
  return hip_check(c, hipGetLastError(), "kernel launch (training)");
}

bh_status bh_mlp_adam(bh_ctx *c, float *params, const float *grad, float *m, float *v, int32_t n, int32_t step,
                      float lr, float beta1, float beta2, float eps) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (n < 1 || step < 1 || !params || !grad || !m || !v) return fail(c, BH_EINVAL, "bad Adam arguments");
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(c, BH_EINVAL, "bad Adam hyper-parameters");
  adam_device(params, grad, m, v, n, lr, beta1, beta2, eps, step, c->stream);
  return hip_check(c, hipGetLastError(), "kernel launch (Adam)");
}

bh_status bh_export_sorted(bh_ctx *c, uint64_t *keys, int32_t *perm) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->have_tree) return fail(c, BH_ESTATE, "no tree");
  if (c->n == 0) return BH_OK;
  if (keys) k_copy_keys<<<blocks_for(c->n), 256, 0, c->stream>>>(c->sorted_keys, keys, c->n);
  if (perm) k_copy_i32<<<blocks_for(c->n), 256, 0, c->stream>>>(P<int32_t>(c->perm), perm, c->n);
  return hip_check(c, hipGetLastError(), "kernel launch (export sorted)");
}

bh_status bh_export_nodes(bh_ctx *c, int32_t *ints, double *reals) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->have_tree) return fail(c, BH_ESTATE, "no tree");
  const int64_t cap = 2 * std::max<int64_t>(c->n, 1) + c->nsys + 1;
  k_export_nodes<<<blocks_for(cap), 256, 0, c->stream>>>(P<NodeRec>(c->nodes), P<int8_t>(c->meta),
                                                          P<DevInfo>(c->info), c->nsys, ints, reals);
  return hip_check(c, hipGetLastError(), "kernel launch (export nodes)");
}

bh_status bh_neighbors(bh_ctx *c, const double *h, int32_t *count, double *rho, const int64_t *offsets,
                       int32_t *nbr) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->have_tree) return fail(c, BH_ESTATE, "neighbour search requested before a tree was built");
  if (!c->have_groups) return fail(c, BH_ESTATE, "neighbour search requested before bh_make_groups");
  if (c->n > 0 && !h) return fail(c, BH_EINVAL, "h must not be NULL");
  if (c->n == 0) {  // nothing to search (empty outputs may come as NULL)
    c->have_neighbors = true;
    return BH_OK;
  }
  if ((offsets == nullptr) != (nbr == nullptr)) return fail(c, BH_EINVAL, "offsets and nbr go together");
  if (!count && !rho && !nbr) return fail(c, BH_EINVAL, "no output requested");
  c->have_neighbors = true;
  const int variant = c->n_crit <= 64 ? 0 : (c->n_crit <= 128 ? 1 : 2);
  if (!c->nb_bpc[variant]) c->nb_bpc[variant] = neighbors_blocks_per_cu(c->n_crit);
  const int grid = c->num_cu * (c->opt.waves_per_cu > 0 ? c->opt.waves_per_cu : c->nb_bpc[variant]);
  NeighborArgs A{};
  A.nodes = P<NodeRec>(c->nodes);
  A.ginfo = P<int32_t>(c->ginfo);
  A.gbox = P<double>(c->gbox);
  A.spos = P<double>(c->spos);
  A.smass = P<double>(c->smass);
  A.perm = P<int32_t>(c->perm);
  A.info = P<DevInfo>(c->info);
  A.nsys = c->nsys;
  A.h = h;
  A.count = count;
  A.rho = rho;
  A.offsets = offsets;
  A.nbr = nbr;
  bh_status st = timer_start(c, c->t_neighbor);
  if (st) return st;
  neighbors_device(A, c->n_crit, grid, c->stream);
  st = timer_stop(c, c->t_neighbor);
  if (st) return st;
  return hip_check(c, hipGetLastError(), "kernel launch (neighbours)");
}

bh_status bh_export_moments(bh_ctx *c, double *moments) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->have_tree) return fail(c, BH_ESTATE, "no tree");
  if (!c->have_quad) return fail(c, BH_ESTATE, "the tree was built without the quadrupole option");
  if (!moments) return fail(c, BH_EINVAL, "moments must not be NULL");
  const int64_t cap = 2 * std::max<int64_t>(c->n, 1) + c->nsys + 1;
  k_export_moments<<<blocks_for(cap), 256, 0, c->stream>>>(P<NodeRec>(c->nodes), P<double>(c->qmom),
                                                            P<DevInfo>(c->info), c->nsys, moments);
  return hip_check(c, hipGetLastError(), "kernel launch (export moments)");
}

bh_status bh_export_groups(bh_ctx *c, int32_t *ints, double *box, int32_t *list_len, double *list_mass) {
  if (!c) return BH_EINVAL;
  c->err.clear();
  if (!c->have_groups) return fail(c, BH_ESTATE, "no groups");
  if ((list_len || list_mass) && !c->have_forces) return fail(c, BH_ESTATE, "no force call since the grouping");
  const int64_t cap = std::max<int64_t>(c->n, 1);
  k_export_groups<<<blocks_for(cap), 256, 0, c->stream>>>(P<int32_t>(c->ginfo), P<double>(c->gbox),
                                                           P<int32_t>(c->glist), P<double>(c->gmass),
                                                           P<DevInfo>(c->info), ints, box, list_len, list_mass);
  return hip_check(c, hipGetLastError(), "kernel launch (export groups)");
}

}  // extern "C"
