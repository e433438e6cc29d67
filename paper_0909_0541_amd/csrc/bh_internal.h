// Internal declarations shared by the HIP sources of libbh.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "bh.h"

namespace bh {

constexpr int kKeyLevels = 21;                 // bits per axis of a Morton key
constexpr uint32_t kQMax = (1u << kKeyLevels) - 1;
constexpr int kWave = 64;

// Node kinds as exported.
enum : int { kCell = 0, kParticle = 1, kBucket = 2, kEmpty = 3 };

// One node record (64 bytes) per slot.  Slots [0, n_systems) hold the system
// roots; the children of a cell occupy consecutive slots in octant order.
struct alignas(16) NodeRec {
  double com[3];  // centre of mass (a particle leaf: its position)
  double m;       // total mass
  double l;       // cell side; +inf for a bucket (always opened); 0 for a leaf
  double s;       // |geometric centre - centre of mass|
  int32_t child;  // first child slot, -1 for a particle leaf or an empty root
  int32_t nchild; // number of children
  int32_t first;  // first particle (Morton index)
  int32_t count;  // number of particles
};
static_assert(sizeof(NodeRec) == 64, "node record must be 64 bytes");

// What the moments pass reads of one cell, written by the level scatter in
// position order (one coalesced record per cell instead of reads scattered
// over the per-position arrays): the children's slots [c0, c0 + nc), the
// cell's own slot and particle range, and its integer coordinates at its
// geometric level (the level, or the chain cell's above a bucket) with that
// level in bits 21-25 of cz_geo and bit 26 set for a bucket that is always
// opened.
struct alignas(16) CellRec {
  int32_t c0, nc, slot, first, count;
  uint32_t cx, cy, cz_geo;
};
static_assert(sizeof(CellRec) == 32, "cell record must be 32 bytes");

// A particle's position and mass in input order, packed by the key pass so
// that the gather into key order reads one aligned 32-byte record per
// particle rather than two scattered reads.
struct alignas(32) PosMass {
  double x, y, z, m;
};

// Per-system geometry in device memory (first/count from the host, the root
// cube from the build).
struct SysInfo {
  double lo[3];
  double side;
  double scale;   // 2^21 / side
  int32_t first;  // first Morton position (systems occupy consecutive ranges)
  int32_t count;
};

// Per-system force parameters (uploaded by every force call).
struct SysParam {
  double eps;
  double theta;
};

constexpr int kLineInts = 32;  // int32 per 128-byte line

// Device-side counters and flags (one instance per context).
struct DevInfo {
  int32_t err;            // error flag bits (kErr*)
  int32_t max_level;
  int32_t n_cells;
  int32_t n_slots;
  int32_t n_groups;
  int32_t queue;          // walk work queue head
  unsigned long long interactions;
  unsigned long long list_entries;
  int32_t max_list;
  int32_t n_items;        // force work items (group, member block)
  unsigned long long nb_pairs;  // neighbour search: neighbours found (sum of the counts)
  unsigned long long nb_tests;  // neighbour search: candidate pairs whose distance was tested
  int32_t theta_fallback;  // groups of the last walk whose per-group theta was NaN (walked with the call's theta)
  int32_t pad0;
  unsigned long long node_visits;   // nodes the last walk tested (all its units)
  unsigned long long near_entries;  // list entries the last walk wrote to near lists
  // Counters that every wave of a kernel updates, each in a 128-byte line of
  // its own (atomics on one line serialise behind each other).
  alignas(128) int32_t queue2;  // force work queue head
  alignas(128) int32_t far_chunks;   // runs of kChunkRun list chunks taken (may exceed the pool: then it is the need)
  alignas(128) int32_t near_chunks;
  alignas(128) int32_t xq[8 * kLineInts];  // walk queue heads, one per XCD: xq[x * kLineInts]
  alignas(128) int32_t fq[8 * kLineInts];  // force queue heads, one per XCD: fq[x * kLineInts]
};

// Interaction lists: chunks (tiles) of T far entries (float4 x - c_g, m) and
// of T/2 near entries (T/2 float4 values, then T/2 float4 rounding
// residues), 16 T bytes each; T = bh_options.list_tile (a power of two in
// [kMinTile, kMaxTile], default kDefaultTile).
constexpr int kDefaultTile = 1024;
constexpr int kMinTile = 128;   // a near tile must hold a batch of 64 entries
constexpr int kMaxTile = 2048;
constexpr int kChunkRun = 4;    // chunks a walk wave takes from a pool per atomic
// Near entries: within kNearFrac times the box half-diagonal of the box.
constexpr double kNearFrac = 0.1;

enum : int32_t {
  kErrNonFinitePos = 1,
  kErrBadMass = 2,
  kErrStack = 4,
  kErrTheta = 8,
  kErrBuild = 16,
  kErrPool = 32,
  kErrWait = 64,          // a bounded wait ended without its condition (walk tasks, sort look-back)
  kErrRadius = 128,      // neighbour search: a radius not positive and finite
  kErrListSpace = 256,   // neighbour search: offsets leave a list too little or too much room
};

// Split walks: a walk that has tested split_visits nodes hands its remaining
// stack to new tasks and ends its own segment of the group's list; waves that
// find no group left take the tasks, in the same launch.  Segments of a group
// are summed separately and reduced in the order of their keys: the group's
// first walk has key 0, and task j of a hand-over by a walk with key K has key
// 17 K + j + 1, so keys are unique, fixed by the walks alone (not by when or
// where tasks ran), and below 17^kSplitDepth.
struct WalkTask {
  int32_t g;       // group
  int32_t roff;    // first of its ranges in the range pool
  int32_t rcount;  // ranges (its initial stack, bottom first); -1 until published
  int32_t key;     // order of its segment within the group
};
struct Segment {
  int32_t g, key;
  int32_t fh, fn, nh, nn;  // far/near chunk list heads and entry counts
  int32_t len, pad;
  double mass;
};
constexpr int kSplitDepth = 5;       // tasks this many hand-overs deep walk to the end
constexpr int kSplitVisits = 12288;  // smallest default node tests before a walk hands over
constexpr int kSplitPerParticle = 16;  // default cap: this many node tests per particle of a walk wave
constexpr int kSplitMeanFactor = 4;    // and at least this many times the previous walk's mean list length
constexpr int kDonateTasks = 16;     // tasks made from one handed-over stack
struct SplitCounters {               // device
  int32_t tasks;                     // task slots reserved
  int32_t queue;                     // task slots claimed by waiting waves
  int32_t ranges;                    // range pool entries taken
  int32_t segs;                      // segments written
  int32_t n_split;                   // groups whose list is in segments
  int32_t pending;                   // units (groups and published tasks) not finished
  int32_t depth;                     // deepest hand-over level reached
  int32_t waiters;                   // waves that wait for tasks
};

// Growable device buffer.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Event pairs recorded around one stage, summed when the stats are read.
struct Timer {
  std::vector<hipEvent_t> ev;  // pairs: ev[2k] start, ev[2k+1] stop
  int used = 0;                // pairs recorded since the last read
  bool open = false;
};

}  // namespace bh

struct bh_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cu = 0;
  std::string err;
  bh_options opt{0, 0, 0, 0, 0, 0};
  int walk_bpc = 0, force_bpc = 0, force_bpc_q = 0, probe_bpc = 0, nb_bpc[3] = {0, 0, 0};  // resident blocks per CU of the persistent kernels

  // current tree
  int64_t n = 0;
  int32_t nsys = 0;
  bool have_tree = false;
  bool have_groups = false;
  bool xq_clean = false;  // the per-XCD group queues are known to be 0 (reset by make_groups, used by walks)
  bool walk_order_valid = false;  // walk_order holds a permutation of the current groups (bh_group_theta)
  bool have_forces = false;
  bool have_quad = false;  // the current tree carries second moments
  bool have_neighbors = false;  // a neighbour search ran since the last build
  bool capturing = false;         // recording a step into a HIP graph: no uploads, syncs or timers
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr; // the captured step
  int32_t n_crit = 0;
  int64_t cap_n = 0;  // particle capacity of the per-particle buffers

  // per-particle workspaces (capacity cap_n)
  bh::DevBuf keys[2], vals[2];  // u64 keys, u32 values (radix sort ping-pong)
  bh::DevBuf sys_in;            // int32 system of each input row
  bh::DevBuf spos, smass;       // FP64 sorted positions [n][3] and masses
  bh::DevBuf pmass;             // PosMass [n] in input order (build scratch)
  bh::DevBuf perm;              // int32 sorted -> input row
  bh::DevBuf delta;             // int8 common-digit count of neighbours
  bh::DevBuf owner;             // int32 owner position of each split (or bucket run start)
  bh::DevBuf level;             // int8 level of the cell owned at a position (-1: none)
  bh::DevBuf cfirst, ccount;    // int32 particle range of the cell owned at a position
  bh::DevBuf cparent;           // int32 parent (owner position) of a cell, or -1 - system
  bh::DevBuf cdigit;            // int8 octant of a cell inside its parent
  bh::DevBuf pparent;           // int32 parent of a particle (owner position), -1 - system for a lone root
  bh::DevBuf pdigit;            // int8 octant of a particle inside its parent cell
  bh::DevBuf mask;              // int32 child octant mask of the cell at a position
  bh::DevBuf nchild;            // int32 children of the cell at a position
  bh::DevBuf cfirst_child;      // int32 first child slot of the cell at a position
  bh::DevBuf cslot;             // int32 slot of the cell at a position
  bh::DevBuf scan_tmp;          // scan block sums
  bh::DevBuf hist;              // radix histograms
  bh::DevBuf nodes;             // NodeRec [slots]
  bh::DevBuf msum;              // FP64 [slots][4] raw sums m, m x, m y, m z
  bh::DevBuf qmom;              // FP64 [slots][6] second moments about the centre of mass (quadrupole option)
  bh::DevBuf qpack;             // FP32 [slots][8] 3 x the same, the trace T and 1.5 T, as read by the force sum
  bh::DevBuf far_slot;          // int32 per far-pool entry: node slot of a cell entry, -1 a particle
  bh::DevBuf meta;              // int8 [slots] 32 * kind + level (inspection only)
  bh::DevBuf levels;            // int32 level counts, offsets and cursors (3 x 24)
  bh::DevBuf lcells;            // CellRec cells grouped by level
  bh::DevBuf gflag;             // int32 group start flags
  bh::DevBuf gidx;              // int32 exclusive scan of the flags (group index)
  bh::DevBuf glen;              // int32 group length at its start position
  bh::DevBuf ginfo;             // int32 [G][3] first, count, system
  bh::DevBuf gbox;              // FP64 [G][6]
  bh::DevBuf glist;             // int32 [G] list length of the last force call
  bh::DevBuf glists;            // int32 [G][4] far head, far count, near head, near count
  bh::DevBuf items;             // force work items in queue order
  bh::DevBuf far_pool, near_pool;  // list chunks
  bh::DevBuf far_next, near_next;  // int32 chunk links
  int32_t far_cap = 0, near_cap = 0;  // pool capacities in chunks
  int32_t pool_tile = 0;              // far entries per chunk the capacities count in
  bh::DevBuf gmass;             // FP64 [G] list mass of the last force call
  bh::DevBuf bbox_part;         // FP64 bbox partials
  bh::DevBuf sys;               // SysInfo [nsys]
  bh::DevBuf par;               // SysParam [nsys]
  bh::DevBuf info;              // DevInfo
  bh::DevBuf direct_part;       // FP64 partial sums of the judge
  double *judge_scratch = nullptr;  // device address of the static judge scratch on this context's device
  bh::DevBuf energy_part;       // FP64 energy partials
  bh::DevBuf feps;              // FP64 [nsys] softening of the feature call
  bh::DevBuf mlp_work;          // training batch workspace
  bh::DevBuf mlp_feat;          // FP32 [n][12] features of bh_group_theta
  bh::DevBuf pp_next;           // int32 per slot: thread pointers of the per-particle walk
  bh::DevBuf order_hist;        // int32 cost bins of the queue orders
  bh::DevBuf walk_order;        // int32 [n] order in which the list walk takes the groups (learned theta)
  bh::DevBuf walk_order_hist;   // int32 cost bins of the walk order (zero between calls)
  bh::DevBuf walk_hist;         // int32 [4]: mean list length of the last force call (automatic split cap)
  // split walks: tasks (ping-pong), range pool, segments, counters, per-group
  // flags, segment sort and partial sums
  bh::DevBuf tasks, ranges, segs, split_ctr, gsplit, gnseg, gsegfirst;
  bh::DevBuf skeys[2], svals[2], shist, sscan, srows, spbase, sgroups, psum;
  bh::SplitCounters *split_host = nullptr;  // pinned
  int32_t task_cap = 0, range_cap = 0, seg_cap = 0;
  int32_t last_split_groups = 0, last_segments = 0, last_depth = 0, last_attempts = 0;
  long long wait_ticks = 0;  // wall-clock ticks a walk wave may wait for a task (2 s)
  std::vector<double> feps_host;
  bh::DevInfo *info_host = nullptr;  // pinned mirror
  std::vector<bh::SysInfo> sys_host;
  std::vector<bh::SysParam> par_host;
  void *stage = nullptr;              // pinned staging buffer of host -> device uploads
  size_t stage_bytes = 0;
  hipEvent_t stage_event = nullptr;   // completion of the last staged upload
  bool stage_event_used = false;
  uint64_t *sorted_keys = nullptr;    // the key buffer holding the sorted keys

  bh::Timer t_build, t_groups, t_walk, t_force, t_particle, t_neighbor, t_theta;
};

namespace bh {

// ---- helpers implemented in bh_api.cpp ------------------------------------
bh_status fail(bh_ctx *c, bh_status st, const std::string &msg);
bh_status hip_check(bh_ctx *c, hipError_t e, const char *what);
bh_status ensure(bh_ctx *c, DevBuf &b, size_t bytes, const char *what);

// ---- kernels launchers (k_*.hip) ------------------------------------------
// scan.hip: exclusive scan of n int32 values (out may alias in); *total
// receives the sum (device int32).  tmp must hold scan_tmp_bytes(n).
size_t scan_tmp_bytes(int64_t n);
void scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, void *tmp,
                        hipStream_t s);

// sort.hip: stable LSD radix sort of (u64 key, u32 value) pairs on bits
// [bit0, bit1) (at most 64 bits); ping-pong buffers; returns the index (0/1)
// holding the result.  hist holds radix_hist_bytes(n); a look-back timeout
// sets kErrWait in *err (when err is not null).
size_t radix_hist_bytes(int64_t n);
int radix_sort_pairs(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit0,
                     int bit1, uint32_t *hist, void *scan_tmp, int32_t *err, hipStream_t s);
// one stable pass on an external 8-bit digit: digit(i) = sys_in[v[i]] >> shift & 255
int radix_pass_by_system(uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int cur, int64_t n,
                         const int32_t *sys_in, int shift, uint32_t *hist, void *scan_tmp, hipStream_t s);

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void iota_u32(uint32_t *v, int64_t n, hipStream_t s);

// k_tree.hip
struct TreeBuffers {
  const double *pos, *mass;
  int64_t n;
  int nsys;
  SysInfo *sys;
  DevInfo *info;
  int32_t *sys_in;  // system of each input row (used when nsys > 1)
  uint64_t *keys[2];
  uint32_t *vals[2];
  uint32_t *hist;
  void *scan_tmp;
  double *bbox_part;
  double *spos, *smass;
  PosMass *pm;      // input positions and masses, packed by the key pass
  int32_t *perm;
  int8_t *delta, *level, *cdigit, *pdigit;
  int32_t *owner, *cfirst, *ccount, *cparent, *pparent, *mask, *nchild, *cfc, *cslot;
  NodeRec *nodes;
  double *msum;
  double *qmom;           // nullable: FP64 [slots][6] second moments (xx, yy, zz, xy, xz, yz)
  float4 *qpack;          // with qmom: FP32 [slots][2] 3 (xx, yy, zz, xy), (3 xz, 3 yz, T, 1.5 T), T the trace
  int8_t *meta;           // per slot: 32 * kind + level (export only)
  int curve;              // key order: 0 Morton, 1 Peano-Hilbert
  bool any_empty;         // some system holds no particle (its root record is written apart)
  int32_t *lcount, *loff, *lcursor;  // cells per level: counts, offsets [23], scatter cursors
  CellRec *lcells;                   // cell records grouped by level
  int64_t slot_cap;       // capacity of nodes/msum/meta in slots
  uint64_t *sorted_keys;  // out: the buffer holding the sorted keys
};
int bbox_blocks_per_system(int nsys);
void build_tree_device(TreeBuffers &B, hipStream_t s);

// k_groups.hip
struct GroupBuffers {
  int64_t n;
  int nsys;
  int n_crit;
  const int8_t *level;
  const int32_t *ccount, *cfc, *nchild;
  const NodeRec *nodes;
  const SysInfo *sys;
  const double *spos;
  DevInfo *info;
  int32_t *gflag, *gidx, *glen, *ginfo;
  double *gbox;
  void *scan_tmp;
  int num_cu;
};
void make_groups_device(GroupBuffers &B, hipStream_t s);
void reset_force_counters(DevInfo *info, hipStream_t s);

// k_walk.hip: group walk writing the interaction lists
struct WalkListArgs {
  const NodeRec *nodes;
  const SysInfo *sys;
  const int32_t *ginfo;
  const double *gbox;
  const SysParam *par;
  const float *theta_group;
  DevInfo *info;
  int nsys;
  float4 *far_pool;
  float4 *near_pool;
  int32_t *far_next;
  int32_t *near_next;
  int far_cap, near_cap;
  int far_tile, near_tile;   // entries per far / near chunk (powers of two)
  int32_t *glists;
  int32_t *glist;
  double *gmass;
  int32_t *far_slot;         // nullable: node slot of each far entry (-1 a particle), for quadrupoles
  // split walks
  int visit_cap;             // node tests before a walk hands over its stack (0: never)
  const int32_t *mean_list;  // nullable: previous mean list length; the cap is raised to kSplitMeanFactor x it
  SplitCounters *ctr;
  WalkTask *tasks;           // task slots (ctr->tasks reserved)
  int task_cap;
  int2 *ranges;
  int range_cap;
  Segment *segs;
  int seg_cap;
  long long wait_ticks;      // wall-clock ticks a wave may wait for a task
  int32_t *gsplit;           // per group: 1 when its list is in segments
  const int32_t *order;      // nullable: the groups in the order the walk takes them; each eighth of
                             // [0, G) a permutation of itself (walk_order_device)
};
void walk_lists_device(const WalkListArgs &a, int grid, hipStream_t s);
// k_neighbors.hip: neighbour search and SPH density over the groups
struct NeighborArgs {
  const NodeRec *nodes;
  const int32_t *ginfo;
  const double *gbox;
  const double *spos, *smass;
  const int32_t *perm;
  DevInfo *info;
  int nsys;
  const double *h;        // [n] input order
  int32_t *count;         // nullable, [n] input order
  double *rho;            // nullable
  const int64_t *offsets; // nullable, [n + 1]: lists are written when set
  int32_t *nbr;
};
void neighbors_device(const NeighborArgs &a, int n_crit, int grid, hipStream_t s);
int neighbors_blocks_per_cu(int n_crit);
// k_particle.hip: the per-particle walk and sum (no shared lists)
void particle_forces_device(const NodeRec *nodes, int nslots, int nsys, const SysInfo *sys, const SysParam *par,
                            const double *spos, const int32_t *perm, int64_t n, int32_t *nxt, float *acc,
                            float *pot, DevInfo *info, hipStream_t s);
// k_split.hip: ordering and reduction of split groups
struct SplitBuffers {
  SplitCounters *ctr;
  Segment *segs;
  int seg_cap;
  uint64_t *keys[2];
  uint32_t *vals[2];
  uint32_t *hist;
  void *scan_tmp;
  uint32_t *order;            // out: sorted position -> segment
  int32_t *gsegfirst, *gnseg;  // per group
  int32_t *rows, *pbase, *total_rows;
  int32_t *sgroups, *nsg;     // split groups (unordered) and their count
  double *psum;
};
void split_finish_device(SplitBuffers &S, const int32_t *ginfo, int32_t *glist, double *gmass, DevInfo *info,
                         hipStream_t s);
void split_reduce_device(const SplitBuffers &S, const int32_t *ginfo, const double *smass, const int32_t *perm,
                         const SysParam *par, float *acc, float *pot, hipStream_t s);
void split_reset(SplitCounters *ctr, const DevInfo *info, WalkTask *tasks, int task_cap, hipStream_t s);
// k_order.hip: longest-first queue order of the force kernel
size_t order_hist_bytes();

// probe walk at theta = 1 for the learned-theta features f6..f10
struct ProbeArgs {
  const NodeRec *nodes;
  const int32_t *ginfo;
  const double *gbox;
  const double *spos, *smass;
  const int32_t *pparent, *cparent, *ccount, *cslot;
  const int8_t *level;
  const double *eps;  // per system
  DevInfo *info;      // queue must be reset before the launch
  int nsys;
  float *feat;        // [G][12]
};
// reset: clear the per-XCD group queues first (not needed right after make_groups)
void probe_device(const ProbeArgs &a, int grid, bool reset, hipStream_t s);
int probe_blocks_per_cu();
int walk_lists_blocks_per_cu();  // resident single-wave blocks per CU

// k_force.hip: force sums over the lists
struct ForceArgs {
  const int32_t *ginfo;
  const double *gbox;
  const int32_t *glists;
  const float4 *far_pool;
  const float4 *near_pool;
  const int32_t *far_next;
  const int32_t *near_next;
  const double *spos;
  const double *smass;
  const int32_t *perm;
  const SysParam *par;
  float *acc;
  float *pot;
  DevInfo *info;
  const int32_t *items;  // [n_items][2] in queue order (eight per-XCD queues, longest group first):
                         // group, member block (+ 256 x (segment + 1) for a split group)
  const int32_t *xstart; // [9]: first queue position of each XCD's queue, then the item count
  const int32_t *glist;  // [G] list length of each group (all segments)
  // split groups: segments sorted by (group, key), the first sorted segment
  // of each group, and the partial sums of each segment's members
  const Segment *segs;
  const uint32_t *seg_order;  // sorted position -> segment
  const int32_t *gsegfirst;   // group -> first sorted position
  const int32_t *pbase;       // sorted position -> first partial-sum row
  double *psum;               // [rows][4] ax, ay, az, pot
  int far_tile, near_tile;    // entries per far / near chunk
  const int32_t *far_slot;    // quadrupole sums: node slot of each far entry (near entries: residue .w)
  const float4 *qpack;        // quadrupole sums: [slots][2] second moments
};
void force_lists_device(const ForceArgs &a, int grid, hipStream_t s);
// The force items in queue order (k_order.hip), with the list statistics and
// the mean list length; hist holds order_hist_bytes() and is zero on entry
// (order_clear_device once after allocation; every call leaves it zero).
void item_order_device(const ForceArgs &f, const int32_t *gsplit, const int32_t *gnseg, int64_t gcap, int32_t *hist,
                       int32_t *mean_list, int32_t *items, hipStream_t s);
void order_clear_device(int32_t *hist, hipStream_t s);
// Walk order of a learned-theta step (k_order.hip): within each eighth of
// the groups, the groups by predicted walk time from their features (FP32
// [cap][12]) and theta, longest first; hist holds order_hist_bytes() and is
// zero on entry (every call leaves it zero).
void walk_order_device(const float *feat, const float *theta, const DevInfo *info, int64_t cap, int32_t *hist,
                       int32_t *order, hipStream_t s);
int force_lists_blocks_per_cu(bool quad);
void reset_list_counters(DevInfo *info, hipStream_t s);

// k_misc.hip
size_t direct_part_bytes(int64_t n, int64_t s, int num_cu, int64_t *chunk, int64_t *nchunk);
// static scratch of the no-allocation judge: its size, and its device address
// on `device` (looked up once per device with that device current)
constexpr size_t kJudgeScratchBytes = (size_t)BH_JUDGE_SCRATCH_BYTES;
hipError_t judge_scratch_address(int device, double **ptr);
void direct_sampled_device(const double *pos, const double *mass, int64_t n, double eps, int64_t s,
                           const int64_t *idx, double *acc, double *pot, double *part, int64_t chunk,
                           int64_t nchunk, hipStream_t st);
void kick_device(int64_t n, double *vel, const float *acc, double dt, hipStream_t s);
void drift_device(int64_t n, double *pos, const double *vel, double dt, hipStream_t s);
size_t energy_part_bytes();
void energy_device(int64_t n, const double *vel, const double *mass, const float *pot, double *part, double *out,
                   hipStream_t s);
void reset_info_device(DevInfo *info, hipStream_t s);

// k_mlp.hip: per-group theta from a 12 -> 64 -> 64 -> 1 network
constexpr int kMlpParams = 64 * 12 + 64 + 64 * 64 + 64 + 64 + 1;
constexpr float kThetaMin = 0.3f, kThetaSpan = 0.7f;
struct MlpWork {  // per-sample activations and gradients of a training batch
  float *xn, *h1, *h2, *dz1, *dz2, *dy, *loss, *wsum;
};
void mlp_infer_device(const float *params, const float *mu, const float *sigma, const float *x, int64_t rows,
                      int64_t cap_rows, const DevInfo *info, float shift, float *theta, hipStream_t s);
void mlp_grad_device(const float *params, const float *mu, const float *sigma, int B, const float *x,
                     const float *target, const float *w, MlpWork ws, float *grad, float *loss, hipStream_t s);
void adam_device(float *params, const float *grad, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t s);

}  // namespace bh
