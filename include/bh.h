/*
 * bh.h -- C ABI of the MI355X grouped Barnes-Hut oct-tree gravity library.
 *
 * Method (N. Nakasato, "Oct-tree Method on GPU"):
 *   Eq. (1)    softened potential and force of particle i, summed over j != i:
 *              acc_i = sum_j m_j (x_j - x_i) / (|x_i - x_j|^2 + eps^2)^(3/2)
 *              pot_i = -sum_j m_j / (|x_i - x_j|^2 + eps^2)^(1/2)
 *              (attractive sign convention, G = 1).
 *   Sec. 3.1   the oct-tree: the cube enclosing all particles is divided into
 *              eight sub-cells recursively until a cell holds one particle;
 *              cells act through their monopole (total mass at the centre of
 *              mass).
 *   Eq. (2)/(3) modified opening criterion: a cell of side l whose centre of
 *              mass lies s from its geometric centre is far enough when
 *              d^2 > (l/theta + s)^2.
 *   Sec. 3.5   Morton ordering of the particles (Peano-Hilbert as an option).
 *   Sec. 1, 3.2 the grouped (vectorised) walk: each group of nearby particles
 *              walks the tree once to build one interaction list that all its
 *              members sum over.  For a group, d is the distance from the
 *              cell's centre of mass to the group's bounding box, so every
 *              member satisfies Eq. (2) on its own.
 *
 * Conventions for every entry point:
 *   - Arrays named "device" are device (HBM) pointers, e.g. torch tensors on
 *     the GPU; arrays named "host" are ordinary host memory.  The caller owns
 *     every array it passes; the library never frees or retains them past the
 *     call.  The context owns all internal workspaces (sorted copies, tree,
 *     groups) until bh_destroy.
 *   - Positions are FP64 [n][3] row-major (x, y, z), masses FP64 [n] (finite,
 *     >= 0).  Forces come back as FP32 acc [n][3] and pot [n] in the caller's
 *     input order.
 *   - Work is enqueued asynchronously on the context's HIP stream; a call
 *     returns before the GPU finishes unless its comment says it synchronises.
 *     One context per host thread; calls on one context must not overlap.
 *   - Every call returns a bh_status and never aborts; after a failure
 *     bh_last_error(ctx) holds a message.  Input checks that need device data
 *     (non-finite positions or masses) are reported by the next synchronising
 *     call (bh_make_groups with a count pointer, bh_get_stats, bh_sync).
 */
#ifndef BH_H
#define BH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bh_ctx bh_ctx;

typedef enum {
  BH_OK = 0,
  BH_EINVAL = -1,    /* bad argument or input data */
  BH_ENOMEM = -2,    /* device allocation failed */
  BH_EHIP = -3,      /* a HIP runtime call failed */
  BH_ESTATE = -4,    /* call out of order (e.g. forces before a tree) */
  BH_EINTERNAL = -5  /* an internal capacity check fired (reported, never silent) */
} bh_status;

/* Largest group size accepted by bh_make_groups. */
#define BH_MAX_NCRIT 256
/* Largest particle count of one tree (all systems together): node slots
 * (at most 2 n + systems) and particle indices are int32 on the device. */
#define BH_MAX_N ((1LL << 30) - (1LL << 17))

typedef struct {
  int64_t n;             /* particles in the current tree (all systems) */
  int32_t n_systems;     /* independent systems in the current tree */
  int32_t n_crit;        /* group size limit of the current groups */
  int64_t n_cells;       /* internal cells (including always-open buckets) */
  int64_t n_slots;       /* node records: cells + particle leaves + system roots */
  int64_t n_groups;      /* groups of the current grouping */
  int64_t interactions;  /* last force call: sum over members of (list length - 1) */
  int64_t list_entries;  /* last force call: sum over groups of the list length */
  int64_t max_list;      /* last force call: longest list */
  int32_t max_level;     /* deepest cell level (root cube = level 0) */
  int32_t error_flags;   /* device-side checks, 0 when all is well */
  /* With timing enabled: summed GPU time (HIP events on the context's stream)
   * of the calls made since the previous bh_get_stats, and their number. */
  double t_build_ms;     /* bh_build_tree / bh_build_batch kernels */
  double t_groups_ms;    /* bh_make_groups kernels */
  double t_walk_ms;      /* group walk kernel of the force calls (lists) */
  double t_force_ms;     /* force-sum kernel of the force calls */
  int32_t n_build_calls;
  int32_t n_groups_calls;
  int32_t n_walk_calls;
  int32_t n_force_calls;
  int32_t n_split_groups;  /* last force call: groups whose walk was handed over to several waves */
  int32_t n_segments;      /* last force call: list segments of those groups */
  int32_t n_split_levels;  /* last force call: deepest hand-over level of a split walk (0: none) */
  int32_t n_walk_attempts; /* last force call: walks run (more than 1 when a list pool had to grow) */
  double t_particle_ms;     /* per-particle walk calls (thread pointers, walk and sum) */
  int32_t n_particle_calls;
  int32_t n_neighbor_calls;
  double t_neighbor_ms;     /* bh_neighbors calls */
  int64_t neighbor_pairs;   /* last bh_neighbors: neighbours found (sum of the counts) */
  int64_t neighbor_tests;   /* last bh_neighbors: member-candidate pairs whose distance was tested */
  double t_theta_ms;        /* bh_group_theta calls (features, probe walk, inference, walk order) */
  int32_t n_theta_calls;
  int32_t n_theta_fallback; /* last force call: groups whose per-group theta was NaN (walked with the
                               call's theta) */
  int64_t node_visits;      /* last force call: nodes the group walk tested */
  int64_t near_entries;     /* last force call: list entries written to near lists (the rest are far) */
} bh_stats;

typedef struct {
  int32_t waves_per_cu;  /* persistent grids = CUs x waves_per_cu; 0 (default): as many as fit */
  int32_t timing;        /* 1: record HIP events around each stage (default 0) */
  int32_t split_visits;  /* a group walk that has tested this many nodes hands the rest of its
                            stack to up to 16 new walk tasks, which waves with no group left
                            take in the same launch, so that long lists are walked and summed
                            by several waves; tasks 5 hand-overs deep walk to the end (0:
                            default, automatic: a single system is not split (its walk then
                            runs without the split machinery, which is faster); a batch
                            splits at 16 per particle of a walk wave, i.e.
                            16 n / (CUs x walk waves per CU), at least 12288, and at least 4
                            times the mean list length of the previous force call on the
                            context, so that only outlier walks split; -1: never; else
                            >= 64, exactly).  Results do not depend on when or where the
                            tasks ran, only on the cap (with the automatic cap, two calls on
                            the same input agree bit for bit when their previous calls had
                            lists of the same mean length). */
  int32_t quadrupole;    /* 1: builds also compute every cell's second mass moments S about its
                            centre of mass (bottom-up, parallel axes, FP64), and bh_compute_forces
                            and bh_compute_forces_batch add to each cell entry of a list the
                            second-order term of the softened potential of its particles,
                            -3 (u.S.u) / (2 R^5) + tr S / (2 R^3) with u = com - x_i,
                            R^2 = |u|^2 + eps^2, and its gradient, in FP32 (an extension of the
                            monopole sums of Eq. 1: same lists, same opening test).  Force calls
                            then need a tree built with the option set (else BH_ESTATE); the
                            per-particle walk rejects it (BH_EINVAL).  0 (default): monopoles. */
  int32_t curve;         /* order of the keys, the particles and the children of a cell (Sec. 3.5
                            uses Morton order; Peano-Hilbert is the alternative it names):
                            0 (default) Morton, bit interleaving; 1 Peano-Hilbert, consecutive
                            cells face-adjacent.  The cells are the same either way; the order,
                            and hence the groups, differ.  Takes effect at the next build. */
  int32_t list_tile;     /* entries per chunk of a group's far interaction list (its near list uses
                            chunks of half as many): the walk hands lists to the force sum in these
                            tiles, and the force sum folds its FP32 partial sums into FP64 after
                            each.  0 (default): 1024; else a power of two in [128, 2048].  Takes
                            effect at the next force call; a tuning knob (bh_graph_capture
                            records the value of the capture). */
} bh_options;

/* ---- context ---------------------------------------------------------- */

/* Create a context on the current HIP device.  stream is a hipStream_t (NULL =
 * the default stream).  *out receives the context; nothing is allocated on
 * the device until the first build. */
bh_status bh_create(bh_ctx **out, void *stream);

/* Free the context and all its device memory.  NULL is allowed. */
void bh_destroy(bh_ctx *ctx);

/* Message of the last failed call on ctx ("" if none).  Valid until the next call. */
const char *bh_last_error(const bh_ctx *ctx);

/* Change the stream used by later calls. */
bh_status bh_set_stream(bh_ctx *ctx, void *stream);

/* Read or change options (opt must not be NULL). */
bh_status bh_get_options(const bh_ctx *ctx, bh_options *opt);
bh_status bh_set_options(bh_ctx *ctx, const bh_options *opt);

/* Wait for all work of ctx and report device-side input errors (BH_EINVAL). */
bh_status bh_sync(bh_ctx *ctx);

/* ---- tree (Sec. 3.1, 3.5) --------------------------------------------- */

/* Build the oct-tree of one system of n particles.
 *   pos  device FP64 [n][3], mass device FP64 [n].
 * Steps: root cube (corner at the per-axis minimum, side = largest extent
 * times (1 + 2^-20), 1 if all points coincide); 21-bit cell coordinates per
 * axis and their 63-bit Morton keys; stable LSD radix sort of (key, index);
 * cells = key prefixes shared by at least two particles that split into at
 * least two sub-cells (single-child chains are skipped: they hold the same
 * particles and, for theta <= 1, give the same interaction list); particles
 * with equal keys form an always-opened bucket; per cell the total mass and
 * centre of mass (FP64 sums over the sub-cells in octant order), side l and s.
 * n = 0 is allowed (empty tree).  BH_EINVAL: n < 0, n > BH_MAX_N, NULL pointers. */
bh_status bh_build_tree(bh_ctx *ctx, int64_t n, const double *pos, const double *mass);

/* Build one tree over several independent systems in one pass.
 *   offsets host int64 [n_systems + 1]: system k owns rows offsets[k] ..
 *   offsets[k+1]-1 of pos/mass (offsets[0] = 0, non-decreasing).
 * Each system gets its own root cube; systems never interact. */
bh_status bh_build_batch(bh_ctx *ctx, int32_t n_systems, const int64_t *offsets, const double *pos,
                         const double *mass);

/* ---- groups ------------------------------------------------------------ */

/* Group the particles of the current tree: a cell holding more than n_crit
 * particles is split further; runs of consecutive sub-cells (octant order)
 * holding at most n_crit particles each are packed greedily into groups of at
 * most n_crit particles; a system with at most n_crit particles is one group.
 * Every group is a contiguous Morton range with an FP64 bounding box.
 *   n_crit in [1, BH_MAX_NCRIT].
 *   n_groups_out host, nullable; when given the call synchronises and reports
 *   device-side input errors. */
bh_status bh_make_groups(bh_ctx *ctx, int32_t n_crit, int64_t *n_groups_out);

/* ---- forces (Eq. 1, 2, 3) ---------------------------------------------- */

/* Tree forces for every particle of a single-system or batched tree, with one
 * eps and theta for all systems.
 *   eps > 0 (eps^2 must be a normal FP32 number), theta in [0, 1]
 *   (theta = 0 opens every cell: exact direct summation).
 *   theta_group device FP32 [n_groups], nullable: per-group theta overriding
 *   theta (values in [0, 1]; a NaN stands for "no value": that group walks
 *   with theta and is counted in stats.n_theta_fallback; other values
 *   outside [0, 1] raise an error flag).
 *   acc device FP32 [n][3], pot device FP32 [n]: input order.
 * Two kernels (the interaction-list method of Sec. 3.2): every group walks
 * the tree once with the FP64 opening test and writes its list to HBM as FP32
 * (x - c_g, m), c_g the group's box centre (entries close to the box also
 * keep the FP32 rounding residue); then members sum Eq. (1) over the list in
 * FP32, folding partial sums into FP64.  The call synchronises once, after
 * the walk, to check that the list pool held every list (the pool grows and
 * the walk is repeated when it did not). */
bh_status bh_compute_forces(bh_ctx *ctx, double eps, double theta, const float *theta_group, float *acc,
                            float *pot);

/* Same with per-system parameters: eps_sys, theta_sys host FP64 [n_systems].
 * A system's results equal, bit for bit, those of the same system run alone
 * with the same split-walk visit cap (the automatic cap depends on the total
 * particle count and the previous call, so give bh_options.split_visits a
 * fixed value for that). */
bh_status bh_compute_forces_batch(bh_ctx *ctx, const double *eps_sys, const double *theta_sys,
                                  const float *theta_group, float *acc, float *pot);

/* The paper's own GPU form (Sec. 3.4, Fig. "treegpu"): every particle walks
 * the tree by itself over a threaded tree ("next" skips a subtree, "more" is
 * the first child) and sums Eq. (1) on the way, with no shared list.  The
 * opening test is the group test of bh_compute_forces with one-particle
 * groups (d = distance from the cell's centre of mass to the particle), so
 * the terms summed are those of the lists of bh_make_groups(1); the lane's
 * own particle is skipped.  FP64 test, FP32 terms from the FP64 relative
 * vector, partial sums folded into FP64.  Needs a tree (not groups).
 *   eps > 0 (eps^2 a normal FP32 number), theta in [0, 1] (theta = 0: direct
 *   summation); acc device FP32 [n][3], pot device FP32 [n], input order.
 * Stats report interactions (list length - 1 per particle), entries and the
 * longest list as for the group path.  Synchronises once (node count). */
bh_status bh_compute_forces_particle(bh_ctx *ctx, double eps, double theta, float *acc, float *pot);

/* Same with per-system parameters: eps_sys, theta_sys host FP64 [n_systems]. */
bh_status bh_compute_forces_particle_batch(bh_ctx *ctx, const double *eps_sys, const double *theta_sys, float *acc,
                                           float *pot);

/* ---- captured steps (HIP graph) ---------------------------------------- */

/* Record one whole step -- tree build (single system or batch), groups, list
 * walk and force sum -- into a HIP graph owned by the context, for replay by
 * bh_graph_launch without host work.  Arguments as for bh_build_batch,
 * bh_make_groups and bh_compute_forces_batch (eps_sys, theta_sys host FP64
 * [n_systems]; theta_group device FP32, nullable).  The call first runs the
 * step eagerly (which sizes every buffer and leaves the results in acc/pot),
 * grows the list pools by a quarter for replays on moved particles, then
 * captures.  A replay reads pos and mass where they were at capture (update
 * them in place between replays) and writes acc and pot.  Sizes, offsets,
 * n_crit, eps and theta are those of the capture.  A replay cannot wait for
 * the list-pool check: if a list does not fit, bh_sync (or bh_get_stats)
 * reports it and the replay's forces are invalid; capture again.  A later
 * call on the context that has to grow a buffer (a larger input, for one)
 * discards the capture.  Synchronises (the eager step). */
bh_status bh_graph_capture(bh_ctx *ctx, int32_t n_systems, const int64_t *offsets, const double *pos,
                           const double *mass, int32_t n_crit, const double *eps_sys, const double *theta_sys,
                           const float *theta_group, float *acc, float *pot);

/* Replay the captured step on the context's stream (asynchronous).
 * BH_ESTATE without a capture. */
bh_status bh_graph_launch(bh_ctx *ctx);

/* Counters of the current tree, groups and last force call, and the timings
 * collected since the previous call (which are then reset).  Synchronises.
 * stats host, not NULL. */
bh_status bh_get_stats(bh_ctx *ctx, bh_stats *stats);

/* ---- FP64 judge (Eq. 1 by direct summation) ---------------------------- */

/* Direct FP64 summation of Eq. (1) for s sampled particles against all n.
 *   pos device FP64 [n][3], mass device FP64 [n], idx device int64 [s]
 *   (0 <= idx < n), acc device FP64 [s][3], pot device FP64 [s].
 * Independent of any tree held by ctx (uses only its stream and scratch). */
bh_status bh_direct_sampled(bh_ctx *ctx, int64_t n, const double *pos, const double *mass, double eps,
                            int64_t s, const int64_t *idx, double *acc, double *pot);

/* Bytes of the static device array behind bh_direct_sampled_noalloc (one per
 * device the library runs on, held until the process ends). */
#define BH_JUDGE_SCRATCH_BYTES (8 << 20)

/* bh_direct_sampled for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results (bit for bit) as
 * bh_direct_sampled, but the FP64 partial sums live in a static device array
 * of BH_JUDGE_SCRATCH_BYTES per device instead of context-owned memory: the
 * call allocates nothing.  The partial sums take 32 bytes per sampled
 * particle and j chunk (a few MiB for any s up to tens of thousands); a
 * sample whose partial sums would not fit is rejected with BH_EINVAL before
 * anything is launched.  Every call on one device shares that device's
 * array: calls that overlap on one device (other contexts or streams) race,
 * so order them on one stream.  The array's address is looked up once per
 * device by bh_create (which does allocate); later calls only launch. */
bh_status bh_direct_sampled_noalloc(bh_ctx *ctx, int64_t n, const double *pos, const double *mass, double eps,
                                    int64_t s, const int64_t *idx, double *acc, double *pot);

/* ---- time integration (kick-drift-kick leapfrog, FP64 state) ----------- */

/* vel += dt * acc (acc FP32 [n][3] from a force call, vel FP64 [n][3]). */
bh_status bh_kick(bh_ctx *ctx, int64_t n, double *vel, const float *acc, double dt);

/* pos += dt * vel (both FP64 [n][3]). */
bh_status bh_drift(bh_ctx *ctx, int64_t n, double *pos, const double *vel, double dt);

/* Kick-drift-kick leapfrog (the time integration of Sec. 4; the scheme is a
 * reading): per step vel += dt/2 acc, pos += dt vel, tree + groups + forces at
 * the new positions, vel += dt/2 acc.  FP64 state, FP32 accelerations.
 *   pos, vel device FP64 [n][3] (updated in place), mass device FP64 [n].
 *   acc, pot device FP32 in/out: on entry the forces at pos (from a
 *   bh_build_tree + bh_make_groups + bh_compute_forces with the same eps,
 *   theta, n_crit, or the previous bh_leapfrog call), on return the forces at
 *   the final positions.  The context's tree and groups are those of the
 *   final positions.  steps >= 0, dt finite; eps, theta, n_crit as for the
 *   force and group calls.  Synchronises once per step (list pool check). */
bh_status bh_leapfrog(bh_ctx *ctx, int64_t n, double *pos, double *vel, const double *mass, double eps,
                      double theta, int32_t n_crit, double dt, int32_t steps, float *acc, float *pot);

/* energy device FP64 [2]: kinetic sum(m v^2 / 2) and potential sum(m pot / 2). */
bh_status bh_energy(bh_ctx *ctx, int64_t n, const double *vel, const double *mass, const float *pot,
                    double *energy);

/* ---- learned per-group theta ------------------------------------------- */

/* The paper fixes one opening angle and studies its accuracy/work trade-off
 * (Sec. 3.5, Table "theta").  These calls let a small network choose theta per group instead:
 * 12 group features -> tanh(64) -> tanh(64) -> theta = 0.3 + 0.7 sigmoid(y +
 * shift).  Features (FP32, per group, from the current tree and groups; c the
 * member count, c_g the box centre, R the box half-diagonal, x_g and m_g the
 * members' centre of mass and mass, A1 the smallest cell with at least two
 * sub-cells (not a bucket of equal keys) holding more than c particles, A2
 * the next such cell above it (A1 at the root)):
 *   f0 = log2 c, f1 = log2(1 + R/eps), f2 = |x_g - c_g| / (R + eps),
 *   f3 = log2(l(A1) / (R + eps)), f4 = log2(m(A1) / m_g),
 *   f5 = |com(A1) - c_g| / l(A1), f11 = log2(m(A2) / m_g)
 * (f3, f4, f5, f11 = 0 for a group that is a whole system), and from the
 * group's interaction list at theta = 1, with d = com - c_g over the entries
 * whose centre of mass lies outside the box:
 *   f6 = log2(|sum m d / (|d|^2 + eps^2)^(3/2)| + 2^-100),
 *   f7 = log2(sum m / (|d|^2 + eps^2) + 2^-100),
 *   f8 = log2(1 + single-particle entries outside the box),
 *   f9 = log2(list length), f10 = log2(mass of the entries inside the box / m_g). */
#define BH_MLP_FEATURES 12
#define BH_MLP_HIDDEN 64
#define BH_MLP_PARAMS 5057

typedef struct bh_mlp {
  const float *params; /* device FP32 [BH_MLP_PARAMS]: W1 [64][12], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 */
  const float *mu;     /* device FP32 [12]: feature offsets */
  const float *sigma;  /* device FP32 [12]: feature scales (nonzero); the network reads (f - mu) / sigma */
} bh_mlp;

/* Features of the current groups.  eps_sys host FP64 [n_systems] (> 0).
 * feat device FP32 [n_groups][12] (n_groups <= max(n, 1)).  Asynchronous.
 * BH_ESTATE without groups. */
bh_status bh_group_features(bh_ctx *ctx, const double *eps_sys, float *feat);

/* theta for rows of features, on the matrix cores in bfloat16 (features
 * after normalisation, the two hidden layers' weights and the first hidden
 * activations are rounded to bfloat16; sums, biases, tanh and the output
 * layer are FP32).  feat device FP32 [rows][12], theta device FP32 [rows]. */
bh_status bh_mlp_infer(bh_ctx *ctx, const bh_mlp *net, int64_t rows, const float *feat, float shift, float *theta);

/* Features and theta of the current groups in one asynchronous call (the
 * features go to a context-owned buffer).  theta device FP32, room for
 * max(n, 1) values; pass it as theta_group to bh_compute_forces.  A row
 * whose network output is not a number gives theta NaN, which the force call
 * replaces by its own theta for that group (the fixed-theta fallback).
 * The call also orders the list walk of the next force calls with a
 * theta_group on these groups (until bh_make_groups): each eighth of the
 * groups, the range one XCD's walk waves take, longest predicted walk first,
 * from the features and theta.  The order changes only which wave walks a
 * group and when, never a list or a result.
 * With timing enabled, stats.t_theta_ms sums these calls. */
bh_status bh_group_theta(bh_ctx *ctx, const bh_mlp *net, const double *eps_sys, float shift, float *theta);

/* bh_graph_capture for a step with learned theta: the captured step is tree
 * build, groups, bh_group_theta (features, probe walk, inference at the
 * given shift, into theta_group), then the list walk and force sum with
 * theta_group; theta_sys is the fixed theta of groups whose network output
 * is NaN.  theta_group device FP32, room for max(n, 1) values, rewritten by
 * every replay; net's arrays must stay in place while the capture is used.
 * Otherwise as bh_graph_capture (same checks, same eager first step, same
 * replay rules).  Synchronises. */
bh_status bh_graph_capture_learned(bh_ctx *ctx, int32_t n_systems, const int64_t *offsets, const double *pos,
                                   const double *mass, int32_t n_crit, const double *eps_sys,
                                   const double *theta_sys, const bh_mlp *net, float shift, float *theta_group,
                                   float *acc, float *pot);

/* FP32 loss and gradient of a training batch: loss = sum_b w_b (theta_b -
 * target_b)^2 / sum_b w_b with theta_b the network output at shift 0 (FP32
 * throughout).  x device FP32 [batch][12], target and weight device FP32
 * [batch] (weights >= 0, positive sum); grad device FP32 [BH_MLP_PARAMS]
 * (summed over the batch in sample order); loss device FP32 [1], nullable.
 * batch in [1, 65536]. */
bh_status bh_mlp_grad(bh_ctx *ctx, const bh_mlp *net, int32_t batch, const float *x, const float *target,
                      const float *weight, float *grad, float *loss);

/* One Adam step (bias-corrected, step >= 1) on device FP32 arrays of n
 * values: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * params -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
bh_status bh_mlp_adam(bh_ctx *ctx, float *params, const float *grad, float *m, float *v, int32_t n, int32_t step,
                      float lr, float beta1, float beta2, float eps);

/* ---- inspection (tests and tools) -------------------------------------- */

/* Sorted keys (Morton or Peano-Hilbert, bh_options.curve) and the permutation: keys device uint64 [n],
 * perm device int32 [n] with perm[k] = input row of the k-th particle in
 * key order (within each system, systems in order).  Either may be NULL. */
bh_status bh_export_sorted(bh_ctx *ctx, uint64_t *keys, int32_t *perm);

/* Node records, one per slot (stats.n_slots): ints device int32 [slots][6] =
 * level, kind (0 cell, 1 particle leaf, 2 bucket, 3 empty system root), first
 * particle (Morton index), count, first child slot (-1 for leaves), number of
 * children; reals device FP64 [slots][6] = mass, centre of mass x, y, z, side
 * l (+inf for buckets), s.  Slot k < n_systems is the root of system k. */
bh_status bh_export_nodes(bh_ctx *ctx, int32_t *ints, double *reals);

/* ---- neighbour search (SPH) ------------------------------------------- */

/* The general treewalk of Sec. 3.3 (Fig. "general_treewalk") applied to a
 * short-range interaction, on the current tree and groups (bh_make_groups
 * first).  The neighbours of particle i are the particles j != i of the same
 * tree with |x_j - x_i| < h_i (each particle's own radius: the "gather"
 * form), the squared distance (dx^2 + dy^2) + dz^2 evaluated in FP64 as
 * written.  h: device FP64 [n], input order, positive and finite (else
 * BH_EINVAL at the next synchronising call).  Outputs, device, input order,
 * each nullable (at least one when n > 0): count int32 [n], the neighbour counts; rho
 * FP64 [n], the SPH density m_i W(0, h_i) + sum over neighbours m_j W(r_ij,
 * h_i) with the cubic spline kernel of compact support h (W = 8/(pi h^3)
 * (1 - 6q^2 + 6q^3) for q = r/h < 1/2, 16/(pi h^3) (1 - q)^3 for q < 1);
 * offsets int64 [n + 1] with nbr int32 [offsets[n]]: the input indices of
 * i's neighbours at nbr[offsets[i] ...], in no particular order (offsets
 * from an exclusive scan of an earlier call's counts; a mismatch is reported
 * as BH_EINVAL).  Systems of a batch are searched separately.  Asynchronous;
 * stats report the pairs found and tested. */
bh_status bh_neighbors(bh_ctx *ctx, const double *h, int32_t *count, double *rho, const int64_t *offsets,
                       int32_t *nbr);

/* Second mass moments of every slot about its centre of mass (tree built
 * with the quadrupole option, else BH_ESTATE): moments device FP64
 * [slots][6] = xx, yy, zz, xy, xz, yz, sum m d_a d_b over the node's
 * particles with d = x - com; zero for particle leaves. */
bh_status bh_export_moments(bh_ctx *ctx, double *moments);

/* Groups (stats.n_groups): ints device int32 [G][3] = first particle, count,
 * system; box device FP64 [G][6] = lo x, y, z, hi x, y, z.  After a force
 * call, list_len device int32 [G] and list_mass device FP64 [G] (sum of the
 * masses of the list entries) describe each group's interaction list.
 * Any pointer may be NULL. */
bh_status bh_export_groups(bh_ctx *ctx, int32_t *ints, double *box, int32_t *list_len, double *list_mass);

#ifdef __cplusplus
}
#endif

#endif /* BH_H */
