/*
 * fmmg.h -- C-ABI of the MI355X (gfx950) octree fast-multipole gravity solve.
 *
 * The operation (arXiv:1908.03121, Sec. 4.3 "The FMM hotspot"): an adaptive
 * octree whose nodes are 8x8x8 sub-grids of cells (Sec. 4.2) carries a mass
 * density in its leaf cells; the solve returns the gravitational potential and
 * acceleration of every leaf cell.  It runs the method's three steps:
 *   1. upward pass: leaf cells are point masses m = rho h^3 at their centres;
 *      refined cells get mass, centre of mass and multipole moments (orders
 *      0..3) from their children, bottom-up;
 *   2. same-level interactions: every cell interacts with the same-level
 *      cells that the opening criterion selects (the 1074-element stencil of
 *      Sec. 4.3), in the four classes refined/leaf target x refined/leaf
 *      source, producing order-3 Taylor coefficients plus the correction that
 *      conserves linear and angular momentum to round-off (Sec. 4.2);
 *   3. downward pass: each parent's expansion is re-expanded at its
 *      children's centres of mass and accumulated, top-down.
 *
 * Interaction rule (opening criterion).  Same-level cells A, B with integer
 * coordinates cA, cB, d = cB - cA, D = floor(cB/2) - floor(cA/2):
 *     evaluated at this level  <=>  (top level under FMMG_TOP_FULL  or |D|^2 <= 8)
 *                                   and (|d|^2 >= 9 or A is a leaf or B is a leaf),
 * which evaluates every ordered pair of leaf cells exactly once.
 *
 * Tree description.  A sub-grid at level l >= 0 with integer coordinates
 * s >= 0 covers origin + L0 * 2^-l * [s, s+1)^3 and holds 8^3 cells of edge
 * h = L0 / (8 * 2^l).  A sub-grid is refined iff its 8 children are listed.
 * Every sub-grid above level 0 has its parent listed; sub-grids without a
 * parent are at level 0 (a forest of level-0 sub-grids is allowed).
 * Several trees (the batched form) never interact with each other.
 *
 * Layouts.  Leaves are numbered in the order they appear in the descriptor,
 * trees concatenated.  rho, phi are [leaf][512] and g is [leaf][3][512]; the
 * 512 cells of a sub-grid are ordered (i*8 + j)*8 + k for cell (i, j, k) along
 * (x, y, z), k fastest.  All three are contiguous float64 device buffers owned
 * by the caller; the library only reads rho and only writes phi and g.
 *
 * Streams.  Every call that takes hip_stream enqueues work on that stream
 * (NULL = the null stream) and returns without waiting for it; the caller
 * synchronises.  A plan is bound to the device that is current when it is
 * created and must be used with that device current.  A plan is not
 * re-entrant: two solves on one plan must not overlap in time (use two
 * plans).  No C++ exception crosses this interface.
 *
 * Errors.  Every call returns an fmmg_status; on failure fmmg_last_error()
 * returns a thread-local text that names the cause.
 */
#ifndef FMMG_H
#define FMMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMMG_VERSION 6

typedef struct fmmg_plan fmmg_plan; /* opaque; owns device tables and workspaces */

typedef enum {
    FMMG_OK = 0,
    FMMG_EINVAL = -1,        /* bad argument: null pointer, size, option value, bad density */
    FMMG_ETREE = -2,         /* malformed tree: duplicate, missing parent, 1..7 children, ... */
    FMMG_ENOMEM = -3,        /* device or host allocation failed                             */
    FMMG_EHIP = -4,          /* a HIP runtime call failed                                    */
    FMMG_EUNSUPPORTED = -5   /* no gfx950 device, or an unsupported combination               */
} fmmg_status;

typedef enum {
    FMMG_FP64 = 0,           /* every step in FP64                                            */
    FMMG_MIXED = 1,          /* same-level Taylor-coefficient pair terms (multipole and
                                monopole) in FP32 with FP32 partial sums per source plane
                                (multipole) or column (monopole), flushed into FP64 sums;
                                the angular-momentum correction's pair terms evaluated and
                                summed in FP64; moments, passes and accumulation in FP64  */
    FMMG_MIXED_F32 = 2       /* as FMMG_MIXED, but the correction's pair terms are also
                                evaluated in FP32 with FP32 partial sums per source plane
                                (faster; its correction is FP32-accurate)                  */
} fmmg_precision;

typedef enum {
    FMMG_TOP_FULL = 0,         /* complete solve: the top level evaluates all its pairs      */
    FMMG_TOP_STENCIL_ONLY = 1  /* the top level uses the parent-near stencil like any other  */
                               /* level (kernel test of one sub-grid neighbourhood)          */
} fmmg_top_mode;

typedef struct {
    int32_t n_subgrids;       /* > 0                                                  */
    const int32_t* level;     /* host [n_subgrids], 0 <= level <= 19                  */
    const int32_t* coord;     /* host [n_subgrids][3], 0 <= coord < 2^19             */
    double origin[3];         /* corner of level-0 sub-grid (0,0,0)                   */
    double L0;                /* edge of a level-0 sub-grid, > 0                       */
} fmmg_tree_desc;

typedef struct {
    fmmg_precision precision;   /* default FMMG_FP64                                    */
    fmmg_top_mode top_mode;     /* default FMMG_TOP_FULL                                */
    double G;                   /* gravitational constant, default 1.0                  */
    int32_t angular_correction; /* 1 (default) | 0 = uncorrected result (tests only)    */
    int32_t use_graph;          /* 1 = capture the launch sequence in a hipGraph on the
                                   first solve and replay it on the solve's stream
                                   (re-captured when the rho/phi/g pointers change);
                                   0 = eager; -1 (default) = 1 for a batched plan
                                   (n_trees > 1) without timing, else 0                 */
    int32_t persistent;         /* 1 = same-level step as one persistent launch over a
                                   work list of all classes and trees; 0 = one launch
                                   per class                                            */
    int32_t timing;             /* 1 = eager solves record a hipEvent at every stage
                                   boundary on the solve's stream (fmmg_get_timings);
                                   not allowed together with use_graph                  */
    int32_t plane_groups;       /* source-plane groups per refined-target item, 1..5
                                   (the 10 source planes split into that many groups,
                                   each writing its own partial sums); 0 = 2.  Partial
                                   buffers are allocated for this many groups, or for
                                   5 when autotune is on                                */
    int32_t blocks_per_cu;      /* persistent launch: resident blocks per compute unit;
                                   0 = the occupancy limit                              */
    int32_t autotune;           /* 1 = the first solve times the candidate launch shapes
                                   (per-class or persistent, plane groups, blocks per
                                   CU, overlap, item queues) on the caller's data, each run as the
                                   plan will run it (captured and replayed when
                                   use_graph is set), keeps the fastest, and records
                                   it in tuning_cache; that solve synchronises the
                                   stream.  A cached entry for the same plan
                                   signature is used without timing.                    */
    const char* tuning_cache;   /* JSON file of tuned launch shapes, or NULL            */
    int32_t overlap;            /* 1 (default) = the coarse levels' passes and
                                   same-level items (the levels below a split level
                                   that carry at most a fifth of the estimated work)
                                   run on a second, plan-owned stream, overlapping
                                   the finer levels' same-level step; the solve still
                                   completes in order on the caller's stream.
                                   2 = as 1, and with one launch per class the fine
                                   levels' monopole class runs on a third plan-owned
                                   stream beside their multipole classes.
                                   0 = everything on the caller's stream.  Timing
                                   solves always run on one stream.  With autotune,
                                   this is the largest value tried.                     */
    int32_t launch_streams;     /* 0 (default) = the launch shapes above.  1..128 = the
                                   execution model of Sec. 5.1 of the paper, kept as a
                                   baseline for comparison: one kernel launch per target
                                   sub-grid and interaction class, issued coarse level
                                   first and round-robin over this many plan-owned
                                   streams (forked from and joined back to the solve's
                                   stream); the passes stay on the solve's stream.
                                   persistent and overlap are then ignored; timing and
                                   autotune are not allowed.  Results are bitwise equal
                                   to those of the default shapes with the same
                                   plane_groups and plane_pairs.                        */
    int32_t xcd_queues;         /* persistent launch: 1 (default) = one item queue per
                                   XCD, each a compact region of the octrees (items in
                                   space-filling-curve order, cut into runs of equal
                                   estimated cost), a block starting on its own XCD's
                                   queue and helping the others once it is drained;
                                   0 = one list, largest estimated cost first.  With
                                   autotune both are tried.  Results are bitwise equal. */
    int32_t plane_pairs;        /* refined-target work items: 1 = an item takes the two
                                   target planes of one plane of parent cells, which
                                   reach the same source planes, so each staged source
                                   plane serves both (half the staging); 0 = an item
                                   per target plane (twice the items, for workloads
                                   too small to fill the GPU otherwise); -1 (default)
                                   = 1 when the paired items number at least 8 per
                                   compute unit, else 0.  With autotune and -1 the
                                   fastest shape is also tried with the other value.
                                   Results agree to rounding (the sums' order differs). */
} fmmg_options;

/* Stages of one solve, in launch order. */
typedef enum {
    FMMG_STAGE_P2M = 0,         /* leaf cell masses                                     */
    FMMG_STAGE_M2M = 1,         /* upward pass, all levels                              */
    FMMG_STAGE_TOP = 2,         /* top level under the all-pairs rule; its reduction    */
    FMMG_STAGE_MONO = 3,        /* leaf targets, leaf sources (class 3)                 */
    FMMG_STAGE_MP_REFINED = 4,  /* refined targets (classes 1 and 2)                    */
    FMMG_STAGE_MP_LEAF = 5,     /* leaf targets, refined sources (class 4)              */
    FMMG_STAGE_FUSED = 6,       /* the persistent launch of all same-level classes      */
    FMMG_STAGE_DOWN = 7,        /* downward pass and leaf output                        */
    FMMG_N_STAGES = 8
} fmmg_stage;

typedef struct {
    double ms[FMMG_N_STAGES];   /* summed stage durations (milliseconds)                */
    int64_t launches[FMMG_N_STAGES]; /* kernel launches per stage and solve             */
    int64_t solves;             /* number of solves summed                              */
} fmmg_timings;

/* Launch shape in use (after tuning, if any). */
typedef struct {
    int32_t persistent;
    int32_t plane_groups;
    int32_t blocks_per_cu;
    int32_t from_cache;         /* 1 if the shape came from the tuning cache           */
    double tuned_ms;            /* best solve time measured by the tuner, or 0         */
    int32_t overlap;            /* 1 if the coarse levels run on the second stream, 2 if
                                   also the fine monopole class runs on a third one      */
    int32_t split_level;        /* levels below this one form the coarse branch        */
    int32_t launch_streams;     /* streams of the per-sub-grid launch model, or 0      */
    int32_t use_graph;          /* 1 if solves are captured and replayed as a hipGraph */
    int32_t xcd_queues;         /* persistent launch: 1 = one item queue per XCD        */
    int32_t plane_pairs;        /* 1 if a refined-target item takes two target planes  */
} fmmg_launch_shape;

typedef struct {
    int64_t pairs[4];      /* ordered cell pairs per class: [0] refined<-leaf,
                              [1] refined<-refined, [2] leaf<-leaf, [3] leaf<-refined   */
    int64_t pairs_top;     /* pairs evaluated at the top level under FMMG_TOP_FULL       */
    int64_t launches;      /* kernel launches enqueued by the last solve                 */
    int64_t solves;        /* solves enqueued on this plan                               */
    double paper_flops;    /* pairs weighted 12 (leaf<-leaf) or 455 (all others) flop,
                              the per-interaction counts of Sec. 4.3                     */
    int64_t n_leaves;
    int64_t n_refined;
    int32_t max_level;
    int32_t n_trees;
    int32_t sweep_y_targets;  /* refined targets whose plane items run along y     */
    int32_t sweep_x_targets;  /* refined targets whose plane items run along x     */
} fmmg_stats;

/* Fills *opt with the defaults listed above (interface convention; no
 * passage of the paper). */
void fmmg_default_options(fmmg_options* opt);

/* Plans the solve of the given octrees (arXiv:1908.03121 Sec. 4.2: an
 * adaptive octree whose nodes are 8x8x8 sub-grids; Sec. 4.3: the opening
 * criterion and its 1074-element stencil, the four interaction classes of
 * refined/leaf targets and sources).  Validates the trees, builds the
 * neighbour/parent/child tables, the stencil tables and the work lists on the
 * host, uploads them, and allocates the device workspaces on the current
 * device.
 * trees: host array [n_trees], n_trees >= 1 (n_trees > 1 is the batched form);
 * read during the call only.  opt may be NULL (defaults).  hip_stream: stream
 * for the table uploads (the call synchronises it).
 * Errors: FMMG_EINVAL for a bad option, FMMG_ETREE for a malformed tree,
 * FMMG_ENOMEM, FMMG_EHIP, FMMG_EUNSUPPORTED if the current device is not
 * gfx950.  On success *out owns everything it allocated (fmmg_plan_destroy);
 * on failure *out is NULL and nothing is kept. */
fmmg_status fmmg_plan_create(fmmg_plan** out, const fmmg_tree_desc* trees, int32_t n_trees,
                             const fmmg_options* opt, void* hip_stream);

/* Number of leaf sub-grids, the leading dimension of rho, phi and g
 * (interface convention). */
fmmg_status fmmg_plan_n_leaves(const fmmg_plan* plan, int64_t* n_leaves);

/* leaf_desc_index: host [n_leaves], caller-owned; entry i = descriptor index of
 * leaf i within its own tree's descriptor (interface convention). */
fmmg_status fmmg_leaf_order(const fmmg_plan* plan, int32_t* leaf_desc_index);

/* The solve (arXiv:1908.03121 Sec. 4.3, its three steps: leaf masses and the
 * upward pass of multipole moments, the same-level stencil interactions of the
 * four classes producing Taylor coefficients, the downward pass; Sec. 4.2 and
 * 4.3: the correction that conserves linear and angular momentum), on
 * hip_stream.
 * rho: device float64 [n_leaves][512], caller-owned, read only; finite and >= 0.
 * phi: device float64 [n_leaves][512]; g: device float64 [n_leaves][3][512];
 *      caller-owned, written.
 * The three buffers must not overlap (FMMG_EINVAL).
 * Asynchronous: returns once the work is enqueued.  The upward pass checks
 * every density it reads; a negative or non-finite one is recorded on the
 * device, without synchronising, and reported as FMMG_EINVAL (naming its flat
 * index, nothing enqueued) by the first fmmg_solve on
 * this plan that starts after that solve has completed, or by
 * fmmg_density_status.  That solve's phi and g are then meaningless. */
fmmg_status fmmg_solve(fmmg_plan* plan, const double* rho, double* phi, double* g,
                       void* hip_stream);

/* Reports a negative or non-finite density read by a completed solve on this
 * plan (the solve's input is cell densities, Sec. 4.3): FMMG_OK with
 * *bad_index = -1, or FMMG_EINVAL with *bad_index = the smallest such flat
 * index into rho of that solve.  Host-only, no device call: synchronise the
 * solves' stream first to cover every enqueued solve.  A report is given once
 * (this call or the next solve takes it). */
fmmg_status fmmg_density_status(fmmg_plan* plan, int64_t* bad_index);

/* Checks on the device that every density is finite and >= 0 (the solve's
 * input, Sec. 4.3); synchronises hip_stream.  Returns FMMG_OK or FMMG_EINVAL
 * (with the first bad index in the error text). */
fmmg_status fmmg_check_density(fmmg_plan* plan, const double* rho, void* hip_stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The check
 * of fmmg_check_density without a plan: records, on hip_stream, in the
 * caller's device word *bad_index the smallest flat index i < n with rho[i]
 * negative or not finite, or -1.  Allocates nothing, does not synchronise and
 * copies nothing to the host (read *bad_index after the stream has reached
 * it).  Its partial results live in a static device array of the library
 * (512 KiB per GPU, held until the process ends) shared by every call on that
 * GPU: calls that overlap in time on one GPU race and must be serialised by
 * the caller.
 * rho: device float64 [n], caller-owned, read only (may be NULL when n = 0).
 * bad_index: device int64 [1], caller-owned, written.
 * Errors: FMMG_EINVAL for n < 0, n > FMMG_NOALLOC_MAX_DENSITIES or a null
 * pointer (nothing enqueued); FMMG_EHIP if a HIP call fails. */
#define FMMG_NOALLOC_MAX_DENSITIES ((int64_t)65536 * 4096)
fmmg_status fmmg_check_density_noalloc(const double* rho, int64_t n, int64_t* bad_index,
                                       void* hip_stream);

/* Sums the stage durations of the solves enqueued with options.timing = 1
 * since the previous call (or plan creation), then starts a new sum.  The
 * caller must have synchronised the solves' stream.  FMMG_EINVAL if the plan
 * was created without timing.  (Measurement; no passage of the paper.) */
fmmg_status fmmg_get_timings(fmmg_plan* plan, fmmg_timings* out);

/* The launch shape the plan uses (launch_streams: the execution model of
 * Sec. 5.1; the other fields are this library's own shapes). */
fmmg_status fmmg_get_launch_shape(const fmmg_plan* plan, fmmg_launch_shape* out);

/* Pair counts and launch counters of the plan (host values; no device work).
 * paper_flops weights the pairs with the per-interaction flop counts of
 * Sec. 4.3 (12 for leaf-leaf, 455 otherwise). */
fmmg_status fmmg_get_stats(const fmmg_plan* plan, fmmg_stats* stats);

/* Releases every device and host resource of the plan; NULL is a no-op.
 * The caller must make sure no solve on the plan is still running. */
void fmmg_plan_destroy(fmmg_plan* plan);

/* Thread-local text for the last non-OK status returned on this thread. */
const char* fmmg_last_error(void);

/* Host-only: validates the trees and counts the ordered pairs per class that
 * a solve with this top_mode evaluates under the interaction rule of Sec. 4.3
 * (no device is touched).  stats->pairs, pairs_top, paper_flops, n_leaves,
 * n_refined, max_level, n_trees, sweep_y_targets and sweep_x_targets are filled; the launch
 * counters are zero. */
fmmg_status fmmg_count_pairs(const fmmg_tree_desc* trees, int32_t n_trees,
                             fmmg_top_mode top_mode, fmmg_stats* stats);

/* Version of this interface (FMMG_VERSION). */
int32_t fmmg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FMMG_H */
