/*
 * lfmm.h -- C ABI of the lattice fast multipole library for MI355X (gfx950).
 *
 * The library evaluates the lattice convolution (eq. 1.7 of Gillman & Martinsson, "A fast
 * solver for Poisson problems on infinite regular lattices")
 *
 *     u(m) = sum over sources n of phi(m - n) f(n),      m, n in Z^2,
 *
 * where phi is the fundamental solution of the 5-point discrete Laplacian (eq. 1.2, eq. 1.8),
 * at the source points themselves (the paper's default, Section 8.1) or at targets of the
 * caller's choosing (the problem statement of Section 1: loads at sources, potentials wanted
 * at finitely many targets).  The fast method is the lattice FMM of Sections 4-8: a quadtree on the sources
 * (Section 6), outgoing/incoming skeleton expansions built by interpolative decomposition
 * (Sections 4.3, 5, 7), the five translation operators (Section 7) and the upward,
 * interaction and downward passes (Section 8.2), with the near field summed against a
 * tabulated phi (Sections 2, 3).
 *
 * Conventions (all calls):
 *  - Every call returns an lfmm_status; nothing throws across the ABI.  On an error the
 *    calling thread's lfmm_last_error() holds a human-readable detail string.
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA tensors on ROCm);
 *    pointers named *_host are host pointers.  The caller owns every buffer it passes; the
 *    library owns the internals of lfmm_ctx, lfmm_plan and lfmm_opset and frees them on
 *    destroy.
 *  - Coordinates are int32 pairs (m1, m2), row i = point i, so xy has 2*n entries.  Loads
 *    f and potentials u are float64.  The extent of the coordinates along either axis must
 *    be below 2^31 (else LFMM_E_RANGE).  Duplicate points are allowed (loads superpose) and
 *    a target on a source gets no self term, since phi(0) = 0.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it in
 *    order; calls that must read sizes back (plan creation) synchronise the stream.
 *  - The well-posedness condition of Section 1 is a zero total load.  The library returns
 *    the finite sum for any loads; a non-zero sum is not an error.  Calls that check the
 *    loads (lfmm_solve always, lfmm_execute* with LFMM_FLAG_CHECK_LOADS) return the warning
 *    LFMM_W_NONZERO_SUM (> 0: the result is computed) when |sum f| > 1e-12 sum |f|, and
 *    LFMM_E_INVAL before any pass is launched when a load is NaN or infinite.
 *  - One host thread per context at a time.  Plans of one context are independent.
 *    Plans draw their device memory from the context's pool: lfmm_ctx_destroy destroys the
 *    servers and plans still alive on the context, whose handles then become invalid.
 */
#ifndef LFMM_H
#define LFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lfmm_status {
    LFMM_OK = 0,
    LFMM_W_NONZERO_SUM = 1,   /* warning: the loads do not sum to zero (|sum f| > 1e-12 sum |f|);
                                 the potentials are computed all the same                 */
    LFMM_E_INVAL = -1,        /* null pointer, bad size, bad option value, NaN/Inf load  */
    LFMM_E_RANGE = -2,        /* coordinate extent >= 2^31, or a size the plan cannot hold */
    LFMM_E_NOMEM = -3,        /* device or host allocation failed (tests can force one:
                                 LFMM_TEST_FAIL_ALLOC=k in the environment fails the k-th
                                 device block requested after it is set)                   */
    LFMM_E_HIP = -4,          /* a HIP runtime call failed; the plan is unusable          */
    LFMM_E_UNSUPPORTED = -5,  /* valid request this build does not implement              */
    LFMM_E_NODEVICE = -6,     /* no GPU visible, or the device id does not exist          */
    LFMM_E_BUSY = -7          /* a wait timed out before the request was done             */
} lfmm_status;

typedef enum lfmm_precision {
    LFMM_FP64 = 0,            /* every step in FP64                                        */
    LFMM_MIXED = 1,           /* M2L as FP32 matrix-core products with hi/lo splitting,
                                 accumulated in FP64; everything else FP64                 */
    LFMM_MIXED_BF16 = 2       /* M2L as bf16 matrix-core products: the operator (less its
                                 constant part, applied in FP64) and q-hat each split into
                                 three bf16 parts, the six products of parts whose orders
                                 sum to at most 2, FP32 sums added to FP64 accumulators
                                 once per interaction; everything else FP64.  Same error
                                 target as LFMM_MIXED (relative 1e-7)                       */
} lfmm_precision;

typedef struct lfmm_options {
    double eps;               /* ID tolerance relative to the first pivot (Section 4:
                                 requested precision); default 1e-12                       */
    int32_t max_leaf;         /* N_leaf of Section 6: most points a leaf may hold before the
                                 tree is refined; default 64; 0 = automatic: the value
                                 lfmm_autotune found for point sets of similar size and
                                 density, else 64                                          */
    int32_t precision;        /* lfmm_precision of the interaction (M2L) pass              */
    int32_t proxy_per_edge;   /* proxy points per edge of the proxy ring once the full ring
                                 is larger (Remark 5.1); default 64                        */
    int32_t max_rank;         /* cap on the skeleton size P, 16..64, multiple of 16;
                                 default 48                                                */
    int32_t flags;            /* LFMM_FLAG_* bits, default 0                               */
    int32_t stencil;          /* lattice operator A whose fundamental solution phi is used
                                 (lfmm_stencil); default LFMM_STENCIL_5                    */
} lfmm_options;

/* The lattice operator of a context (A phi = delta).  The method needs only phi (Sections 1,
 * 3.1: it carries over to other constant-coefficient difference operators). */
typedef enum lfmm_stencil {
    LFMM_STENCIL_5 = 0,       /* 4 u(m) - sum of the 4 neighbours, eq. (1.2)               */
    LFMM_STENCIL_9 = 1        /* isotropic 9-point: (20 u(m) - 4 (4 neighbours) - (4 diagonal
                                 neighbours)) / 6; phi by the same reduced integral, its far
                                 field by an expansion of the form of eq. (3.1) fitted to the
                                 tabulated values                                         */
} lfmm_stencil;

/* options.flags: lfmm_execute / lfmm_execute_instances replay a HIP graph of the evaluation
 * passes, recorded at the plan's first execute (one graph launch per execute instead of one
 * launch per pass and height).  Per-phase timing is not available in this mode. */
#define LFMM_FLAG_GRAPH 1
/* options.flags: lfmm_execute / lfmm_execute_instances check the loads first (a reduction on
 * the device and a read-back, so the call synchronises the stream): NaN or infinite loads
 * give LFMM_E_INVAL with nothing launched, a non-zero total load LFMM_W_NONZERO_SUM. */
#define LFMM_FLAG_CHECK_LOADS 2
/* options.flags: plans use the adaptive tree of Section 6 (closing paragraph): a box is
 * refined while it holds more than max_leaf points, so leaves sit at different levels and
 * the far field goes through the lists of Carrier, Greengard and Rokhlin: V (interaction
 * lists, M2L), W (multipole expansions of small boxes evaluated at a leaf's points), X (a
 * large leaf's sources evaluated into a small box's incoming expansion) and U (adjacent
 * leaves, summed directly).  Outgoing and incoming expansions of a leaf above the finest
 * level are those of its descendants moved up by T_ofo and down by T_ofo^T, which composes
 * the leaf's own T_ofs and T_tfi.  Suited to strongly non-uniform point sets.  Not with
 * lfmm_solve_static or a server (LFMM_E_UNSUPPORTED). */
#define LFMM_FLAG_ADAPTIVE 4

typedef struct lfmm_ctx lfmm_ctx;     /* device, phi table, per-leaf-side operator cache  */
typedef struct lfmm_plan lfmm_plan;   /* one or more point sets (instances): sorted points,
                                         trees, lists and expansion storage, resident until
                                         destroyed                                          */
typedef struct lfmm_opset lfmm_opset; /* host copy of the operators for one leaf side     */

typedef struct lfmm_plan_info {
    int64_t n_points;         /* over all instances                                        */
    int32_t n_instances;
    int32_t root_bits;        /* instance 0: root box side is 2^root_bits                  */
    int32_t leaf_level;       /* instance 0: L, leaves are the boxes of level L (Section 6) */
    int64_t leaf_side;        /* instance 0: lattice side of a leaf, 2^(root_bits - L)     */
    int32_t rank;             /* padded skeleton size P used by the kernels                */
    int32_t leaf_kind;        /* 0: dense-model outgoing operator (Remark 8.2)             */
    int64_t n_boxes;          /* non-empty boxes over all levels and instances             */
    int64_t n_leaves;         /* non-empty leaves over all instances                       */
    int64_t near_pairs;       /* (target, source) pairs summed directly (Section 2)        */
    int64_t m2l_pairs;        /* (box, interaction-list box) pairs (Section 8.2, step 3)   */
    int64_t device_bytes;     /* device memory the plan holds between executes             */
    int64_t n_targets;        /* potentials one execute writes, over all instances         */
    int32_t adaptive;         /* 1: adaptive tree (LFMM_FLAG_ADAPTIVE); n_leaves, near_pairs
                                 and m2l_pairs then count its leaves, U and V lists        */
    int32_t pad0;
    int64_t m2p_terms;        /* adaptive: sum over leaves of targets x W-list skeleton
                                 points (multipole evaluations at targets)                 */
    int64_t p2l_terms;        /* adaptive: sum over boxes of skeleton points x X-list
                                 sources (sources evaluated into incoming expansions)      */
} lfmm_plan_info;

/* Fills *opt with the defaults listed above. */
lfmm_status lfmm_options_init(lfmm_options* opt);

/* Creates a context on HIP device `device` (Section 8.1 precompute that does not depend on
 * the points: the phi table of Section 3 is built on the host and uploaded; operators are
 * built per leaf side on first use and cached).  opt may be NULL for the defaults.
 * LFMM_E_NODEVICE if the device does not exist. */
lfmm_status lfmm_ctx_create(int32_t device, const lfmm_options* opt, lfmm_ctx** out);
lfmm_status lfmm_ctx_destroy(lfmm_ctx* ctx);

/* Builds the tree of Section 6 (Morton keys, sort, levels, parent/child, neighbor and
 * interaction lists of Definition 6.1) and the operators for its leaf side if the context
 * lacks them, for the n_src sources src_xy_dev[2 n_src] (device, int32) and:
 *  - tgt_xy_dev == NULL: targets = sources (Section 8.1); n_tgt must be 0 or n_src;
 *  - else the n_tgt targets tgt_xy_dev[2 n_tgt] (device, int32), 1 <= n_tgt: the potentials
 *    are wanted there (Section 1).  The tree is built over the union of sources and targets
 *    (a target carries no load), so a box holding targets gets its incoming expansion and its
 *    near field like any other; targets may coincide with sources or with each other.
 * The coordinates are copied; the buffers may be freed afterwards.  1 <= n_src and
 * n_src + n_tgt <= 2^30.  The leaf level is the smallest at which no leaf holds more than
 * max_leaf points, raised where needed so that a leaf is at most 128 cells wide (the
 * dense-model outgoing operator of Remark 8.2 is tabulated up to that side). */
lfmm_status lfmm_plan_create(lfmm_ctx* ctx, int64_t n_src, const int32_t* src_xy_dev, int64_t n_tgt,
                             const int32_t* tgt_xy_dev, void* stream, lfmm_plan** out);

/* Builds one plan over n_inst independent problems (instances): instance k has
 * n_src_host[k] >= 1 sources at src_xy_dev[k][2 n_src_host[k]] (device, int32) and, if
 * tgt_xy_dev is not NULL and tgt_xy_dev[k] is not NULL, n_tgt_host[k] targets of its own at
 * tgt_xy_dev[k] (else its targets are its sources).  The count and pointer arrays are host
 * memory; n_tgt_host and tgt_xy_dev may be NULL together.  Each instance gets its own root
 * box and tree, exactly as lfmm_plan_create would build it alone, so its potentials equal the
 * ones of a plan of its own bit for bit; all instances share every construction and
 * evaluation launch.  At most 2^30 points in total; LFMM_E_RANGE if the instance count and
 * coordinate extents do not fit the 64-bit sort key (2 * root bits + bits of n_inst - 1 <=
 * 64). */
lfmm_status lfmm_plan_create_batch(lfmm_ctx* ctx, int32_t n_inst, const int64_t* n_src_host,
                                   const int32_t* const* src_xy_dev, const int64_t* n_tgt_host,
                                   const int32_t* const* tgt_xy_dev, void* stream, lfmm_plan** out);

/* Evaluates u_dev[i] = sum_j phi(t_i - s_j) f_dev[j] for the plan's targets t_i and sources
 * s_j (eq. 1.7) by the passes of Section 8.2: P2M (T_ofs), M2M (T_ofo), M2L (T_ifo), L2L
 * (T_ifi = T_ofo^T), L2P (T_tfi = T_ofs^T) and the direct near field.  f_dev (n_src) and
 * u_dev (n_tgt, or n_src when targets = sources) are device float64 arrays in the caller's
 * order.  Enqueued on `stream`; no sync (unless LFMM_FLAG_CHECK_LOADS).  Executes of one
 * plan share its expansion storage: the caller orders them (one stream, or events), and
 * an execute on another stream than the plan was built on waits for the build. */
lfmm_status lfmm_execute(lfmm_plan* plan, const double* f_dev, double* u_dev, void* stream);

/* lfmm_execute with loads and potentials in the plan's own point order, for callers that keep
 * their vectors in that order across many executes of one plan (iterative solvers, repeated
 * right-hand sides): P2M then reads the loads, and the near field writes the potentials, as
 * contiguous runs instead of one scattered word per point.  Index s runs over every point of
 * the plan (n_points of lfmm_plan_get_info: sources and separate targets of all instances,
 * concatenated in instance order, Morton-ordered inside each; LFMM_EXPORT_PERM gives the
 * caller index perm[s] of each).  f_sorted_dev[s] is the load of point s where perm[s] is a
 * source index (perm[s] < n_src of its instance); other entries are not read.  u_sorted_dev[s]
 * receives the potential of point s where it is a target (with separate targets, perm[s] >=
 * n_src: target perm[s] - n_src); other entries are not written.  Same arithmetic as
 * lfmm_execute, so u_sorted_dev[s] equals u_dev[perm[s]] of the same loads bit for bit.
 * Device float64 arrays of n_points entries; enqueued on `stream`, no sync (with
 * LFMM_FLAG_CHECK_LOADS all n_points loads are checked).  Works for every plan, including
 * several instances, adaptive trees and graph replays. */
lfmm_status lfmm_execute_sorted(lfmm_plan* plan, const double* f_sorted_dev, double* u_sorted_dev, void* stream);

/* lfmm_execute for a plan of several instances: f_dev[k] and u_dev[k] (device arrays of
 * n_host[k] float64, in instance k's caller order) belong to instance k; the pointer arrays
 * are host memory read during the call.  One launch per pass covers every instance. */
lfmm_status lfmm_execute_instances(lfmm_plan* plan, const double* const* f_dev,
                                   double* const* u_dev, void* stream);

/* Runs lfmm_execute on each single-instance plan of one context, in order, on one stream
 * (separate launches per plan; build one plan with lfmm_plan_create_batch to share them). */
lfmm_status lfmm_execute_batch(lfmm_ctx* ctx, int32_t n_plans, lfmm_plan* const* plans,
                               const double* const* f_dev, double* const* u_dev, void* stream);

lfmm_status lfmm_plan_get_info(lfmm_plan* plan, lfmm_plan_info* out);

/* Autotuner of N_leaf (Section 6), which sets the leaf size and with it the balance between
 * the near field (pairs grow with N_leaf) and the matrix passes (boxes shrink with it):
 * builds the plan of the n points xy_dev[2n] with each of the n_cand candidates cand_host[]
 * (each in [1, 4096]), evaluates it `reps` times with zero loads, and stores in *best_host
 * the candidate with the least time per solve (objective 0: plan build plus one execute) or
 * per execute (objective 1: the plan is reused).  ms_host[n_cand] (optional) receives each
 * candidate's time.  The context remembers the choice for point sets of the same size and
 * density class (log2 of n and of n / root-box area, rounded) and uses it for later plans
 * when options.max_leaf is 0.  Synchronises the stream. */
lfmm_status lfmm_autotune(lfmm_ctx* ctx, int64_t n, const int32_t* xy_dev, int32_t n_cand,
                          const int32_t* cand_host, int32_t objective, int32_t reps, void* stream,
                          int32_t* best_host, double* ms_host);

/* lfmm_autotune for a plan of several instances (lfmm_plan_create_batch): every candidate is
 * applied to all n_inst instances at once (n_host[k] points at xy_dev[k], host arrays of
 * device pointers) and the whole plan is timed, so the choice accounts for the launches the
 * instances share (instances of mixed N_leaf split them into more, smaller groups).  The
 * fastest candidate is recorded for the size and density class of every instance, where a
 * context in automatic mode (max_leaf 0) finds it when it builds such instances again. */
lfmm_status lfmm_autotune_batch(lfmm_ctx* ctx, int32_t n_inst, const int64_t* n_host,
                                const int32_t* const* xy_dev, int32_t n_cand, const int32_t* cand_host,
                                int32_t objective, int32_t reps, void* stream, int32_t* best_host,
                                double* ms_host);

/* Phases of lfmm_execute, in launch order, for lfmm_plan_phase_times. */
typedef enum lfmm_phase {
    LFMM_PHASE_GATHER = 0,    /* loads into Morton order (empty: P2M gathers them)         */
    LFMM_PHASE_P2M = 1,       /* T_ofs, Section 8.2 step 1                                 */
    LFMM_PHASE_M2M = 2,       /* T_ofo, step 2                                             */
    LFMM_PHASE_M2L = 3,       /* T_ifo, step 3                                             */
    LFMM_PHASE_L2L = 4,       /* T_ifi, step 4                                             */
    LFMM_PHASE_LEAF = 5,      /* T_tfi + near field + caller order, step 5                 */
    LFMM_NUM_PHASES = 6
} lfmm_phase;

/* Turns per-phase timing of later lfmm_execute calls on or off (HIP events recorded on
 * the execute stream around each phase; off by default). */
lfmm_status lfmm_plan_set_timing(lfmm_plan* plan, int32_t enable);

/* Times only the phases in phase_mask (bit k = lfmm_phase k; 0 turns timing off): later
 * lfmm_execute calls record just the events that bound those phases, each event costing a
 * few microseconds of device time.  LFMM_E_INVAL for bits above the last phase. */
lfmm_status lfmm_plan_set_timing_phases(lfmm_plan* plan, uint32_t phase_mask);

/* Milliseconds spent in each phase by the most recent timed lfmm_execute of this plan,
 * ms_host[LFMM_NUM_PHASES] (NaN for phases that execute did not time); waits for that
 * execute to finish.  LFMM_E_INVAL before any timed execute. */
lfmm_status lfmm_plan_phase_times(lfmm_plan* plan, double* ms_host);

/* Plan internals that lfmm_plan_export copies to the host, for inspection and tests.
 * Points of all instances are concatenated in instance order, Morton-ordered inside each
 * instance.  Boxes are numbered by height above their instance's leaf level (all leaves
 * first), then by instance, then by Morton key. */
typedef enum lfmm_export_item {
    LFMM_EXPORT_POINTS = 0,     /* int32 [n][2]: points in Morton order, shifted so that the
                                   instance's root box is [0, 2^root_bits)^2                 */
    LFMM_EXPORT_PERM = 1,       /* int32 [n]: index of each Morton-ordered point in its
                                   instance's caller order                                   */
    LFMM_EXPORT_LEVEL_BASE = 2, /* int32 [L+1], instance 0: boxes of level l are
                                   [base[l], base[l] + count[l])                             */
    LFMM_EXPORT_BOX_KEY = 3,    /* uint64 [n_boxes]: Morton key of the box at its level      */
    LFMM_EXPORT_BOX_BEGIN = 4,  /* int32 [n_boxes]: first Morton-ordered point of the box    */
    LFMM_EXPORT_BOX_END = 5,    /* int32 [n_boxes]: one past its last point                  */
    LFMM_EXPORT_BOX_PARENT = 6, /* int32 [n_boxes]: parent box, -1 for a root                */
    LFMM_EXPORT_BOX_CHILD = 7,  /* int32 [n_boxes][4]: child c = x bit + 2 y bit, or -1      */
    LFMM_EXPORT_INTERACTION = 8,/* int32 [n_boxes][27]: interaction list slots, in the order
                                   dy = -3..3 outer, dx = -3..3 inner over the 7x7 block of
                                   the parent's neighbours minus the 3x3 block around the
                                   box; -1 = empty slot or level < 2                         */
    LFMM_EXPORT_NEIGHBOR = 9,   /* int32 [n_boxes][9]: 3x3 neighbourhood, dy outer, dx inner */
    LFMM_EXPORT_QHAT = 10,      /* float64 [n_boxes][48]: outgoing expansions (last execute) */
    LFMM_EXPORT_UHAT = 11,      /* float64 [n_boxes][48]: incoming expansions (last execute) */
    LFMM_EXPORT_LOADS = 12,     /* float64 [n]: loads of the last execute in Morton order   */
    LFMM_EXPORT_LEVEL_COUNT = 13, /* int32 [L+1], instance 0: boxes of level l              */
    LFMM_EXPORT_BOX_LEVEL = 14, /* int8 [n_boxes]: level of the box in its instance's tree   */
    LFMM_EXPORT_BOX_INSTANCE = 15, /* int32 [n_boxes]: instance of the box                   */
    LFMM_EXPORT_BOX_ROLE = 16,  /* int8 [n_boxes]: 0 below an adaptive leaf, 1 refined box,
                                   2 leaf (uniform plans: the level-L boxes are the leaves)  */
    LFMM_EXPORT_LIST_U = 17,    /* int32, adaptive plans: [n_boxes + 1] row starts, then the
                                   entries (box indices); row of a leaf: its U list          */
    LFMM_EXPORT_LIST_W = 18,    /* int32, adaptive plans: the same for the W lists           */
    LFMM_EXPORT_LIST_X = 19     /* int32, adaptive plans: the same for the X lists (rows of
                                   every box of the adaptive tree)                          */
} lfmm_export_item;

/* Copies plan item `item` into host_out.  With host_out NULL, stores the byte size in *bytes;
 * otherwise *bytes must hold at least that size.  Waits for the device. */
lfmm_status lfmm_plan_export(lfmm_plan* plan, int32_t item, void* host_out, size_t* bytes);

/* Bound on the device bytes a single-instance plan of n_src sources and n_tgt separate targets
 * (0: targets = sources) holds while it is built (tree, lists, expansions, construction
 * temporaries, each counted at the pool block that serves it), given the bits of its root
 * box, root_bits = ceil(log2(coordinate extent)) in [0, 31], or -1 if unknown (the bound for
 * any extent below 2^31).  Level l of a tree holds at most min(4^l, n) boxes, so the bound
 * grows with root_bits for sparse point sets.  Used for admission by memory footprint; the
 * bytes a built plan holds are lfmm_plan_info.device_bytes.  Uniform trees only:
 * LFMM_E_UNSUPPORTED for a context with LFMM_FLAG_ADAPTIVE (its list lengths depend on how
 * the points cluster). */
lfmm_status lfmm_plan_footprint_bytes(const lfmm_ctx* ctx, int64_t n_src, int64_t n_tgt, int32_t root_bits,
                                      size_t* out);

/* Frees a plan.  When every execute of the plan ran on the stream it was built on (and it
 * does not replay a HIP graph), this returns without waiting: the plan's device memory goes
 * back to the context's pool once that stream has passed this call, and results written by
 * earlier executes are ordered on that stream as usual.  Otherwise it waits for the device. */
lfmm_status lfmm_plan_destroy(lfmm_plan* plan);

/* One-shot: plan, execute, destroy, for targets = sources.  Checks the loads first (see
 * LFMM_FLAG_CHECK_LOADS: LFMM_E_INVAL for NaN/Inf loads, LFMM_W_NONZERO_SUM for a non-zero
 * total, with u_dev written).  Synchronises the stream before returning. */
lfmm_status lfmm_solve(lfmm_ctx* ctx, int64_t n, const int32_t* xy_dev, const double* f_dev,
                       double* u_dev, void* stream);

/* lfmm_solve for callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same solve (targets = sources, loads
 * checked as by lfmm_solve, stream synchronised before return), with every device buffer the
 * tree, the expansions and the construction need taken from the library's static workspace,
 * a 64 MiB device array per GPU held until the process ends.  It calls no hipMalloc, hipFree,
 * pinned-memory or other allocating routine.  Limits: 1 <= n <= 65536 (else LFMM_E_RANGE),
 * and the point set's tree must fit the workspace (sparse sets make deep trees; else
 * LFMM_E_RANGE, nothing computed).  The operators for the point set's leaf side must be in
 * the context already (an earlier plan or solve of a point set with that leaf side and depth
 * builds them); else LFMM_E_UNSUPPORTED.  Calls on one device share its workspace: the
 * library makes them take turns; the caller must not overlap them with its own use of the
 * results of an earlier call, which the next call overwrites only in the workspace. */
lfmm_status lfmm_solve_static(lfmm_ctx* ctx, int64_t n, const int32_t* xy_dev, const double* f_dev,
                              double* u_dev, void* stream);

/* Direct O(n_t n_s) sum on the GPU, u_dev[t] = sum_s phi(txy_t - sxy_s) f_dev[s] (eq. 1.7),
 * with phi from the table (|m|_inf <= 128) or the expansion eq. (3.1).  For small inputs and
 * for checking. */
lfmm_status lfmm_direct(lfmm_ctx* ctx, int64_t n_t, const int32_t* txy_dev, int64_t n_s,
                        const int32_t* sxy_dev, const double* f_dev, double* u_dev, void* stream);

const char* lfmm_status_string(lfmm_status s);
const char* lfmm_last_error(void);

/* ---- serving: continuous batching of solve requests on one context ------------------- */

/* A server owns a worker thread that drives its context (the caller must not use that
 * context while the server lives).  Requests are admitted in arrival order, as many per
 * scheduling iteration as the limits below allow; each iteration builds one forest plan over
 * its admitted requests (lfmm_plan_create_batch) and evaluates it, on one of max_inflight
 * streams, so that the tree construction of a new iteration overlaps on the device with
 * the evaluation of earlier ones.  A request's potentials equal, bit for bit, those of
 * lfmm_solve on the same input alone, whatever it was batched with.  Plans stay resident
 * until their evaluation has completed, then their memory returns to the context's pool. */
typedef struct lfmm_server lfmm_server;

typedef struct lfmm_server_options {
    size_t hbm_budget_bytes;  /* bound on lfmm_plan_footprint_bytes (with each request's own
                                 root bits, measured on the device before admission) summed
                                 over the requests on the device; 0 = half of the device's
                                 free memory                                              */
    int32_t max_batch;        /* most requests admitted in one iteration; 0 = 256          */
    int32_t max_inflight;     /* iterations on the device at once (one stream each); 0 = 3 */
    int64_t max_batch_points; /* most points admitted in one iteration; 0 = 2^24           */
} lfmm_server_options;

typedef struct lfmm_request_stats {
    int32_t status;           /* lfmm_status of the request                                */
    int32_t batch_size;       /* requests in the iteration that served it                  */
    int64_t batch_id;         /* scheduling iteration, counted from 0                      */
    double t_submit;          /* seconds since server creation: submit call                */
    double t_admit;           /* admitted into an iteration                                */
    double t_done;            /* its evaluation was seen complete on the device            */
} lfmm_request_stats;

/* Starts a server on ctx (opt may be NULL for the defaults). */
lfmm_status lfmm_server_create(lfmm_ctx* ctx, const lfmm_server_options* opt, lfmm_server** out);

/* Queues a solve of n points: xy_dev[2n] int32, f_dev[n] and u_dev[n] float64, all device
 * memory that the caller keeps valid and untouched until lfmm_server_wait reports the
 * request done.  producer_stream is the stream on which the caller wrote xy_dev and f_dev
 * (NULL = the default stream): submit records an event there and the server reads the
 * buffers only after it.  Thread-safe.  *ticket identifies the request.  A request whose
 * footprint alone exceeds the memory budget finishes with LFMM_E_NOMEM. */
lfmm_status lfmm_server_submit(lfmm_server* srv, int64_t n, const int32_t* xy_dev,
                               const double* f_dev, double* u_dev, void* producer_stream,
                               uint64_t* ticket);

/* Waits up to timeout_s seconds (< 0: without limit) for request `ticket`; fills *out when
 * it is done and forgets the ticket.  LFMM_E_BUSY if it is not done in time.  Returns the
 * request's own status otherwise.  Thread-safe. */
lfmm_status lfmm_server_wait(lfmm_server* srv, uint64_t ticket, double timeout_s,
                             lfmm_request_stats* out);

/* Finishes every queued request, stops the worker and frees the server. */
lfmm_status lfmm_server_destroy(lfmm_server* srv);

/* ---- Section 10: iterative solves with the lattice convolution as the fast operator ---- */

/* Restarted GMRES (classical Gram-Schmidt run twice) on device vectors; the operator is applied
 * through resident plans.  tol: relative residual |b - A x| / |b| (default 1e-12); max_iter:
 * default 500; restart: Krylov dimension per cycle (default 50, at most 512).  Fields <= 0
 * take the defaults. */
typedef struct lfmm_solver_options {
    double tol;
    int32_t max_iter;
    int32_t restart;
} lfmm_solver_options;

typedef struct lfmm_solver_stats {
    int32_t iterations;       /* operator applications inside the Krylov cycles           */
    int32_t converged;        /* 1 if the true relative residual is <= tol                */
    double rel_residual;      /* true |b - A x| / |b| of the returned solution             */
} lfmm_solver_stats;

/* Lattice with inclusions (Section 10.1, eq. 10.1-10.4).  The lattice's bars are modified by B:
 * bar k joins the nodes (bars_host[4k], bars_host[4k+1]) and (bars_host[4k+2], bars_host[4k+3])
 * and changes its conductance by delta_host[k] (-1 removes a unit bar of the 5-point lattice;
 * a bar between nodes that had none is added with delta > 0), so that
 * (B w)(a) += delta (w(a) - w(b)) and (B w)(b) += delta (w(b) - w(a)).  The problem is
 * (A + B) u = 0 with u -> v = c1 m1 + c2 m2 at infinity (eq. 10.2).  Create builds the
 * node set Omega_inc (the bars' end points, in first-appearance order), B on it, and a
 * resident plan for S (convolution with phi) on Omega_inc; host arrays are read during the
 * call.  LFMM_E_INVAL for a bar from a node to itself or a non-finite delta.  The caller
 * keeps (A + B) invertible on decaying functions (no part of the lattice cut off). */
typedef struct lfmm_inclusions lfmm_inclusions;
lfmm_status lfmm_inclusions_create(lfmm_ctx* ctx, int64_t n_bars, const int32_t* bars_host,
                                   const double* delta_host, void* stream, lfmm_inclusions** out);
/* Number of nodes of Omega_inc and, if nodes_xy_host is not NULL, their coordinates [n][2]. */
lfmm_status lfmm_inclusions_nodes(const lfmm_inclusions* inc, int64_t* n_nodes, int32_t* nodes_xy_host);
/* Solves mu + B S mu = -B S B v on Omega_inc (eq. 10.4) by GMRES, each iteration one
 * execute of the resident plan; mu_dev[n_nodes] (device) receives mu.  Synchronises. */
lfmm_status lfmm_inclusions_solve(lfmm_inclusions* inc, double c1, double c2, const lfmm_solver_options* opt,
                                  double* mu_dev, lfmm_solver_stats* stats, void* stream);
/* u = v - S (B v + mu) at n_tgt targets tgt_xy_dev[2 n_tgt] (device) into u_dev[n_tgt]: the
 * recovery of the potential after eq. 10.4, read with +mu (with the paper's definitions,
 * A w = -(B v + B w) for w = u - v; the printed minus sign does not satisfy eq. 10.1). */
lfmm_status lfmm_inclusions_potential(lfmm_inclusions* inc, double c1, double c2, const double* mu_dev,
                                      int64_t n_tgt, const int32_t* tgt_xy_dev, double* u_dev, void* stream);
/* Frees the object and its plan; call it before lfmm_ctx_destroy of its context. */
lfmm_status lfmm_inclusions_destroy(lfmm_inclusions* inc);

/* Dirichlet problem on a finite lattice (Section 10.2, eq. 10.5-10.7).  gamma_xy_host[n][2]:
 * the boundary nodes Gamma (outside the domain, next to it); normal_host[n]: each node's
 * outward unit normal nu(n) as a code 0: +x, 1: -x, 2: +y, 3: -y, chosen so that n + nu(n)
 * lies outside the domain.  The double-layer-like operator of eq. 10.6, read as the difference
 * along nu acting on the source variable,
 *     [D q](m) = sum_{n in Gamma} [phi(m - n - nu(n)) - phi(m - n)] q(n),
 * is the field of a dipole per boundary node, so A (D q) = 0 in the domain.  Create builds a
 * resident plan with the 2n dipole ends as sources and Gamma as targets. */
typedef struct lfmm_dirichlet lfmm_dirichlet;
lfmm_status lfmm_dirichlet_create(lfmm_ctx* ctx, int64_t n, const int32_t* gamma_xy_host, const int8_t* normal_host,
                                  void* stream, lfmm_dirichlet** out);
/* out_dev[n] = (D q)(Gamma) for q_dev[n]: the matrix of eq. 10.7 applied by the FMM. */
lfmm_status lfmm_dirichlet_apply(lfmm_dirichlet* dir, const double* q_dev, double* out_dev, void* stream);
/* Solves D q = g on Gamma (eq. 10.7) by GMRES (the paper cites an O(N_Gamma) direct inversion
 * that it does not describe); g_dev, q_dev: device [n].  Synchronises. */
lfmm_status lfmm_dirichlet_solve(lfmm_dirichlet* dir, const double* g_dev, const lfmm_solver_options* opt,
                                 double* q_dev, lfmm_solver_stats* stats, void* stream);
/* u_dev[n_tgt] = (D q)(t) at n_tgt targets tgt_xy_dev (device): the solution of eq. 10.5 at
 * interior nodes once q solves eq. 10.7. */
lfmm_status lfmm_dirichlet_potential(lfmm_dirichlet* dir, const double* q_dev, int64_t n_tgt,
                                     const int32_t* tgt_xy_dev, double* u_dev, void* stream);
/* Frees the object and its plan; call it before lfmm_ctx_destroy of its context. */
lfmm_status lfmm_dirichlet_destroy(lfmm_dirichlet* dir);

/* ---- host-only calls (no GPU needed): the library's own phi and operators ------------ */

/* phi of lattice operator `stencil` (lfmm_stencil) at n integer offsets mxy_host[2n] (table
 * for |m|_inf <= 128 from the reduced 1-D integral of the remark closing Section 3, the
 * far-field expansion beyond: eq. (3.1) for the 5-point operator), into out_host[n]. */
lfmm_status lfmm_host_phi(int32_t stencil, int64_t n, const int32_t* mxy_host, double* out_host);

/* Builds the operators of Sections 5 and 7 for leaves of side leaf_side and n_levels
 * heights above the leaf (opt may be NULL). */
lfmm_status lfmm_host_opset_create(int64_t leaf_side, int32_t n_levels, const lfmm_options* opt,
                                   lfmm_opset** out);
/* Side and skeleton size of height h (h = 0 is the leaf). */
lfmm_status lfmm_host_opset_level(const lfmm_opset* ops, int32_t h, int64_t* side, int32_t* rank);
/* Skeleton points of height h relative to the box corner, out_host[2*rank]. */
lfmm_status lfmm_host_opset_skeleton(const lfmm_opset* ops, int32_t h, int64_t* out_host);
/* T_ofo for child c (0..3, c = x bit + 2 y bit) of height h >= 1, row-major
 * rank(h) x rank(h-1). */
lfmm_status lfmm_host_opset_ofo(const lfmm_opset* ops, int32_t h, int32_t c, double* out_host);
/* Dense-model T_ofs of the leaf (Remark 8.2), row-major rank(0) x side^2, column
 * x + side*y for the cell (x, y).  LFMM_E_UNSUPPORTED if the leaf is not dense. */
lfmm_status lfmm_host_opset_leaf(const lfmm_opset* ops, double* out_host);
lfmm_status lfmm_host_opset_destroy(lfmm_opset* ops);

#ifdef __cplusplus
}
#endif

#endif /* LFMM_H */
