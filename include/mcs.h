/*
 * mcs.h -- C ABI of the MI355X (gfx950) maximum common induced subgraph search.
 *
 * Problem (paper Sec. II.A): given graphs G and H, find the largest injective
 * partial map f: V_G -> V_H such that every ordered pair of distinct mapped
 * vertices agrees on adjacency (A_G(u,u') = A_H(f(u),f(u'))) and, for
 * vertex-labelled graphs, mapped vertices carry equal labels.  The common
 * subgraph need not be connected.
 *
 * Method (paper Sec. II.B, Eq. 1, Algorithm 1): McSplit branch and bound.
 * Each open search node holds label classes (L subset of V_G, R subset of V_H);
 * a child (v, w) splits every class by adjacency to v in G and to w in H, and
 * is pruned when |M| + sum over classes of min(|L|, |R|) cannot beat the
 * incumbent.  The library runs this on the GPU: many depth-first searches per
 * wavefront (one per segment of 16 or 8 lanes, a node's bitset classes
 * across the segment's lanes), a device work queue shared by all of them for
 * load balancing, and a per-instance incumbent updated with atomics.
 *
 * Conventions for every entry point:
 *   - No exception crosses the ABI; every call returns an mcs_status.
 *   - Host pointers (graphs, results, tuning) are borrowed for the duration of
 *     the call only.  Device memory is the caller's: the library never
 *     allocates or frees device memory.
 *   - A negative status means no result was written except size = -1 in each
 *     result; mcs_last_error() then names the cause.
 *   - Vertex ids in results are the caller's original ids.
 *   - libmcs.so links no HIP runtime of its own: it uses the one the process
 *     already has (link the program with -lamdhip64, or load that runtime
 *     with RTLD_GLOBAL before libmcs.so), so streams and device memory passed
 *     in belong to the same runtime that launches the kernels.
 */
#ifndef MCS_H
#define MCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCS_OK = 0,           /* solved to proven optimality */
    MCS_LIMIT = 1,        /* a node or time limit stopped the search: sizes and
                             mappings are valid, optimal = 0 where not proven */
    MCS_E_INVALID = -1,   /* malformed input (see mcs_last_error) */
    MCS_E_TOO_LARGE = -2, /* a graph has more than MCS_MAX_N vertices */
    MCS_E_DEVICE = -3,    /* a HIP call or the search kernel failed */
    MCS_E_WORKSPACE = -4, /* workspace missing, too small or misaligned */
    MCS_E_INTERNAL = -5   /* an internal check fired (a bug): a capacity check, a
                             mapping larger than the smaller graph, or a frame
                             past the class stack's worst case; the search
                             stops instead of writing out of bounds */
} mcs_status;

/* The paper's limit (Sec. III.B): vertex indices and stack entries are
 * bytes, with 255 reserved. */
#define MCS_MAX_N 254

/* One graph.  adj holds n rows of rw 64-bit words each, rw = ceil(n / 64)
 * (at least 1; 1 up to 64, 2 up to 128, 3 up to 192, 4 up to 254): the arc i -> j
 * exists iff bit j % 64 of adj[i * rw + j / 64] is set.  Undirected graphs
 * must be symmetric.  No self loops (diagonal bits) and no bits at or above
 * n.  label is NULL (unlabelled) or n vertex labels; G and H of a pair must
 * agree on directed and on labelled.  One batch may mix directed and
 * undirected pairs, and labelled and unlabelled ones.  A batch whose
 * largest graph has more than 64 vertices runs the slower one-search-per-
 * wavefront kernel with 128-bit rows for all its pairs (two classes per
 * lane in nodes of more than 64 classes), and one whose largest graph has
 * more than 128 vertices the same kernel with 256-bit rows (up to four
 * classes per lane). */
typedef struct {
    int32_t n;
    int32_t directed;
    const uint64_t *adj;
    const int32_t *label;
} mcs_graph;

/* Launch and scheduling knobs of the search kernel; zero fields take the
 * defaults the library derives from the instance sizes. */
typedef struct {
    int32_t waves_per_cu;      /* resident search wavefronts per CU (0: about
                                  96 searches per instance; segmented
                                  searches: 16, 12 or 8 per CU, the most that
                                  leave each search about 40 classes of LDS
                                  stack; one search per wavefront: 8 to 24;
                                  always capped by what LDS and registers let
                                  stay resident together) */
    int32_t children_per_wave; /* how many sibling children one wavefront may
                                  evaluate at once (1, 2, 4 or 8; 0: 8) */
    int32_t ring_slots;        /* total capacity of the device node queue, split
                                  over 8 per-XCD rings (0: auto) */
    int32_t donate_low;        /* records each XCD's queue ring is kept stocked
                                  with: a busy wavefront whose periodic check
                                  finds fewer waiting donates its shallowest
                                  open node (0: 2; < 0: never donate) */
    int32_t donate_depth;      /* only nodes with |M| <= this are donated, as the
                                  paper delegates only above PART_LEVEL
                                  (0: any depth -- the largest min(nG, nH)) */
    int32_t check_interval;    /* search steps between queue/limit checks (0: 128) */
    int32_t no_reprune;        /* 1: do not re-test a frame's bound against the
                                  incumbent when the search returns to it */
    int32_t single_wave;       /* 1: one search alone (the first segment of one
                                  wavefront, or one wavefront with seg_lanes
                                  64), in the sequential order: no queue, no
                                  donations (debugging and node-count
                                  comparisons with the oracle) */
    int32_t use_graph;         /* 1: mcs_plan_run replays a HIP graph that holds
                                  a whole solve: the input copy (from pinned
                                  host memory the plan allocates once), the
                                  reset and search kernels, and the result
                                  copy back (mcs_plan_results then only waits
                                  and decodes) */
    int32_t stack_classes;     /* segmented searches: classes of each search's
                                  stack kept in LDS (0: the worst case
                                  m(m+1)/2, m the largest min(nG, nH), or
                                  less if that keeps waves_per_cu from
                                  fitting in LDS; never below m, so any one
                                  frame fits at the stack's start).  The
                                  rest of the worst case is in HBM, so a
                                  child always has room: a frame that might
                                  not fit in the LDS part goes to the HBM
                                  part.  One search per wavefront always
                                  keeps the whole worst case (in LDS, or in
                                  HBM with 128- and 256-bit rows); this field does not
                                  apply to it. */
    int32_t backoff_max;       /* an idle wavefront that finds no work sleeps
                                  1, 2, 4, ... up to this many times about
                                  3.4 us before polling again (0: 32) */
    int32_t seg_lanes;         /* search layout: 16, 8 or 4 -- each wavefront runs
                                  64 / seg_lanes independent searches, one per
                                  segment of that many lanes (a node's classes
                                  across the segment); 64 -- one search per
                                  wavefront, whose sibling children share the
                                  lanes; 0: 8.  Rows of more than 64 bits and
                                  the learned policy always use 64.  With
                                  segments, waves_per_cu counts wavefronts
                                  and children_per_wave is not used. */
} mcs_tuning;

typedef struct {
    int64_t node_limit;        /* stop after about this many nodes (0: none) */
    double time_limit_s;       /* stop after this much kernel time (<= 0: 600 s) */
    const mcs_tuning *tuning;  /* NULL: all defaults */
    const uint16_t *policy;    /* device pointer, 16-byte aligned, to the learned
                                  branching policy's half-precision parameters
                                  (mcs_policy_pack_half; graphs of at most 64
                                  vertices, else MCS_E_INVALID), or NULL: branch on the
                                  smallest vertex index
                                  (descending degree) and try partners in index
                                  order */
    int32_t policy_depth;      /* the policy orders choices at nodes with
                                  |M| <= policy_depth (ignored if policy is NULL) */
    int32_t policy_mode;       /* bit 0: the policy picks v within the selected
                                  class; bit 1: it orders the partners w
                                  (0: order the partners only) */
    int32_t ordering;          /* static vertex order of both graphs (Sec. IV.A):
                                  0: descending degree (total degree if
                                  directed), ties by index; 1: connected
                                  components, a component with more non-zero
                                  rows per non-zero column first, each in a
                                  bordered block-triangular order (the column
                                  meeting the most shortest active rows next);
                                  2: both, as a portfolio (Sec. IV): each pair
                                  is searched twice in the same launch, under
                                  order 0 and under order 1, and the two
                                  searches share one incumbent (a mapping
                                  either finds prunes the other) and stop
                                  together once either has finished; nodes
                                  are summed over both, the mapping is the
                                  one of the search that found the final
                                  size.  Sizes do not depend on the order;
                                  node counts do. */
    int32_t deadend_ratio;     /* dead-end forecast (paper Sec. IV.A), with
                                  deadend_nodes: an instance is given up once
                                  its search has gone more than deadend_nodes
                                  nodes and more than deadend_ratio times the
                                  nodes that led to its last improvement
                                  (0: the absolute threshold alone) without
                                  raising its incumbent.  Its result is then
                                  the best mapping so far, optimal = 0, and
                                  the call returns MCS_LIMIT;
                                  mcs_solve_goals strategies 2 and 3 answer a
                                  forecast by stepping the bound. */
    int64_t deadend_nodes;     /* 0: no dead-end forecast */
} mcs_opts;

/* Per-instance result.  map_g/map_h are caller-owned arrays of capacity
 * min(nG, nH) (either may be NULL); size pairs are written. */
typedef struct {
    int32_t size;
    int32_t optimal;           /* 1: the search finished, size is the MCS */
    int32_t *map_g;
    int32_t *map_h;
    int64_t nodes;             /* search nodes evaluated for this instance
                                  (the root and every child whose bound was
                                  computed) */
    double t_best_s;           /* kernel time at which the final size was found */
    double t_proof_s;          /* kernel time at which the search of this
                                  instance finished (0 if it did not) */
} mcs_result;

/* Whole-launch statistics, filled by mcs_plan_stats. */
typedef struct {
    int64_t nodes;             /* sum over instances */
    int64_t batches;           /* child batches evaluated by all wavefronts */
    int64_t children;          /* children evaluated (with re-evaluations) */
    int64_t lane_slots;        /* lanes holding a class in those batches */
    int64_t donations;         /* nodes published to the shared queue */
    int64_t pops;              /* nodes taken from the shared queue */
    int32_t waves;             /* wavefronts launched */
    int32_t blocks;            /* workgroups launched */
    int32_t lds_per_wave;      /* bytes of LDS per wavefront */
    int32_t stopped;           /* 1 if a limit stopped the search */
    double kernel_ms;          /* search kernel time of the last run */
    double busy_wave_s;        /* wavefront-seconds spent searching; the rest
                                  of waves x kernel time went to looking for
                                  work (load imbalance and queue latency) */
    int64_t hbm_frames;        /* frames placed in the HBM part of a segmented
                                  search's class stack */
    int32_t stack_classes;     /* class-stack capacity per wavefront */
    int32_t max_stack_used;    /* most classes any wavefront's stack held */
    double sleep_wave_s;       /* wavefront-seconds idle wavefronts spent in
                                  back-off sleeps (part of the time not busy) */
    int64_t lds_bytes;         /* algorithmic bytes through LDS: the adjacency
                                  rows each child batch reads (v's and its
                                  partners'), and the classes of each pushed
                                  frame, written once and read twice (headers
                                  and mapping entries are not counted) */
    int64_t node_classes;      /* classes split by the matched children counted
                                  in nodes, each counted once (siblings that a
                                  batch evaluates again after a descent are
                                  not): the algorithmic unit of the split and
                                  Eq. 1 work */
} mcs_stats;

typedef struct mcs_plan mcs_plan;

/* Validate count pairs (G[i], H[i]), order vertices by descending degree
 * (total degree when directed; ties by index), pack bit rows and root classes
 * on the host (Sec. IV.A ordering; root classes: all vertices, or one class
 * per label present in both graphs).  No device work.  *out must be released
 * with mcs_plan_destroy.  Errors: MCS_E_INVALID, MCS_E_TOO_LARGE. */
mcs_status mcs_plan_create(int32_t count, const mcs_graph *G, const mcs_graph *H,
                           const mcs_opts *opts, mcs_plan **out);

/* Bytes of device workspace the plan needs (256-byte aligned base). */
size_t mcs_plan_workspace_size(const mcs_plan *plan);

/* Bind the caller's device workspace and copy the packed instances into it
 * (asynchronous on stream, a hipStream_t or NULL).  The workspace must stay
 * allocated and untouched by the caller until the plan is destroyed or bound
 * again.  Errors: MCS_E_WORKSPACE, MCS_E_DEVICE. */
mcs_status mcs_plan_upload(mcs_plan *plan, void *workspace, size_t bytes, void *stream);

/* Reset the search state and launch the search over all instances
 * (asynchronous on stream).  Inputs are already resident in the workspace.
 * Errors: MCS_E_WORKSPACE (no upload yet), MCS_E_DEVICE. */
mcs_status mcs_plan_run(mcs_plan *plan, void *stream);

/* Wait for the last run, copy results back and map them to original vertex
 * ids.  results has one entry per instance.  Returns MCS_OK, MCS_LIMIT, or
 * an error (MCS_E_DEVICE; MCS_E_INTERNAL if the kernel flagged a broken
 * invariant). */
mcs_status mcs_plan_results(mcs_plan *plan, mcs_result *results, void *stream);

/* Statistics of the last run (valid after mcs_plan_results). */
mcs_status mcs_plan_stats(const mcs_plan *plan, mcs_stats *stats);

/* Goal-directed runs (paper Sec. IV.A, top-down search and bound
 * correction).  goal[i] > 0: the next run asks only whether instance i has a
 * common induced subgraph of at least goal[i] vertices -- its incumbent starts
 * at goal[i] - 1 and its search stops at the first such mapping (the result
 * then has size >= goal[i] and optimal = 1 means the question was settled:
 * either such a mapping was found, or, with size < goal[i], none exists).
 * goal[i] == 0: plain search; goal[i] < 0: skip instance i.  Goals stay set
 * until changed.  Errors: MCS_E_INVALID (a goal above min(nG, nH)),
 * MCS_E_WORKSPACE, MCS_E_DEVICE. */
mcs_status mcs_plan_set_goals(mcs_plan *plan, const int32_t *goal, void *stream);

/* Eq. 1 at the root of each instance (an upper bound on its MCS size). */
mcs_status mcs_plan_root_bounds(const mcs_plan *plan, int32_t *bounds);

void mcs_plan_destroy(mcs_plan *plan);

/* Workspace bytes mcs_solve_batch needs for these instances. */
size_t mcs_workspace_size(int32_t count, const mcs_graph *G, const mcs_graph *H,
                          const mcs_opts *opts);

/* Solve MCS(G[i], H[i]) for count pairs in one launch: create, upload, run,
 * results, destroy.  workspace: device memory of mcs_workspace_size bytes. */
mcs_status mcs_solve_batch(int32_t count, const mcs_graph *G, const mcs_graph *H,
                           const mcs_opts *opts, void *workspace, size_t bytes,
                           void *stream, mcs_result *results);

/* Bytes of the library's static device scratch (64 MiB). */
#define MCS_STATIC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation:
 * mcs_solve_batch with the library's own static device scratch (a
 * file-scope array of MCS_STATIC_SCRATCH_BYTES per device, held by every
 * device the library runs on until the process ends) as the workspace.  The
 * caller still passes the inputs (host graphs, borrowed for the call) and
 * the results (host, caller-owned).  No device memory, pinned host memory or
 * event is allocated; the HIP graph mode (tuning->use_graph) is refused, as
 * it stages through pinned memory.  Every call on one device reuses that
 * device's scratch, whose contents the previous call left: the search state
 * is cleared by the reset kernel at the start of each run.  Calls that
 * overlap on one device (other host threads, other streams) race on the
 * scratch: serialize them.  Synchronous on stream.  Errors: as
 * mcs_solve_batch; MCS_E_WORKSPACE if the batch needs more than
 * MCS_STATIC_SCRATCH_BYTES (mcs_workspace_size tells; fewer wavefronts per
 * CU or one search per wavefront need less); MCS_E_INVALID for use_graph;
 * MCS_E_DEVICE if the scratch's address cannot be looked up. */
mcs_status mcs_solve_batch_static(int32_t count, const mcs_graph *G, const mcs_graph *H,
                                  const mcs_opts *opts, void *stream, mcs_result *results);

/* Goal-directed search over a batch, as the paper's top-down and
 * bound-correction variants (Sec. IV.A).  strategy 0: goals root bound,
 * root bound - 1, ...; the first goal reached is the optimum.  strategy 1:
 * a plain run bounded by opts->node_limit gives a lower bound, then a binary
 * search on the goal between it and the root bound.  Each launch gets the
 * whole opts->time_limit_s; the call stops with MCS_LIMIT once their sum
 * exceeds it.  results as for mcs_solve_batch (nodes summed over launches);
 * *launches (may be NULL) = kernel launches used. */
mcs_status mcs_solve_goals(int32_t count, const mcs_graph *G, const mcs_graph *H,
                           const mcs_opts *opts, int32_t strategy, void *workspace,
                           size_t bytes, void *stream, mcs_result *results,
                           int32_t *launches);

/* One pair: mcs_solve_batch with count = 1. */
mcs_status mcs_solve(const mcs_graph *G, const mcs_graph *H, const mcs_opts *opts,
                     void *workspace, size_t bytes, void *stream, mcs_result *result);

/* ---- learned branching policy -------------------------------------------
 * A 16 -> 64 -> 64 -> 1 ReLU network scores a candidate vertex from 16
 * features of the search node (degrees, class sizes, depth, neighbours per
 * class-size bucket).  At nodes with |M| <= policy_depth the search tries the
 * partners w of v best-scored first and, if asked (policy_mode bit 0),
 * branches on the best-scored vertex v of the selected class.  Order only: every child is still explored or bounded by Eq. 1, so
 * results are the same as without the policy (the paper has no learned part;
 * its Solve leaves both choices to "some heuristic", Sec. II.B).
 *
 * Parameters: float32, packed W1[64][16], b1[64], W2[64][64], b2[64], w3[64],
 * b3 (mcs_policy_param_count() values).  Rows: 16 half-precision features.
 * Every pointer below is device memory owned by the caller; calls are
 * asynchronous on stream.  Multiplies use the half-rounded weights with
 * float32 accumulation, as the search does. */

/* Number of float parameters (5313). */
int32_t mcs_policy_param_count(void);

/* Device bytes of workspace mcs_policy_grad needs for rows rows. */
size_t mcs_policy_workspace_size(int32_t rows);

/* logits[r] = network(x[r]) for r < rows.  Errors: MCS_E_INVALID. */
mcs_status mcs_policy_forward(const uint16_t *x, int32_t rows, const float *params,
                              float *logits, void *stream);

/* grads = gradient of the mean binary cross-entropy of sigmoid(logit) against
 * labels y (0/1 floats) over rows rows; *loss (device, may be NULL) = the
 * mean loss.  Deterministic (fixed reduction order).  Errors: MCS_E_INVALID,
 * MCS_E_WORKSPACE. */
mcs_status mcs_policy_grad(const uint16_t *x, const float *y, int32_t rows, const float *params,
                           float *grads, float *loss, void *workspace, size_t bytes,
                           void *stream);

/* params -= lr * grads. */
mcs_status mcs_policy_sgd(float *params, const float *grads, float lr, void *stream);

/* half_params = params rounded to half precision (the form mcs_opts.policy takes). */
mcs_status mcs_policy_pack_half(const float *params, uint16_t *half_params, void *stream);

/* Static description of a status code. */
const char *mcs_status_string(mcs_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char *mcs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCS_H */
