/*
 * lpr.h -- C ABI of the lock-free push-relabel library for AMD Instinct
 * MI355X (gfx950).
 *
 * Two forms of the same lock-free push-relabel method ("Parallel
 * implementation of flow and matching algorithms", A. Lupinska):
 *
 *   1. Maximum flow / minimum cut on 4-connected grid networks (Section 4:
 *      flow network definitions in Section 3, the lock-free push/relabel of
 *      Algorithm 4.5 with the global and gap relabelling of Section 4.2 and
 *      Algorithm 4.8).
 *   2. The dense assignment problem by cost scaling (Section 5: the reduction
 *      to min-cost flow, the Min-Cost loop of Algorithm 5.0, the Refine of
 *      Algorithm 5.2 and the lock-free push/relabel of Algorithm 5.4).
 *
 * Built on the same machinery: form 1 on any directed network given as an
 * arc list (lpr_graph_maxflow), assignment on a sparse bipartite graph
 * (lpr_assign_sparse_solve) and min-cost flow with node supplies on any
 * capacitated network (lpr_mincost_flow, Algorithm 5.0 with the generic
 * Refine).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers documented as "device" must be device memory of the current HIP
 *    device (hipMalloc'd or a torch CUDA tensor); "host" pointers are read
 *    only during the call.  All buffers are caller-owned; the library keeps
 *    no pointer after it returns.
 *  - `workspace` is a caller-owned device buffer of at least the size the
 *    matching *_workspace() function returns (any alignment is accepted; the
 *    library aligns internally).  The solve entry points allocate no device
 *    memory of their own; the grid solvers keep instantiated HIP graphs of
 *    their round loops in a process-wide cache, and lpr_mincost_flow
 *    creates a stream and a HIP graph for its passes, released before it
 *    returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it and every solve call RETURNS AFTER COMPLETION
 *    (it synchronises the stream), so the status covers convergence.
 *  - The return code is the only error channel; the library never aborts.
 *    lpr_last_error() gives a thread-local description of the last failure.
 *  - Results that are unique (flow value, minimal source side, optimal
 *    total cost) are deterministic.  The flow decomposition, the permutation
 *    among equal-cost optima and the prices may differ between runs: this is
 *    inherent to lock-free execution.
 */
#ifndef LPR_H
#define LPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LPR_OK = 0,
    LPR_EINVAL = -1,  /* bad shape, offset, pointer or a negative capacity */
    LPR_ERANGE = -2,  /* a value too large for the fixed-width arithmetic  */
    LPR_ENOMEM = -3,  /* workspace smaller than required                   */
    LPR_EDEVICE = -4, /* a HIP runtime error (text in lpr_last_error)      */
    LPR_EBUDGET = -5, /* the round / operation budget ran out              */
    LPR_ENOMATCH = -6,   /* a sparse assignment has no perfect matching    */
    LPR_EINFEASIBLE = -7 /* no flow meets the supplies                     */
} lpr_status;

/* Thread-local, NUL-terminated description of the most recent failure of a
 * call made by this thread ("" if none).  Owned by the library. */
const char *lpr_last_error(void);

/* Library version string, e.g. "lpr 0.1.0 gfx950".  Owned by the library. */
const char *lpr_version(void);

/* ======================================================================== */
/* Form 1: 4-connected grid maximum flow / minimum cut                      */
/* ======================================================================== */

/* Limits: every capacity must lie in [0, LPR_GRID_MAX_CAP]; larger values
 * give LPR_ERANGE.  Excesses and residuals are int32 on the device; with this
 * bound no sum of a pixel's incident capacities can overflow. */
#define LPR_GRID_MAX_CAP ((1 << 26) - 1)

/* Option flags for lpr_grid_opts.flags. */
#define LPR_GRID_TIME_KERNELS 0x1 /* time every push-sweep and BFS launch
                                     with HIP events into lpr_grid_stats */
#define LPR_GRID_NO_GRAPH 0x2     /* launch every round's kernels one by one
                                     instead of replaying a captured graph */
#define LPR_GRID_ASYNC_RELABEL 0x4 /* asynchronous global relabel (ARG,
                                     Section 4.6): each round's global
                                     relabel runs on a library stream beside
                                     the push sweeps, on a snapshot of the
                                     residual arcs taken at the previous
                                     round boundary, and its labels become
                                     the heights at the next boundary; an
                                     instance retires when the exact count
                                     of a snapshot is 0 */
#define LPR_GRID_SYNC_RELABEL 0x8 /* global relabel between the sweeps (the
                                     scheme of Algorithm 4.8); with neither
                                     flag the tuned schedule decides */
#define LPR_GRID_SEGMENTED_SCAN 0x10 /* relax the rows of the global relabel
                                     and of the cut closure with segmented
                                     scans that test every lane, the form a
                                     batch uses anyway when an instance has
                                     more than 2^25 - 66 pixels (the default
                                     form offsets the labels by multiples
                                     of 2^25); same results, for testing */

typedef struct {
    int32_t sweeps_per_relabel; /* push-sweep launches between global
                                   relabels (the paper's CYCLE, counted in
                                   launches); 0 = tuned default; an odd
                                   count is rounded up to even            */
    int32_t local_iters;        /* push/relabel iterations each tile runs in
                                   on-chip memory per sweep launch; 0 =
                                   tuned default                          */
    int32_t tile_rows;          /* push-sweep tile height in pixels: 4, 8,
                                   16 or 32 (tile width is 64); 0 = tuned
                                   default                                */
    int32_t max_rounds;         /* budget of global-relabel rounds; 0 =
                                   default (1 << 16)                       */
    int32_t flags;              /* LPR_GRID_* bits                          */
    int32_t rounds_per_check;   /* rounds enqueued between two reads of the
                                   device status (1..16); 0 = tuned default */
    int32_t reserved[2];        /* must be 0                                */
} lpr_grid_opts;

typedef struct {
    int64_t rounds;          /* global relabels performed (BFS + gap) while
                                an instance was still unretired            */
    int64_t sweeps;          /* push-sweep launches enqueued                */
    int64_t bfs_passes;      /* relaxation launches of the global relabels
                                enqueued (a launch whose list is empty
                                returns at once)                          */
    int64_t tiles_swept;     /* tiles processed, summed over sweep launches */
    int64_t pushes;          /* push operations                             */
    int64_t relabels;        /* relabel operations                          */
    int64_t cut_passes;      /* tile-relaxation launches of the cut closure */
    int64_t tiles_relaxed;   /* tiles processed by the BFS relaxation       */
    int64_t device_atomics;  /* device-scope atomic updates the push sweeps
                                made (edge-pixel excess deltas and the three
                                words of every push across a tile edge);
                                pushes inside a tile update registers      */
    int32_t tile_rows;       /* push-sweep tile height actually used        */
    int32_t local_iters;     /* local iterations actually used              */
    int32_t sweeps_per_relabel;
    int32_t relax_tile_rows; /* tile height of the relaxation passes (the
                                tiles counted by tiles_relaxed; width 64)   */
    double sweep_ms;         /* with LPR_GRID_TIME_KERNELS: summed duration
                                of all push-sweep launches (HIP events)    */
    double bfs_ms;           /* same, for the BFS relaxation launches       */
    double total_ms;         /* wall time of the device work (HIP events)   */
    int32_t async_relabel;   /* 1 if the asynchronous global relabel ran    */
    int32_t rounds_per_check;/* rounds between host reads actually used     */
    int64_t bfs_passes_with_work; /* relaxation launches that relaxed a tile */
} lpr_grid_stats;

/* Device workspace bytes needed by lpr_grid_maxflow for an H x W grid. */
size_t lpr_grid_maxflow_workspace(int32_t H, int32_t W);

/*
 * Maximum s-t flow value and minimal minimum-cut source side of one grid.
 *
 * Network (Section 3; grid construction of Section 4.3): nodes are the H*W
 * pixels p = i*W + j (row-major) plus a source s and a sink t.  Arcs:
 *   s -> p     capacity cap_src[p]
 *   p -> t     capacity cap_snk[p]
 *   p -> p+1   capacity cap_right[p]  (ignored in the last column)
 *   p -> p-1   capacity cap_left[p]   (ignored in the first column)
 *   p -> p+W   capacity cap_down[p]   (ignored in the last row)
 *   p -> p-W   capacity cap_up[p]     (ignored in the first row)
 * All six arrays are device int32 [H*W], read only.
 *
 * Outputs (device):
 *   flow_value   int64 [1]: |f*|, the maximum flow value = min cut capacity.
 *   source_side  uint8 [H*W] or NULL: 1 iff p belongs to S_min, the source
 *                side of the unique minimal minimum cut (the residual closure
 *                of the pixels that hold excess in the maximum preflow).
 * opts may be NULL (defaults).  stats may be NULL.
 * Errors: LPR_EINVAL (H or W < 1, H*W >= 2^28, NULL inputs, negative
 * capacity), LPR_ERANGE (capacity > LPR_GRID_MAX_CAP), LPR_ENOMEM (workspace
 * too small), LPR_EBUDGET (max_rounds exhausted, or a global relabel that
 * needs more tile passes than 16 x tiles + 1024; outputs unspecified),
 * LPR_EDEVICE.
 */
lpr_status lpr_grid_maxflow(int32_t H, int32_t W,
                            const int32_t *cap_src, const int32_t *cap_snk,
                            const int32_t *cap_right, const int32_t *cap_left,
                            const int32_t *cap_down, const int32_t *cap_up,
                            int64_t *flow_value, uint8_t *source_side,
                            const lpr_grid_opts *opts, lpr_grid_stats *stats,
                            void *workspace, size_t workspace_bytes,
                            void *stream);

/*
 * Allocation-free variant of lpr_grid_maxflow, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same network, arguments, outputs and errors as
 * lpr_grid_maxflow, without the workspace: the solve's state lives in a
 * device array of the library (lpr_grid_maxflow_noalloc_max_bytes() bytes,
 * 40 MiB; one copy per GPU the library runs on, held until the process
 * ends).  The call allocates no device or pinned host memory and creates no
 * graph, stream or event; it still synchronises `stream` before it returns.
 * It runs the global relabel between the sweeps (LPR_GRID_ASYNC_RELABEL and
 * LPR_GRID_TIME_KERNELS give LPR_EINVAL: they need a stream or events).
 * Limit: grids whose lpr_grid_maxflow_workspace(H, W) exceeds that size
 * (about 1.25 M pixels; 1024 x 1024 fits) give LPR_ENOMEM.
 * Concurrency: all calls on one GPU share its array; calls that overlap on
 * one GPU (other threads or streams) race and give unspecified results.  A
 * call needs nothing from the previous call's contents.
 */
size_t lpr_grid_maxflow_noalloc_max_bytes(void);
lpr_status lpr_grid_maxflow_noalloc(int32_t H, int32_t W,
                                    const int32_t *cap_src, const int32_t *cap_snk,
                                    const int32_t *cap_right, const int32_t *cap_left,
                                    const int32_t *cap_down, const int32_t *cap_up,
                                    int64_t *flow_value, uint8_t *source_side,
                                    const lpr_grid_opts *opts, lpr_grid_stats *stats,
                                    void *stream);

/* Device workspace bytes for lpr_grid_maxflow_batched (H, W: host [B]). */
size_t lpr_grid_maxflow_batched_workspace(int32_t B, const int32_t *H,
                                          const int32_t *W);

/*
 * B independent grid networks solved together: every phase launch covers the
 * tiles of all unfinished instances, and finished instances retire.
 *   H, W         host int32 [B]: shape of instance b.
 *   node_offset  host int64 [B+1]: node_offset[0] = 0 and node_offset[b+1] =
 *                node_offset[b] + H[b]*W[b]; instance b occupies elements
 *                [node_offset[b], node_offset[b+1]) of every packed array.
 *   cap_*        device int32 [node_offset[B]], packed as above, each
 *                instance laid out as in lpr_grid_maxflow.
 *   flow_values  device int64 [B].
 *   source_side  device uint8 [node_offset[B]] (packed) or NULL.
 * Errors as for lpr_grid_maxflow; offsets that are not the prefix sums of
 * H*W, or a batch of 2^30 pixels or more, give LPR_EINVAL.
 */
lpr_status lpr_grid_maxflow_batched(int32_t B, const int32_t *H,
                                    const int32_t *W,
                                    const int64_t *node_offset,
                                    const int32_t *cap_src,
                                    const int32_t *cap_snk,
                                    const int32_t *cap_right,
                                    const int32_t *cap_left,
                                    const int32_t *cap_down,
                                    const int32_t *cap_up,
                                    int64_t *flow_values,
                                    uint8_t *source_side,
                                    const lpr_grid_opts *opts,
                                    lpr_grid_stats *stats, void *workspace,
                                    size_t workspace_bytes, void *stream);

/*
 * Schedule autotuner for the grid solver.  Solves the given batch (same
 * arguments as lpr_grid_maxflow_batched; flow_values device int64 [B]
 * receives the flow values) under every schedule of tile rows {4,8,16,32} x
 * local iterations {4,8,16,32} x sweeps per relabel {2,4,8} x relabel mode
 * {between sweeps, asynchronous} at 4 rounds per check, then the winner at
 * {1,2,4,8} rounds per check; each schedule `reps` times after one warm-up
 * run (1 <= reps <= 100), timed with HIP events.  It returns the fastest in
 * `best` (host, may be NULL; its flags name the relabel mode) with its time
 * in ms
 * (host, may be NULL).  The winner becomes the default schedule of this
 * process for the batch's size class (floor(log2(total pixels))) -- used
 * whenever opts is NULL or leaves a schedule field 0 -- and is written to
 * the file named by the environment variable LPR_GRID_TUNE_FILE, if set,
 * which later processes read.  Every schedule must produce the same flow
 * values; a disagreement returns LPR_EDEVICE.  Other errors as for
 * lpr_grid_maxflow_batched.
 */
lpr_status lpr_grid_tune(int32_t B, const int32_t *H, const int32_t *W,
                         const int64_t *node_offset, const int32_t *cap_src,
                         const int32_t *cap_snk, const int32_t *cap_right,
                         const int32_t *cap_left, const int32_t *cap_down,
                         const int32_t *cap_up, int64_t *flow_values,
                         int32_t reps, lpr_grid_opts *best, double *best_ms,
                         void *workspace, size_t workspace_bytes, void *stream);

/* ======================================================================== */
/* Form 2: dense assignment by cost scaling                                  */
/* ======================================================================== */

/* Costs must satisfy |c| <= LPR_ASSIGN_MAX_COST; n <= LPR_ASSIGN_MAX_N. */
#define LPR_ASSIGN_MAX_COST ((1 << 24) - 1)
#define LPR_ASSIGN_MAX_N 2048

#define LPR_ASSIGN_TIME_KERNELS 0x1 /* time the solve kernel with HIP events */
#define LPR_ASSIGN_NO_START_UPDATE 0x2 /* skip the global price update that
                                          otherwise runs right after each
                                          refine's first push of every row  */
#define LPR_ASSIGN_ARC_FIXING 0x4 /* arc fixing (Section 5): once
                                     (4n+2) eps < max|c| S, each refine
                                     ends by keeping per row only the arcs
                                     less than (4n+2) eps above the row
                                     minimum
                                     (a reduced cost above 2|V| eps never
                                     carries flow again) and later row
                                     scans read that list; after the last
                                     refine every row is checked for
                                     1-optimality over all arcs, and a
                                     failure reruns that refine with full
                                     scans (fixing_reruns).  Off by
                                     default: on the measured workloads
                                     the lists stay long until the last
                                     refines and the solve is not faster */

typedef struct {
    int32_t alpha;                  /* epsilon divisor per refine; 0 -> the
                                       tuned default (lpr_assign_tune), else
                                       6 for dense calls whose largest
                                       instance has n >= 1024, 16 for dense
                                       calls from the plain start whose
                                       largest instance has n <= 512, 8
                                       otherwise                           */
    int32_t flags;                  /* LPR_ASSIGN_* bits                     */
    int64_t eps0;                   /* initial epsilon of the Min-Cost loop in
                                       scaled units (costs times 2n+1); the
                                       first refine runs at eps0/alpha.
                                       0 -> max|c| * (2n+1)                  */
    const int64_t *init_col_prices; /* device int64 [n] (packed for batched)
                                       scaled starting prices of Y, or NULL
                                       for all zero                          */
    int64_t max_ops;                /* budget of push+relabel operations per
                                       instance; 0 -> 64 n^2 + 2^20          */
    int64_t max_ms;                 /* wall-clock budget of the solve kernel,
                                       checked on the device after every
                                       phase; 0 -> 20000 ms                  */
    const int64_t *eps0_per_instance; /* device int64 [B] or NULL: initial
                                       epsilon per instance (> 0), overrides
                                       eps0 (for starts whose accuracy is
                                       known per instance)                   */
    int64_t price_update_period;    /* pushes between global price updates
                                       (Algorithm 5.3), which run when a
                                       refine reaches its last few active
                                       rows; 0 -> n q / 4 for an instance of
                                       size n (q = price_update_quarters),
                                       -1 -> never                         */
    int32_t tail_rows;              /* a refine switches to one wavefront
                                       running operations back to back once
                                       at most this many rows are active;
                                       0 -> the tuned default, else 32 for
                                       dense calls whose largest instance
                                       has n <= 512 and min(32, max(8,
                                       8192 / n)) per instance otherwise   */
    int32_t fixing_shift;           /* for tests of the rerun path: divides
                                       the arc-fixing bound by
                                       2^fixing_shift (0..63; 0 = the
                                       bound above, 63 keeps only each
                                       row's matched arc); a bound that
                                       drops needed arcs is caught by the
                                       final check and costs a rerun       */
    int64_t warm_max_ops;           /* fallback of a warm start: an
                                       instance started from given prices
                                       (init_col_prices) or a given epsilon
                                       (eps0, eps0_per_instance) that has
                                       spent this many push+relabel
                                       operations without finishing
                                       restarts once from the plain start
                                       of Algorithm 5.0 (prices 0, epsilon
                                       max|c| (2n+1)); max_ops still bounds
                                       the whole solve.  0 -> 2 n^2 + 2^16,
                                       -1 -> never                         */
    int32_t price_update_quarters;  /* q of the default period n q / 4
                                       (1..64); 0 -> the tuned default, else
                                       1 for dense warm starts (given prices
                                       or epsilon) whose largest instance
                                       has n <= 512, and per instance 2 for
                                       n <= 512 and 4 above (measured best
                                       on the batched and the n = 1024
                                       workloads)                          */
    int32_t reserved;               /* must be 0                            */
} lpr_assign_opts;

typedef struct {
    int64_t refines;    /* refine calls (summed over instances)           */
    int64_t phases;     /* X-phase / Y-phase rounds (summed)              */
    int64_t pushes;     /* push operations                                */
    int64_t relabels;   /* relabel operations                             */
    int64_t scans;      /* arc scans of X rows (each reads n costs)       */
    int64_t price_updates; /* global price updates (Algorithm 5.3)        */
    int64_t price_update_us; /* time inside them, summed over instances   */
    int64_t fixing_reruns;   /* last refines rerun with full scans because
                                the arc-fixed matching failed the
                                1-optimality check (expected 0)          */
    int64_t warm_restarts;   /* instances whose warm start ran past
                                warm_max_ops and restarted from the plain
                                start                                     */
    int64_t scan_entries;    /* cost entries read by row scans: scans x n,
                                summed over instances                     */
    int64_t price_update_steps; /* bucket steps of the price updates (one
                                per distinct label reached), summed       */
    double kernel_ms;   /* with LPR_ASSIGN_TIME_KERNELS: solve kernel time */
    double total_ms;    /* device time of the whole call (HIP events)      */
    int32_t alpha;      /* schedule used: epsilon divisor per refine,       */
    int32_t price_update_quarters; /* q of the period n q / 4 (0: the rule
                                of 2 for n <= 512 and 4 above, or a
                                price_update_period was given),            */
    int32_t tail_rows;  /* and the tail threshold (0: min(32, max(8,
                                8192 / n)) per instance)                   */
    int32_t reserved;
} lpr_assign_stats;

/* Device workspace bytes needed by lpr_assign_solve for size n. */
size_t lpr_assign_workspace(int32_t n);

/*
 * Optimal assignment of the complete bipartite graph X x Y, |X| = |Y| = n,
 * given as a device int32 row-major n x n matrix `cost` (row x in X, column y
 * in Y).  maximize = 1 solves the problem as stated in Section 3 (maximum
 * total weight; internally the weights are negated), maximize = 0 minimises.
 *
 * Method (Section 5): costs are scaled by S = 2n+1; starting from eps0 the
 * Min-Cost loop runs Refine at eps <- max(1, floor(eps/alpha)) until a refine
 * at eps = 1 (i.e. 1/(2n+1) < 1/n in cost units) has finished.  Each refine
 * unmatches everything, sets row prices by Algorithm 5.2 and applies the
 * push/relabel of Algorithm 5.4 to active nodes until the pseudoflow is a
 * flow (a perfect matching).  The result is optimal for any starting prices.
 *
 * Outputs (device): row_to_col int32 [n] (a permutation), total int64 [1]
 * (sum of the given cost entries on the assignment), col_prices int64 [n] or
 * NULL (final scaled prices of Y for the minimised costs, a 1-optimality
 * certificate together with the assignment).
 * Errors: LPR_EINVAL (n < 1 or n > LPR_ASSIGN_MAX_N, NULL pointers),
 * LPR_ERANGE (|cost| > LPR_ASSIGN_MAX_COST), LPR_ENOMEM, LPR_EBUDGET,
 * LPR_EDEVICE.
 */
lpr_status lpr_assign_solve(int32_t n, const int32_t *cost, int32_t maximize,
                            int32_t *row_to_col, int64_t *total,
                            int64_t *col_prices, const lpr_assign_opts *opts,
                            lpr_assign_stats *stats, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Device workspace bytes for lpr_assign_solve_batched (n: host [B]). */
size_t lpr_assign_batched_workspace(int32_t B, const int32_t *n);

/*
 * B independent assignment instances solved in one launch (one workgroup
 * per instance, largest first).
 *   n            host int32 [B].
 *   cost_offset  host int64 [B+1]: prefix sums of n[b]^2; instance b's matrix
 *                is costs[cost_offset[b] .. cost_offset[b+1]) (row-major).
 *   costs        device int32 [cost_offset[B]].
 *   row_to_col   device int32 [sum n] packed by the prefix sums of n.
 *   totals       device int64 [B].
 *   col_prices   device int64 [sum n] packed, or NULL.
 *   opts->init_col_prices, when given, is packed like col_prices.
 * Errors as for lpr_assign_solve.
 */
lpr_status lpr_assign_solve_batched(int32_t B, const int32_t *n,
                                    const int64_t *cost_offset,
                                    const int32_t *costs, int32_t maximize,
                                    int32_t *row_to_col, int64_t *totals,
                                    int64_t *col_prices,
                                    const lpr_assign_opts *opts,
                                    lpr_assign_stats *stats, void *workspace,
                                    size_t workspace_bytes, void *stream);

/*
 * Schedule autotuner for the assignment solver (the tuning the paper does
 * by hand for its refine: alpha and the price-update heuristic, Section 5).
 * Solves the given batch (the arguments of lpr_assign_solve_batched; `base`
 * may be NULL or carry a start -- init_col_prices, eps0, eps0_per_instance
 * -- and budgets, which every trial keeps; its alpha, period, quarters and
 * tail fields must be 0) under every schedule of alpha {4, 6, 8, 16} x
 * price-update period n q / 4, q in {1, 2, 4, 8} x tail rows {per-instance
 * rule, 8, 32}, each `reps` times after one warm-up run (1 <= reps <= 100),
 * timed with HIP events.  It returns the fastest in `best` (host, may be
 * NULL; a copy of `base` with the schedule fields set) with its time in ms
 * (host, may be NULL).  The winner becomes this process's default for the
 * batch's size class (floor(log2(sum of n^2))) and kind of start (plain, or
 * from given prices or epsilon) -- used whenever those fields of the options
 * are 0 -- and is written to the file named by the environment variable
 * LPR_ASSIGN_TUNE_FILE, if set, which later processes read.  Every schedule
 * must give the same optimal totals; a disagreement returns LPR_EDEVICE.
 * Other errors as for lpr_assign_solve_batched.
 */
lpr_status lpr_assign_tune(int32_t B, const int32_t *n, const int64_t *cost_offset,
                           const int32_t *costs, int32_t maximize, int32_t *row_to_col,
                           int64_t *totals, const lpr_assign_opts *base, int32_t reps,
                           lpr_assign_opts *best, double *best_ms, void *workspace,
                           size_t workspace_bytes, void *stream);

/* Most arcs a sparse assignment instance may list (parallel arcs included). */
#define LPR_ASSIGN_SPARSE_MAX_ARCS (1 << 26)

/* Device workspace bytes for lpr_assign_sparse_solve (0 for bad n or m). */
size_t lpr_assign_sparse_workspace(int32_t n, int32_t m);

/*
 * Optimal assignment on a sparse bipartite graph X x Y, |X| = |Y| = n
 * (Section 3's problem on a graph with fewer arcs than the complete one),
 * by the same cost scaling (Section 5).  The arcs are given in CSR by row,
 * all device int32:
 *   row_ptr [n+1]  row_ptr[0] = 0, non-decreasing, row_ptr[n] = m;
 *   col     [m]    the columns of row x are col[row_ptr[x] .. row_ptr[x+1]);
 *   cost    [m]    |cost| <= 32767.
 * Parallel arcs are allowed; the best of them (least cost to minimise,
 * largest weight to maximise) is the arc.  Every row scan of every refine
 * reads the row's arcs only.  The price update (Algorithm 5.3) runs over a
 * dense copy in which a missing arc costs as much as the costliest arc and
 * has a length of at least 0; labels over a graph with such extra arcs
 * still bound every real arc, so the update stays valid.  Before the refines, a unit-capacity max-flow on
 * the arbitrary-network solver checks that a perfect matching exists.
 * Outputs as for lpr_assign_solve (total: the given costs of the chosen
 * arcs).  opts as for lpr_assign_solve; LPR_ASSIGN_ARC_FIXING is ignored.
 * Errors: LPR_EINVAL (n outside [1, LPR_ASSIGN_MAX_N], m outside
 * [0, LPR_ASSIGN_SPARSE_MAX_ARCS], a bad row_ptr, a column outside [0, n),
 * NULL pointers), LPR_ERANGE (|cost| > 32767), LPR_ENOMATCH (no perfect
 * matching), LPR_ENOMEM, LPR_EBUDGET, LPR_EDEVICE.
 */
lpr_status lpr_assign_sparse_solve(int32_t n, int32_t m, const int32_t *row_ptr,
                                   const int32_t *col, const int32_t *cost,
                                   int32_t maximize, int32_t *row_to_col,
                                   int64_t *total, int64_t *col_prices,
                                   const lpr_assign_opts *opts,
                                   lpr_assign_stats *stats, void *workspace,
                                   size_t workspace_bytes, void *stream);

/* ======================================================================== */
/* Learned warm start for cost scaling (not part of the paper's method)     */
/* ======================================================================== */
/*
 * A permutation-equivariant price network predicts the column prices p(Y)
 * that cost scaling starts from, so that the Min-Cost loop of Algorithm 5.0
 * can start at a small epsilon.  Refine recomputes the row prices from p(Y)
 * (Algorithm 5.2), so lpr_assign_solve stays exact whatever is predicted.
 *
 * Features: 16 per column, symmetric over rows -- with sc = mean|c| and
 * z = c/sc, rr = z - rowmin(z): the 8 smallest z of the column, mean and std
 * of z, the 2 smallest rr, mean rr, a two-pass min-plus dual estimate, the
 * column potential of an annealed Sinkhorn (entropic) dual of the assignment
 * (16 alternating log-sum-exp updates, temperature 0.3 falling by 0.7 per
 * step to 0.003; both centred per instance), and log(n)/6.
 * Network per instance (columns as the set): H_l = relu(H_{l-1} W_l +
 * mean_cols(H_{l-1}) U_l + b_l) for l = 1..3 (width 128), q = H_3 w_o + b_o
 * + f14: the network predicts a correction to the Sinkhorn potential, which
 * reaches the prediction at float32 precision (a skip connection).
 * Parameters: one float32 vector of lpr_pricenet_param_count() values,
 * W1 [16,128], U1 [16,128], b1 [128], W2 [128,128], U2 [128,128], b2 [128],
 * W3, U3 [128,128], b3 [128], w_o [128], b_o [1], row-major, concatenated.
 * Matrix products run on BF16 matrix cores with FP32 accumulation.
 *
 * Instances are described as for lpr_assign_solve_batched (host n [B], host
 * cost_offset [B+1], device costs); per-column arrays are packed by the
 * prefix sums of n.  maximize negates the costs first.  All calls return
 * after completion.  Errors: LPR_EINVAL, LPR_ENOMEM, LPR_EDEVICE.
 */
#define LPR_PRICENET_FEATURES 16
#define LPR_PRICENET_WIDTH 128

size_t lpr_pricenet_param_count(void);

/* Device workspace bytes for any lpr_pricenet_* call on these instances. */
size_t lpr_pricenet_workspace(int32_t B, const int32_t *n);

/* Column features (device float [sum n, 16], or NULL) and cost scales
 * sc (device float [B], or NULL). */
lpr_status lpr_pricenet_features(int32_t B, const int32_t *n,
                                 const int64_t *cost_offset,
                                 const int32_t *costs, int32_t maximize,
                                 float *feats, float *scales, void *workspace,
                                 size_t workspace_bytes, void *stream);

/* Forward pass.  params: device float [param_count], or NULL for a model
 * whose correction is zero: the prediction is then f14 alone, and the
 * feature passes only the network reads and the network itself are skipped
 * (the same q as a network with w_o = 0, b_o = 0).  Outputs (device, each
 * may be NULL): q float [sum n] (raw prediction); col_prices int64
 * [sum n], the scaled start prices rint((q - mean q) * sc * (2n+1)) to pass
 * as lpr_assign_opts.init_col_prices; eps0 int64 [B], the starting epsilon
 * max(1, rint(kappa * sc * (2n+1))) per instance to pass as
 * lpr_assign_opts.eps0_per_instance (kappa > 0 is the calibrated error of
 * the network in units of sc). */
lpr_status lpr_pricenet_infer(int32_t B, const int32_t *n,
                              const int64_t *cost_offset, const int32_t *costs,
                              int32_t maximize, const float *params,
                              float kappa, float *q, int64_t *col_prices,
                              int64_t *eps0, void *workspace,
                              size_t workspace_bytes, void *stream);

/* Prediction and warm-started batched solve in one call: lpr_pricenet_infer
 * (col_prices and eps0 into the workspace) followed by
 * lpr_assign_solve_batched with init_col_prices and eps0_per_instance set to
 * them (Algorithm 5.0 from the predicted prices; exact whatever is
 * predicted).  The solve's instance tables and cost copies are enqueued on a
 * second stream of the library's (created on the first call of a thread on a
 * device, default priority, kept until the process ends) so that they
 * overlap the prediction; the call waits for everything the caller enqueued
 * on `stream` before it and returns after completion like the other solves.
 * params and kappa as for lpr_pricenet_infer (kappa > 0); row_to_col,
 * totals, col_prices, opts and stats as for lpr_assign_solve_batched, where
 * opts (or NULL) must leave init_col_prices, eps0 and eps0_per_instance
 * unset.  workspace: device, at least lpr_assign_learned_workspace(B, n)
 * bytes.  Errors: LPR_EINVAL (arguments, kappa <= 0, start fields set in
 * opts), LPR_ENOMEM (workspace too small), and those of the two calls. */
size_t lpr_assign_learned_workspace(int32_t B, const int32_t *n);
lpr_status lpr_assign_solve_learned(int32_t B, const int32_t *n,
                                    const int64_t *cost_offset,
                                    const int32_t *costs, int32_t maximize,
                                    const float *params, float kappa,
                                    int32_t *row_to_col, int64_t *totals,
                                    int64_t *col_prices,
                                    const lpr_assign_opts *opts,
                                    lpr_assign_stats *stats, void *workspace,
                                    size_t workspace_bytes, void *stream);

/* One training step on a batch.  target_prices: device int64 [sum n], scaled
 * column prices of an optimal solution (e.g. lpr_assign_solve's col_prices);
 * they are normalised to t = (p - mean p) / (sc (2n+1)) internally.  Loss
 * (1/sum n) sum ((q - mean q) - t)^2 goes to loss_out (device float [1], or
 * NULL) and its gradient to grad_out (device float [param_count], or NULL).
 * step = 0 computes loss and gradient only; step >= 1 also applies Adam
 * (beta 0.9 / 0.999, bias correction for that step) to params with the
 * caller-owned moments adam_m, adam_v (device float [param_count]). */
lpr_status lpr_pricenet_train_step(int32_t B, const int32_t *n,
                                   const int64_t *cost_offset,
                                   const int32_t *costs, int32_t maximize,
                                   const int64_t *target_prices, float *params,
                                   float *grad_out, float *adam_m,
                                   float *adam_v, int32_t step, float lr,
                                   float *loss_out, void *workspace,
                                   size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Form 1 on an arbitrary directed graph (Section 4 with the node/adjacency
 * representation of the paper's implementation).
 * ------------------------------------------------------------------------- */
#define LPR_GRAPH_MAX_N (1 << 27)

typedef struct {
    int32_t cycle;       /* push/relabel attempts per node per sweep (the
                            paper's CYCLE); 0 -> 16                         */
    int32_t max_rounds;  /* rounds (sweeps_per_relabel sweeps, then a
                            global relabel); 0 -> 100000                    */
    int32_t sweeps_per_relabel; /* 1..1024; 0 -> 16                        */
    int32_t reserved;    /* must be 0                                       */
} lpr_graph_opts;

typedef struct {
    int64_t rounds;      /* rounds (each ends with a global relabel)         */
    int64_t pushes;      /* push operations                                  */
    int64_t relabels;    /* relabel operations (in the sweeps)               */
    int64_t bfs_levels;  /* BFS levels launched (global relabels, closure)   */
    double total_ms;     /* device time of the whole call (HIP events)       */
} lpr_graph_stats;

/* Device workspace bytes for lpr_graph_maxflow (0 if n < 2, m < 0 or m odd). */
size_t lpr_graph_maxflow_workspace(int32_t n, int32_t m);

/*
 * Maximum s-t flow of a directed network (Section 3's flow network; Section
 * 4's lock-free push-relabel with global relabel and gap).
 *   n                nodes 0..n-1 (2 <= n <= LPR_GRAPH_MAX_N); s != t.
 *   m                arcs, even: arcs a and a^1 are each other's reverse
 *                    (tail[a^1] == head[a], head[a^1] == tail[a]); an
 *                    undirected edge or a one-way arc is a pair with the
 *                    reverse capacity given (0 for one-way).
 *   tail, head, cap  device int32 [m]; cap >= 0 and cap[a] + cap[a^1] <=
 *                    2^31 - 1.  Parallel arcs and self-loops are allowed.
 *   flow_value       host int64 [1]: the maximum flow value.
 *   source_side      device uint8 [n] or NULL: 1 for the nodes of the
 *                    minimal source side of a minimum cut (the residual
 *                    closure of s and of the nodes left with excess).
 * Errors: LPR_EINVAL (arguments, arcs not in mate pairs or out of range),
 * LPR_ERANGE (capacity), LPR_ENOMEM (workspace too small), LPR_EBUDGET
 * (max_rounds), LPR_EDEVICE.  Returns after completion.
 */
lpr_status lpr_graph_maxflow(int32_t n, int32_t m, const int32_t *tail,
                             const int32_t *head, const int32_t *cap, int32_t s,
                             int32_t t, int64_t *flow_value, uint8_t *source_side,
                             const lpr_graph_opts *opts, lpr_graph_stats *stats,
                             void *workspace, size_t workspace_bytes,
                             void *stream);

/* ---------------------------------------------------------------------------
 * Minimum-cost flow with node supplies (Section 5, Algorithm 5.0: the cost
 * scaling Min-Cost loop with the generic Refine, push and relabel) on a
 * directed network given as arcs in mate pairs, as for lpr_graph_maxflow.
 * ------------------------------------------------------------------------- */

#define LPR_MCF_MAX_N (1 << 20)
#define LPR_MCF_MAX_COST ((1 << 16) - 1)
#define LPR_MCF_MAX_SUPPLY (1 << 30)

typedef struct {
    int32_t alpha;           /* eps divisor per refine (0: 8; >= 2)          */
    int32_t iters_per_check; /* push + relabel passes between host checks of
                                the active count (0: 32)                     */
    int64_t max_iters;       /* budget of passes over all refines (0: 2^20)  */
} lpr_mcf_opts;

typedef struct {
    int64_t refines;    /* Refine calls                                      */
    int64_t iterations; /* push + relabel passes launched                    */
    int64_t pushes;     /* push operations                                   */
    int64_t relabels;   /* relabel operations                                */
    double total_ms;    /* device time of the whole call (HIP events)        */
} lpr_mcf_stats;

/* Device workspace bytes for lpr_mincost_flow (0 for bad n or m). */
size_t lpr_mincost_flow_workspace(int32_t n, int32_t m);

/*
 * A flow meeting every node's supply (out-flow minus in-flow = supply[v])
 * within the arc capacities, of least total cost.
 *   n       nodes 0..n-1, 1 <= n <= LPR_MCF_MAX_N.
 *   m       arcs, even: arc a ^ 1 reverses arc a (as for lpr_graph_maxflow).
 *   tail, head, cap  device int32 [m] as for lpr_graph_maxflow; cap[a] bounds
 *           the flow along a, so a pair carries a net flow in
 *           [-cap[a ^ 1], cap[a]].
 *   cost    device int32 [m], cost[a ^ 1] = -cost[a], |cost| <=
 *           LPR_MCF_MAX_COST.
 *   supply  device int32 [n], |supply| <= LPR_MCF_MAX_SUPPLY, summing to 0.
 * Method: costs scaled by S = n + 1; eps starts at max|cost| x S and each
 * Refine divides it by alpha (at least 1) until a refine at eps = 1 (i.e.
 * 1/(n+1) < 1/n in cost units) has ended, which makes the flow optimal.
 * Refine saturates every arc of negative reduced cost, then alternates a
 * push pass (every node with excess pushes along its admissible arcs, with
 * atomic updates of residuals and excesses, prices fixed) and a relabel
 * pass (every node with excess and no admissible arc relabels, reading its
 * neighbours' prices, which only fall) until no node has excess; a global
 * price update (Algorithm 5.3: distances in units of eps over residual arcs
 * to the nodes with a deficit) runs at the start of a refine and between
 * batches of passes.  A maximum flow from the supplies to the demands on
 * the arbitrary-network solver first checks that a feasible flow exists.
 * Outputs: *total_cost (host) = sum over pairs of net flow x cost[a], in
 * int64 (callers keep it in range); residual (device int32 [m] or NULL):
 * final residual capacities, net flow along a = cap[a] - residual[a];
 * prices (device int64 [n] or NULL): final prices for the scaled costs,
 * with cost[a] S + p[tail] - p[head] >= -1 on every residual arc (the
 * optimality certificate).
 * Errors: LPR_EINVAL (n, m, pairs, nodes out of range, supplies not summing
 * to 0, costs not antisymmetric, NULL pointers), LPR_ERANGE (capacity, cost
 * or supply out of range), LPR_EINFEASIBLE (no flow meets the supplies),
 * LPR_ENOMEM, LPR_EBUDGET (max_iters), LPR_EDEVICE.
 */
lpr_status lpr_mincost_flow(int32_t n, int32_t m, const int32_t *tail,
                            const int32_t *head, const int32_t *cap,
                            const int32_t *cost, const int32_t *supply,
                            int64_t *total_cost, int32_t *residual,
                            int64_t *prices, const lpr_mcf_opts *opts,
                            lpr_mcf_stats *stats, void *workspace,
                            size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Measurement helper (not part of the method).  Section 4's pushes each
 * update four words with atomics; this gives the device's rate for such
 * updates: `blocks` x 256 threads each add 1 with a non-returning
 * device-scope 32-bit atomic to `per_thread` counters picked by their own
 * xorshift32 sequence among 2^log2_counters.
 *   counters       device int32 [2^log2_counters], caller-owned (zero it to
 *                  check that the counts sum to blocks * 256 * per_thread).
 *   log2_counters  6 .. 28;  blocks  1 .. 2^20;  per_thread  1 .. 4096.
 *   ms             host double [1]: the kernel's time (HIP events).
 * Returns after completion.  Errors: LPR_EINVAL (argument out of range or
 * NULL), LPR_EDEVICE.
 * ------------------------------------------------------------------------- */
lpr_status lpr_atomic_probe(int32_t *counters, int32_t log2_counters,
                            int32_t blocks, int32_t per_thread, double *ms,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LPR_H */
