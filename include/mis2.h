/*
 * mis2.h -- C ABI of the MI355X (gfx950) library for the deterministic
 * distance-2 maximal independent set (MIS-2) and MIS-2 aggregation of
 * Kelley & Rajamanickam, "Parallel, Portable Algorithms for Distance-2
 * Maximal Independent Set and Graph Coarsening" (arXiv 2204.02934).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Graphs are symmetric CSR: row_ptr (int64, n+1 entries, row_ptr[0] = 0,
 * non-decreasing, row_ptr[n] = nnz) and col (int32, nnz entries, each in
 * [0, n), no self-loops).  Duplicate entries are harmless to MIS-2 but
 * change the coupling counts of aggregation, so aggregation and coarsening
 * expect deduplicated rows.  n may be 0; n must be at most 2^31 - 2 so that
 * id + 1 fits the 32-bit packed tuple (Section V-C, Eq. 1).
 *
 * Every array argument is DEVICE memory on the context's GPU unless it is
 * documented as host memory.  The caller owns all inputs, outputs and the
 * workspace; the library allocates no device memory after mis2_create and
 * never frees caller memory.  Work is enqueued on the HIP stream passed as
 * `stream` (NULL = the null stream).  Entry points that return host
 * scalars synchronise that stream before returning.
 *
 * Every function returns MIS2_OK (0) or a negative error code; on error no
 * output is guaranteed and mis2_last_error() describes the failure.
 * Results are bit-identical for every launch plan, run and stream: all
 * reductions are min / any / all or integer sums, and every numbering is an
 * order-preserving prefix sum.
 *
 * A context is not thread-safe: one context per host thread and stream.
 */
#ifndef MIS2_H
#define MIS2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define MIS2_OK         0
#define MIS2_EINVAL    -1  /* bad argument (null pointer, negative size, n too large) */
#define MIS2_EGRAPH    -2  /* invalid CSR, detected when validation is enabled */
#define MIS2_ENOSPACE  -3  /* workspace missing or smaller than mis2_workspace_bytes() */
#define MIS2_EHIP      -4  /* HIP runtime error */
#define MIS2_EINTERNAL -5  /* an invariant the paper guarantees failed */

/* Operations, for mis2_workspace_bytes(). */
#define MIS2_OP_MIS2      0
#define MIS2_OP_AGGREGATE 1
#define MIS2_OP_COARSEN   2

/* Options, for mis2_set_option(). */
#define MIS2_OPT_VALIDATE      0  /* 1: check the CSR on the GPU before each call (default 0) */
#define MIS2_OPT_LANES_PER_ROW 1  /* 0 = automatic; -1 = flat (merge-path) sweeps; -2 =
                                     MIS2_LANES_STAGED; else 1, 2, 4, 8, 16, 32 or 64 lanes
                                     per CSR row */
#define MIS2_LANES_STAGED     (-2) /* one row per lane, each row's column indices staged in LDS
                                     by 16-byte loads (rows of more than 32 entries go to the
                                     whole wavefront); on graphs without such rows, once
                                     fewer than n/4 rows are left in worklist2, the rounds
                                     run 4 lanes per row */
#define MIS2_OPT_GRID_BLOCKS   2  /* 0 = automatic; else 1..8192 256-thread workgroups per sweep */
#define MIS2_OPT_PROFILE       3  /* 1: time every sweep launch with HIP events on the call's stream */
#define MIS2_OPT_ACCOUNT       4  /* 1: sweeps also sum the CSR row lengths they visit (extra atomics) */
#define MIS2_OPT_PERSISTENT    5  /* 0 (default): two launches per round; 1: all rounds of a MIS-2
                                     run in one cooperative launch (falls back to 0 when the
                                     grid cannot be co-resident) */
#define MIS2_OPT_COMPACT       6  /* 1 (default): when the workspace has room (see
                                     mis2_workspace_bytes_csr) and the graph has rows longer
                                     than the cooperative threshold (32 entries per lane of
                                     the lane plan, 1024 at 64 lanes), Refresh Column rewrites
                                     those rows without their OUT neighbours and reads the
                                     shorter rows in later rounds; 0: never (lane plans > 0
                                     only; results are the same either way) */
#define MIS2_OPT_TAIL          8  /* 1: once both worklists of a run hold fewer than 4096
                                     vertices (round 2 on), its remaining rounds run in one
                                     workgroup with the lists in LDS (one launch instead of
                                     two per round, and no round issued past the end); 0
                                     (default): every round is launched.  The plan tuner
                                     tries both.  Results are the same either way. */
#define MIS2_OPT_QUEUE_DEPTH   9  /* rounds the host keeps queued beyond the running one: 0
                                     (default) = 2; else 1..8.  Deeper queues issue more
                                     rounds past the end of a run (they find empty
                                     worklists); results never change */
#define MIS2_OPT_AUTOTUNE      7  /* 1 (default): while lanes and grid are automatic and the
                                     launch is not persistent, each graph of at least 16384
                                     vertices runs with the fastest of a few launch plans for
                                     its class (half octave of n and degree histogram), timed
                                     once per class and device on its first sight in the
                                     process (candidates in a fixed order; a later one wins
                                     only when at least 1% faster, the last one, the fastest
                                     with the one-workgroup tail, when no slower); 2: the
                                     plan of a class tuned before in the
                                     process, never a tuning run (a class not seen yet takes
                                     the degree rule); 0: the fixed degree rule.  Plans never
                                     change results. */

typedef struct mis2_ctx mis2_ctx;

/* A CSR graph in device memory (see the conventions above). */
typedef struct mis2_graph {
    int64_t n;              /* number of vertices */
    int64_t nnz;            /* stored entries, = row_ptr[n] */
    const int64_t *row_ptr; /* device, [n+1] */
    const int32_t *col;     /* device, [nnz] */
} mis2_graph;

/* Create a context bound to HIP device `device`.  Allocates only a small
 * pinned host buffer for scalar read-back.  *ctx receives the handle. */
int mis2_create(mis2_ctx **ctx, int device);

/* Destroy a context (NULL is ignored).  Does not free the workspace. */
void mis2_destroy(mis2_ctx *ctx);

/* Text of the last error on this context (never NULL). */
const char *mis2_last_error(const mis2_ctx *ctx);

/* Set an option (MIS2_OPT_*).  Launch-plan options never change results. */
int mis2_set_option(mis2_ctx *ctx, int option, int64_t value);

/* Bytes of device workspace that operation `op` (MIS2_OP_*) needs for a
 * graph with n vertices; written to *bytes (host).  Depends on n only. */
int mis2_workspace_bytes(int64_t n, int op, size_t *bytes);

/* Bytes of device workspace for operation `op` on a graph with n vertices
 * and nnz stored entries that also hold the compacted adjacency of Refresh
 * Column (4 * nnz + 4 * n bytes more than mis2_workspace_bytes, aligned);
 * written to *bytes (host).  A workspace of at least this size lets
 * mis2_run and mis2_aggregate read the long rows (MIS2_OPT_COMPACT), from
 * round 2 of a MIS-2 run on (round 0 of the phase-2 induced subgraph), as
 * only the neighbours whose tuple was not yet OUT when the row was last
 * swept: OUT is final and never lowers a minimum, so results are the same
 * with either size.  mis2_coarsen and mis2_aggregate_batched compact in
 * buffers of their own workspaces that are idle during the aggregation. */
int mis2_workspace_bytes_csr(int64_t n, int64_t nnz, int op, size_t *bytes);

/* Hand the context a caller-owned device workspace of `bytes` bytes,
 * 256-byte aligned.  It stays in use until replaced or the context is
 * destroyed; the caller frees it afterwards. */
int mis2_set_workspace(mis2_ctx *ctx, void *dev_ptr, size_t bytes);

/*
 * mis2_run -- Algorithm 1 (Section III-A): the deterministic MIS-2.
 *
 * Each round gives every undecided vertex v the packed tuple
 * (h(iter, v) << b) | (v + 1) (Section V-A hash, Section V-C packing,
 * b = ceil(log2(n + 2))), takes the minimum tuple over each closed
 * neighbourhood (Refresh Column), decides IN/OUT from the distance-2
 * information (Decide Set) and compacts the two worklists (Section V-B),
 * until no vertex is undecided.
 *
 *   seed      64-bit seed; the hash's first argument is (seed << 32) ^ iter,
 *             so seed 0 is the paper's h(iter, v)
 *   status    device out, uint8[n]: 1 if v is in the MIS-2, else 0
 *   n_roots   host out (may be NULL): |MIS-2|
 *   n_iters   host out (may be NULL): rounds executed
 * Needs a workspace of mis2_workspace_bytes(n, MIS2_OP_MIS2).
 */
int mis2_run(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, uint8_t *status,
             int64_t *n_roots, int32_t *n_iters, void *stream);

/*
 * mis2_run_noalloc -- mis2_run for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as mis2_run, but the
 * workspace is a static device array of the library (48 MiB, one copy per
 * GPU, held until the process ends) instead of the one set with
 * mis2_set_workspace, which is neither needed nor touched.  The call makes
 * no hipMalloc, hipFree or other allocating call.  The array's device
 * address is taken by mis2_create on each device.
 *
 * Limit: n <= mis2_run_noalloc_max_n() (about 2 million vertices); a larger
 * graph returns MIS2_ENOSPACE before any GPU work.  MIS2_OPT_PROFILE must be
 * off (MIS2_EINVAL otherwise: profiling creates events).
 * Every call on one GPU shares that GPU's array: two calls that overlap in
 * time on the same GPU (other threads, contexts or streams) race and may
 * return wrong results.  Calls in sequence are safe: each run initialises
 * every word it reads.
 */
int mis2_run_noalloc(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, uint8_t *status,
                     int64_t *n_roots, int32_t *n_iters, void *stream);

/* Largest n that mis2_run_noalloc accepts; written to *max_n (host). */
int mis2_run_noalloc_max_n(int64_t *max_n);

/*
 * mis2_run_ablation -- Algorithm 1 with the optimizations of Section V taken
 * away, for the comparison of Fig. 2 and Table I.  flags (bitwise or):
 */
#define MIS2_ABL_FIXED_PRIORITY 1   /* priorities drawn once, round 0's hash in every round
                                       (Bell et al.); changes the result */
#define MIS2_ABL_XORSHIFT       2   /* f = xorshift (shifts 12, 25, 27, no multiplication) instead
                                       of xorshift* (Table I's "Xor Hash"); changes the result */
#define MIS2_ABL_NO_WORKLISTS   4   /* every round sweeps every vertex (Section V-B taken away) */
#define MIS2_ABL_UNPACKED       8   /* three-field tuples (status, priority, id) in three arrays
                                       (Section V-C taken away) */
#define MIS2_ABL_ONE_LANE      16   /* one lane per CSR row (Section V-D taken away) */
#define MIS2_ABL_SIMPLE        32   /* the simple kernels even with none of the flags above */
#define MIS2_ABL_ALL_FLAGS     63
/*
 * With none of flags 1, 2, 4, 8 or 32 the production kernels run (as mis2_run,
 * with one lane per row under MIS2_ABL_ONE_LANE).  Otherwise simple kernels
 * run: one lane per row, a plain loop over each row, packed or three-field
 * tuples, worklists or every vertex.  The priority field of a three-field
 * tuple holds the same bits as the packed tuple, so only flags 1 and 2
 * change the result; the others change only the work done.  Outputs as in
 * mis2_run; per-round sizes and launch records as after mis2_run.  Needs a
 * workspace of mis2_ablation_workspace_bytes(n, flags).
 */
int mis2_run_ablation(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int flags,
                      uint8_t *status, int64_t *n_roots, int32_t *n_iters, void *stream);

/* Bytes of device workspace mis2_run_ablation needs (written to *bytes, host). */
int mis2_ablation_workspace_bytes(int64_t n, int flags, size_t *bytes);

/*
 * Cluster multicolor Gauss-Seidel (Algorithm 4, Section III-C).
 *
 * Setup coarsens the graph with mis2_aggregate (each row's aggregate is its
 * cluster; point != 0: every row is its own cluster, "point multicolor
 * Gauss-Seidel"), colours the coarse (quotient) graph -- the paper leaves
 * the colouring to other work; here Jones-Plassmann with the fixed priorities
 * of h(seed, 0, v) packed as in Section V-C: each round every uncoloured
 * vertex below all its uncoloured neighbours takes the smallest colour no
 * coloured neighbour has -- and orders the rows by colour, then cluster id,
 * then row id.  Apply runs that order: colour by colour, clusters of one
 * colour in parallel (they share no edge), the rows of a cluster one after
 * the other, each with x_i = (b_i - sum over j != i of A_ij x_j) / A_ii in
 * CSR order (no fused multiply-add); the symmetric form runs the order
 * forward, then backward.
 */
typedef struct mis2_cgs_plan {
    int64_t n;              /* rows (set by the caller) */
    int64_t n_clusters;     /* out */
    int32_t n_colors;       /* out */
    int32_t *cluster;       /* device out, int32[n]: cluster of each row */
    int32_t *cluster_color; /* device out, int32[n]: colour of cluster a at [a] (a < n_clusters) */
    int32_t *rows;          /* device out, int32[n]: rows in sweep order */
    int32_t *pos;           /* device out, int32[n]: sweep position of each row (rows[pos[i]] == i) */
    int64_t *cluster_off;   /* device out, int64[n + 1]: the k-th cluster of the sweep order holds
                               rows[cluster_off[k] .. cluster_off[k+1]) */
    int64_t *color_off;     /* host out, int64[n + 1]: colour c holds the sweep-order clusters
                               [color_off[c], color_off[c+1]) */
} mis2_cgs_plan;

/* Bytes of device workspace mis2_cgs_setup needs (written to *bytes, host). */
int mis2_cgs_workspace_bytes(int64_t n, int64_t nnz, size_t *bytes);

/* Fill a plan for graph g (the caller allocates its arrays, sizes above).
 * Synchronises the stream (the colouring reads a count back each round). */
int mis2_cgs_setup(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int point,
                   mis2_cgs_plan *plan, void *stream);

/* sweeps applications of the plan to x (device, double[n], in place) for the
 * matrix with off-diagonal entries val (device, double[nnz], in g's CSR order)
 * and diagonal diag (device, double[n]); b: device, double[n].  symmetric != 0:
 * each sweep runs forward and then backward.  Enqueues the launches and
 * returns (no synchronisation); needs no workspace. */
int mis2_cgs_apply(mis2_ctx *ctx, const mis2_graph *g, const double *val, const double *diag,
                   const mis2_cgs_plan *plan, const double *b, double *x, int32_t sweeps,
                   int symmetric, void *stream);

/* Per-round worklist sizes of the last mis2_run (or of the two MIS-2 runs
 * of the last mis2_aggregate, phase 1 then phase 2): host out
 * sizes[r*2 + 0] = |worklist1|, sizes[r*2 + 1] = |worklist2| at the start of
 * round r, for r < min(rounds, cap).  *rounds (host) receives the total
 * number of rounds recorded.  Reads host-side state only. */
int mis2_last_trace(const mis2_ctx *ctx, int phase, int64_t *sizes, int32_t cap,
                    int32_t *rounds);

/* One sweep launch of the last mis2_run / mis2_aggregate call. */
/* One launch plan timed by the plan tuner (MIS2_OPT_AUTOTUNE). */
typedef struct mis2_tune_record {
    int32_t lanes;   /* lanes per row (MIS2_LANES_STAGED for the staged sweeps) */
    int32_t blocks;  /* workgroups per sweep */
    int32_t tail;    /* 1: the last rounds in one workgroup (MIS2_OPT_TAIL) */
    float ms;        /* best of two timed MIS-2 runs of the graph, host wall clock */
} mis2_tune_record;

typedef struct mis2_sweep_record {
    int32_t kind;      /* 0 = Refresh Column (worklist2), 1 = Decide Set (worklist1),
                          2 = one persistent launch running every round of the phase
                          (then rows and edges are totals over its sweeps, rows_out is
                          the round count, and the per-sweep records carry ms = -1),
                          3 = the one-workgroup tail launch (MIS2_OPT_TAIL) running the
                          phase's rounds from `round` on (totals as for 2; its sweeps'
                          records come before it, with ms = -1),
                          4 / 5 = a Refresh Column / Decide Set launch of a round issued
                          after the run had ended (it found empty worklists; rows 0) */
    int32_t phase;     /* 0 = MIS-2 of G; 1 = MIS-2 of the phase-2 induced subgraph */
    int32_t round;     /* round of Algorithm 1, from 0 (-1 for kind 2) */
    int32_t lanes;     /* lanes per CSR row used by the launch */
    int64_t rows;      /* worklist entries processed */
    int64_t rows_out;  /* entries kept for the next round */
    int64_t edges;     /* sum of the processed CSR row lengths with MIS2_OPT_ACCOUNT, else -1 */
    float ms;          /* launch duration with MIS2_OPT_PROFILE, else -1 */
    int32_t compact;   /* Refresh Column and compacted rows (see MIS2_OPT_COMPACT): 0 = none,
                          1 = read the CSR's rows and rewrote the long ones compacted,
                          2 = read the long rows in compacted form and rewrote them */
    int64_t written;   /* Refresh Column with MIS2_OPT_ACCOUNT: column indices written into
                          compacted rows; else -1 */
} mis2_sweep_record;

/* Copy up to `cap` records of the last call's sweep launches to host array
 * `out`, in launch order; *count (host) receives the total number. */
int mis2_last_sweeps(const mis2_ctx *ctx, mis2_sweep_record *out, int32_t cap, int32_t *count);

/* Launch plan of the last mis2_run / mis2_aggregate / mis2_aggregate_basic on
 * this context (the last level's for multilevel and batched calls): lanes per
 * row (MIS2_LANES_STAGED for the staged sweeps), workgroups per sweep,
 * whether the last rounds ran in one workgroup (MIS2_OPT_TAIL), and
 * *source = 0 (set by options or the degree rule), 1 (tuned plan from the
 * cache) or 2 (tuned during this call).  Any pointer may be NULL. */
int mis2_last_plan(const mis2_ctx *ctx, int32_t *lanes, int32_t *blocks, int32_t *tail,
                   int32_t *source);

/* The candidate plans the last tuning on this context timed (see
 * MIS2_OPT_AUTOTUNE): lanes 1, 2, 4, 8 and the staged sweeps, each at its
 * grid rule, then the fastest with the one-workgroup tail when MIS2_OPT_TAIL
 * is automatic; up to cap of them into out (host); *count = how many there
 * were (0 if this context never tuned). */
int mis2_last_tuning(const mis2_ctx *ctx, mis2_tune_record *out, int32_t cap, int32_t *count);

/*
 * mis2_aggregate -- Algorithm 3 (Section III-B): MIS-2 based aggregation.
 *
 * Phase 1: the roots of an MIS-2 of G, numbered 0..n1-1 in increasing
 * vertex id, each aggregated with its neighbours.  Phase 2: an MIS-2 of the
 * subgraph induced by the still unaggregated vertices (original ids, same b,
 * round counter restarted at 0); each of its roots with at least two
 * unaggregated neighbours forms aggregate n1 + k (k in increasing id) with
 * those neighbours.  Phase 3: every remaining vertex joins the aggregate
 * holding most of its neighbours, ties to the smaller aggregate, then to the
 * smaller aggregate id, all counted on the labels frozen after phase 2.
 *
 *   agg_id    device out, int32[n]: aggregate of every vertex, 0..n_agg-1
 *   n_agg     host out (may be NULL)
 *   roots     device out, uint8[n] (may be NULL): 1 = phase-1 root,
 *             2 = accepted phase-2 root, 0 otherwise
 * Needs a workspace of mis2_workspace_bytes(n, MIS2_OP_AGGREGATE).
 * MIS2_EINTERNAL if a phase-3 vertex has no aggregated neighbour (the
 * maximality of the phase-1 MIS-2 rules this out).
 */
int mis2_aggregate(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int32_t *agg_id,
                   int64_t *n_agg, uint8_t *roots, void *stream);

/*
 * mis2_aggregate_basic -- Algorithm 2 (Section III-B): basic MIS-2 coarsening.
 *
 * Every vertex of an MIS-2 of G becomes a root; each root and its neighbours
 * form one aggregate, numbered 0..n_agg-1 in increasing root id (as phase 1
 * of mis2_aggregate).  Every vertex left over then joins the aggregate of a
 * neighbour: the smallest aggregate id among its neighbours aggregated by
 * the first step (the paper leaves the choice open; this one is
 * deterministic and reads only the first step's labels).
 *
 *   agg_id    device out, int32[n]: aggregate of every vertex
 *   n_agg     host out (may be NULL): |MIS-2|
 *   roots     device out, uint8[n] (may be NULL): 1 = root, 0 otherwise
 * Needs a workspace of mis2_workspace_bytes(n, MIS2_OP_AGGREGATE) (or the
 * _csr size for compacted long rows).  MIS2_EINTERNAL if a leftover vertex
 * has no aggregated neighbour (the maximality of the MIS-2 rules this out).
 * The per-round sizes of its MIS-2 are phase 0 of mis2_last_trace.
 */
int mis2_aggregate_basic(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int32_t *agg_id,
                         int64_t *n_agg, uint8_t *roots, void *stream);

/*
 * mis2_quotient -- the coarse graph of an aggregation, for multilevel
 * coarsening.  The paper coarsens recursively (Sections I and II) but does
 * not say how the coarse graph is formed; here it is the quotient graph:
 * vertex a of the coarse graph is aggregate a, and a and c are adjacent iff
 * some edge (u, w) of g has agg_id[u] = a, agg_id[w] = c and a != c.
 *
 *   agg_id          device, int32[n]: labels in [0, n_agg) (as from mis2_aggregate)
 *   n_agg           number of aggregates, 0 <= n_agg <= n
 *   coarse_row_ptr  device out, int64[n_agg + 1]
 *   coarse_col      device out, int32[g->nnz] (capacity; the coarse graph has at
 *                   most g->nnz entries), ascending and distinct in every row,
 *                   no self-loops
 *   coarse_nnz      host out (may be NULL)
 * Needs a workspace of mis2_workspace_bytes(n, MIS2_OP_COARSEN).
 */
int mis2_quotient(mis2_ctx *ctx, const mis2_graph *g, const int32_t *agg_id, int64_t n_agg,
                  int64_t *coarse_row_ptr, int32_t *coarse_col, int64_t *coarse_nnz, void *stream);

/*
 * mis2_smoothed -- smoothed aggregation on an aggregation of g (the
 * multigrid setup of Section VI-E smooths the prolongator of the aggregates;
 * the paper gives no formula): the damped-Jacobi prolongator
 * P = (I - omega D^-1 A) P_tent, with P_tent[i][agg i] = 1/sqrt(n_a) as in
 * mis2_galerkin, and the coarse operator A_c = P^T A P.
 *
 *   val, diag    device: A's off-diagonal values in g's CSR order, and its
 *                diagonal (nonzero)
 *   agg, n_agg   device labels in [0, n_agg), every aggregate non-empty
 *   omega        the damping factor (finite)
 *   prow/pcol/pval  device out: P as an n x n_agg CSR, p_cap entries of room
 *                (n + nnz always suffice); row i holds the distinct
 *                aggregates of i and its neighbours, ascending
 *   crow/ccol/cval  device out: A_c as an n_agg x n_agg CSR (diagonal
 *                included), c_cap entries of room, columns ascending
 *   p_nnz, c_nnz host out: entries of P and A_c (-1 when not reached)
 *   ws_need      host out (may be NULL): workspace bytes needed, when the
 *                context's is too small
 * Order of operations (bit-exact with the CPU reference): S = sum of A_ij
 * over j in N[i] with agg j = a, the diagonal first, then CSR order, from
 * 0.0; P[i][a] = (1{a = agg i} - (omega / d_i) * S) / sqrt(n_a); AP[i][b] =
 * sum over j in N[i] (i first, then CSR order) of A_ij * P[j][b]; A_c[a][b] =
 * sum over the rows i holding P[i][a], increasing, of P[i][a] * AP[i][b];
 * each product rounded on its own.
 * Errors: MIS2_ENOSPACE when p_cap, c_cap or the workspace is too small
 * (the counts known so far are set; call again with more room) or when a row
 * of A P or A_c has more than 2048 columns; MIS2_EINVAL for labels out of
 * range.  Synchronises the stream several times (setup work).
 */
int mis2_smoothed(mis2_ctx *ctx, const mis2_graph *g, const double *val, const double *diag,
                  const int32_t *agg, int64_t n_agg, double omega, int64_t *prow, int32_t *pcol,
                  double *pval, int64_t p_cap, int64_t *crow, int32_t *ccol, double *cval,
                  int64_t c_cap, int64_t *p_nnz, int64_t *c_nnz, size_t *ws_need, void *stream);

/*
 * mis2_galerkin -- the Galerkin coarse operator of an aggregation, the
 * multigrid hookup of the aggregates (Section VI-E builds smoothed-aggregation
 * multigrid on them; the paper takes the operator from its multigrid
 * package).  With the tentative prolongator for the constant near-null space,
 * P[i][a] = 1/sqrt(n_a) when agg_id[i] = a (n_a = members of a), it computes
 * A_c = P^T A P:  (A_c)[a][b] = (sum of A[i][j] over i in a, j in b)
 * / sqrt(n_a * n_b).  Each sum runs over the fine rows in increasing id,
 * within a row its diagonal first and then its entries in CSR order, from
 * 0.0, followed by one division (IEEE fp64, no fused multiply-add), so the
 * result does not depend on the launch.
 *
 *   g            the fine graph; A's off-diagonal entries are val (device,
 *                double[g->nnz], in g's CSR order), its diagonal diag (device,
 *                double[g->n])
 *   agg_id       device, int32[n]: labels in [0, coarse->n)
 *   coarse       the quotient graph of agg_id (as from mis2_quotient):
 *                coarse->n = number of aggregates
 *   coarse_val   device out, double[coarse->nnz]: A_c off the diagonal, in the
 *                coarse graph's CSR order
 *   coarse_diag  device out, double[coarse->n]: A_c's diagonal (the fine
 *                diagonal plus every coupling inside an aggregate)
 * Needs a workspace of mis2_galerkin_workspace_bytes(n, coarse->n).
 * Synchronises the stream.  MIS2_EINVAL if a label or coarse column is outside
 * [0, coarse->n) (nothing is written) or if the coarse graph lacks a coupling
 * of the aggregation (the outputs are then incomplete).
 */
int mis2_galerkin_workspace_bytes(int64_t n, int64_t n_agg, size_t *bytes);
int mis2_galerkin(mis2_ctx *ctx, const mis2_graph *g, const double *val, const double *diag,
                  const int32_t *agg_id, const mis2_graph *coarse, double *coarse_val,
                  double *coarse_diag, void *stream);

/* Bytes of device workspace mis2_coarsen needs for a graph with n vertices
 * and nnz stored entries (written to *bytes, host). */
int mis2_coarsen_workspace_bytes(int64_t n, int64_t nnz, size_t *bytes);

/*
 * mis2_coarsen -- multilevel coarsening: MIS-2 aggregation (Algorithm 3),
 * then the quotient graph, repeated while the current graph has at least
 * stop_below vertices, at most max_levels times, and stopping early when a
 * level does not shrink.  Every level uses the same seed.
 *
 *   agg_out     device out, int32[agg_cap]: the labels of level l start at
 *               the sum of the vertex counts of levels 0..l-1
 *   level_n, level_nnz, level_nagg
 *               host out, int64[max_levels]: vertices, stored entries and
 *               aggregates of each level's input graph
 *   n_levels    host out: levels computed (0 if g->n < stop_below)
 * Needs a workspace of mis2_coarsen_workspace_bytes(n, nnz).
 * MIS2_ENOSPACE if agg_cap is too small for the levels' labels.
 */
int mis2_coarsen(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int64_t stop_below,
                 int32_t max_levels, int32_t *agg_out, int64_t agg_cap, int64_t *level_n,
                 int64_t *level_nnz, int64_t *level_nagg, int32_t *n_levels, void *stream);

/* Bytes of device workspace mis2_aggregate_batched needs for n_graphs graphs
 * whose union has n vertices and nnz stored entries (written to *bytes). */
int mis2_batch_workspace_bytes(int32_t n_graphs, int64_t n, int64_t nnz, size_t *bytes);

/*
 * mis2_aggregate_batched -- mis2_coarsen for many graphs in one call.
 *
 * The graphs of the batch are given as their disjoint union g: graph k owns
 * the union's vertices [vtx_off[k], vtx_off[k+1]) and its rows there, with
 * columns in union ids; no edge may join two graphs.  Each graph gets exactly
 * what mis2_coarsen gives it alone (same seed, stop_below and max_levels):
 * Algorithm 1's tuples use the graph's own vertex ids and id width b (Section
 * V-C), and Algorithm 3's aggregate numbering is the graph's own.  Every
 * level runs all still-coarsening graphs together as one union.
 *
 *   vtx_off     host, int64[n_graphs + 1], vtx_off[0] = 0, non-decreasing,
 *               vtx_off[n_graphs] = g->n
 *   agg_out     device out, int32[agg_cap]: one block per level.  Level 0's
 *               block has g->n entries, the graph-local aggregate id of each
 *               vertex (-1 for graphs with no level, i.e. fewer than
 *               stop_below vertices); level l >= 1's block holds, in graph
 *               order, the coarse vertices of the graphs with more than l
 *               levels.  Blocks follow each other without gaps.
 *   level_n, level_nnz, level_nagg
 *               host out, int64[max_levels * n_graphs], entry l * n_graphs + k:
 *               vertices, stored entries and aggregates of graph k's level-l
 *               input (0 past its last level)
 *   n_levels    host out, int32[n_graphs]: levels computed per graph
 * Nothing is written to agg_out when no graph has a level.
 * Needs a workspace of mis2_batch_workspace_bytes(n_graphs, g->n, g->nnz).
 * MIS2_EINVAL for bad offsets; MIS2_ENOSPACE if agg_cap is too small.  Edges
 * between graphs are not detected; they give wrong results (aggregates that
 * would cross graphs are dropped as -1) but no out-of-bounds access.
 */
int mis2_aggregate_batched(mis2_ctx *ctx, const mis2_graph *g, int32_t n_graphs,
                           const int64_t *vtx_off, uint64_t seed, int64_t stop_below,
                           int32_t max_levels, int32_t *agg_out, int64_t agg_cap,
                           int64_t *level_n, int64_t *level_nnz, int64_t *level_nagg,
                           int32_t *n_levels, void *stream);

/*
 * Serving: continuous batching of coarsening jobs.
 *
 * A server owns a device arena (caller-allocated, 256-byte aligned, of
 * mis2_server_bytes() bytes) for a union of at most max_vertices vertices,
 * max_nnz stored entries and max_graphs graphs, plus its own context on
 * `device`.  Each job is mis2_coarsen of one graph with the server's seed,
 * stop_below and max_levels, and gets exactly mis2_coarsen's labels and level
 * sizes.  mis2_server_step admits queued jobs first come first served while
 * the union fits the arena, copying their CSRs in, then runs one level of
 * Algorithm 3 for every graph in the union at once (graphs at different levels
 * side by side); graphs that go on stay in the union as their coarse graphs,
 * so new jobs join at the next step.  Not thread-safe; one stream at a time.
 * A union's make-up changes from step to step, so the server's context never
 * runs a tuning pass inside a step (MIS2_OPT_AUTOTUNE = 2): a union takes the
 * plan of its class when that class was tuned earlier in the process, else
 * the degree rule.
 */
#define MIS2_SERVE_MAX_LEVELS 32

typedef struct mis2_server mis2_server;

typedef struct mis2_job_result {
    int64_t tag;             /* the submit() tag */
    int32_t n_levels;        /* levels computed */
    int32_t truncated;       /* 1 if coarsening stopped because agg_out was full */
    int64_t level_n[MIS2_SERVE_MAX_LEVELS];     /* vertices of each level's graph */
    int64_t level_nnz[MIS2_SERVE_MAX_LEVELS];   /* stored entries */
    int64_t level_nagg[MIS2_SERVE_MAX_LEVELS];  /* aggregates */
} mis2_job_result;

/* Arena bytes for the given capacities (written to *bytes, host). */
int mis2_server_bytes(int64_t max_vertices, int64_t max_nnz, int32_t max_graphs, size_t *bytes);

/* max_levels in [1, MIS2_SERVE_MAX_LEVELS]; max_vertices <= 2^31 - 3.
 * MIS2_EINVAL for bad capacities or an arena that is too small or misaligned. */
int mis2_server_create(mis2_server **srv, int device, void *arena, size_t arena_bytes,
                       int64_t max_vertices, int64_t max_nnz, int32_t max_graphs, uint64_t seed,
                       int64_t stop_below, int32_t max_levels);
void mis2_server_destroy(mis2_server *srv);
const char *mis2_server_last_error(const mis2_server *srv);

/* Queue a job.  g: device CSR that must stay valid (and unchanged) until the
 * job is admitted, i.e. until a later mis2_server_step returns.  agg_out:
 * device int32[agg_cap], at least g->n; receives each level's labels one
 * after the other, as mis2_coarsen's agg_out (a job whose next level might
 * not fit stops early with truncated = 1).  Jobs with fewer than stop_below
 * vertices finish at once with no level.  MIS2_ENOSPACE if the graph alone
 * exceeds the server's capacities. */
int mis2_server_submit(mis2_server *srv, const mis2_graph *g, int32_t *agg_out, int64_t agg_cap,
                       int64_t tag);

/* One step (admission + one level of every admitted graph) on `stream`;
 * returns after the stream has finished it.  *n_pending (host, may be NULL):
 * jobs queued or still coarsening afterwards. */
int mis2_server_step(mis2_server *srv, void *stream, int32_t *n_pending);

/* Finished jobs since the last poll, in completion order, at most cap of
 * them; *count gets how many were written. */
int mis2_server_poll(mis2_server *srv, mis2_job_result *out, int32_t cap, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* MIS2_H */
