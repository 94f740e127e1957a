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
#define MIS2_OPT_LANES_PER_ROW 1  /* 0 = automatic; -1 = flat (merge-path) sweeps; else 1, 2, 4,
                                     8, 16, 32 or 64 lanes per CSR row */
#define MIS2_OPT_GRID_BLOCKS   2  /* 0 = automatic; else the number of 256-thread workgroups per sweep */
#define MIS2_OPT_PROFILE       3  /* 1: time every sweep launch with HIP events on the call's stream */
#define MIS2_OPT_ACCOUNT       4  /* 1: sweeps also sum the CSR row lengths they visit (extra atomics) */
#define MIS2_OPT_PERSISTENT    5  /* 1 (default): all rounds of a MIS-2 run in one cooperative launch;
                                     0: two launches per round (also the fallback) */

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

/* Per-round worklist sizes of the last mis2_run (or of the two MIS-2 runs
 * of the last mis2_aggregate, phase 1 then phase 2): host out
 * sizes[r*2 + 0] = |worklist1|, sizes[r*2 + 1] = |worklist2| at the start of
 * round r, for r < min(rounds, cap).  *rounds (host) receives the total
 * number of rounds recorded.  Reads host-side state only. */
int mis2_last_trace(const mis2_ctx *ctx, int phase, int64_t *sizes, int32_t cap,
                    int32_t *rounds);

/* One sweep launch of the last mis2_run / mis2_aggregate call. */
typedef struct mis2_sweep_record {
    int32_t kind;      /* 0 = Refresh Column (worklist2), 1 = Decide Set (worklist1),
                          2 = one persistent launch running every round of the phase
                          (then rows and edges are totals over its sweeps, rows_out is
                          the round count, and the per-sweep records carry ms = -1) */
    int32_t phase;     /* 0 = MIS-2 of G; 1 = MIS-2 of the phase-2 induced subgraph */
    int32_t round;     /* round of Algorithm 1, from 0 (-1 for kind 2) */
    int32_t lanes;     /* lanes per CSR row used by the launch */
    int64_t rows;      /* worklist entries processed */
    int64_t rows_out;  /* entries kept for the next round */
    int64_t edges;     /* sum of the processed CSR row lengths with MIS2_OPT_ACCOUNT, else -1 */
    float ms;          /* launch duration with MIS2_OPT_PROFILE, else -1 */
    int32_t reserved;
} mis2_sweep_record;

/* Copy up to `cap` records of the last call's sweep launches to host array
 * `out`, in launch order; *count (host) receives the total number. */
int mis2_last_sweeps(const mis2_ctx *ctx, mis2_sweep_record *out, int32_t cap, int32_t *count);

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

#ifdef __cplusplus
}
#endif

#endif /* MIS2_H */
