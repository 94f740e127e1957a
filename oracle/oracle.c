/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the deterministic
 * distance-2 maximal independent set (MIS-2) and the MIS-2 aggregation of
 * Kelley & Rajamanickam, "Parallel, Portable Algorithms for Distance-2 Maximal
 * Independent Set and Graph Coarsening" (arXiv 2204.02934).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the HIP library is
 * compared against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it; the product path never does.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Every loop below runs sequentially, in increasing vertex order, exactly in
 * the order the paper states the steps; nothing is blocked, fused or
 * reordered.  Readings taken where the paper is silent are marked "Reading".
 *
 * Pins (in tests/): the worked example of Fig. 1 (exact intermediate values),
 * a brute-force Luby-on-G^2 implementation (Section IV, Lemma 2) on small
 * graphs, breadth-first validity checks of the definitions (Section I),
 * closed-form special cases, exhaustive packing checks (Section V-C, Eq. 1),
 * brute-force aggregation invariants (Section III-B, Alg. 3) and Table III
 * counts (soft: the paper does not fix the hash bits, see oracle_hash); for
 * the Galerkin coarse operator, the dense product P^T A P, its special cases
 * and exact rounding on integer-valued matrices.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The phase loops of Alg. 1 are pure maps (each writes only its own
 * vertex's entry and reads only arrays the phase does not write), so a
 * build with -DORACLE_OMP -fopenmp may run them on several threads with
 * identical results; the default build is sequential. */
#ifdef ORACLE_OMP
#define ORACLE_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define ORACLE_PARALLEL_FOR
#endif

#define ORACLE_IN  0u           /* Section V-C: IN is the value 0          */
#define ORACLE_OUT 0xFFFFFFFFu  /* Section V-C: OUT is UINT_MAX (32 bits)  */

/* ------------------------------------------------------------------------- */
/* Section V-A: f is 64-bit xorshift* (an xorshift step followed by a         */
/* multiplicative linear congruential step).  The paper gives no constants;  */
/* Reading: Vigna's published xorshift64* (ACM TOMS 2016): shifts 12, 25, 27 */
/* and multiplier 2685821657736338717, arithmetic modulo 2^64.               */
/* ------------------------------------------------------------------------- */
uint64_t oracle_xorshift64star(uint64_t x)
{
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    return x * UINT64_C(2685821657736338717);
}

/* Section V-A: h(iter, v) = f(f(iter) XOR f(v)).
 * Reading (seed): the paper has no seed; the first argument of h becomes
 * (seed << 32) XOR iter, so seed 0 is the paper's formula unchanged. */
uint64_t oracle_hash(uint64_t seed, uint64_t iter, uint64_t v)
{
    uint64_t i = (seed << 32) ^ iter;
    return oracle_xorshift64star(oracle_xorshift64star(i) ^ oracle_xorshift64star(v));
}

/* Section V-A, Table I ("Xor Hash"): f is 64-bit xorshift instead.
 * Reading: the paper defines xorshift* as xorshift followed by a linear
 * congruential step, so this xorshift is the first stage of the xorshift*
 * above -- shifts 12, 25, 27 with no multiplication.  (On the 7-point 100^3
 * Laplacian it gives 19 rounds where Table I reports 20; Marsaglia's triple
 * 13, 7, 17 would give 10.) */
uint64_t oracle_xorshift64(uint64_t x)
{
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    return x;
}

/* Priority choices of the Section V-A comparison (Table I), for
 * oracle_mis2_ablation: */
#define ORACLE_PRIO_FIXED    1  /* Bell et al.: priorities drawn once (round 0's hash in every round) */
#define ORACLE_PRIO_XORSHIFT 2  /* f = xorshift instead of xorshift* */

static uint64_t oracle_priority(uint64_t seed, uint64_t iter, uint64_t v, int pflags)
{
    if (pflags & ORACLE_PRIO_FIXED) iter = 0;
    if (pflags & ORACLE_PRIO_XORSHIFT) {
        uint64_t i = (seed << 32) ^ iter;
        return oracle_xorshift64(oracle_xorshift64(i) ^ oracle_xorshift64(v));
    }
    return oracle_hash(seed, iter, v);
}

/* Section V-C, Eq. (1): b = ceil(log2(|V| + 2)), i.e. the smallest integer b
 * with 2^b >= |V| + 2, computed with integers only. */
int oracle_id_bits(int64_t n)
{
    int b = 0;
    while (b < 63 && (INT64_C(1) << b) < n + 2)
        b++;
    return b;
}

/* Section V-C: an undecided tuple is (priority << b) | (id + 1) in 32 bits.
 * Reading: the priority keeps the low 32 - b bits of the hash (the shift in
 * a 32-bit type drops the rest); with b = 32 there are no priority bits. */
uint32_t oracle_pack(uint64_t prio, int64_t v, int b)
{
    int pb = 32 - b;
    uint64_t p = (pb <= 0) ? 0 : (prio & ((UINT64_C(1) << pb) - 1));
    return (uint32_t)((p << b) | (uint64_t)(v + 1));
}

/*
 * Algorithm 1 (Section III-A), optionally on the subgraph induced by the
 * vertices with active[v] != 0 (the second MIS-2 of Alg. 3).
 *
 *   n, row_ptr[n+1], col[nnz]  symmetric CSR without self-loops
 *   active                     NULL = every vertex; else induced subgraph
 *   seed                       hash seed (see oracle_hash)
 *   prio, prio_rounds          NULL = hash priorities; else injected
 *                              priorities prio[r*n + v] for rounds r <
 *                              prio_rounds (used for the Fig. 1 example)
 *   status[n]                  out: 1 if v is IN, else 0
 *   n_iters                    out: loop executions (Table I's count)
 *   trace[cap][4]              out, may be NULL: per round, at its start,
 *                              |wl1|, |wl2|, sum of CSR row lengths over wl1
 *                              and over wl2
 *   T_hist, M_hist, D_hist     out, may be NULL: [cap][n] snapshots of T
 *                              after Refresh Row, M after Refresh Column and
 *                              T after Decide Set
 * Returns 0, -1 on bad arguments, -6 if injected priorities ran out.
 */
static int mis2_core(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const uint8_t *active, uint64_t seed,
                     const uint64_t *prio, int32_t prio_rounds,
                     uint8_t *status, int32_t *n_iters,
                     int64_t *trace, int32_t trace_cap,
                     uint32_t *T_hist, uint32_t *M_hist, uint32_t *D_hist,
                     int32_t hist_cap, int pflags);

int oracle_mis2_ex(int64_t n, const int64_t *row_ptr, const int32_t *col,
                   const uint8_t *active, uint64_t seed,
                   const uint64_t *prio, int32_t prio_rounds,
                   uint8_t *status, int32_t *n_iters,
                   int64_t *trace, int32_t trace_cap,
                   uint32_t *T_hist, uint32_t *M_hist, uint32_t *D_hist,
                   int32_t hist_cap)
{
    return mis2_core(n, row_ptr, col, active, seed, prio, prio_rounds, status, n_iters,
                     trace, trace_cap, T_hist, M_hist, D_hist, hist_cap, 0);
}

/*
 * Algorithm 1 with the priorities of the Section V-A comparison (Table I):
 * pflags = 0 is Algorithm 1 itself, ORACLE_PRIO_FIXED draws the priorities
 * once (Bell et al.), ORACLE_PRIO_XORSHIFT uses xorshift as f.  The other
 * optimizations of Section V (worklists, packed tuples, SIMD) change how
 * much work a round does, not what it computes, so they have no switch here.
 * Outputs as in oracle_mis2_ex.
 */
int oracle_mis2_ablation(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         uint64_t seed, int pflags, uint8_t *status, int32_t *n_iters,
                         int64_t *trace, int32_t trace_cap)
{
    return mis2_core(n, row_ptr, col, NULL, seed, NULL, 0, status, n_iters,
                     trace, trace_cap, NULL, NULL, NULL, 0, pflags);
}

static int mis2_core(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const uint8_t *active, uint64_t seed,
                     const uint64_t *prio, int32_t prio_rounds,
                     uint8_t *status, int32_t *n_iters,
                     int64_t *trace, int32_t trace_cap,
                     uint32_t *T_hist, uint32_t *M_hist, uint32_t *D_hist,
                     int32_t hist_cap, int pflags)
{
    if (n < 0 || (n > 0 && (!row_ptr || !status || !n_iters)))
        return -1;
    if (n == 0) {
        if (n_iters) *n_iters = 0;
        return 0;
    }
    int b = oracle_id_bits(n);
    if (b > 32)
        return -1;

    uint32_t *T = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *M = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    int64_t *wl1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *wl2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!T || !M || !wl1 || !wl2) {
        free(T); free(M); free(wl1); free(wl2);
        return -1;
    }

    /* Alg. 1, set-up: both worklists start as every vertex of the
     * (sub)graph, in increasing id.  Inactive vertices are never touched
     * and count as absent. */
    int64_t n1 = 0, n2 = 0;
    for (int64_t v = 0; v < n; v++) {
        T[v] = ORACLE_OUT;
        M[v] = ORACLE_OUT;
        if (!active || active[v]) {
            wl1[n1++] = v;
            wl2[n2++] = v;
        }
    }

    int32_t iter = 0;
    int rc = 0;
    while (n1 > 0) {
        if (trace && iter < trace_cap) {
            int64_t d1 = 0, d2 = 0;
            for (int64_t i = 0; i < n1; i++) d1 += row_ptr[wl1[i] + 1] - row_ptr[wl1[i]];
            for (int64_t i = 0; i < n2; i++) d2 += row_ptr[wl2[i] + 1] - row_ptr[wl2[i]];
            trace[4 * iter + 0] = n1;
            trace[4 * iter + 1] = n2;
            trace[4 * iter + 2] = d1;
            trace[4 * iter + 3] = d2;
        }

        /* Alg. 1, Refresh Row: every undecided vertex draws this round's
         * hash priority and packs it above its id (Section V-C). */
        if (prio && iter >= prio_rounds) { rc = -6; goto done; }
        ORACLE_PARALLEL_FOR
        for (int64_t i = 0; i < n1; i++) {
            int64_t v = wl1[i];
            uint64_t p;
            if (prio) {
                p = prio[(int64_t)iter * n + v];
            } else {
                p = oracle_priority(seed, (uint64_t)iter, (uint64_t)v, pflags);
            }
            T[v] = oracle_pack(p, v, b);
        }
        if (T_hist && iter < hist_cap)
            memcpy(T_hist + (int64_t)iter * n, T, sizeof(uint32_t) * (size_t)n);

        /* Alg. 1, Refresh Column: each vertex of worklist2 stores the
         * smallest tuple of its closed neighbourhood (itself and its
         * neighbours); when that smallest tuple is IN it stores OUT.
         * Reading: the neighbourhood includes v itself -- Fig. 1 shows
         * M = (1,1) at vertex 1, whose only neighbour carries (3,2). */
        ORACLE_PARALLEL_FOR
        for (int64_t i = 0; i < n2; i++) {
            int64_t v = wl2[i];
            uint32_t m = T[v];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
                int64_t w = col[e];
                if (active && !active[w]) continue;
                if (T[w] < m) m = T[w];
            }
            if (m == ORACLE_IN) m = ORACLE_OUT;
            M[v] = m;
        }
        if (M_hist && iter < hist_cap)
            memcpy(M_hist + (int64_t)iter * n, M, sizeof(uint32_t) * (size_t)n);

        /* Decide Set for v in worklist1, both tests against t0 = T_v as it
         * was after Refresh Row.  Reading: the two ifs are exclusive ("if
         * some M_w is OUT then OUT, else if every M_w equals T_v then IN");
         * for an undecided t0 they cannot both hold.  Decide Set writes only
         * T_v and reads only M, so the order of this loop is immaterial. */
        ORACLE_PARALLEL_FOR
        for (int64_t i = 0; i < n1; i++) {
            int64_t v = wl1[i];
            uint32_t t0 = T[v];
            int any_out = (M[v] == ORACLE_OUT);
            int all_eq = (M[v] == t0);
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
                int64_t w = col[e];
                if (active && !active[w]) continue;
                if (M[w] == ORACLE_OUT) any_out = 1;
                if (M[w] != t0) all_eq = 0;
            }
            if (any_out)
                T[v] = ORACLE_OUT;
            else if (all_eq)
                T[v] = ORACLE_IN;
        }
        if (D_hist && iter < hist_cap)
            memcpy(D_hist + (int64_t)iter * n, T, sizeof(uint32_t) * (size_t)n);

        /* Compact the worklists, keeping their order (a stable filter). */
        int64_t k = 0;
        for (int64_t i = 0; i < n1; i++) {
            int64_t v = wl1[i];
            if (T[v] != ORACLE_IN && T[v] != ORACLE_OUT) wl1[k++] = v;
        }
        n1 = k;
        k = 0;
        for (int64_t i = 0; i < n2; i++) {
            int64_t v = wl2[i];
            if (M[v] != ORACLE_OUT) wl2[k++] = v;
        }
        n2 = k;
        iter++;
    }

    /* The result: the vertices whose tuple ended IN. */
    for (int64_t v = 0; v < n; v++)
        status[v] = (uint8_t)((!active || active[v]) && T[v] == ORACLE_IN);
    *n_iters = iter;

done:
    free(T); free(M); free(wl1); free(wl2);
    return rc;
}

/* Algorithm 1 on the whole graph with hash priorities. */
int oracle_mis2(int64_t n, const int64_t *row_ptr, const int32_t *col,
                uint64_t seed, uint8_t *status, int32_t *n_iters)
{
    return oracle_mis2_ex(n, row_ptr, col, NULL, seed, NULL, 0, status, n_iters,
                          NULL, 0, NULL, NULL, NULL, 0);
}

/*
 * Algorithm 3 (Section III-B): MIS-2 based aggregation.
 *
 *   agg[n]      out: aggregate of every vertex, numbered 0..n_agg-1
 *   n_agg       out
 *   info[8]     out, may be NULL: roots of phase 1, accepted roots of
 *               phase 2, vertices joined in phase 3, rounds of the two
 *               MIS-2 runs, size of the phase-2 MIS-2, vertices left
 *               unaggregated after phase 1, 0
 *   roots[n]    out, may be NULL: 1 = phase-1 root, 2 = accepted phase-2
 *               root, 0 otherwise
 *   trace1/2    out, may be NULL: per-round traces of the two MIS-2 runs
 *               ([cap][4], as in oracle_mis2_ex)
 * Returns 0; -1 on bad arguments; -5 if an invariant the paper guarantees
 * fails (overlapping phase-1 aggregates, or a phase-3 vertex with no
 * aggregated neighbour).
 */
int oracle_aggregate_ex(int64_t n, const int64_t *row_ptr, const int32_t *col,
                        uint64_t seed, int32_t *agg, int64_t *n_agg,
                        int64_t *info, uint8_t *roots,
                        int64_t *trace1, int64_t *trace2, int32_t trace_cap)
{
    if (n < 0 || !n_agg || (n > 0 && (!row_ptr || !agg)))
        return -1;
    if (info) memset(info, 0, 8 * sizeof(int64_t));
    if (n == 0) { *n_agg = 0; return 0; }

    uint8_t *st1 = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *st2 = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *act = (uint8_t *)calloc((size_t)n, 1);
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *label1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *tent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *aggsize = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *coupling = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int rc = 0;
    if (!st1 || !st2 || !act || !label || !label1 || !tent || !aggsize || !coupling) {
        rc = -1;
        goto done;
    }
    for (int64_t v = 0; v < n; v++) label[v] = -1;
    if (roots) memset(roots, 0, (size_t)n);

    /* Alg. 3, first phase: an MIS-2 of the whole graph; every root takes
     * its neighbours into one aggregate.  Reading: roots are numbered in
     * increasing vertex id. */
    int32_t it1 = 0;
    rc = oracle_mis2_ex(n, row_ptr, col, NULL, seed, NULL, 0, st1, &it1,
                        trace1, trace_cap, NULL, NULL, NULL, 0);
    if (rc) goto done;
    int64_t na = 0;
    for (int64_t v = 0; v < n; v++) {
        if (!st1[v]) continue;
        if (label[v] != -1) { rc = -5; goto done; }
        label[v] = (int32_t)na;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int64_t w = col[e];
            if (label[w] != -1) { rc = -5; goto done; }  /* roots are >= 3 apart */
            label[w] = (int32_t)na;
        }
        if (roots) roots[v] = 1;
        na++;
    }
    int64_t n1 = na;

    /* Alg. 3, second phase: an MIS-2 of the subgraph the first phase left
     * unaggregated.  Reading: that subgraph keeps the original vertex ids
     * and the same b, and its round counter starts again at 0. */
    int64_t unagg = 0;
    for (int64_t v = 0; v < n; v++) {
        act[v] = (uint8_t)(label[v] == -1);
        unagg += act[v];
        label1[v] = label[v];
    }
    int32_t it2 = 0;
    rc = oracle_mis2_ex(n, row_ptr, col, act, seed, NULL, 0, st2, &it2,
                        trace2, trace_cap, NULL, NULL, NULL, 0);
    if (rc) goto done;
    int64_t m2 = 0;
    for (int64_t v = 0; v < n; v++) {
        if (!st2[v]) continue;
        m2++;
        /* "v has >= 2 unaggregated neighbours": neighbours u != v that are
         * unlabelled after phase 1. */
        int64_t cnt = 0;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
            if (label1[col[e]] == -1) cnt++;
        if (cnt < 2) continue;
        label[v] = (int32_t)na;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int64_t u = col[e];
            if (label1[u] != -1) continue;
            if (label[u] != -1) { rc = -5; goto done; }
            label[u] = (int32_t)na;
        }
        if (roots) roots[v] = 2;
        na++;
    }
    int64_t n2 = na - n1;

    /* Alg. 3, third phase: the labels are copied and frozen; aggregate
     * sizes and each leftover vertex's coupling to an aggregate are counted
     * on that copy.  A leftover vertex joins the aggregate it shares the
     * most edges with, a tie going to the smaller aggregate.
     * Reading: a remaining tie goes to the smaller aggregate id. */
    for (int64_t v = 0; v < n; v++) {
        tent[v] = label[v];
        if (tent[v] >= 0) aggsize[tent[v]]++;
    }
    int64_t joined = 0;
    for (int64_t v = 0; v < n; v++) {
        if (tent[v] != -1) continue;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t a = tent[col[e]];
            if (a >= 0) coupling[a]++;
        }
        int64_t best = -1;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t a = tent[col[e]];
            if (a < 0) continue;
            if (best < 0 || coupling[a] > coupling[best] ||
                (coupling[a] == coupling[best] &&
                 (aggsize[a] < aggsize[best] ||
                  (aggsize[a] == aggsize[best] && a < best))))
                best = a;
        }
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t a = tent[col[e]];
            if (a >= 0) coupling[a] = 0;
        }
        if (best < 0) { rc = -5; goto done; }
        label[v] = (int32_t)best;
        joined++;
    }

    memcpy(agg, label, sizeof(int32_t) * (size_t)n);
    *n_agg = na;
    if (info) {
        info[0] = n1; info[1] = n2; info[2] = joined;
        info[3] = it1; info[4] = it2; info[5] = m2; info[6] = unagg;
    }

done:
    free(st1); free(st2); free(act); free(label); free(label1); free(tent);
    free(aggsize); free(coupling);
    return rc;
}

int oracle_aggregate(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     uint64_t seed, int32_t *agg, int64_t *n_agg)
{
    return oracle_aggregate_ex(n, row_ptr, col, seed, agg, n_agg, NULL, NULL,
                               NULL, NULL, 0);
}

/* ------------------------------------------------------------------------- */
/* Algorithm 2 (Section III-B): basic MIS-2 coarsening.                       */
/*                                                                           */
/*   agg[n]      out: aggregate of every vertex, numbered 0..n_agg-1          */
/*   n_agg       out: |MIS-2| (every aggregate has one root)                  */
/*   roots[n]    out, may be NULL: 1 = root, 0 otherwise                      */
/*   joined      out, may be NULL: vertices that joined a neighbour's         */
/*               aggregate in the second loop                                 */
/* Each MIS-2 vertex becomes a root, and the root with its neighbours one    */
/* aggregate (roots numbered in increasing vertex id, as in Alg. 3).  Every  */
/* vertex left over then joins the aggregate of a neighbour.                 */
/* Reading: "any neighbour" is the smallest aggregate id among the           */
/* neighbours aggregated by the first loop (the second loop is a parallel    */
/* for, so it reads the first loop's labels, not its own writes).            */
/* Returns 0; -1 on bad arguments; -5 if a leftover vertex has no aggregated */
/* neighbour (maximality of the MIS-2 rules it out).                         */
/* ------------------------------------------------------------------------- */
int oracle_aggregate_basic(int64_t n, const int64_t *row_ptr, const int32_t *col,
                           uint64_t seed, int32_t *agg, int64_t *n_agg,
                           uint8_t *roots, int64_t *joined)
{
    if (n < 0 || !n_agg || (n > 0 && (!row_ptr || !agg)))
        return -1;
    if (joined) *joined = 0;
    if (n == 0) { *n_agg = 0; return 0; }

    uint8_t *st = (uint8_t *)calloc((size_t)n, 1);
    int32_t *first = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int rc = 0;
    if (!st || !first) { rc = -1; goto done; }
    if (roots) memset(roots, 0, (size_t)n);

    /* Alg. 2: an MIS-2 of the whole graph first. */
    int32_t it = 0;
    rc = oracle_mis2_ex(n, row_ptr, col, NULL, seed, NULL, 0, st, &it,
                        NULL, 0, NULL, NULL, NULL, 0);
    if (rc) goto done;

    /* Each root of that set forms an aggregate with its neighbours. */
    for (int64_t v = 0; v < n; v++) first[v] = -1;
    int64_t na = 0;
    for (int64_t v = 0; v < n; v++) {
        if (!st[v]) continue;
        if (first[v] != -1) { rc = -5; goto done; }
        first[v] = (int32_t)na;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int64_t w = col[e];
            if (first[w] != -1) { rc = -5; goto done; }  /* roots are >= 3 apart */
            first[w] = (int32_t)na;
        }
        if (roots) roots[v] = 1;
        na++;
    }

    /* for v in V not aggregated: join the aggregate of a neighbour */
    int64_t nj = 0;
    for (int64_t v = 0; v < n; v++) {
        agg[v] = first[v];
        if (first[v] != -1) continue;
        int32_t best = -1;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t a = first[col[e]];
            if (a >= 0 && (best < 0 || a < best)) best = a;
        }
        if (best < 0) { rc = -5; goto done; }
        agg[v] = best;
        nj++;
    }
    *n_agg = na;
    if (joined) *joined = nj;

done:
    free(st); free(first);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Coarse graph for the next level of a multilevel coarsening.  The paper     */
/* coarsens recursively (Sections I and II) but does not say how the coarse  */
/* graph is formed.  Reading: the quotient graph -- vertices are the          */
/* aggregates, and a and c are adjacent iff some edge (u, v) has agg u = a,   */
/* agg v = c and a != c; no self-loops, no duplicates, columns ascending.     */
/* ------------------------------------------------------------------------- */
typedef struct { int32_t a, c; } oracle_pair;

static int oracle_pair_cmp(const void *x, const void *y)
{
    const oracle_pair *p = (const oracle_pair *)x, *q = (const oracle_pair *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->c != q->c) return p->c < q->c ? -1 : 1;
    return 0;
}

/* crow_ptr[n_agg+1] and ccol[cap] are caller-owned.  Returns the coarse nnz,
 * -1 on bad arguments, -3 if cap is too small. */
int64_t oracle_quotient(int64_t n, const int64_t *row_ptr, const int32_t *col,
                        const int32_t *agg, int64_t n_agg,
                        int64_t *crow_ptr, int32_t *ccol, int64_t cap)
{
    if (n < 0 || n_agg < 0 || !crow_ptr || (n > 0 && (!row_ptr || !agg)))
        return -1;
    int64_t nnz = n > 0 ? row_ptr[n] : 0;
    oracle_pair *p = (oracle_pair *)malloc(sizeof(oracle_pair) * (size_t)(nnz > 0 ? nnz : 1));
    if (!p) return -1;
    int64_t k = 0;
    for (int64_t u = 0; u < n; u++)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            int32_t a = agg[u], c = agg[col[e]];
            if (a < 0 || a >= n_agg || c < 0 || c >= n_agg) { free(p); return -1; }
            if (a != c) { p[k].a = a; p[k].c = c; k++; }
        }
    qsort(p, (size_t)k, sizeof(oracle_pair), oracle_pair_cmp);
    int64_t m = 0;
    for (int64_t i = 0; i < k; i++)
        if (i == 0 || oracle_pair_cmp(&p[i], &p[i - 1]) != 0)
            p[m++] = p[i];
    if (m > cap || (m > 0 && !ccol)) { free(p); return -3; }
    for (int64_t a = 0; a <= n_agg; a++) crow_ptr[a] = 0;
    for (int64_t i = 0; i < m; i++) {
        crow_ptr[p[i].a + 1]++;
        ccol[i] = p[i].c;
    }
    for (int64_t a = 0; a < n_agg; a++) crow_ptr[a + 1] += crow_ptr[a];
    free(p);
    return m;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 4 (Section III-C): cluster multicolor Gauss-Seidel.              */
/*                                                                           */
/* Setup: coarsen the graph (Algorithm 3), take each row's aggregate as its  */
/* cluster, colour the coarse graph, and order the rows by colour, then by   */
/* cluster, then by row: clusters of one colour share no edge, so updating   */
/* them in parallel is the same as updating them one after the other.       */
/* Apply: for each colour in turn, each of its clusters updates its rows in  */
/* order with the Gauss-Seidel step.                                         */
/*                                                                           */
/* Reading (colouring): the paper takes the colouring from other work.  Here  */
/* it is Jones-Plassmann with fixed priorities, the packed tuple of          */
/* h(seed, 0, v) (Sections V-A, V-C): each round every uncoloured vertex     */
/* whose tuple is below those of all its uncoloured neighbours takes the     */
/* smallest colour no coloured neighbour has.                                */
/* Reading (update): the row step of Alg. 4 is the Gauss-Seidel update,     */
/* the new x_i is b_i minus the off-diagonal products A_ij x_j (j != i,      */
/* subtracted in CSR order), divided by A_ii.                                */
/* Reading (order): rows of a cluster in increasing id; clusters of a colour */
/* in increasing id; the symmetric sweep runs the reverse order afterwards   */
/* (colours backward, rows of each cluster backward).                        */
/* ------------------------------------------------------------------------- */

/* Jones-Plassmann colouring.  color[n] out (0-based), *n_colors out.
 * Returns 0, -1 on bad arguments. */
int oracle_color_jp(int64_t n, const int64_t *row_ptr, const int32_t *col, uint64_t seed,
                    int32_t *color, int32_t *n_colors, int32_t *rounds)
{
    if (n < 0 || !n_colors || (n > 0 && (!row_ptr || !color)))
        return -1;
    *n_colors = 0;
    if (rounds) *rounds = 0;
    if (n == 0) return 0;
    int b = oracle_id_bits(n);
    if (b > 32) return -1;
    uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *used = (uint8_t *)calloc((size_t)n + 1, 1);
    if (!pr || !next || !used) { free(pr); free(next); free(used); return -1; }
    for (int64_t v = 0; v < n; v++) {
        pr[v] = oracle_pack(oracle_hash(seed, 0, (uint64_t)v), v, b);
        color[v] = -1;
    }
    int64_t left = n;
    int32_t r = 0, nc = 0;
    while (left > 0) {
        /* decisions of this round read the colours of the round start */
        for (int64_t v = 0; v < n; v++) {
            next[v] = color[v];
            if (color[v] != -1) continue;
            int local_min = 1;
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
                int64_t w = col[e];
                if (color[w] == -1 && pr[w] < pr[v]) local_min = 0;
            }
            if (!local_min) continue;
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
                if (color[col[e]] >= 0) used[color[col[e]]] = 1;
            int32_t c = 0;
            while (used[c]) c++;
            next[v] = c;
            if (c + 1 > nc) nc = c + 1;
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
                if (color[col[e]] >= 0) used[color[col[e]]] = 0;
        }
        for (int64_t v = 0; v < n; v++) {
            if (color[v] == -1 && next[v] != -1) left--;
            color[v] = next[v];
        }
        r++;
    }
    *n_colors = nc;
    if (rounds) *rounds = r;
    free(pr); free(next); free(used);
    return 0;
}

/* The sweep order of Algorithm 4.  point = 0: clusters are the aggregates of
 * Algorithm 3 and the coarse (quotient) graph is coloured; point = 1: every
 * row is its own cluster and the graph itself is coloured (point multicolor
 * Gauss-Seidel).
 *   cluster[n]        out: cluster of each row
 *   cluster_color[n]  out: colour of each cluster (first *n_clusters)
 *   rows[n]           out: rows in sweep order
 *   cluster_off[n+1]  out: the k-th cluster of the sweep order holds
 *                     rows[cluster_off[k] .. cluster_off[k+1])
 *   color_off[n+1]    out: colour c holds the sweep-order clusters
 *                     [color_off[c], color_off[c+1])
 * Returns 0, -1 on bad arguments, -5 if a step fails. */
int oracle_cgs_plan(int64_t n, const int64_t *row_ptr, const int32_t *col, uint64_t seed,
                    int point, int32_t *cluster, int32_t *cluster_color, int32_t *rows,
                    int64_t *cluster_off, int64_t *color_off, int64_t *n_clusters,
                    int32_t *n_colors)
{
    if (n < 0 || !n_clusters || !n_colors ||
        (n > 0 && (!row_ptr || !cluster || !cluster_color || !rows || !cluster_off || !color_off)))
        return -1;
    *n_clusters = 0;
    *n_colors = 0;
    if (n == 0) { if (cluster_off) cluster_off[0] = 0; if (color_off) color_off[0] = 0; return 0; }
    int rc = 0;
    int64_t nc = 0;
    int64_t *crow = NULL;
    int32_t *ccol = NULL;
    int64_t *size = NULL, *start = NULL;
    int64_t nnz = row_ptr[n];
    if (point) {
        for (int64_t v = 0; v < n; v++) cluster[v] = (int32_t)v;
        nc = n;
        rc = oracle_color_jp(n, row_ptr, col, seed, cluster_color, n_colors, NULL);
        if (rc) goto done;
    } else {
        rc = oracle_aggregate(n, row_ptr, col, seed, cluster, &nc);
        if (rc) goto done;
        crow = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
        ccol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        if (!crow || !ccol) { rc = -1; goto done; }
        if (oracle_quotient(n, row_ptr, col, cluster, nc, crow, ccol, nnz) < 0) { rc = -5; goto done; }
        rc = oracle_color_jp(nc, crow, ccol, seed, cluster_color, n_colors, NULL);
        if (rc) goto done;
    }
    *n_clusters = nc;
    /* clusters by colour, then id; rows of a cluster by id */
    size = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
    start = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    if (!size || !start) { rc = -1; goto done; }
    for (int64_t v = 0; v < n; v++) size[cluster[v]]++;
    int64_t k = 0, pos = 0;
    color_off[0] = 0;
    for (int32_t c = 0; c < *n_colors; c++) {
        for (int64_t a = 0; a < nc; a++) {
            if (cluster_color[a] != c) continue;
            cluster_off[k] = pos;
            start[a] = pos;
            pos += size[a];
            k++;
        }
        color_off[c + 1] = k;
    }
    cluster_off[k] = pos;
    for (int64_t v = 0; v < n; v++) rows[start[cluster[v]]++] = (int32_t)v;
done:
    free(crow); free(ccol); free(size); free(start);
    return rc;
}

/* Gauss-Seidel step of row i (see the reading above).  val[nnz] are the
 * off-diagonal entries in CSR order, diag[n] the diagonal. */
static void oracle_gs_row(int64_t i, const int64_t *row_ptr, const int32_t *col,
                          const double *val, const double *diag, const double *b, double *x)
{
    double r = b[i];
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++)
        r -= val[e] * x[col[e]];
    x[i] = r / diag[i];
}

/* sweeps applications of Algorithm 4 to x (in place), forward only or,
 * with symmetric, forward then backward.  The plan is oracle_cgs_plan's. */
int oracle_cgs_apply(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const double *diag, const int32_t *rows, const int64_t *cluster_off,
                     const int64_t *color_off, int32_t n_colors, const double *b, double *x,
                     int32_t sweeps, int symmetric)
{
    if (n < 0 || sweeps < 0 || (n > 0 && (!row_ptr || !diag || !rows || !cluster_off ||
                                          !color_off || !b || !x)))
        return -1;
    for (int32_t s = 0; s < sweeps; s++) {
        for (int32_t c = 0; c < n_colors; c++)
            for (int64_t k = color_off[c]; k < color_off[c + 1]; k++)
                for (int64_t t = cluster_off[k]; t < cluster_off[k + 1]; t++)
                    oracle_gs_row(rows[t], row_ptr, col, val, diag, b, x);
        if (!symmetric) continue;
        for (int32_t c = n_colors - 1; c >= 0; c--)
            for (int64_t k = color_off[c + 1] - 1; k >= color_off[c]; k--)
                for (int64_t t = cluster_off[k + 1] - 1; t >= cluster_off[k]; t--)
                    oracle_gs_row(rows[t], row_ptr, col, val, diag, b, x);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Galerkin coarse operator of an aggregation (a multigrid hookup: Section   */
/* VI-E sets up smoothed-aggregation multigrid on these aggregates).         */
/*                                                                           */
/* Reading: the tentative prolongator for the constant near-null space,      */
/* P[i][a] = 1/sqrt(n_a) when agg(i) = a (n_a = members of a), so that       */
/* P^T P = I, and the coarse operator A_c = P^T A P:                         */
/*   (A_c)[a][b] = (sum of A[i][j] over i in a, j in b) / sqrt(n_a * n_b).   */
/* A is given as the graph's CSR with off-diagonal values val (CSR order)    */
/* and a diagonal diag.  The off-diagonal part of A_c is laid out on the     */
/* quotient graph (rows by aggregate, ascending columns, no self); its       */
/* diagonal gets the fine diagonal and every coupling inside an aggregate.   */
/* Reading (summation order): each sum runs over the fine rows i in         */
/* increasing id, and within row i first diag_i (for the diagonal), then its */
/* entries in CSR order, starting from 0.0; the scaling is one division by   */
/* sqrt((double)n_a * n_b) (the product is exact below 2^53).                */
/* ------------------------------------------------------------------------- */
static int64_t oracle_find_col(const int32_t *c, int64_t lo, int64_t hi, int32_t key)
{
    /* plain binary search: position of key in the ascending c[lo .. hi) */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (c[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

int oracle_galerkin(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                    const double *diag, const int32_t *agg, int64_t n_agg,
                    const int64_t *crow_ptr, const int32_t *ccol, double *cval, double *cdiag)
{
    if (n < 0 || n_agg < 0 || (n > 0 && (!row_ptr || !agg || !diag)) || !crow_ptr ||
        (n_agg > 0 && !cdiag))
        return -1;
    int64_t cnnz = crow_ptr[n_agg];
    if (cnnz > 0 && (!ccol || !cval)) return -1;
    int64_t *size = (int64_t *)calloc((size_t)(n_agg > 0 ? n_agg : 1), sizeof(int64_t));
    if (!size) return -1;
    for (int64_t i = 0; i < n; i++) {
        if (agg[i] < 0 || agg[i] >= n_agg) { free(size); return -2; }
        size[agg[i]]++;
    }
    for (int64_t e = 0; e < cnnz; e++) cval[e] = 0.0;
    for (int64_t a = 0; a < n_agg; a++) cdiag[a] = 0.0;
    for (int64_t i = 0; i < n; i++) {
        int32_t a = agg[i];
        cdiag[a] = cdiag[a] + diag[i];
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            int32_t b = agg[col[e]];
            if (b == a) {
                cdiag[a] = cdiag[a] + val[e];
                continue;
            }
            int64_t p = oracle_find_col(ccol, crow_ptr[a], crow_ptr[a + 1], b);
            if (p >= crow_ptr[a + 1] || ccol[p] != b) { free(size); return -3; }
            cval[p] = cval[p] + val[e];
        }
    }
    for (int64_t a = 0; a < n_agg; a++) {
        for (int64_t p = crow_ptr[a]; p < crow_ptr[a + 1]; p++)
            cval[p] = cval[p] / sqrt((double)size[a] * (double)size[ccol[p]]);
        if (size[a] > 0) cdiag[a] = cdiag[a] / sqrt((double)size[a] * (double)size[a]);
    }
    free(size);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Smoothed aggregation (the multigrid setup of Section VI-E smooths the     */
/* prolongator built on these aggregates; the paper takes the method from    */
/* its multigrid package and prints no formula).                             */
/* Reading: with the tentative prolongator of oracle_galerkin,               */
/* P_tent[i][agg i] = 1/sqrt(n_a), the smoothed prolongator is the damped    */
/* Jacobi step P = (I - omega D^-1 A) P_tent for a given omega (D = the      */
/* diagonal of A), and the coarse operator is P^T A P.  Three sparse         */
/* products, each with a fixed order of operations:                          */
/*   P[i][a]  = (1{a = agg i} - (omega / d_i) * S) / sqrt(n_a), where S is    */
/*              the sum of A_ij over j in N[i] with agg j = a: from 0.0, the  */
/*              diagonal first, then row i's entries in CSR order;            */
/*   AP[i][b] = sum of A_ij * P[j][b] over j in N[i] (i first, then row i's  */
/*              entries in CSR order), from 0.0, absent P[j][b] skipped;      */
/*   Ac[a][b] = sum of P[i][a] * AP[i][b] over the rows i that hold P[i][a],  */
/*              in increasing i, from 0.0, absent AP[i][b] skipped.           */
/* Patterns are structural and columns ascend in every row: P row i = the    */
/* distinct aggregates of N[i]; AP row i = the union of the P rows of N[i];  */
/* Ac row a = the union of the AP rows i with P[i][a] present.               */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t *ptr;   /* [rows + 1] */
    int32_t *col;
    double *val;
    int64_t nnz, cap;
} oracle_csr;

static int oracle_cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return a < b ? -1 : a > b ? 1 : 0;
}

/* Sorts c[0 .. k) and drops repeats; returns the count kept. */
static int64_t oracle_sort_unique(int32_t *c, int64_t k)
{
    if (k <= 1) return k;
    qsort(c, (size_t)k, sizeof(int32_t), oracle_cmp_i32);
    int64_t m = 1;
    for (int64_t t = 1; t < k; t++)
        if (c[t] != c[m - 1]) c[m++] = c[t];
    return m;
}

/* Appends columns c[0 .. k) as the next row of m (values 0.0). */
static int oracle_csr_push(oracle_csr *m, int64_t row, const int32_t *c, int64_t k)
{
    if (m->nnz + k > m->cap) {
        int64_t cap = m->cap * 2 + k + 16;
        int32_t *nc = (int32_t *)realloc(m->col, (size_t)cap * sizeof(int32_t));
        if (!nc) return -1;
        m->col = nc;
        double *nv = (double *)realloc(m->val, (size_t)cap * sizeof(double));
        if (!nv) return -1;
        m->val = nv;
        m->cap = cap;
    }
    for (int64_t t = 0; t < k; t++) {
        m->col[m->nnz + t] = c[t];
        m->val[m->nnz + t] = 0.0;
    }
    m->nnz += k;
    m->ptr[row + 1] = m->nnz;
    return 0;
}

static void oracle_csr_free(oracle_csr *m)
{
    free(m->ptr);
    free(m->col);
    free(m->val);
}

/* Value of (row, c) in m, or NULL when absent. */
static double *oracle_csr_at(const oracle_csr *m, int64_t row, int32_t c)
{
    int64_t p = oracle_find_col(m->col, m->ptr[row], m->ptr[row + 1], c);
    if (p < m->ptr[row + 1] && m->col[p] == c) return &m->val[p];
    return NULL;
}

/* Computes P and Ac (see above).  Outputs (any may be NULL to only count):
 * prow[n+1], pcol / pval[p_cap]; crow[n_agg+1], ccol / cval[c_cap].
 * *p_nnz and *c_nnz receive the entry counts.  Returns 0, -1 (bad
 * argument or memory), -2 (label out of range), -4 (a capacity too small;
 * the counts are still set). */
int oracle_smoothed(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                    const double *diag, const int32_t *agg, int64_t n_agg, double omega,
                    int64_t *prow, int32_t *pcol, double *pval, int64_t p_cap,
                    int64_t *crow, int32_t *ccol, double *cval, int64_t c_cap,
                    int64_t *p_nnz, int64_t *c_nnz)
{
    if (n < 0 || n_agg < 0 || (n > 0 && (!row_ptr || !agg || !diag)) || !p_nnz || !c_nnz)
        return -1;
    int rc = -1;
    int64_t *size = (int64_t *)calloc((size_t)(n_agg > 0 ? n_agg : 1), sizeof(int64_t));
    oracle_csr P = {0}, AP = {0}, C = {0}, R = {0};
    int32_t *buf = NULL;
    int64_t buf_cap = 0;
    if (!size) goto out;
    for (int64_t i = 0; i < n; i++) {
        if (agg[i] < 0 || agg[i] >= n_agg) { rc = -2; goto out; }
        size[agg[i]]++;
    }
    P.ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    AP.ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    C.ptr = (int64_t *)calloc((size_t)n_agg + 1, sizeof(int64_t));
    R.ptr = (int64_t *)calloc((size_t)n_agg + 1, sizeof(int64_t));
    if (!P.ptr || !AP.ptr || !C.ptr || !R.ptr) goto out;
#define ORACLE_BUF(k)                                                            \
    do {                                                                         \
        if ((k) > buf_cap) {                                                     \
            buf_cap = (k) * 2;                                                   \
            int32_t *nb_ = (int32_t *)realloc(buf, (size_t)buf_cap * sizeof(int32_t)); \
            if (!nb_) goto out;                                                  \
            buf = nb_;                                                           \
        }                                                                        \
    } while (0)
    /* P: pattern, then values */
    for (int64_t i = 0; i < n; i++) {
        int64_t k = 0, deg = row_ptr[i + 1] - row_ptr[i];
        ORACLE_BUF(deg + 1);
        buf[k++] = agg[i];
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) buf[k++] = agg[col[e]];
        k = oracle_sort_unique(buf, k);
        if (oracle_csr_push(&P, i, buf, k)) goto out;
    }
    for (int64_t i = 0; i < n; i++) {
        double w = omega / diag[i];
        for (int64_t p = P.ptr[i]; p < P.ptr[i + 1]; p++) {
            int32_t a = P.col[p];
            double s = 0.0;
            if (agg[i] == a) s = s + diag[i];
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++)
                if (agg[col[e]] == a) s = s + val[e];
            double ind = agg[i] == a ? 1.0 : 0.0;
            double t = w * s;
            double r = ind - t;
            P.val[p] = r / sqrt((double)size[a]);
        }
    }
    /* AP = A P */
    for (int64_t i = 0; i < n; i++) {
        int64_t k = 0;
        int64_t need = P.ptr[i + 1] - P.ptr[i];
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++)
            need += P.ptr[col[e] + 1] - P.ptr[col[e]];
        ORACLE_BUF(need + 1);
        for (int64_t p = P.ptr[i]; p < P.ptr[i + 1]; p++) buf[k++] = P.col[p];
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++)
            for (int64_t p = P.ptr[col[e]]; p < P.ptr[col[e] + 1]; p++) buf[k++] = P.col[p];
        k = oracle_sort_unique(buf, k);
        if (oracle_csr_push(&AP, i, buf, k)) goto out;
    }
    for (int64_t i = 0; i < n; i++) {
        for (int64_t q = AP.ptr[i]; q < AP.ptr[i + 1]; q++) {
            int32_t b = AP.col[q];
            double acc = 0.0;
            double *pib = oracle_csr_at(&P, i, b);
            if (pib) acc = acc + diag[i] * *pib;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
                double *pjb = oracle_csr_at(&P, col[e], b);
                if (pjb) acc = acc + val[e] * *pjb;
            }
            AP.val[q] = acc;
        }
    }
    /* R: for each aggregate a, the rows i holding P[i][a], increasing i */
    for (int64_t i = 0; i < n; i++)
        for (int64_t p = P.ptr[i]; p < P.ptr[i + 1]; p++) R.ptr[P.col[p] + 1]++;
    for (int64_t a = 0; a < n_agg; a++) R.ptr[a + 1] += R.ptr[a];
    R.nnz = R.ptr[n_agg];
    R.col = (int32_t *)malloc((size_t)(R.nnz > 0 ? R.nnz : 1) * sizeof(int32_t));
    if (!R.col) goto out;
    {
        int64_t *fill = (int64_t *)malloc((size_t)(n_agg > 0 ? n_agg : 1) * sizeof(int64_t));
        if (!fill) goto out;
        for (int64_t a = 0; a < n_agg; a++) fill[a] = R.ptr[a];
        for (int64_t i = 0; i < n; i++)
            for (int64_t p = P.ptr[i]; p < P.ptr[i + 1]; p++) R.col[fill[P.col[p]]++] = (int32_t)i;
        free(fill);
    }
    /* Ac = P^T AP */
    for (int64_t a = 0; a < n_agg; a++) {
        int64_t k = 0, need = 0;
        for (int64_t t = R.ptr[a]; t < R.ptr[a + 1]; t++)
            need += AP.ptr[R.col[t] + 1] - AP.ptr[R.col[t]];
        ORACLE_BUF(need + 1);
        for (int64_t t = R.ptr[a]; t < R.ptr[a + 1]; t++)
            for (int64_t q = AP.ptr[R.col[t]]; q < AP.ptr[R.col[t] + 1]; q++) buf[k++] = AP.col[q];
        k = oracle_sort_unique(buf, k);
        if (oracle_csr_push(&C, a, buf, k)) goto out;
    }
    for (int64_t a = 0; a < n_agg; a++) {
        for (int64_t q = C.ptr[a]; q < C.ptr[a + 1]; q++) {
            int32_t b = C.col[q];
            double acc = 0.0;
            for (int64_t t = R.ptr[a]; t < R.ptr[a + 1]; t++) {
                int64_t i = R.col[t];
                double *apb = oracle_csr_at(&AP, i, b);
                if (apb) acc = acc + *oracle_csr_at(&P, i, (int32_t)a) * *apb;
            }
            C.val[q] = acc;
        }
    }
#undef ORACLE_BUF
    *p_nnz = P.nnz;
    *c_nnz = C.nnz;
    rc = 0;
    if ((prow || pcol || pval) && (!prow || P.nnz > p_cap || (P.nnz > 0 && (!pcol || !pval))))
        rc = -4;
    if ((crow || ccol || cval) && (!crow || C.nnz > c_cap || (C.nnz > 0 && (!ccol || !cval))))
        rc = -4;
    if (rc == 0 && prow) {
        memcpy(prow, P.ptr, ((size_t)n + 1) * sizeof(int64_t));
        if (P.nnz > 0) {
            memcpy(pcol, P.col, (size_t)P.nnz * sizeof(int32_t));
            memcpy(pval, P.val, (size_t)P.nnz * sizeof(double));
        }
    }
    if (rc == 0 && crow) {
        memcpy(crow, C.ptr, ((size_t)n_agg + 1) * sizeof(int64_t));
        if (C.nnz > 0) {
            memcpy(ccol, C.col, (size_t)C.nnz * sizeof(int32_t));
            memcpy(cval, C.val, (size_t)C.nnz * sizeof(double));
        }
    }
out:
    free(size);
    free(buf);
    oracle_csr_free(&P);
    oracle_csr_free(&AP);
    oracle_csr_free(&C);
    oracle_csr_free(&R);
    return rc;
}
