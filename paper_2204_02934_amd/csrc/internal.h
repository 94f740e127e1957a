// internal.h -- shared declarations of the gfx950 MIS-2 library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "mis2.h"

namespace mis2 {

// Packed status values (Section V-C): IN = 0 < undecided tuples < OUT = UINT_MAX.
constexpr uint32_t kIn = 0u;
constexpr uint32_t kOut = 0xFFFFFFFFu;
// M value of a vertex outside the induced subgraph of a masked run.  A real
// M is never 0 because Refresh Column turns an IN minimum into OUT, so the
// value can mark "absent" without a separate mask array.
constexpr uint32_t kAbsent = 0u;

constexpr int kBlock = 256;       // threads per workgroup (4 wave64s)
constexpr int kTraceCap = 4096;   // most rounds of one MIS-2 run
constexpr int kRing = 4;          // per-round counter slots, slot = round % kRing
constexpr int kScalars = 64;      // misc device scalars
// Round table: row r holds the size of worklist1 (word 0) and worklist2
// (word 1) at the start of round r and, for the persistent kernel, device
// wall-clock stamps (two words each) taken by workgroup 0 at the start of
// round r and after its two grid barriers.
constexpr int kRoundStride = 8;
constexpr int kRtStamp0 = 2, kRtStamp1 = 4, kRtStamp2 = 6;
// Size counters.  The sweeps of round r add each workgroup's kept count to
// one of kSplit counters per list, each in its own 128-byte line (atomics on
// one line serialise across the whole chip), in ring slot (r + 1) % kRing.
// A slot holds worklist1's counters, then worklist2's.
constexpr int kSplit = 64;
constexpr int kCtrLine = 32;                     // words per counter (one cache line)
constexpr int kCtrList = kSplit * kCtrLine;      // words per list of a slot
constexpr int kCtrSlot = 2 * kCtrList;           // words per slot
constexpr int kCtrRing = 4;                      // slots

// Section V-A: f = xorshift64* (Vigna's parameters 12, 25, 27 and multiplier
// 2685821657736338717, arithmetic mod 2^64); h(i, v) = f(f(i) ^ f(v)).
__host__ __device__ __forceinline__ uint64_t xs64star(uint64_t x) {
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    return x * 0x2545F4914F6CDD1Dull;
}

// Graphs of a batch: graph g owns the union's vertex ids [voff[g], voff[g+1]);
// its tuples use graph-local ids and the graph's own id width gb[g], so a
// batch computes exactly what each graph computes alone (there are no edges
// between graphs).  voff == nullptr means a single graph.
struct BatchInfo {
    const int64_t *voff = nullptr;  // device [G + 1]
    const uint32_t *gb = nullptr;   // device [G]
    const int32_t *gid = nullptr;   // device [n]: graph of each union vertex (or null)
    int32_t G = 0;
    int32_t steps = 0;              // binary-search steps, ceil(log2(G + 1))
};

// What a kernel needs to build the packed tuple of one round.
struct TupleParams {
    uint64_t f_iter;  // f((seed << 32) ^ iter): the per-round half of h
    uint64_t pmask;   // 2^(32-b) - 1, or 0 when b = 32
    uint32_t b;       // id bits, the smallest b with 2^b >= n + 2
    BatchInfo batch;
};

// Graph of union vertex v: one load from the per-vertex table when there is
// one, else a binary search (fixed trip count, the same in every lane).
__device__ __forceinline__ int32_t graph_of(const BatchInfo &bt, int64_t v) {
    if (bt.gid) return bt.gid[v];
    int32_t lo = 0, hi = bt.G;
    for (int k = 0; k < bt.steps; k++) {
        const int32_t mid = (lo + hi) >> 1;
        if (bt.voff[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// Section V-C: (priority << b) | (v + 1); the priority keeps the low 32 - b
// bits of h.
__device__ __forceinline__ uint32_t make_tuple(const TupleParams &p, uint32_t v) {
    uint64_t l = v, pmask = p.pmask;
    uint32_t b = p.b;
    if (p.batch.voff) {
        const int32_t g = graph_of(p.batch, v);
        l = (uint64_t)((int64_t)v - p.batch.voff[g]);
        b = p.batch.gb[g];
        pmask = b >= 32 ? 0ull : ((1ull << (32 - b)) - 1ull);
    }
    const uint64_t h = xs64star(p.f_iter ^ xs64star(l));
    return (uint32_t)(((h & pmask) << b) | (l + 1u));
}

int id_bits(int64_t n);
TupleParams tuple_params(int64_t n, uint64_t seed, uint64_t iter);

// Scalar slots in Workspace::scalars.
enum Scalar {
    kS_Roots = 0,   // |MIS-2| of mis2_run
    kS_Count1 = 1,  // phase-1 root count (aggregation)
    kS_Count2 = 3,  // accepted phase-2 roots
    kS_Err = 5,     // error bits
};

// Accounting sums per round: Decide Set's row lengths, Refresh Column's,
// and the column indices Refresh Column wrote into compacted rows.
constexpr int kDegStride = 4;

constexpr int kMaxBlocks = 8192;              // most workgroups of a sweep grid
constexpr int kMaxWaves = kMaxBlocks * (kBlock / 64);

// The caller's workspace, carved into arrays (all 256-byte aligned).
struct Workspace {
    uint32_t *T = nullptr;        // [n] packed row status tuples
    uint32_t *M = nullptr;        // [n] radius-1 minima
    uint8_t *near = nullptr;      // [n] 1: within distance 2 of an IN vertex of round 0 (k_push_near)
    int32_t *wl1[2] = {};         // [n] undecided vertices (per-wave segments), double buffered
    int32_t *wl2[2] = {};         // [n] vertices without an IN neighbour, double buffered
    uint32_t *cnt1[2] = {};       // [kMaxWaves] per-wave sizes of wl1[i]
    uint32_t *cnt2[2] = {};       // [kMaxWaves] per-wave sizes of wl2[i]
    uint32_t *rt = nullptr;       // [kTraceCap + 2][kRoundStride] round table
    uint32_t *ctr = nullptr;      // [kCtrRing][kCtrSlot] size counters
    uint32_t *scalars = nullptr;  // [kScalars]
    unsigned long long *degs = nullptr;  // [2][kTraceCap][kDegStride] row-length sums per sweep
    unsigned long long *dsplit = nullptr;  // [2][kSplit][16] their partial sums in flight
    uint32_t *blocksum = nullptr; // [compact_blocks(n) + 1]
    uint32_t *bar = nullptr;      // [kBarWords] persistent-kernel barrier state
    // compacted adjacency of Refresh Column (both null: none), from a
    // workspace tail or from buffers the caller is not using during the call
    int32_t *colc = nullptr;      // [nnz]
    int32_t *lenc = nullptr;      // [n]
    uint32_t *lflag = nullptr;    // [kSplit * kCtrLine] long-row flags of round 0
    // aggregation only
    int32_t *label = nullptr;     // [n] aggregate labels, -1 = none
    int32_t *list = nullptr;      // [n] ordered vertex lists
    uint8_t *flag = nullptr;      // [n]
    int32_t *aggsize = nullptr;   // [n]
    // coarsening only
    struct {
        uint32_t *cnt = nullptr;
        int64_t *moff = nullptr;
        int32_t *members = nullptr;
        unsigned long long *part = nullptr;
        int32_t *big = nullptr;
        uint32_t *big_count = nullptr;
        uint32_t *gbits = nullptr;   // [kGiantSlots * giant_words(n)]
        uint32_t *gmeta = nullptr;   // [kGiantMeta]
        uint8_t *cls = nullptr;      // [n] which pass handles each coarse row
    } q;
};

size_t workspace_bytes(int64_t n, int op);
// Extra bytes for the compacted adjacency of Refresh Column (colc, lenc).
size_t compact_bytes(int64_t n, int64_t nnz);
bool carve(void *base, size_t bytes, int64_t n, int op, Workspace *ws);

// Launch-plan knobs; never change results.
// Plan value of the staged sweeps (one row per lane, each row's column
// indices staged in LDS by 16-byte loads); the template argument L of the
// sweep kernels takes it too.
constexpr int kStagedLanes = 128;

// Lanes per row of the group kernels that have no staged form (Algorithm 2's
// join, phase 3 of Algorithm 3): 4 in place of the staged plan.
__host__ __device__ constexpr int group_lanes(int lanes) {
    return lanes == kStagedLanes ? 4 : lanes;
}

// Class of a graph for the plan tuner: its size (half octaves of n) and
// degree histogram (the share of rows in each bin of deg_bin, in sixteenths,
// and the bin of the largest degree).
struct GraphClass {
    int32_t size_bucket = 0;
    uint8_t share[9] = {};
    int32_t max_bin = 0;
    bool operator==(const GraphClass &o) const {
        if (size_bucket != o.size_bucket || max_bin != o.max_bin) return false;
        for (int k = 0; k < 9; k++)
            if (share[k] != o.share[k]) return false;
        return true;
    }
};

struct Plan {
    int lanes = 0;       // lanes per CSR row (power of two <= 64, or kStagedLanes); 0 = automatic
    int blocks = 0;      // workgroups per sweep (<= kMaxBlocks); 0 = automatic
    int persistent = 0;  // 1: one cooperative launch per MIS-2 run; 0: two launches per round
    int compact = 1;     // 1: Refresh Column skips OUT neighbours when the workspace has room
    int tail = -1;       // 1: the last rounds (worklists of < kTailCap) run in one workgroup;
                         // 0: never; -1: as the plan tuner finds (off untuned)
    int ahead = 0;       // rounds queued beyond the running one (0: 2)
};

// One sweep's worklists.  Wavefront w owns slots [w*seg, w*seg + cnt[w]) of
// each list.  cnt_in == nullptr means the identity lists (w's whole vertex
// range).  trace_out (may be null) points at the kSplit counters (stride
// kCtrLine) whose sum becomes the output size; deg_sum (may be null)
// accumulates the visited CSR row lengths.
struct SegIO {
    const int32_t *wl_in;
    const uint32_t *cnt_in;
    int32_t *wl_out;
    uint32_t *cnt_out;
    uint32_t *trace_out;
    unsigned long long *deg_sum;
    int64_t n;
    int64_t seg;
    int64_t S;
    // Refresh Column only.  Compacted adjacency: the row of v keeps, at
    // [row_ptr[v], row_ptr[v] + len[v]), the column indices whose T was not
    // OUT when the row was last swept.  ccol_in / lenc_in (both null: read
    // the CSR's own rows) are the rows to read; ccol_out / lenc_out (null: no
    // writes) receive the kept rows' compacted form (the same arrays: a row
    // is rewritten in place by the lane group that reads it).
    const int32_t *ccol_in;
    const int32_t *lenc_in;
    int32_t *ccol_out;
    int32_t *lenc_out;
    // Refresh Column of round 0 (unmasked): a wavefront that meets a row
    // longer than the cooperative threshold sets one of kSplit flags
    // (stride kCtrLine), or null.
    uint32_t *long_flag;
    int64_t nnz;  // entries of the CSR (the staged sweeps' 16-byte loads stay below it)
    // Refresh Column of rounds 0 and 1 of an unmasked run on one graph: a
    // neighbour's tuple is computed, make_tuple(t0, u), instead of gathered
    // from T.  gen0 1 (round 0): every tuple is still that.  2 (round 1):
    // round 0's Decide Set made no vertex OUT, and every IN vertex has set M
    // to OUT on itself and its neighbours since (k_push_in); a row with M
    // OUT keeps M OUT, any other has no IN neighbour, so all its
    // neighbours' tuples are round 1's function of the id.
    int gen0;
    TupleParams t0;
    // Decide Set of round 0: no vertex is IN yet, so no M is OUT and a row
    // whose own M differs from its tuple stays undecided without reading its
    // neighbours (dec0 true).
    bool dec0;
    // Decide Set of round 1 after k_push_near (dec1 true): a neighbour's M is
    // OUT exactly when an IN vertex of round 0 lies within distance 2, which
    // near[v] records, so a row whose own M differs from its tuple (it
    // cannot join) reads near[v] instead of its neighbours.
    bool dec1;
    const uint8_t *near;
};

// Arguments of the persistent round kernel.  bar: [kMaxBlocks] per-workgroup
// epoch flags, then the published epoch at [kMaxBlocks], the abort word at
// [kMaxBlocks + 16] and the executed round count at [kMaxBlocks + 32]; all
// zero before the launch.
constexpr int kBarWords = kMaxBlocks + 64;
// Also the arguments of the launched round kernels (k_col_round /
// k_dec_round, which take the round number as a second argument).
// alive_host (may be null): host-pinned word where workgroup 0 of every
// Refresh Column stores (epoch << 48) | (round << 32) | |worklist1| at the
// start of its round (and word 1 the same with |worklist2|).  The epoch tells
// the host's poll of one run from the late rounds of the run before it,
// which may still be starting when the next run resets the words.
struct RoundsArgs {
    BatchInfo batch;
    int32_t *wl1[2];
    int32_t *wl2[2];
    uint32_t *cnt1[2];
    uint32_t *cnt2[2];
    uint32_t *rt;
    uint32_t *rt_host;   // host-pinned copy of the round table rows (may be null)
    uint32_t *ctr;
    unsigned long long *alive_host;
    uint32_t epoch;            // 1 .. kEpochMax, a new one per run of rounds
    unsigned long long *degs;  // [kTraceCap][kDegStride] or null
    unsigned long long *dsplit;  // [2][kSplit][16] partial row-length sums, or null
    uint32_t *bar;
    int32_t *colc;   // [nnz] compacted rows, or null (no compaction)
    int32_t *lenc;   // [n] their lengths
    uint32_t *lflag; // [kSplit][kCtrLine] set by round 0 when a row is long (zero at the start)
    int abl;         // ablation kernels only: kAblFixed | kAblXorshift
    int gen0;        // 1: rounds 0 and 1 of Refresh Column may compute the tuples they gather
    uint8_t *near;   // Workspace::near
    int64_t n, seg, S;
    int64_t nnz;
    uint64_t seed, pmask;
    uint32_t b;
    int masked;
    int max_rounds;
};

// Refresh Column drops OUT neighbours from the long rows it keeps from this
// round on (unmasked runs): no vertex is OUT before round 0's Decide Set and
// few are before round 1's, so earlier rewrites would copy nearly whole
// rows.  A masked run starts with every absent vertex OUT and compacts from
// round 0.
constexpr int kCompactFrom = 2;
// Priority choices of the ablation kernels (Section V-A, Table I).
constexpr int kAblFixed = 1;     // priorities drawn once (Bell et al.)
constexpr int kAblXorshift = 2;  // f = xorshift (xorshift*'s first stage)

// Tuples of the ablation kernels: packed (s only, as T / M) or three
// fields (status, priority, id) in three arrays.
struct AblTuples {
    uint32_t *s = nullptr;
    uint32_t *p = nullptr;
    uint32_t *i = nullptr;
};

// Bit of the host-reported |worklist1| word that says round 0 met rows long
// enough for the cooperative pass (|worklist1| < 2^31 always).
constexpr uint32_t kLongRowsBit = 0x80000000u;
constexpr uint32_t kEpochMax = 0x7FFFu;  // epochs in the top 16 bits of a host word
// A host word: epoch, round and a 32-bit value.
__host__ __device__ inline unsigned long long host_word(uint32_t epoch, int round, uint32_t value) {
    return ((unsigned long long)epoch << 48) | ((unsigned long long)((uint32_t)round & 0xFFFFu) << 32) |
           value;
}

// mis2_kernels.hip
// Degree histogram of the plan tuner: kHistBlocks partial rows of kHistWords
// (kDegBins row counts, then the largest degree) at part.
constexpr int kDegBins = 9;
constexpr int kHistWords = kDegBins + 1;
constexpr int kHistBlocks = 64;
hipError_t launch_degree_hist(int64_t n, const int64_t *row_ptr, unsigned long long *part,
                              hipStream_t s);
int rounds_max_blocks(int lanes, int num_cus);
// Workgroups of a sweep grid that are resident at once (staged sweeps only; 0 otherwise).
int sweep_resident_blocks(int lanes, int num_cus);
// The last rounds of a run in one workgroup, from round r0 with both
// worklists of at most kTailCap vertices (see k_tail).  cstart: first
// compacting round (< 0: none); thr: the plan's cooperative threshold;
// rt_host: this phase's host-pinned round table; end_host receives the
// rounds of the run plus one.
constexpr int kTailCap = 4096;
hipError_t launch_tail(const int64_t *row_ptr, const int32_t *col, uint32_t *T, uint32_t *M,
                       const RoundsArgs &a, int r0, int cstart, int64_t thr, uint32_t *rt_host,
                       unsigned long long *end_host, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
// Rows longer than this go to the whole wavefront in the sweeps of `lanes`
// (and only they are compacted).
int64_t coop_threshold(int lanes);
hipError_t launch_rounds(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                         uint32_t *T, uint32_t *M, const RoundsArgs &a, hipStream_t s);
// e0 / e1 (may be null): events stamped by the launch itself at the kernel's
// start and end.
// smoothed.hip: smoothed aggregation.  kind 0: P rows (sources N[i], one
// aggregate each), 1: AP rows (P rows of N[i]), 2: coarse rows (AP rows of
// the rows holding P[i][a]); count pass (fill == false) writes count[r] and
// sets *err |= 1 for a row of more than 2048 distinct columns; fill pass
// writes the ascending columns at out_ptr[r].
hipError_t launch_smoothed_sym(int kind, bool fill, int64_t rows, const int64_t *row_ptr,
                               const int32_t *col, const int32_t *agg, const int64_t *sptr,
                               const int32_t *scol, const int64_t *moff, const int32_t *members,
                               const int32_t *prow_of, uint32_t *count, const int64_t *out_ptr,
                               int32_t *out_col, uint32_t *err, uint8_t *cls, hipStream_t s);
hipError_t launch_p_values(int64_t n, int64_t p_nnz, const int64_t *row_ptr, const int32_t *col,
                           const double *val, const double *diag, const int32_t *agg,
                           const uint32_t *size, double omega, const int64_t *prow,
                           const int32_t *pcol, double *pval, int32_t *prow_of, hipStream_t s);
hipError_t launch_ap_values(int64_t n, int64_t ap_nnz, const int64_t *row_ptr, const int32_t *col,
                            const double *val, const double *diag, const int64_t *prow,
                            const int32_t *pcol, const double *pval, const int64_t *aptr,
                            const int32_t *acol, double *aval, hipStream_t s);
hipError_t launch_c_values(int64_t n_agg, int64_t c_nnz, const int64_t *moff,
                           const int32_t *members, const int32_t *prow_of, const double *pval,
                           const int64_t *aptr, const int32_t *acol, const double *aval,
                           const int64_t *crow, const int32_t *ccol, double *cval, hipStream_t s);
// cgs.hip: Algorithm 4 (cluster multicolor Gauss-Seidel).
hipError_t launch_jp_init(int64_t n, const TupleParams &tp, uint32_t *pr, int32_t *cround,
                          int32_t *color, hipStream_t s);
hipError_t launch_jp_round(int64_t n, const int64_t *row_ptr, const int32_t *col,
                           const uint32_t *pr, int32_t *cround, int32_t *color, int r,
                           uint32_t *d_left, uint32_t *d_maxc, hipStream_t s);
hipError_t launch_iota(int64_t n, int32_t *out, hipStream_t s);
hipError_t launch_count_of(int64_t n, const int32_t *key, uint32_t *cnt, hipStream_t s);
hipError_t launch_color_hist(int64_t n, const int32_t *color, int32_t n_colors, uint32_t *hist,
                             hipStream_t s);
// members[moff[a] .. moff[a+1]) = the rows of cluster a in increasing id
// (cursor zero on entry).
hipError_t launch_sorted_members(int64_t n, const int32_t *cluster, int64_t nc,
                                 const int64_t *moff, uint32_t *cursor, int32_t *members,
                                 hipStream_t s);
hipError_t launch_gather_sizes(int64_t nk, const int32_t *order, const uint32_t *cnt,
                               uint32_t *out, hipStream_t s);
hipError_t launch_place_rows(int64_t nk, const int32_t *order, const int64_t *moff,
                             const int32_t *members, const int64_t *cluster_off, int32_t *rows,
                             hipStream_t s);
hipError_t launch_scatter_pos(int64_t n, const int32_t *rows, int32_t *pos, hipStream_t s);
// galerkin.hip: *flag |= 1 (an aggregate id outside [0, n_agg)), 2 (a coarse
// column outside it), 4 (a coupling missing from the coarse graph).
hipError_t launch_check_ids(int64_t n, const int32_t *agg, int64_t cnnz, const int32_t *ccol,
                            int64_t n_agg, uint32_t *flag, hipStream_t s);
hipError_t launch_galerkin(const int64_t *row_ptr, const int32_t *col, const double *val,
                           const double *diag, const int32_t *agg, int64_t n_agg,
                           const int64_t *moff, const int32_t *members, const int64_t *crow,
                           const int32_t *ccol, double *cval, double *cdiag, uint32_t *flag,
                           int64_t nnz, hipStream_t s);
hipError_t launch_cgs_sweep(const int64_t *row_ptr, const int32_t *col, const double *val,
                            const double *diag, const double *b, double *x, const int32_t *rows,
                            const int32_t *pos, const int64_t *cluster_off, int64_t k0, int64_t k1,
                            bool backward, hipStream_t s);
hipError_t launch_cgs_point(const int64_t *row_ptr, const int32_t *col, const double *val,
                            const double *diag, const double *b, double *x, const int32_t *rows,
                            int64_t t0, int64_t t1, hipStream_t s);

// Ablation kernels (one lane per row): round 0's tuples, and the Refresh
// Column (kind 0) / Decide Set (kind 1) of round r; e0 / e1 (may be null)
// are recorded around the launch.
hipError_t launch_abl_init(bool unpacked, const AblTuples &t, const RoundsArgs &a, hipStream_t s);
hipError_t launch_abl_round(int kind, bool unpacked, bool all, int blocks,
                            const int64_t *row_ptr, const int32_t *col, const AblTuples &T,
                            const AblTuples &M, const RoundsArgs &a, int r, hipStream_t s,
                            hipEvent_t e0, hipEvent_t e1);
// mode: 0 plain, 1 write compacted rows from the CSR's, 2 read and rewrite
// them (1 and 2 need lanes > 0 and a.colc / a.lenc).
hipError_t launch_col_round(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                            const uint32_t *T, uint32_t *M, const RoundsArgs &a, int r, int mode,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1);
// M = OUT on every IN vertex of T and on its neighbours (after round 0's
// Decide Set, for round 1's computed tuples).
hipError_t launch_push_in(int64_t n, const int64_t *row_ptr, const int32_t *col, const uint32_t *T,
                          uint32_t *M, hipStream_t s);
// near = 1 on every vertex whose M is OUT (after launch_push_in: the IN
// vertices of round 0 and their neighbours) and on its neighbours.
hipError_t launch_push_near(int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const uint32_t *M, uint8_t *near, hipStream_t s);
hipError_t launch_dec_round(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                            uint32_t *T, const uint32_t *M, const RoundsArgs &a, int r,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1);
int64_t status_blocks(int64_t n);
hipError_t launch_status(int64_t n, const uint32_t *T, uint8_t *status, uint32_t *blocksum,
                         uint32_t *d_total, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s);
// up to kFillSpans fills of 32-bit words (p[k][0 .. n[k]) = v[k]) in one launch
constexpr int kFillSpans = 4;
struct FillSpans {
    uint32_t *p[kFillSpans];
    uint32_t v[kFillSpans];
    int64_t n[kFillSpans];
    int k = 0;
    void add(uint32_t *ptr, uint32_t value, int64_t count) {
        if (count <= 0) return;
        p[k] = ptr;
        v[k] = value;
        n[k] = count;
        k++;
    }
};
hipError_t launch_fill_spans(const FillSpans &f, hipStream_t s);
// The fills of f (p[k][0 .. n[k]) = v[k]), spread over the launch's grid of
// kBlock-thread workgroups; for kernels that carry fills beside their work.
__device__ __forceinline__ void fill_span_words(const FillSpans &f) {
    int64_t total = 0;
    for (int k = 0; k < f.k; k++) total += f.n[k];
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * kBlock) {
        int64_t o = t;
        int k = 0;  // the span of word t (a fixed trip count: no early exit)
        for (int q = 0; q + 1 < kFillSpans; q++)
            if (k == q && q + 1 < f.k && o >= f.n[q]) {
                o -= f.n[q];
                k = q + 1;
            }
        f.p[k][o] = f.v[k];
    }
}
// Round-0 tuples (T), then the fills f, in one launch.
hipError_t launch_init_tuples(const TupleParams &tp, int64_t n, uint32_t *T, const FillSpans &f,
                              hipStream_t s);
// Induced-subgraph start (T, M, both round-0 worklists into io) and the fills
// f, in one launch.
hipError_t launch_init_masked(int blocks, const TupleParams &tp, int64_t n, const int32_t *label,
                              uint32_t *T, uint32_t *M, const SegIO &io, const FillSpans &f,
                              hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t count, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint8_t value, int64_t count, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long value, int64_t count,
                           hipStream_t s);
hipError_t launch_validate(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                           uint32_t *err, hipStream_t s);

// compact.hip: out = [v : pred(v)] in increasing v, size -> *d_count.
// blocksum needs compact_blocks(n) + 1 entries.
constexpr int kCompactTile = 2048;  // vertices per compaction tile
int64_t compact_blocks(int64_t n);
// Phase 1's start: the fills f, zero_u8[0 .. n) = 0 (when not null), and the
// per-tile counts of T == IN into blocksum, in one launch.
hipError_t count_in_with_fills(const uint32_t *T, int64_t n, const FillSpans &f, uint8_t *zero_u8,
                               uint32_t *blocksum, hipStream_t s);
// The rest of an ordered compaction whose per-tile counts are in blocksum:
// out = the indices i with a[i] == value (or a8[i] != 0), in increasing
// order, *d_count = how many.  One launch up to kOnePassTiles tiles (each
// workgroup sums the counts of the tiles before it), else scan and scatter.
hipError_t scatter_counted_u32_eq(const uint32_t *a, uint32_t value, int64_t n, int32_t *out,
                                  uint32_t *d_count, uint32_t *blocksum, hipStream_t s);
hipError_t scatter_counted_u8_nz(const uint8_t *a8, int64_t n, int32_t *out, uint32_t *d_count,
                                 uint32_t *blocksum, hipStream_t s);
// Per-tile counts of a8[i] != 0 into blocksum (plain stores, every tile).
hipError_t count_u8_nz(const uint8_t *a8, int64_t n, uint32_t *blocksum, hipStream_t s);
hipError_t compact_u32_eq(const uint32_t *a, uint32_t value, int64_t n, int32_t *out,
                          uint32_t *d_count, uint32_t *blocksum, hipStream_t s);
hipError_t compact_u8_nz(const uint8_t *a, int64_t n, int32_t *out, uint32_t *d_count,
                         uint32_t *blocksum, hipStream_t s);
// Exclusive prefix sum of n u32 values into int64 out[0..n]; part needs
// scan_parts(n) entries.
int64_t scan_parts(int64_t n);
hipError_t exclusive_scan_u32_i64(const uint32_t *in, int64_t n, int64_t *out,
                                  unsigned long long *part, hipStream_t s);
// Exclusive scan of blocksum[0..nb) in place; total -> blocksum[nb], *d_total.
hipError_t launch_scan_tiles(uint32_t *blocksum, int64_t nb, uint32_t *d_total, hipStream_t s);

// quotient.hip: coarse graph of an aggregation.
// Coarse rows with more than kGiantCand candidates take one of kGiantSlots
// bitmap slots (a bit per coarse id) filled by the whole grid.
constexpr int kGiantSlots = 8;
constexpr int64_t kGiantCand = 65536;
constexpr int kGiantMeta = 3 * kGiantSlots + 1;  // rows, smallest and largest ids, count
inline size_t giant_words(int64_t n) { return (size_t)((n + 31) / 32); }
struct QuotientWs {
    uint32_t *cnt;              // [n_agg] member / row counts
    int64_t *moff;              // [n_agg + 1] member offsets
    int32_t *members;           // [n]
    unsigned long long *part;   // [scan_parts(n)]
    int32_t *big;               // [n_agg] coarse rows left to whole workgroups
    uint32_t *big_count;        // [1]
    uint32_t *gbits;            // [kGiantSlots * giant_words(n_agg)] bitmaps of giant rows
    uint32_t *gmeta;            // [kGiantMeta]
    uint8_t *cls;               // [n_agg] the pass of each coarse row (small, middle, large)
};
// nnz: stored entries of the fine graph (no coarse row has more candidates).
hipError_t quotient_graph(const int64_t *row_ptr, const int32_t *col, int64_t n, int64_t nnz,
                          const int32_t *agg, int64_t n_agg, int64_t *crow, int32_t *ccol,
                          const QuotientWs &q, hipStream_t s);

// batch.hip: graph-local numbering of a union's aggregates.
hipError_t launch_graph_bounds(const int32_t *list, const uint32_t *d_count, const int64_t *voff,
                               int32_t G, uint32_t *P, hipStream_t s);
hipError_t launch_batch_local(int64_t n, const BatchInfo &bt, const uint32_t *P1,
                              const uint32_t *P2, int32_t *agg, const uint8_t *live,
                              const uint8_t *cont, const int64_t *newoff, int32_t *map,
                              hipStream_t s);
hipError_t launch_gather_i64(const int64_t *src, const int64_t *idx, int64_t count, int64_t *out,
                             hipStream_t s);
hipError_t launch_graph_ids(int64_t n, const BatchInfo &bt, int32_t *gid, hipStream_t s);

// aggregate.hip
hipError_t launch_label_roots(int64_t n, const int64_t *row_ptr, const int32_t *col,
                              const int32_t *roots, const uint32_t *d_count,
                              const uint32_t *d_base, bool only_unlabelled, int32_t *label,
                              int32_t *aggsize, uint8_t *root_mark, uint8_t mark, hipStream_t s);
// flag[v] = 1 for the phase-2 roots that become aggregates, else 0.
hipError_t launch_accept_phase2(int64_t n, const int64_t *row_ptr, const int32_t *col,
                                const uint32_t *T, const int32_t *label, uint8_t *flag,
                                hipStream_t s);
// Lists the vertices still unlabelled (label -1), and copies label to copy_to.
hipError_t launch_list_unlabelled(int blocks, int64_t n, const int32_t *label, int32_t *copy_to,
                                  const SegIO &io,
                                  hipStream_t s);
// io: the unaggregated rows (wl_in / cnt_in) and the list of long rows it
// leaves (wl_out / cnt_out); io_long: that list as input.
// Algorithm 2's second loop over the unaggregated vertices listed in io
// (wl_in / cnt_in): agg_out[v] = the smallest first-loop label among v's
// neighbours; bit 1 of *err if there is none.
hipError_t launch_join_min(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                           const int32_t *label, const SegIO &io, int32_t *agg_out,
                           uint32_t *err, hipStream_t s);
hipError_t launch_phase3(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                         const int32_t *label, const int32_t *aggsize, const SegIO &io,
                         const SegIO &io_long, int32_t *agg_out, uint32_t *err, hipStream_t s);

// Batched coarsening (abi.hip).  The arena is the caller's workspace: the
// coarsening workspace of the union, two coarse-union CSR buffers, the
// coarse-id map and the per-graph tables.
struct BatchArena {
    size_t head;           // bytes of the coarsening workspace at the start
    int64_t *crow[2];      // [n + 1]
    int32_t *ccol[2];      // [nnz]
    int32_t *map;          // [n]
    int32_t *gid;          // [n]
    int64_t *voff, *newoff, *bnd;  // [G + 1]
    uint32_t *gb, *P1, *P2;        // [G + 1]
    uint8_t *cont, *live;          // [G + 1]
};
size_t batch_bytes(int32_t G, int64_t n, int64_t nnz);
BatchArena carve_batch_arena(void *base, int32_t G, int64_t n, int64_t nnz);

// One level of a union of graphs.  In: voff (the graphs' vertex offsets in
// the union), live (graph takes part: its labels are kept), allow (graph may
// go on to another level).  Out: per-graph aggregate counts and stored
// entries, cont (graph goes on), and the coarse union of the graphs that go
// on (next_voff, n_next, nnz_next) in crow_next / ccol_next.  agg_dst gets
// graph-local labels (-1 for graphs that are not live).
struct BatchLevel {
    std::vector<int64_t> voff;
    std::vector<uint8_t> live, allow;
    std::vector<int64_t> nagg, nnz;
    std::vector<uint8_t> cont;
    std::vector<int64_t> next_voff;
    int64_t n_next = 0, nnz_next = 0;
};

}  // namespace mis2

struct mis2_ctx;
namespace mis2 {
int batch_level(mis2_ctx *ctx, const mis2_graph &cur, uint64_t seed, int64_t stop_below,
                int32_t *agg_dst, const BatchArena &ar, int64_t *crow_next, int32_t *ccol_next,
                BatchLevel *bl, hipStream_t s);
}  // namespace mis2

// Context (abi.hip).
struct mis2_ctx {
    int device = 0;
    int num_cus = 256;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t *pinned = nullptr;  // host-pinned scalars for read-back
    uint32_t *pinned_ctr = nullptr;  // host-pinned [2][kCtrList]: worklist1 counters per chunk
    uint32_t epoch = 0;                        // of the last run of rounds (host words)
    unsigned long long *alive_host = nullptr;  // host-pinned [8]: (round << 32) | |worklist1|,
                                               // (round << 32) | |worklist2|, tail row counts
    uint32_t *pinned_rt = nullptr;  // host-pinned [2][kTraceCap + 2][kRoundStride] round tables
    int trace_rounds[2] = {0, 0};   // rows of pinned_rt copied per phase
    int tail_used[2] = {0, 0};      // the phase's last rounds ran in the tail kernel
                                    // (it writes their rows of pinned_rt itself and the
                                    // row count to alive_host[2 + phase])
    int stamps_valid[2] = {0, 0};   // the rows hold persistent-kernel stamps
    std::string err;
    int validate = 0;
    int profile = 0;
    int account = 0;
    mis2::Plan plan;
    mis2::BatchInfo batch;  // graphs of the union being processed (batched calls only)
    std::vector<int64_t> trace[2];  // per-round |wl1|, |wl2| of the last run(s)
    std::vector<mis2_sweep_record> sweeps;  // launches of the last call
    std::vector<float> stamp_ms[2];         // persistent kernel: per-round sweep times
    double wall_khz = 100000.0;             // device wall-clock rate
    std::vector<hipEvent_t> events;         // profiling event pool
    size_t events_used = 0;
    mutable int staged_blocks = -1;         // resident workgroups of the staged sweeps (-1: not yet asked)
    // plan tuner
    int autotune = 1;                        // MIS2_OPT_AUTOTUNE
    struct SeenGraph {                       // graphs already classified (most recent last)
        const int64_t *row_ptr;
        int64_t n, nnz;
        mis2::GraphClass cls;
    };
    std::vector<SeenGraph> seen;
    int last_lanes = 0, last_blocks = 0, last_tail = 0, last_source = 0;  // plan of the last call
    std::vector<mis2_tune_record> tuning;    // candidate timings of the last tuning
};
