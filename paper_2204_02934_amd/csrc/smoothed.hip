// smoothed.hip -- smoothed aggregation on gfx950: the damped-Jacobi
// prolongator P = (I - omega D^-1 A) P_tent of an aggregation and the coarse
// operator P^T A P (the multigrid setup Section VI-E runs on these
// aggregates smooths its prolongator; the paper prints no formula).
//
// P_tent[i][agg i] = 1/sqrt(n_a) as in galerkin.hip.  Three sparse products,
// each with one fixed sequence of roundings:
//   P[i][a]  = (1{a = agg i} - (omega / d_i) * S) / sqrt(n_a), S = the sum of
//              A_ij over j in N[i] with agg j = a, from 0.0, the diagonal
//              first, then row i's entries in CSR order;
//   AP[i][b] = the sum of A_ij * P[j][b] over j in N[i] (i first, then row
//              i's entries in CSR order), from 0.0, absent P[j][b] skipped;
//   Ac[a][b] = the sum of P[i][a] * AP[i][b] over the rows i holding
//              P[i][a], in increasing i, from 0.0, absent AP[i][b] skipped.
// Patterns are structural, columns ascending: P row i = the distinct
// aggregates of N[i]; AP row i = the union of the P rows of N[i]; Ac row a =
// the union of the AP rows i with P[i][a].
//
// Structure (symbolic) kernels: one wavefront per output row.  The row's
// candidate columns -- each source row's columns, sources in order -- are
// inserted into an LDS hash set (kSetCap slots, open addressing with
// compare-and-swap); a count pass records the number of distinct columns,
// and after a prefix sum a fill pass lists the set's columns and places each
// at its rank among them (so rows come out ascending).  A row with more than
// kSetMax distinct columns sets an error flag.
// Value (numeric) kernels: P one group of lanes per row (k_p_values); AP
// and Ac one group per output row (k_row_values).  Each entry folds its terms one after the other in the
// stated order, each term one rounded product (the file is compiled without
// contraction into fused multiply-adds).
#include "internal.h"
#include "lanes.h"

#pragma clang fp contract(off)

namespace mis2 {

namespace {

constexpr int kSetCap = 4096;       // LDS hash-set slots per wavefront (large set)
constexpr int kSetMax = 2048;       // distinct columns a row may have (load factor 1/2)
constexpr int kSmallCap = 512;      // slots of the small set of the first pass
constexpr int kSmallMax = 256;      // distinct columns a row may have there
constexpr int kSThreads = 128;      // large-set pass: 2 wavefronts per workgroup (50 KB of LDS)
constexpr int kSWaves = kSThreads / 64;
constexpr int kSmallThreads = 256;  // small-set pass: 4 wavefronts per workgroup (17 KB)
constexpr int32_t kEmpty = -1;
constexpr int kSU = 4;              // candidates per lane whose loads go out together

int grid_of_s(int64_t work, int per_block, int cap) {
    const int64_t b = (work + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// A wavefront's hash set of CAP slots and the list of its columns (at most
// MAX are kept; a row with more is bad for this set).
template <int CAP, int MAX>
struct SetLds {
    int32_t slot[CAP];
    int32_t list[MAX];      // the columns in the set, in insertion order
    int64_t src_lo[64];     // a batch of 64 source rows: first entry
    int64_t src_end[65];    // inclusive prefix of their lengths (src_end[0] = 0)
    uint32_t n;             // columns inserted (may pass MAX: the row is then bad)
};

__device__ __forceinline__ void wave_sync_s() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CAP>
__device__ __forceinline__ uint32_t set_hash(int32_t c) {
    static_assert((CAP & (CAP - 1)) == 0 && CAP >= 64, "CAP: a power of two");
    return ((uint32_t)c * 2654435761u) >> (32 - __builtin_ctz(CAP));
}

// Inserts c (c >= 0) into the set, appending it to the list when it is new
// (while the list has room); returns 1 if it was new, 0 if present, and 2 if
// the set is full (the row is bad for this set).
template <int CAP, int MAX>
__device__ __forceinline__ int set_insert(SetLds<CAP, MAX> &sh, int32_t c) {
    uint32_t h = set_hash<CAP>(c) & (CAP - 1);
    for (int probe = 0; probe < CAP; probe++) {
        const int32_t old = atomicCAS(&sh.slot[h], kEmpty, c);
        if (old == kEmpty) {
            const uint32_t k = atomicAdd(&sh.n, 1u);
            if (k < (uint32_t)MAX) sh.list[k] = c;
            return 1;
        }
        if (old == c) return 0;
        h = (h + 1) & (CAP - 1);
    }
    return 2;
}

// The three kinds of rows.  For output row r, sources(r) gives the source
// rows in order; each source s contributes the columns col_of(s, k) for k in
// [0, len(s)).
//   kP:  sources = i, then i's neighbours; a source j contributes agg[j].
//   kAP: sources = i, then i's neighbours; a source j contributes P row j.
//   kC:  sources = the rows holding P[i][a] (members of R_a, increasing i);
//        a source i contributes AP row i.
enum { kP = 0, kAP = 1, kC = 2 };

struct SymArgs {
    int64_t rows;
    // the graph
    const int64_t *row_ptr;
    const int32_t *col;
    const int32_t *agg;
    // source CSR (P for kAP, AP for kC)
    const int64_t *sptr;
    const int32_t *scol;
    // kC: the members of R_a as P entry indices, and the row of each P entry
    const int64_t *moff;
    const int32_t *members;
    const int32_t *prow_of;
    // output
    uint32_t *count;          // count pass
    const int64_t *out_ptr;   // fill pass
    int32_t *out_col;
    uint32_t *err;            // |= 1: a row with more than kSetMax columns
    uint8_t *cls;             // [rows] 1: the row is left to the large-set pass
};

// Source rows of output row r: [first, last) of an index range, and the row
// id of source index t.
template <int K>
__device__ __forceinline__ void source_range(const SymArgs &a, int64_t r, int64_t &first,
                                             int64_t &last) {
    if (K == kC) {
        first = a.moff[r];
        last = a.moff[r + 1];
    } else {
        first = a.row_ptr[r] - 1;  // index first - 1 ... stands for r itself
        last = a.row_ptr[r + 1];
    }
}

template <int K>
__device__ __forceinline__ int64_t source_row(const SymArgs &a, int64_t r, int64_t t) {
    if (K == kC) return a.prow_of[a.members[t]];
    return t < a.row_ptr[r] ? r : (int64_t)a.col[t];
}

// Inserts every candidate column of output row r; returns the number of new
// columns this lane inserted, and sets *full when the set overflowed.
template <int K, class Set>
__device__ uint32_t insert_row(Set &sh, const SymArgs &a, int64_t r, bool *full) {
    const int lane = (int)(threadIdx.x & 63u);
    uint32_t added = 0;
    bool ovf = false;
    int64_t first, last;
    source_range<K>(a, r, first, last);
    if (K == kP) {
        // one column per source: 64 sources at a time
        for (int64_t t0 = first; t0 < last; t0 += 64) {
            const int64_t t = t0 + lane;
            if (t < last) {
                const int rc = set_insert(sh, a.agg[source_row<K>(a, r, t)]);
                added += rc == 1;
                ovf |= rc == 2;
            }
        }
    } else {
        for (int64_t t0 = first; t0 < last; t0 += 64) {
            // a batch of up to 64 source rows: their extents and prefix
            const int64_t t = t0 + lane;
            int64_t lo = 0, len = 0;
            if (t < last) {
                const int64_t s = source_row<K>(a, r, t);
                lo = a.sptr[s];
                len = a.sptr[s + 1] - lo;
            }
            int64_t incl = len;
            for (int off = 1; off < 64; off <<= 1) {
                const int64_t y = __shfl_up(incl, off, 64);
                if (lane >= off) incl += y;
            }
            sh.src_lo[lane] = lo;
            sh.src_end[lane + 1] = incl;
            if (lane == 0) sh.src_end[0] = 0;
            wave_sync_s();
            const int64_t total = sh.src_end[64];
            for (int64_t k0 = 0; k0 < total; k0 += 64 * kSU) {
                // kSU candidates per lane, every load issued before any insert
                // (candidates past the total reread the last one and are dropped)
                int32_t cand[kSU];
                bool ok[kSU];
#pragma unroll
                for (int u = 0; u < kSU; u++) {
                    const int64_t k = k0 + u * 64 + lane;
                    ok[u] = k < total;
                    const int64_t kk = ok[u] ? k : total - 1;
                    // the source holding candidate kk: last q with src_end[q] <= kk
                    int q = 0;
                    for (int step = 32; step > 0; step >>= 1)
                        if (q + step <= 63 && sh.src_end[q + step] <= kk) q += step;
                    cand[u] = a.scol[sh.src_lo[q] + (kk - sh.src_end[q])];
                }
#pragma unroll
                for (int u = 0; u < kSU; u++) {
                    if (ok[u]) {
                        const int rc = set_insert(sh, cand[u]);
                        added += rc == 1;
                        ovf |= rc == 2;
                    }
                }
            }
            wave_sync_s();
        }
    }
    *full = ovf;
    return added;
}

// One output row per wavefront.  SMALL: the first pass, with the small set
// (kSmallCap slots, kSmallMax columns), over every row; a row with more
// columns is marked in a.cls[r] = 1 (count pass) and left to the second
// pass.  Else: the large set over the rows marked 1 (64 marks read at a
// time over rows spread across all wavefronts); a row with more than
// kSetMax columns sets the error flag.
// (the small-set pass asks for 8 workgroups per CU, 8 waves per SIMD: its LDS
// allows them, and the register cap, 64, spills nothing)
template <int K, bool FILL, bool SMALL>
__global__ __launch_bounds__(SMALL ? kSmallThreads : kSThreads, SMALL ? 8 : 1) void k_sym(SymArgs a) {
    constexpr int CAP = SMALL ? kSmallCap : kSetCap;
    constexpr int MAX = SMALL ? kSmallMax : kSetMax;
    constexpr int WAVES = (SMALL ? kSmallThreads : kSThreads) / 64;
    __shared__ SetLds<CAP, MAX> sh_all[WAVES];
    SetLds<CAP, MAX> &sh = sh_all[threadIdx.x >> 6];
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t w0 = (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6);
    const int64_t stride = (int64_t)gridDim.x * WAVES;
    // the set starts empty and is emptied after each row by clearing the
    // slots of the listed columns only (the whole table after a bad row)
    for (int q = lane; q < CAP; q += 64) sh.slot[q] = kEmpty;
    if (lane == 0) sh.n = 0u;
    wave_sync_s();
    auto row = [&](const int64_t r) {
        bool full = false;
        insert_row<K>(sh, a, r, &full);
        wave_sync_s();
        const uint32_t distinct = sh.n;
        const bool bad = __ballot(full) != 0 || distinct > (uint32_t)MAX;
        if (!FILL && lane == 0) {
            if (SMALL) {
                a.cls[r] = bad ? 1 : 0;
                if (!bad) a.count[r] = distinct;
            } else {
                a.count[r] = bad ? 0u : distinct;
                if (bad) atomicOr(a.err, 1u);
            }
        }
        if (FILL && !bad) {
            // place each column at its rank among the row's columns
            int32_t *out = a.out_col + a.out_ptr[r];
            for (uint32_t x0 = 0; x0 < distinct; x0 += 64) {
                const uint32_t x = x0 + lane;
                const int32_t c = x < distinct ? sh.list[x] : 0;
                uint32_t rank = 0;
                for (uint32_t y = 0; y < distinct; y++) rank += sh.list[y] < c;
                if (x < distinct) out[rank] = c;
            }
        }
        wave_sync_s();
        if (bad) {
            for (int q = lane; q < CAP; q += 64) sh.slot[q] = kEmpty;
        } else {
            for (uint32_t x = lane; x < distinct; x += 64) {
                const int32_t c = sh.list[x];
                uint32_t h = set_hash<CAP>(c) & (CAP - 1);
                while (sh.slot[h] != c) h = (h + 1) & (CAP - 1);
                sh.slot[h] = kEmpty;
            }
        }
        wave_sync_s();
        if (lane == 0) sh.n = 0u;
        wave_sync_s();
    };
    if (SMALL) {
        for (int64_t r = w0; r < a.rows; r += stride) {
            // the fill pass skips the rows the count pass left to the large set
            if (FILL && a.cls[r] != 0) continue;  // uniform: one row per wavefront
            row(r);
        }
    } else {
        for (int64_t j0 = 0; w0 + j0 * stride < a.rows; j0 += 64) {
            const int64_t v = w0 + (j0 + lane) * stride;
            uint64_t mask = __ballot(v < a.rows && a.cls[v] != 0);
            while (mask) {
                const int q = __ffsll((unsigned long long)mask) - 1;
                mask &= mask - 1;
                row(w0 + (j0 + q) * stride);
            }
        }
    }
}

// P values: one group of kPG lanes per row i, one lane per entry (i, a) of
// P's row (kPG at a time).  The row of A goes kPG entries at a time, each
// lane loading one entry's aggregate and value; the group then folds them in
// CSR order by shuffles, every lane adding the entries of its own aggregate.
constexpr int kPG = 8;

__global__ __launch_bounds__(kBlock) void k_p_values(int64_t n, const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ diag,
                                                     const int32_t *__restrict__ agg,
                                                     const uint32_t *__restrict__ size,
                                                     double omega, const int64_t *__restrict__ prow,
                                                     const int32_t *__restrict__ pcol,
                                                     double *__restrict__ pval,
                                                     int32_t *__restrict__ prow_of) {
    const int gl = (int)(threadIdx.x & (kPG - 1));
    const int64_t NG = (int64_t)gridDim.x * (kBlock / kPG);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / kPG) + threadIdx.x / kPG; i < n; i += NG) {
        const int64_t p0 = prow[i], pm = prow[i + 1] - p0;
        const int64_t rs = row_ptr[i], re = row_ptr[i + 1];
        const int32_t ai = agg[i];
        const double di = diag[i];
        for (int64_t s0 = 0; s0 < pm; s0 += kPG) {
            const bool mine = s0 + gl < pm;
            const int32_t a = mine ? pcol[p0 + s0 + gl] : -1;
            double sum = 0.0;
            if (ai == a) sum = sum + di;
            for (int64_t e0 = rs; e0 < re; e0 += kPG) {
                const int cnt = (int)min<int64_t>(kPG, re - e0);
                int32_t ag = -1;
                double v = 0.0;
                if (gl < cnt) {
                    ag = agg[col[e0 + gl]];
                    v = val[e0 + gl];
                }
                // every lane of the group runs the shuffles
                for (int t = 0; t < cnt; t++) {
                    const int32_t at = __shfl(ag, t, kPG);
                    const double vt = __shfl(v, t, kPG);
                    if (at == a) sum = sum + vt;
                }
            }
            if (mine) {
                const double w = omega / di;
                const double ind = ai == a ? 1.0 : 0.0;
                const double t = w * sum;
                const double r = ind - t;
                pval[p0 + s0 + gl] = r / sqrt((double)size[a]);
                prow_of[p0 + s0 + gl] = (int32_t)i;
            }
        }
    }
}

// AP and Ac values: one group of G lanes per output row (G = 32 for AP,
// whose rows are short, so a wavefront has two rows in flight; 64 for Ac).
// An output entry (r, b) is the sum, over the row's terms t in their stated
// order, of coef_t * S[src_t][b] (skipped where S has no such entry).  The
// row's columns go to LDS, G at a time (a slot pass); the terms go kVT at a
// time: each entry of the chunk's source rows finds its column's slot by
// binary search and writes its rounded product into a kVT x G table cleared
// to +0.0, and then every lane folds its slot's column of the table in term
// order.  An absent term reads +0.0, and adding +0.0 changes no sum that
// starts from +0.0 (such a sum is never -0.0), so the result is that of
// skipping it.  Entries of a term have distinct columns, so no two writes
// meet.
// terms per chunk: 12 leaves a 32-lane group's table small enough (14 KB per
// workgroup) for registers, not LDS, to set the occupancy (5 waves per SIMD
// against 4 at 16 terms); the sums are the same term by term for any chunk
constexpr int kVT = 12;
constexpr int kVU = 4;            // staged entries per lane per step
constexpr int kValThreads = 128;  // 2 wavefronts per workgroup

template <int G>
struct ValLds {
    double table[kVT][G];
    double coef[kVT];
    int64_t lo[kVT];        // first entry of each term's source row
    uint32_t pre[kVT + 1];  // prefix of the chunk's source row lengths
    int32_t outc[G];        // the slot pass's output columns
};

// Inclusive prefix sum over each aligned group of G lanes.
template <int G>
__device__ __forceinline__ uint32_t group_incl_scan(uint32_t x) {
    const int gl = (int)(threadIdx.x & (G - 1));
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const uint32_t y = __shfl_up(x, (unsigned)d, G);
        if (gl >= d) x += y;
    }
    return x;
}

// Terms of AP row i: (i, d_i), then (j, A_ij) for row i's entries in CSR order.
struct ApTerms {
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
    const double *diag;
    struct Row {
        int64_t r, base, count;
    };
    __device__ Row row(int64_t r) const {
        const int64_t b = row_ptr[r];
        return {r, b, 1 + row_ptr[r + 1] - b};
    }
    __device__ void term(const Row &w, int64_t t, int64_t &src, double &coef) const {
        if (t == 0) {
            src = w.r;
            coef = diag[w.r];
        } else {
            src = col[w.base + t - 1];
            coef = val[w.base + t - 1];
        }
    }
};

// Terms of Ac row a: (i, P[i][a]) for the rows i holding P[i][a], increasing i.
struct CTerms {
    const int64_t *moff;
    const int32_t *members;
    const int32_t *prow_of;
    const double *pval;
    struct Row {
        int64_t base, count;
    };
    __device__ Row row(int64_t a) const {
        const int64_t b = moff[a];
        return {b, moff[a + 1] - b};
    }
    __device__ void term(const Row &w, int64_t t, int64_t &src, double &coef) const {
        const int32_t p = members[w.base + t];
        src = prow_of[p];
        coef = pval[p];
    }
};

// Stages one chunk of tc <= kVT terms (group lane t < tc holds term t's
// source row start lo, length len and coefficient cf) into the table and
// folds it into acc (group lanes < ns).  The group's lanes run it together;
// LDS accesses are ordered for the whole wavefront.
template <int G>
__device__ __forceinline__ void fold_chunk(ValLds<G> &sh, int gl, int tc, int64_t lo, uint32_t len,
                                           double cf, int ns, int32_t cmin, int32_t cmax,
                                           const int32_t *__restrict__ scol,
                                           const double *__restrict__ sval, double &acc) {
    const uint32_t incl = group_incl_scan<G>(len);
    const uint32_t E = (uint32_t)__shfl((int)incl, G - 1, G);
    if (gl < tc) {
        sh.lo[gl] = lo;
        sh.coef[gl] = cf;
        sh.pre[gl + 1] = incl;
    }
    if (gl == 0) sh.pre[0] = 0u;
    for (int t = 0; t < tc; t++) sh.table[t][gl] = 0.0;
    wave_sync_s();
    for (uint32_t k0 = 0; k0 < E; k0 += G * kVU) {
        // kVU entries per lane, every load issued before any is used (entries
        // past E reread entry E - 1 and are dropped)
        int tt[kVU];
        int32_t c[kVU];
        double v[kVU];
#pragma unroll
        for (int u = 0; u < kVU; u++) {
            const uint32_t k = k0 + (uint32_t)(u * G + gl);
            const uint32_t kk = k < E ? k : E - 1;
            int lo_t = 0, hi_t = tc - 1;  // the term of entry kk: last t with pre[t] <= kk
            while (lo_t < hi_t) {
                const int mid = (lo_t + hi_t + 1) >> 1;
                if (sh.pre[mid] <= kk) lo_t = mid; else hi_t = mid - 1;
            }
            const int64_t e = sh.lo[lo_t] + (int64_t)(kk - sh.pre[lo_t]);
            tt[u] = k < E ? lo_t : -1;
            c[u] = scol[e];
            v[u] = sval[e];
        }
#pragma unroll
        for (int u = 0; u < kVU; u++) {
            if (tt[u] >= 0 && c[u] >= cmin && c[u] <= cmax) {
                int l = 0, h = ns;  // its slot: the first output column >= c
                while (l < h) {
                    const int mid = (l + h) >> 1;
                    if (sh.outc[mid] < c[u]) l = mid + 1; else h = mid;
                }
                if (l < ns && sh.outc[l] == c[u]) sh.table[tt[u]][l] = sh.coef[tt[u]] * v[u];
            }
        }
    }
    wave_sync_s();
    if (gl < ns)
        for (int t = 0; t < tc; t++) acc = acc + sh.table[t][gl];
    wave_sync_s();
}

template <int G, class Terms>
__global__ __launch_bounds__(kValThreads) void k_row_values(
    int64_t rows, Terms tm, const int64_t *__restrict__ sptr, const int32_t *__restrict__ scol,
    const double *__restrict__ sval, const int64_t *__restrict__ optr,
    const int32_t *__restrict__ ocol, double *__restrict__ oval) {
    static_assert(G == 32 || G == 64, "a group is half or all of a wavefront");
    __shared__ ValLds<G> sh_all[kValThreads / G];
    ValLds<G> &sh = sh_all[threadIdx.x / G];
    const int gl = (int)(threadIdx.x & (G - 1));
    const int64_t NG = (int64_t)gridDim.x * (kValThreads / G);
    for (int64_t r = (int64_t)blockIdx.x * (kValThreads / G) + threadIdx.x / G; r < rows;
         r += NG) {
        const int64_t o0 = optr[r], m = optr[r + 1] - o0;
        const typename Terms::Row w = tm.row(r);
        for (int64_t s0 = 0; s0 < m; s0 += G) {
            const int ns = (int)min<int64_t>(G, m - s0);
            const int32_t myc = gl < ns ? ocol[o0 + s0 + gl] : INT32_MAX;
            const int32_t cmin = __shfl(myc, 0, G), cmax = __shfl(myc, ns - 1, G);
            sh.outc[gl] = myc;
            double acc = 0.0;
            for (int64_t tb = 0; tb < w.count; tb += G) {
                // the source rows and coefficients of G terms, one per lane,
                // in one round of loads; each chunk takes its own by shuffles
                const int tn = (int)min<int64_t>(G, w.count - tb);
                int64_t my_lo = 0;
                uint32_t my_len = 0;
                double my_cf = 0.0;
                if (gl < tn) {
                    int64_t src;
                    tm.term(w, tb + gl, src, my_cf);
                    my_lo = sptr[src];
                    my_len = (uint32_t)(sptr[src + 1] - my_lo);
                }
                for (int c0 = 0; c0 < tn; c0 += kVT) {
                    const int tc = min(kVT, tn - c0);
                    // every lane of the group shuffles (a lane that is switched
                    // off in a shuffle cannot be read from), then lanes past tc
                    // drop it
                    const int from = c0 + (gl < tc ? gl : 0);
                    const int64_t lo = __shfl(my_lo, from, G);
                    const uint32_t len_from = (uint32_t)__shfl((int)my_len, from, G);
                    const double cf = __shfl(my_cf, from, G);
                    const uint32_t len = gl < tc ? len_from : 0u;
                    fold_chunk<G>(sh, gl, tc, lo, len, cf, ns, cmin, cmax, scol, sval, acc);
                }
            }
            if (gl < ns) oval[o0 + s0 + gl] = acc;
        }
    }
}

}  // namespace

hipError_t launch_smoothed_sym(int kind, bool fill, int64_t rows, const int64_t *row_ptr,
                               const int32_t *col, const int32_t *agg, const int64_t *sptr,
                               const int32_t *scol, const int64_t *moff, const int32_t *members,
                               const int32_t *prow_of, uint32_t *count, const int64_t *out_ptr,
                               int32_t *out_col, uint32_t *err, uint8_t *cls, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    SymArgs a{rows, row_ptr, col, agg, sptr, scol, moff, members, prow_of, count, out_ptr,
              out_col, err, cls};
    // the small-set pass over every row, then the large-set pass over the
    // rows it left
    const dim3 g1(grid_of_s(rows, kSmallThreads / 64, 16384)), b1(kSmallThreads);
    const dim3 g2(grid_of_s(rows, kSWaves, 8192)), b2(kSThreads);
#define MIS2_SYM2(K, F)                                                        \
    hipLaunchKernelGGL((k_sym<K, F, true>), g1, b1, 0, s, a);                  \
    hipLaunchKernelGGL((k_sym<K, F, false>), g2, b2, 0, s, a);
    switch (kind * 2 + (fill ? 1 : 0)) {
        case 0: MIS2_SYM2(kP, false) break;
        case 1: MIS2_SYM2(kP, true) break;
        case 2: MIS2_SYM2(kAP, false) break;
        case 3: MIS2_SYM2(kAP, true) break;
        case 4: MIS2_SYM2(kC, false) break;
        case 5: MIS2_SYM2(kC, true) break;
        default: return hipErrorInvalidValue;
    }
#undef MIS2_SYM2
    return hipGetLastError();
}

hipError_t launch_p_values(int64_t n, int64_t p_nnz, const int64_t *row_ptr, const int32_t *col,
                           const double *val, const double *diag, const int32_t *agg,
                           const uint32_t *size, double omega, const int64_t *prow,
                           const int32_t *pcol, double *pval, int32_t *prow_of, hipStream_t s) {
    if (n <= 0 || p_nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_p_values, dim3(grid_of_s(n, kBlock / kPG, 16384)), dim3(kBlock), 0, s, n,
                       row_ptr, col, val, diag, agg, size, omega, prow, pcol, pval, prow_of);
    return hipGetLastError();
}

hipError_t launch_ap_values(int64_t n, int64_t ap_nnz, const int64_t *row_ptr, const int32_t *col,
                            const double *val, const double *diag, const int64_t *prow,
                            const int32_t *pcol, const double *pval, const int64_t *aptr,
                            const int32_t *acol, double *aval, hipStream_t s) {
    if (n <= 0 || ap_nnz <= 0) return hipSuccess;
    const ApTerms tm{row_ptr, col, val, diag};
    hipLaunchKernelGGL((k_row_values<32, ApTerms>), dim3(grid_of_s(n, kValThreads / 32, 16384)),
                       dim3(kValThreads), 0, s, n, tm, prow, pcol, pval, aptr, acol, aval);
    return hipGetLastError();
}

hipError_t launch_c_values(int64_t n_agg, int64_t c_nnz, const int64_t *moff,
                           const int32_t *members, const int32_t *prow_of, const double *pval,
                           const int64_t *aptr, const int32_t *acol, const double *aval,
                           const int64_t *crow, const int32_t *ccol, double *cval, hipStream_t s) {
    if (n_agg <= 0 || c_nnz <= 0) return hipSuccess;
    const CTerms tm{moff, members, prow_of, pval};
    hipLaunchKernelGGL((k_row_values<64, CTerms>), dim3(grid_of_s(n_agg, kValThreads / 64, 16384)),
                       dim3(kValThreads), 0, s, n_agg, tm, aptr, acol, aval, crow, ccol, cval);
    return hipGetLastError();
}

}  // namespace mis2
