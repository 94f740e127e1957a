// mis2_kernels.hip -- the per-round sweeps of Algorithm 1 (Section III-A) for gfx950.
//
// One round is two CSR sweeps:
//   Refresh Column over worklist2:  M_v = min T_w over the closed neighbourhood,
//                                   an IN minimum becomes OUT; v stays in
//                                   worklist2 iff M_v != OUT.
//   Decide Set over worklist1:      OUT if some M_w in the closed neighbourhood
//                                   is OUT, else IN if every M_w equals T_v;
//                                   a still undecided v gets the next round's
//                                   tuple at once (Refresh Row of round r+1 is
//                                   fused here) and stays in worklist1.
// Decide Set reads only M and writes only T_v, so rows are independent, and
// every per-row reduction is a min / any / all.
//
// Worklists are segmented by wavefront.  Wavefront w of the grid owns the
// vertex range [w*seg, (w+1)*seg) for the whole run; its part of a worklist
// lives in list[w*seg ...] with its own count cnt[w].  A sweep compacts its
// survivors in order with a wave ballot (Section V-B's prefix sum, at wave
// scope), so worklists need no atomics and no grid-wide scan, and a vertex is
// always handled by the same wavefront -- and the same XCD, because blocks are
// mapped so that each XCD's wavefronts own one contiguous slice of the ids.
// Inside a wavefront a group of L lanes (a power of two up to 64) streams one
// row's column indices (Section V-D uses SIMD lanes for the same coalescing)
// and combines partial results with cross-lane shuffles.
#include <hip/hip_ext.h>

#include <algorithm>

#include "internal.h"
#include "lanes.h"

namespace mis2 {

namespace {

constexpr int kUnroll = 4;  // rows per lane in flight (flat sweeps)
// L-lane sweeps: each lane group holds kRows rows and issues the loads of
// kChunks<L> chunks of L column indices per row before it gathers, so about
// 2 * kRows * kChunks<L> independent loads per lane are in flight (32 column
// indices per row for L <= 4).  Measured on gfx950 with the 27-point 100^3
// graph: one chunk per batch took 55 us per full Refresh Column sweep, eight
// chunks 30 us.  One row per group (rather than 2 or 4) keeps the sweeps at
// 64-80 registers, so more wavefronts stay resident: MIS-2 took 0.46 ms
// against 0.49 ms with 2 rows and 0.61 ms with 4.
constexpr int kRows = 1;
template <int L>
constexpr int kChunks = L >= 32 ? 1 : (32 / L > 8 ? 8 : 32 / L);

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Global wavefront id with the XCD-aware block order: workgroups are handed to
// the 8 XCDs round-robin, so logical block (b % 8) * (B / 8) + b / 8 gives
// each XCD a contiguous run of logical blocks (when B is a multiple of 8).
__device__ __forceinline__ int64_t wave_id() {
    const int64_t B = gridDim.x;
    const int64_t b = blockIdx.x;
    const int64_t lb = (B % 8 == 0) ? (b % 8) * (B / 8) + b / 8 : b;
    return lb * (kBlock / 64) + (threadIdx.x >> 6);
}

// Sum of the L-lane groups' row lengths over the workgroup, added to one of
// kSplit partial sums (stride kDegLine words, one cache line each) by thread
// 0 (accounting runs only; fold_deg collects the partial sums).  All threads
// must call it.
constexpr int kDegLine = 16;
// A second figure w (column indices written into compacted rows) goes to
// word 1 of the same lines.
__device__ __forceinline__ void wave_degsum(unsigned long long *split, unsigned long long d,
                                            unsigned long long w = 0) {
    __shared__ unsigned long long part[2][kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        d += __shfl_xor(d, off, 64);
        w += __shfl_xor(w, off, 64);
    }
    if ((threadIdx.x & 63u) == 0) {
        part[0][threadIdx.x >> 6] = d;
        part[1][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0, tw = 0;
        for (int k = 0; k < kBlock / 64; k++) {
            t += part[0][k];
            tw += part[1][k];
        }
        if (t) atomicAdd(&split[(blockIdx.x % kSplit) * kDegLine], t);
        if (tw) atomicAdd(&split[(blockIdx.x % kSplit) * kDegLine + 1], tw);
    }
}

// *target += the kSplit partial sums (word 0 of each line) and, when
// target_w is not null, *target_w += those of word 1; both are cleared
// (threads 0..63 of one workgroup).
__device__ __forceinline__ void fold_deg(unsigned long long *split, unsigned long long *target,
                                         unsigned long long *target_w) {
    unsigned long long x = split[(threadIdx.x & 63u) * kDegLine];
    unsigned long long y = split[(threadIdx.x & 63u) * kDegLine + 1];
    split[(threadIdx.x & 63u) * kDegLine] = 0ull;
    split[(threadIdx.x & 63u) * kDegLine + 1] = 0ull;
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off, 64);
        y += __shfl_xor(y, off, 64);
    }
    if (threadIdx.x == 0) {
        *target += x;
        if (target_w) *target_w += y;
    }
}

// The rows of wavefront w: either its identity range or its list segment.
struct Seg {
    int64_t base;   // first slot of the segment (= first vertex id of the range)
    int64_t count;  // rows in this round
};

__device__ __forceinline__ Seg seg_of(const SegIO &io, int64_t w) {
    Seg s;
    s.base = w * io.seg;
    if (io.cnt_in) {
        s.count = w < io.S ? (int64_t)io.cnt_in[w] : 0;
    } else {
        const int64_t hi = min(io.n, s.base + io.seg);
        s.count = hi > s.base ? hi - s.base : 0;
    }
    return s;
}

// Appends v (lanes with keep) to the wavefront's output segment in lane order.
__device__ __forceinline__ void seg_append(const SegIO &io, const Seg &sg, bool keep, int32_t v,
                                           uint32_t &kept) {
    const int lane = (int)(threadIdx.x & 63u);
    const uint64_t mask = __ballot(keep);
    if (keep) io.wl_out[sg.base + kept + (uint32_t)__popcll(mask & lanes_below(lane))] = v;
    kept += (uint32_t)__popcll(mask);
}

// Ends a sweep: the wavefront's count, and the workgroup's total added to one
// of kSplit size counters, each on its own cache line (one shared word or
// line would serialise thousands of workgroups).  All threads must call it.
__device__ __forceinline__ void seg_finish(const SegIO &io, int64_t w, uint32_t kept) {
    __shared__ uint32_t part[kBlock / 64];
    if ((threadIdx.x & 63u) == 0) {
        if (w < io.S) io.cnt_out[w] = kept;
        part[threadIdx.x >> 6] = kept;
    }
    if (!io.trace_out) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kBlock / 64; k++) t += part[k];
        if (t) atomicAdd(&io.trace_out[(blockIdx.x % kSplit) * kCtrLine], t);
    }
}

// Sum of the kSplit counters of one list (wavefront 0 of the workgroup; the
// result is in every lane of that wavefront).
__device__ __forceinline__ uint32_t ctr_sum(const uint32_t *list) {
    return group_sum<64>(list[(threadIdx.x & 63u) * kCtrLine]);
}

// Workgroup 0 clears the counter slot of round r + 2 at the start of round
// r's Refresh Column (nobody reads or writes that slot during round r).
__device__ __forceinline__ void clear_slot(uint32_t *ctr, int r) {
    if (blockIdx.x == 0 && threadIdx.x < 2 * kSplit)
        ctr[(size_t)((r + 2) % kCtrRing) * kCtrSlot + (threadIdx.x / kSplit) * kCtrList +
            (threadIdx.x % kSplit) * kCtrLine] = 0u;
}

// Largest row length among the rows this lane's group holds, over the
// wavefront (so every lane runs the same number of chunk steps).
template <int U>
__device__ __forceinline__ int64_t wave_max_len(const int64_t (&s)[U], const int64_t (&e)[U]) {
    int64_t m = 0;
#pragma unroll
    for (int u = 0; u < U; u++) m = max(m, e[u] - s[u]);
    return group_max64<64>(m);
}

// The U rows of this lane group for the step starting at row i0 of the
// segment; rows past the end repeat the last row (a valid address) with
// ok = false.
template <int L, int U>
__device__ __forceinline__ void load_rows(const SegIO &io, const Seg &sg, int64_t i0,
                                          int32_t (&v)[U], bool (&ok)[U]) {
    constexpr int G = 64 / L;
    const int lane = (int)(threadIdx.x & 63u);
    // The list slot address does not depend on the count (slots past the
    // segment's end are clamped into the array, and what they hold is not
    // used), so the entries load in the same trip as the wavefront's count.
    int64_t slot[U];
#pragma unroll
    for (int u = 0; u < U; u++) slot[u] = min(sg.base + i0 + u * G + lane / L, io.n - 1);
    int32_t x[U];
    if (io.wl_in) {
#pragma unroll
        for (int u = 0; u < U; u++) x[u] = io.wl_in[slot[u]];
    } else {
#pragma unroll
        for (int u = 0; u < U; u++) x[u] = (int32_t)slot[u];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
        ok[u] = i0 + u * G + lane / L < sg.count;
        v[u] = ok[u] ? x[u] : 0;  // vertex 0: a valid address for the lanes without a row
    }
}

// Rows longer than this many column indices are streamed by the whole
// wavefront (8 loads per lane in flight) instead of by their L-lane group,
// so one high-degree row does not hold the wavefront for len / L steps.
template <int L>
__device__ __forceinline__ int64_t heavy_threshold() {
    return L >= 64 ? 1024 : (int64_t)32 * L;
}
constexpr int kCoopLoads = 8;  // loads per lane per cooperative step

// Minimum of T over the column indices [s, e), by the whole wavefront.
// With out != null the indices whose T is not OUT are also written, in
// order, to out[s ...] (out may be the array read: every store lands at or
// below the position of an index already loaded), and *written gets their
// count.
__device__ __forceinline__ uint32_t coop_min_T(const int32_t *col, const uint32_t *__restrict__ T,
                                               int64_t s, int64_t e, int32_t *out = nullptr,
                                               uint32_t *written = nullptr,
                                               const SegIO *gio = nullptr) {
    const int lane = (int)(threadIdx.x & 63u);
    uint32_t m = kOut;
    uint32_t wc = 0;
    for (int64_t b = s; b < e; b += 64 * kCoopLoads) {
        int32_t x[kCoopLoads];
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++) {
            const int64_t j = b + (int64_t)k * 64 + lane;
            x[k] = col[j < e ? j : s];  // entry s exists: the row is not empty
        }
        uint32_t t[kCoopLoads];
        if (gio && gio->gen0) {
#pragma unroll
            for (int k = 0; k < kCoopLoads; k++) t[k] = make_tuple(gio->t0, (uint32_t)x[k]);
        } else {
#pragma unroll
            for (int k = 0; k < kCoopLoads; k++) t[k] = T[x[k]];
        }
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++)
            if (b + (int64_t)k * 64 + lane < e) m = min(m, t[k]);
        if (out) {
#pragma unroll
            for (int k = 0; k < kCoopLoads; k++) {
                const bool kp = b + (int64_t)k * 64 + lane < e && t[k] != kOut;
                const uint64_t bal = __ballot(kp);
                if (kp) out[s + wc + (uint32_t)__popcll(bal & lanes_below(lane))] = x[k];
                wc += (uint32_t)__popcll(bal);
            }
        }
    }
    if (written) *written = wc;
    return group_min<64>(m);
}

// Any M_w == OUT and all M_w in {t0, absent} over [s, e), by the whole wavefront.
__device__ __forceinline__ void coop_decide(const int32_t *__restrict__ col,
                                            const uint32_t *__restrict__ M, int64_t s, int64_t e,
                                            uint32_t t0, int &any_out, int &all_eq) {
    const int lane = (int)(threadIdx.x & 63u);
    int ao = 0, ae = 1;
    for (int64_t b = s; b < e; b += 64 * kCoopLoads) {
        int32_t x[kCoopLoads];
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++) {
            const int64_t j = b + (int64_t)k * 64 + lane;
            x[k] = col[j < e ? j : s];
        }
        uint32_t mw[kCoopLoads];
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++) mw[k] = M[x[k]];
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++) {
            if (b + (int64_t)k * 64 + lane < e) {
                ao |= (mw[k] == kOut);
                ae &= (mw[k] == t0) | (mw[k] == kAbsent);
            }
        }
    }
    any_out = (int)group_or<64>((uint32_t)ao);
    all_eq = (int)group_and<64>((uint32_t)ae);
}

// Refresh Column over the wavefront's segment: U rows per lane group per
// step, and K chunks of each row's column indices loaded before any of their
// gathers, so that U * K independent loads are in flight.  Loads are issued
// unconditionally from clamped, always valid addresses and their results
// selected afterwards: a predicated load would become a branch with a full
// wait after it and serialise the streams.
//
// Long rows (more than heavy_threshold<L>() entries when the CSR's, the rows
// the whole wavefront streams) may carry a compacted form: with io.ccol_out
// set, the cooperative pass rewrites each long row it sweeps without its OUT
// entries (T = OUT is final and never lowers a minimum) and records the
// length; with RD, rows that were long in the CSR are read from that form.
// A row stays a superset of its live neighbours whether or not it was
// rewritten in the last round, so short rows and rows that shrank below the
// threshold are simply read as they are.
template <int L, int U, int K, bool RD, bool WR>
__device__ __forceinline__ uint32_t sweep_column(const int64_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col,
                                                 const uint32_t *__restrict__ T,
                                                 uint32_t *__restrict__ M, const SegIO &io,
                                                 const Seg &sg) {
    constexpr int G = 64 / L;  // rows per wavefront per unrolled slot
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & (L - 1);
    const int32_t *colc = io.ccol_in;
    const int32_t *lenc = io.lenc_in;
    int32_t *wout = WR ? io.ccol_out : nullptr;
    uint32_t kept = 0;
    unsigned long long dsum = 0, wsum = 0;
    // The rows of step i + 1 (list entries, extents, own T) are loaded while
    // step i's column indices and gathers are in flight.
    int32_t v[U];
    bool ok[U];
    int64_t s[U], e[U];
    uint32_t m[U];
    int32_t lc[U];  // RD: compacted length (meaningful for rows long in the CSR)
    bool cf[U];     // RD: the row is read from its compacted form
    if (sg.count > 0) {
        load_rows<L, U>(io, sg, 0, v, ok);
#pragma unroll
        for (int u = 0; u < U; u++) {
            s[u] = row_ptr[v[u]];
            e[u] = row_ptr[v[u] + 1];
            m[u] = T[v[u]];
            lc[u] = RD ? lenc[v[u]] : 0;
        }
    }
    for (int64_t i0 = 0; i0 < sg.count; i0 += G * U) {
        const bool more = i0 + G * U < sg.count;
        int32_t vn[U];
        bool okn[U];
        int64_t sn[U] = {}, en[U] = {};
        uint32_t mn[U] = {};
        int32_t lcn[U] = {};
        if (more) load_rows<L, U>(io, sg, i0 + G * U, vn, okn);
        bool fetched = !more;
        uint32_t wc[U];  // entries of a rewritten long row
        bool wrote[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (!ok[u]) e[u] = s[u];
            cf[u] = RD && e[u] - s[u] > heavy_threshold<L>();
            if (cf[u]) e[u] = s[u] + lc[u];
            wc[u] = 0;
            wrote[u] = false;
            if (sub != 0) m[u] = kOut;
            if (sub == 0) dsum += (unsigned long long)(e[u] - s[u]);
        }
        // high-degree rows: the whole wavefront streams each one in turn
#pragma unroll
        for (int u = 0; u < U; u++) {
            uint64_t heavy = __ballot(sub == 0 && e[u] - s[u] > heavy_threshold<L>());
            // round 0 reports that the graph has such rows (compaction pays
            // only for them)
            if (!RD && !WR && heavy && io.long_flag && lane == 0)
                io.long_flag[(blockIdx.x % kSplit) * kCtrLine] = 1u;
            while (heavy) {
                const int src = __ffsll((unsigned long long)heavy) - 1;
                heavy &= heavy - 1;
                const int64_t hs = __shfl(s[u], src, 64), he = __shfl(e[u], src, 64);
                uint32_t hm, hw = 0;
                if (RD && __shfl((int)cf[u], src, 64) != 0)
                    hm = coop_min_T(colc, T, hs, he, wout, &hw, &io);
                else
                    hm = coop_min_T(col, T, hs, he, wout, &hw, &io);
                if (WR && lane == 0) wsum += hw;
                if ((lane & ~(L - 1)) == (src & ~(L - 1))) {
                    m[u] = (sub == 0) ? min(m[u], hm) : kOut;
                    e[u] = s[u];  // its group skips the row below
                    wc[u] = hw;
                    wrote[u] = WR;
                }
            }
        }
        const int64_t steps = wave_max_len<U>(s, e);
        for (int64_t c0 = 0; c0 < steps; c0 += (int64_t)L * K) {
            int32_t x[U][K];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int32_t *rs = (RD && cf[u]) ? colc : col;
#pragma unroll
                for (int k = 0; k < K; k++) {
                    const int64_t j = s[u] + c0 + k * L + sub;
                    x[u][k] = rs[j < e[u] ? j : 0];
                    // entry 0 of the compacted array may never have been
                    // written: lanes past the row's end gather at vertex 0
                    if (RD && j >= e[u]) x[u][k] = 0;
                }
            }
            if (!fetched) {
#pragma unroll
                for (int u = 0; u < U; u++) {
                    sn[u] = row_ptr[vn[u]];
                    en[u] = row_ptr[vn[u] + 1];
                    mn[u] = T[vn[u]];
                    lcn[u] = RD ? lenc[vn[u]] : 0;
                }
                fetched = true;
            }
            uint32_t t[U][K];
            if (io.gen0) {
#pragma unroll
                for (int u = 0; u < U; u++)
#pragma unroll
                    for (int k = 0; k < K; k++) t[u][k] = make_tuple(io.t0, (uint32_t)x[u][k]);
            } else {
#pragma unroll
                for (int u = 0; u < U; u++)
#pragma unroll
                    for (int k = 0; k < K; k++) t[u][k] = T[x[u][k]];
            }
#pragma unroll
            for (int u = 0; u < U; u++)
#pragma unroll
                for (int k = 0; k < K; k++)
                    if (s[u] + c0 + k * L + sub < e[u]) m[u] = min(m[u], t[u][k]);
        }
        if (!fetched) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                sn[u] = row_ptr[vn[u]];
                en[u] = row_ptr[vn[u] + 1];
                mn[u] = T[vn[u]];
                lcn[u] = RD ? lenc[vn[u]] : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            m[u] = group_min<L>(m[u]);
            bool keep = false;
            if (ok[u] && sub == 0) {
                if (io.gen0 == 2 && M[v[u]] == kOut) m[u] = kOut;  // pushed by an IN vertex
                if (m[u] == kIn) m[u] = kOut;
                M[v[u]] = m[u];
                keep = (m[u] != kOut);
                if (WR && keep && wrote[u]) io.lenc_out[v[u]] = (int32_t)wc[u];
            }
            seg_append(io, sg, keep, v[u], kept);
        }
        if (more) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                v[u] = vn[u];
                ok[u] = okn[u];
                s[u] = sn[u];
                e[u] = en[u];
                m[u] = mn[u];
                lc[u] = lcn[u];
            }
        }
    }
    if (io.deg_sum) wave_degsum(io.deg_sum, dsum, wsum);
    return kept;
}

// Decide Set over the wavefront's segment, with the next round's Refresh Row
// for the vertices that stay undecided (loads as in sweep_column).
template <int L, int U, int K>
__device__ __forceinline__ uint32_t sweep_decide(const int64_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col,
                                                 uint32_t *__restrict__ T,
                                                 const uint32_t *__restrict__ M,
                                                 const TupleParams &next, const SegIO &io,
                                                 const Seg &sg) {
    constexpr int G = 64 / L;
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & (L - 1);
    uint32_t kept = 0;
    unsigned long long dsum = 0;
    // The rows of step i + 1 are loaded while step i's gathers are in flight
    // (as in sweep_column).
    int32_t v[U];
    bool ok[U];
    int64_t s[U], e[U];
    uint32_t t0[U], mv[U];
    if (sg.count > 0) {
        load_rows<L, U>(io, sg, 0, v, ok);
#pragma unroll
        for (int u = 0; u < U; u++) {
            s[u] = row_ptr[v[u]];
            e[u] = row_ptr[v[u] + 1];
            t0[u] = T[v[u]];
            mv[u] = M[v[u]];
        }
    }
    for (int64_t i0 = 0; i0 < sg.count; i0 += G * U) {
        const bool more = i0 + G * U < sg.count;
        int32_t vn[U];
        bool okn[U];
        int64_t sn[U] = {}, en[U] = {};
        uint32_t tn[U] = {}, mvn[U] = {};
        if (more) load_rows<L, U>(io, sg, i0 + G * U, vn, okn);
        bool fetched = !more;
        int any_out[U], all_eq[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (!ok[u]) e[u] = s[u];
            any_out[u] = (sub == 0) & (mv[u] == kOut);
            all_eq[u] = (sub != 0) | (mv[u] == t0[u]);
            if (sub == 0) dsum += (unsigned long long)(e[u] - s[u]);
            // M_v = OUT already decides the row (OUT), whatever the neighbours
            // hold; in round 0, M_v != T_v keeps it undecided
            if (mv[u] == kOut || (io.dec0 && mv[u] != t0[u])) e[u] = s[u];
            // in round 1, near[v] stands for the neighbours' OUT test
            if (io.dec1 && ok[u] && mv[u] != kOut && mv[u] != t0[u]) {
                any_out[u] = (sub == 0) & (io.near[v[u]] != 0);
                e[u] = s[u];
            }
        }
        // high-degree rows: the whole wavefront streams each one in turn
#pragma unroll
        for (int u = 0; u < U; u++) {
            uint64_t heavy = __ballot(sub == 0 && e[u] - s[u] > heavy_threshold<L>());
            while (heavy) {
                const int src = __ffsll((unsigned long long)heavy) - 1;
                heavy &= heavy - 1;
                const int64_t hs = __shfl(s[u], src, 64), he = __shfl(e[u], src, 64);
                const uint32_t ht0 = __shfl(t0[u], src, 64);
                int hao, hae;
                coop_decide(col, M, hs, he, ht0, hao, hae);
                if ((lane & ~(L - 1)) == (src & ~(L - 1))) {
                    if (sub == 0) {
                        any_out[u] |= hao;
                        all_eq[u] &= hae;
                    }
                    e[u] = s[u];  // its group skips the row below
                }
            }
        }
        const int64_t steps = wave_max_len<U>(s, e);
        for (int64_t c0 = 0; c0 < steps; c0 += (int64_t)L * K) {
            int32_t x[U][K];
#pragma unroll
            for (int u = 0; u < U; u++)
#pragma unroll
                for (int k = 0; k < K; k++) {
                    const int64_t j = s[u] + c0 + k * L + sub;
                    x[u][k] = col[j < e[u] ? j : 0];
                }
            if (!fetched) {
#pragma unroll
                for (int u = 0; u < U; u++) {
                    sn[u] = row_ptr[vn[u]];
                    en[u] = row_ptr[vn[u] + 1];
                    tn[u] = T[vn[u]];
                    mvn[u] = M[vn[u]];
                }
                fetched = true;
            }
            uint32_t mw[U][K];
#pragma unroll
            for (int u = 0; u < U; u++)
#pragma unroll
                for (int k = 0; k < K; k++) mw[u][k] = M[x[u][k]];
#pragma unroll
            for (int u = 0; u < U; u++)
#pragma unroll
                for (int k = 0; k < K; k++) {
                    if (s[u] + c0 + k * L + sub < e[u]) {
                        any_out[u] |= (mw[u][k] == kOut);
                        all_eq[u] &= (mw[u][k] == t0[u]) | (mw[u][k] == kAbsent);
                    }
                }
        }
        if (!fetched) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                sn[u] = row_ptr[vn[u]];
                en[u] = row_ptr[vn[u] + 1];
                tn[u] = T[vn[u]];
                mvn[u] = M[vn[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            any_out[u] = group_or<L>((uint32_t)any_out[u]);
            all_eq[u] = group_and<L>((uint32_t)all_eq[u]);
            bool keep = false;
            if (ok[u] && sub == 0) {
                uint32_t nt;
                if (any_out[u]) {
                    nt = kOut;
                } else if (all_eq[u]) {
                    nt = kIn;
                } else {
                    nt = make_tuple(next, (uint32_t)v[u]);
                    keep = true;
                }
                T[v[u]] = nt;
            }
            seg_append(io, sg, keep, v[u], kept);
        }
        if (more) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                v[u] = vn[u];
                ok[u] = okn[u];
                s[u] = sn[u];
                e[u] = en[u];
                t0[u] = tn[u];
                mv[u] = mvn[u];
            }
        }
    }
    if (io.deg_sum) wave_degsum(io.deg_sum, dsum);
    return kept;
}

// ---------------------------------------------------------------------------
// Staged sweeps: one row per lane.  A wavefront takes the rows of its segment
// 64 at a time.  Groups of 4 lanes load each row's column indices with
// 16-byte loads (up to kStagedCap entries, two loads per lane) into the row's
// slot of LDS; then every lane walks its own row from LDS and gathers the
// neighbour values.  The k-th gathers of consecutive rows are thereby issued
// by consecutive lanes of one instruction (for a stencil graph: nearby
// addresses, few cache lines per instruction), while the column indices are
// read in whole 64-byte pieces.  Rows longer than kStagedCap entries go to
// the whole wavefront, as in the L-lane sweeps.
//
// Measured on gfx950 (27-point 100^3 graph, round 0 of Refresh Column): 4
// lanes per row took 34 us, the staged sweep with one lane per row (64 rows
// per step) 26 us at 1024 workgroups; two lanes per row (32 rows per step,
// half the LDS) 36 us at 1536 and 29 us at 2048 workgroups.  The slots take
// 8.4 KB of LDS per wavefront, so 4 workgroups fit on a compute unit.
// ---------------------------------------------------------------------------
constexpr int kStagedCap = 32;     // column indices per LDS row slot
constexpr int kStagedStride = 33;  // words per slot: a lane's k-th read hits bank (slot + k) % 32
constexpr int kStagedUnroll = 13;  // gathers in flight per lane

typedef int32_t v4i32 __attribute__((ext_vector_type(4), aligned(4)));

// H lanes per row (1 or 2): 64 / H rows per step.
template <int H>
struct StagedLds {
    int32_t idx[(64 / H) * kStagedStride];
};

// p[j .. j + 3] for 0 <= j < nnz (nnz >= 4): one 16-byte load from
// min(j, nnz - 4), whose elements are moved down near the end of the array
// so that element q is p[j + q] whenever j + q < nnz.  Elements past nnz are
// not meaningful.  The move is register work only (no load in the branch).
__device__ __forceinline__ v4i32 load4_clamped(const int32_t *p, int64_t j, int64_t nnz) {
    const int64_t jj = min(j, nnz - 4);
    v4i32 x = *(const v4i32 *)(p + jj);
    const int64_t d = j - jj;
    if (d == 1) {
        x.x = x.y; x.y = x.z; x.z = x.w;
    } else if (d == 2) {
        x.x = x.z; x.y = x.w;
    } else if (d == 3) {
        x.x = x.w;
    }
    return x;
}

// Copies the column indices of the step's rows into their LDS slots: groups
// of 4 lanes take one row each (16 rows per pass), `chunks` (1 or 2)
// 16-byte loads per lane, 16 entries per chunk.  Row r's start s and length
// len are held by lane r * H; cf (same lanes) selects the compacted copy.  A
// chunk is loaded only when the row reaches into it (a row of length 0, one
// that needs no scan, loads nothing); entries past a row's end are written
// too and never read.
template <int H>
__device__ __forceinline__ void stage_rows(StagedLds<H> &sh, const int32_t *col,
                                           const int32_t *colc, const int64_t s, const int len,
                                           const int cf, int chunks, int64_t nnz) {
    constexpr int R = 64 / H;
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & 3;
#pragma unroll
    for (int g = 0; g < R / 16; g++) {
        const int rr = g * 16 + (lane >> 2);
        const int64_t sr = __shfl(s, rr * H, 64);
        const int rlen = __shfl(len, rr * H, 64);
        const int rcf = __shfl(cf, rr * H, 64);
        const int32_t *src = rcf ? colc : col;
        v4i32 x[2];
#pragma unroll
        for (int c = 0; c < 2; c++)
            if (c < chunks && rlen > c * 16) x[c] = load4_clamped(src, sr + c * 16 + sub * 4, nnz);
#pragma unroll
        for (int c = 0; c < 2; c++) {
            if (c < chunks && rlen > c * 16) {
                int32_t *d = &sh.idx[rr * kStagedStride + c * 16 + sub * 4];
                d[0] = x[c].x;
                d[1] = x[c].y;
                d[2] = x[c].z;
                d[3] = x[c].w;
            }
        }
    }
}

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Refresh Column over the wavefront's segment, staged (see above), with H
// lanes per row (lane h of a row gathers its entries h, h + H, ...).  RD /
// WR: as in sweep_column, with "long" meaning more than kStagedCap entries
// in the CSR.
template <int H, bool RD, bool WR>
__device__ __forceinline__ uint32_t sweep_column_staged(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const uint32_t *__restrict__ T,
                                                        uint32_t *__restrict__ M, const SegIO &io,
                                                        const Seg &sg, StagedLds<H> &sh) {
    constexpr int R = 64 / H;
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & (H - 1);
    const int32_t *colc = io.ccol_in;
    const int32_t *lenc = io.lenc_in;
    int32_t *wout = WR ? io.ccol_out : nullptr;
    uint32_t kept = 0;
    unsigned long long dsum = 0, wsum = 0;
    int32_t v[1];
    bool ok[1];
    int64_t s = 0, e = 0;
    uint32_t m = 0;
    int32_t lc = 0;
    if (sg.count > 0) {
        load_rows<H, 1>(io, sg, 0, v, ok);
        s = row_ptr[v[0]];
        e = row_ptr[v[0] + 1];
        m = T[v[0]];
        lc = RD ? lenc[v[0]] : 0;
    }
    for (int64_t i0 = 0; i0 < sg.count; i0 += R) {
        const bool more = i0 + R < sg.count;
        int32_t vn[1] = {0};
        bool okn[1] = {false};
        if (more) load_rows<H, 1>(io, sg, i0 + R, vn, okn);
        if (!ok[0]) e = s;
        const int cf = RD && e - s > kStagedCap;
        if (cf) e = s + lc;
        if (sub == 0) dsum += (unsigned long long)(e - s);
        uint32_t wc = 0;
        bool wrote = false;
        // long rows: the whole wavefront streams each one in turn
        uint64_t heavy = __ballot(sub == 0 && e - s > kStagedCap);
        if (!RD && !WR && heavy && io.long_flag && lane == 0)
            io.long_flag[(blockIdx.x % kSplit) * kCtrLine] = 1u;
        while (heavy) {
            const int src = __ffsll((unsigned long long)heavy) - 1;
            heavy &= heavy - 1;
            const int64_t hs = __shfl(s, src, 64), he = __shfl(e, src, 64);
            uint32_t hm, hw = 0;
            if (RD && __shfl(cf, src, 64) != 0)
                hm = coop_min_T(colc, T, hs, he, wout, &hw, &io);
            else
                hm = coop_min_T(col, T, hs, he, wout, &hw, &io);
            if (WR && lane == 0) wsum += hw;
            if ((lane & ~(H - 1)) == src) {
                m = min(m, hm);
                e = s;  // skipped below
                wc = hw;
                wrote = WR;
            }
        }
        const int len = (int)(e - s);
        const int maxlen = (int)group_max<64>((uint32_t)len);
        if (maxlen > 0) stage_rows<H>(sh, col, colc, s, len, cf, maxlen > 16 ? 2 : 1, io.nnz);
        // the next rows' extents and own values load while this step's
        // gathers are in flight
        int64_t sn = 0, en = 0;
        uint32_t mn = 0;
        int32_t lcn = 0;
        if (more) {
            sn = row_ptr[vn[0]];
            en = row_ptr[vn[0] + 1];
            mn = T[vn[0]];
            lcn = RD ? lenc[vn[0]] : 0;
        }
        wave_lds_fence();
        const int32_t *slot = &sh.idx[(lane / H) * kStagedStride];
        for (int k0 = 0; k0 < maxlen; k0 += H * kStagedUnroll) {
            int32_t x[kStagedUnroll];
#pragma unroll
            for (int u = 0; u < kStagedUnroll; u++) {
                const int k = k0 + H * u + sub;
                const int32_t y = slot[k < kStagedCap ? k : 0];
                x[u] = k < len ? y : v[0];
            }
            uint32_t t[kStagedUnroll];
            if (io.gen0) {
#pragma unroll
                for (int u = 0; u < kStagedUnroll; u++) t[u] = make_tuple(io.t0, (uint32_t)x[u]);
            } else {
#pragma unroll
                for (int u = 0; u < kStagedUnroll; u++) t[u] = T[x[u]];
            }
#pragma unroll
            for (int u = 0; u < kStagedUnroll; u++) m = min(m, t[u]);
        }
        m = group_min<H>(m);
        bool keep = false;
        if (ok[0] && sub == 0) {
            if (io.gen0 == 2 && M[v[0]] == kOut) m = kOut;  // pushed by an IN vertex
            if (m == kIn) m = kOut;
            M[v[0]] = m;
            keep = (m != kOut);
            if (WR && keep && wrote) io.lenc_out[v[0]] = (int32_t)wc;
        }
        seg_append(io, sg, keep, v[0], kept);
        wave_lds_fence();  // the slots are rewritten by the next step
        if (more) {
            v[0] = vn[0];
            ok[0] = okn[0];
            s = sn;
            e = en;
            m = mn;
            lc = lcn;
        }
    }
    if (io.deg_sum) wave_degsum(io.deg_sum, dsum, wsum);
    return kept;
}

// Decide Set over the wavefront's segment, staged, with the next round's
// Refresh Row for the vertices that stay undecided.
template <int H>
__device__ __forceinline__ uint32_t sweep_decide_staged(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        uint32_t *__restrict__ T,
                                                        const uint32_t *__restrict__ M,
                                                        const TupleParams &next, const SegIO &io,
                                                        const Seg &sg, StagedLds<H> &sh) {
    constexpr int R = 64 / H;
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & (H - 1);
    uint32_t kept = 0;
    unsigned long long dsum = 0;
    int32_t v[1];
    bool ok[1];
    int64_t s = 0, e = 0;
    uint32_t t0 = 0, mv = 0;
    if (sg.count > 0) {
        load_rows<H, 1>(io, sg, 0, v, ok);
        s = row_ptr[v[0]];
        e = row_ptr[v[0] + 1];
        t0 = T[v[0]];
        mv = M[v[0]];
    }
    for (int64_t i0 = 0; i0 < sg.count; i0 += R) {
        const bool more = i0 + R < sg.count;
        int32_t vn[1] = {0};
        bool okn[1] = {false};
        if (more) load_rows<H, 1>(io, sg, i0 + R, vn, okn);
        if (!ok[0]) e = s;
        int any_out = (sub == 0) & (mv == kOut);
        int all_eq = (sub != 0) | (mv == t0);
        if (sub == 0) dsum += (unsigned long long)(e - s);
        // M_v = OUT already decides the row (OUT), whatever the neighbours
        // hold; in round 0, M_v != T_v keeps it undecided
        if (mv == kOut || (io.dec0 && mv != t0)) e = s;
        // in round 1, near[v] stands for the neighbours' OUT test
        if (io.dec1 && ok[0] && mv != kOut && mv != t0) {
            any_out = (sub == 0) & (io.near[v[0]] != 0);
            e = s;
        }
        uint64_t heavy = __ballot(sub == 0 && e - s > kStagedCap);
        while (heavy) {
            const int src = __ffsll((unsigned long long)heavy) - 1;
            heavy &= heavy - 1;
            const int64_t hs = __shfl(s, src, 64), he = __shfl(e, src, 64);
            const uint32_t ht0 = __shfl(t0, src, 64);
            int hao, hae;
            coop_decide(col, M, hs, he, ht0, hao, hae);
            if ((lane & ~(H - 1)) == src) {
                if (sub == 0) {
                    any_out |= hao;
                    all_eq &= hae;
                }
                e = s;
            }
        }
        const int len = (int)(e - s);
        const int maxlen = (int)group_max<64>((uint32_t)len);
        if (maxlen > 0) stage_rows<H>(sh, col, col, s, len, 0, maxlen > 16 ? 2 : 1, io.nnz);
        int64_t sn = 0, en = 0;
        uint32_t tn = 0, mvn = 0;
        if (more) {
            sn = row_ptr[vn[0]];
            en = row_ptr[vn[0] + 1];
            tn = T[vn[0]];
            mvn = M[vn[0]];
        }
        wave_lds_fence();
        const int32_t *slot = &sh.idx[(lane / H) * kStagedStride];
        for (int k0 = 0; k0 < maxlen; k0 += H * kStagedUnroll) {
            int32_t x[kStagedUnroll];
#pragma unroll
            for (int u = 0; u < kStagedUnroll; u++) {
                const int k = k0 + H * u + sub;
                const int32_t y = slot[k < kStagedCap ? k : 0];
                x[u] = k < len ? y : v[0];
            }
            uint32_t mw[kStagedUnroll];
#pragma unroll
            for (int u = 0; u < kStagedUnroll; u++) mw[u] = M[x[u]];
#pragma unroll
            for (int u = 0; u < kStagedUnroll; u++) {
                if (k0 + H * u + sub < len) {
                    any_out |= (mw[u] == kOut);
                    all_eq &= (mw[u] == t0) | (mw[u] == kAbsent);
                }
            }
        }
        any_out = (int)group_or<H>((uint32_t)any_out);
        all_eq = (int)group_and<H>((uint32_t)all_eq);
        bool keep = false;
        if (ok[0] && sub == 0) {
            uint32_t nt;
            if (any_out) {
                nt = kOut;
            } else if (all_eq) {
                nt = kIn;
            } else {
                nt = make_tuple(next, (uint32_t)v[0]);
                keep = true;
            }
            T[v[0]] = nt;
        }
        seg_append(io, sg, keep, v[0], kept);
        wave_lds_fence();
        if (more) {
            v[0] = vn[0];
            ok[0] = okn[0];
            s = sn;
            e = en;
            t0 = tn;
            mv = mvn;
        }
    }
    if (io.deg_sum) wave_degsum(io.deg_sum, dsum);
    return kept;
}

// ---------------------------------------------------------------------------
// Flat ("merge path") sweeps.  A wavefront takes its rows 64 at a time, one
// per lane, lays their column indices out as one flat range (offsets and
// starts in LDS) and lets every lane stream kFlatEP consecutive indices of
// that range per step.  All loads of a step are independent, so a batch of
// 64 rows needs about 2 + 2 * ceil(edges / (64 * kFlatEP)) dependent memory
// steps instead of one chain per row.  Each lane folds its edges into a
// partial result per row it touches and merges it into the row's LDS slot
// with an order-free atomic (min, or, and).  High-degree rows are handled
// first by the whole wavefront (coop_min_T / coop_decide) and leave the
// flat range.
// ---------------------------------------------------------------------------
constexpr int kFlatEP = 8;     // consecutive edges per lane per step
constexpr int kFlatRows = 64;  // rows per batch (one per lane)
constexpr int64_t kFlatHeavy = 4096;  // rows longer than this take the cooperative path

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wavefront LDS of a flat batch.
struct FlatLds {
    uint32_t off[kFlatRows + 1];  // flat offsets of the compacted non-empty rows
    int64_t start[kFlatRows];     // their first column index
    uint32_t t0[kFlatRows];       // their T_v (Decide Set)
    uint32_t acc[kFlatRows];      // min (Refresh Column) or any-OUT (Decide Set)
    uint32_t acc2[kFlatRows];     // all-equal (Decide Set)
};

// Loads the batch's rows (one per lane), compacts the non-empty light rows
// into the LDS table and returns this lane's table index (-1 if none).
// total: flat length of the batch.
__device__ __forceinline__ int flat_table(FlatLds &sh, int64_t s, int64_t len, bool light,
                                          uint32_t &total) {
    const int lane = (int)(threadIdx.x & 63u);
    const bool in = light && len > 0;
    const uint64_t mask = __ballot(in);
    const int idx = (int)__popcll(mask & lanes_below(lane));
    // exclusive prefix of the lengths over the compacted rows
    uint32_t l32 = in ? (uint32_t)len : 0u;
    uint32_t incl = l32;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
        if (lane >= o) incl += y;
    }
    total = (uint32_t)__shfl((int)incl, 63, 64);
    if (in) {
        sh.off[idx] = incl - l32;
        sh.start[idx] = s;
    }
    if (lane == 0) sh.off[__popcll(mask)] = total;
    return in ? idx : -1;
}

// Row of flat edge f: the last table row whose offset is <= f (7 fixed steps).
__device__ __forceinline__ int flat_row(const FlatLds &sh, int nrows, uint32_t f) {
    int lo = 0, hi = nrows;
    for (int k = 0; k < 7; k++) {
        const int mid = (lo + hi) >> 1;
        if (mid > lo && sh.off[mid] <= f) lo = mid; else if (mid > lo) hi = mid;
    }
    return lo;
}

template <int U>
__device__ __forceinline__ uint32_t flat_column(const int64_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col,
                                                const uint32_t *__restrict__ T,
                                                uint32_t *__restrict__ M, const SegIO &io,
                                                const Seg &sg, FlatLds &sh) {
    const int lane = (int)(threadIdx.x & 63u);
    uint32_t kept = 0;
    unsigned long long dsum = 0;
    for (int64_t i0 = 0; i0 < sg.count; i0 += kFlatRows) {
        const int64_t i = i0 + lane;
        const bool ok = i < sg.count;
        const int64_t ic = ok ? i : sg.count - 1;
        const int32_t v = io.wl_in ? io.wl_in[sg.base + ic] : (int32_t)(sg.base + ic);
        const int64_t s = row_ptr[v], e = row_ptr[v + 1];
        uint32_t m = T[v];
        const int64_t len = ok ? e - s : 0;
        dsum += (unsigned long long)len;
        // high-degree rows: the whole wavefront, one at a time
        uint64_t heavy = __ballot(len > kFlatHeavy);
        while (heavy) {
            const int src = __ffsll((unsigned long long)heavy) - 1;
            heavy &= heavy - 1;
            const uint32_t hm =
                coop_min_T(col, T, __shfl(s, src, 64), __shfl(e, src, 64), nullptr, nullptr, &io);
            if (lane == src) m = min(m, hm);
        }
        uint32_t total;
        const int me = flat_table(sh, s, len, len <= kFlatHeavy, total);
        const int nrows = (int)__popcll(__ballot(me >= 0));
        if (me >= 0) sh.acc[me] = kOut;
        wave_lds_sync();
        for (uint32_t c0 = 0; c0 < total; c0 += 64 * kFlatEP) {
            const uint32_t f0 = c0 + (uint32_t)lane * kFlatEP;
            int r = f0 < total ? flat_row(sh, nrows, f0) : 0;
            int32_t x[kFlatEP];
            int rr[kFlatEP];
#pragma unroll
            for (int j = 0; j < kFlatEP; j++) {
                const uint32_t f = f0 + j;
                if (f < total && r + 1 < nrows && sh.off[r + 1] <= f) r++;
                rr[j] = r;
                x[j] = col[f < total ? sh.start[r] + (int64_t)(f - sh.off[r]) : 0];
            }
            uint32_t t[kFlatEP];
            if (io.gen0) {
#pragma unroll
                for (int j = 0; j < kFlatEP; j++) t[j] = make_tuple(io.t0, (uint32_t)x[j]);
            } else {
#pragma unroll
                for (int j = 0; j < kFlatEP; j++) t[j] = T[x[j]];
            }
            uint32_t part = kOut;
            int pr = rr[0];
#pragma unroll
            for (int j = 0; j < kFlatEP; j++) {
                if (f0 + j < total) {
                    if (rr[j] != pr) {
                        atomicMin(&sh.acc[pr], part);
                        part = kOut;
                        pr = rr[j];
                    }
                    part = min(part, t[j]);
                }
            }
            if (f0 < total) atomicMin(&sh.acc[pr], part);
        }
        wave_lds_sync();
        if (me >= 0) m = min(m, sh.acc[me]);
        bool keep = false;
        if (ok) {
            if (io.gen0 == 2 && M[v] == kOut) m = kOut;  // pushed by an IN vertex
            if (m == kIn) m = kOut;
            M[v] = m;
            keep = (m != kOut);
        }
        seg_append(io, sg, keep, v, kept);
        wave_lds_sync();
    }
    if (io.deg_sum) wave_degsum(io.deg_sum, dsum);
    return kept;
}

template <int U>
__device__ __forceinline__ uint32_t flat_decide(const int64_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col,
                                                uint32_t *__restrict__ T,
                                                const uint32_t *__restrict__ M,
                                                const TupleParams &next, const SegIO &io,
                                                const Seg &sg, FlatLds &sh) {
    const int lane = (int)(threadIdx.x & 63u);
    uint32_t kept = 0;
    unsigned long long dsum = 0;
    for (int64_t i0 = 0; i0 < sg.count; i0 += kFlatRows) {
        const int64_t i = i0 + lane;
        const bool ok = i < sg.count;
        const int64_t ic = ok ? i : sg.count - 1;
        const int32_t v = io.wl_in ? io.wl_in[sg.base + ic] : (int32_t)(sg.base + ic);
        const int64_t s = row_ptr[v], e = row_ptr[v + 1];
        const uint32_t t0 = T[v];
        const uint32_t mv = M[v];
        int any_out = mv == kOut;
        int all_eq = mv == t0;
        // in round 1, near[v] stands for the neighbours' OUT test
        const bool by_near = io.dec1 && ok && mv != kOut && mv != t0;
        if (by_near) any_out = io.near[v] != 0;
        dsum += (unsigned long long)(ok ? e - s : 0);
        // M_v = OUT already decides the row (OUT), whatever the neighbours
        // hold; in round 0, M_v != T_v keeps it undecided
        const int64_t len = ok && mv != kOut && !(io.dec0 && mv != t0) && !by_near ? e - s : 0;
        uint64_t heavy = __ballot(len > kFlatHeavy);
        while (heavy) {
            const int src = __ffsll((unsigned long long)heavy) - 1;
            heavy &= heavy - 1;
            int hao, hae;
            coop_decide(col, M, __shfl(s, src, 64), __shfl(e, src, 64), __shfl(t0, src, 64), hao,
                        hae);
            if (lane == src) {
                any_out |= hao;
                all_eq &= hae;
            }
        }
        uint32_t total;
        const int me = flat_table(sh, s, len, len <= kFlatHeavy, total);
        const int nrows = (int)__popcll(__ballot(me >= 0));
        if (me >= 0) {
            sh.t0[me] = t0;
            sh.acc[me] = 0u;
            sh.acc2[me] = 1u;
        }
        wave_lds_sync();
        for (uint32_t c0 = 0; c0 < total; c0 += 64 * kFlatEP) {
            const uint32_t f0 = c0 + (uint32_t)lane * kFlatEP;
            int r = f0 < total ? flat_row(sh, nrows, f0) : 0;
            int32_t x[kFlatEP];
            int rr[kFlatEP];
#pragma unroll
            for (int j = 0; j < kFlatEP; j++) {
                const uint32_t f = f0 + j;
                if (f < total && r + 1 < nrows && sh.off[r + 1] <= f) r++;
                rr[j] = r;
                x[j] = col[f < total ? sh.start[r] + (int64_t)(f - sh.off[r]) : 0];
            }
            uint32_t mw[kFlatEP];
#pragma unroll
            for (int j = 0; j < kFlatEP; j++) mw[j] = M[x[j]];
            int pr = rr[0];
            uint32_t pt0 = sh.t0[pr];
            uint32_t pao = 0u, pae = 1u;
#pragma unroll
            for (int j = 0; j < kFlatEP; j++) {
                if (f0 + j < total) {
                    if (rr[j] != pr) {
                        if (pao) atomicOr(&sh.acc[pr], 1u);
                        if (!pae) atomicAnd(&sh.acc2[pr], 0u);
                        pao = 0u;
                        pae = 1u;
                        pr = rr[j];
                        pt0 = sh.t0[pr];
                    }
                    pao |= (mw[j] == kOut);
                    pae &= (mw[j] == pt0) | (mw[j] == kAbsent);
                }
            }
            if (f0 < total) {
                if (pao) atomicOr(&sh.acc[pr], 1u);
                if (!pae) atomicAnd(&sh.acc2[pr], 0u);
            }
        }
        wave_lds_sync();
        if (me >= 0) {
            any_out |= (int)sh.acc[me];
            all_eq &= (int)sh.acc2[me];
        }
        bool keep = false;
        if (ok) {
            uint32_t nt;
            if (any_out) {
                nt = kOut;
            } else if (all_eq) {
                nt = kIn;
            } else {
                nt = make_tuple(next, (uint32_t)v);
                keep = true;
            }
            T[v] = nt;
        }
        seg_append(io, sg, keep, v, kept);
        wave_lds_sync();
    }
    if (io.deg_sum) wave_degsum(io.deg_sum, dsum);
    return kept;
}

// lanes == 0 in the plan selects the flat sweeps.
template <int L, bool RD = false, bool WR = false>
__device__ __forceinline__ uint32_t any_column(const int64_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col,
                                               const uint32_t *__restrict__ T,
                                               uint32_t *__restrict__ M, const SegIO &io,
                                               const Seg &sg) {
    if constexpr (L == 0) {
        __shared__ FlatLds sh[kBlock / 64];
        return flat_column<kUnroll>(row_ptr, col, T, M, io, sg, sh[threadIdx.x >> 6]);
    } else if constexpr (L == kStagedLanes) {
        __shared__ StagedLds<1> sh[kBlock / 64];
        return sweep_column_staged<1, RD, WR>(row_ptr, col, T, M, io, sg, sh[threadIdx.x >> 6]);
    } else {
        return sweep_column<L, kRows, kChunks<L>, RD, WR>(row_ptr, col, T, M, io, sg);
    }
}

template <int L>
__device__ __forceinline__ uint32_t any_decide(const int64_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col,
                                               uint32_t *__restrict__ T,
                                               const uint32_t *__restrict__ M,
                                               const TupleParams &next, const SegIO &io,
                                               const Seg &sg) {
    if constexpr (L == 0) {
        __shared__ FlatLds sh[kBlock / 64];
        return flat_decide<kUnroll>(row_ptr, col, T, M, next, io, sg, sh[threadIdx.x >> 6]);
    } else if constexpr (L == kStagedLanes) {
        __shared__ StagedLds<1> sh[kBlock / 64];
        return sweep_decide_staged<1>(row_ptr, col, T, M, next, io, sg, sh[threadIdx.x >> 6]);
    } else {
        return sweep_decide<L, kRows, kChunks<L>>(row_ptr, col, T, M, next, io, sg);
    }
}

// ---------------------------------------------------------------------------
// Launched rounds.  A round past the end of the run finds empty per-wavefront
// lists and does nothing; workgroup 0 of each Refresh Column records the
// round's sizes and reports |worklist1| to the host.
// ---------------------------------------------------------------------------
__device__ __forceinline__ SegIO round_col_io(const RoundsArgs &a, int r) {
    const int cur = r & 1, nxt = cur ^ 1;
    const bool first = r == 0;
    SegIO io{};
    io.wl_in = first ? (a.masked ? a.wl1[0] : nullptr) : a.wl2[cur];
    io.cnt_in = first ? (a.masked ? a.cnt1[0] : nullptr) : a.cnt2[cur];
    io.wl_out = a.wl2[nxt];
    io.cnt_out = a.cnt2[nxt];
    io.trace_out = a.ctr + (size_t)((r + 1) % kCtrRing) * kCtrSlot + kCtrList;
    io.deg_sum = a.dsplit ? a.dsplit + (size_t)kSplit * kDegLine : nullptr;
    io.n = a.n;
    io.seg = a.seg;
    io.S = a.S;
    io.nnz = a.nnz;
    if (r == 0 && !a.masked) io.long_flag = a.lflag;
    if (r <= 1 && a.gen0 && !a.masked && !a.batch.voff && !a.abl) {
        io.gen0 = r + 1;
        io.t0 = TupleParams{xs64star((a.seed << 32) ^ (uint64_t)r), a.pmask, a.b, a.batch};
    }
    return io;
}

__device__ __forceinline__ SegIO round_dec_io(const RoundsArgs &a, int r) {
    const int cur = r & 1, nxt = cur ^ 1;
    const bool first = r == 0;
    SegIO io{};
    io.wl_in = first ? (a.masked ? a.wl1[0] : nullptr) : a.wl1[cur];
    io.cnt_in = first ? (a.masked ? a.cnt1[0] : nullptr) : a.cnt1[cur];
    io.wl_out = a.wl1[nxt];
    io.cnt_out = a.cnt1[nxt];
    io.trace_out = a.ctr + (size_t)((r + 1) % kCtrRing) * kCtrSlot;
    io.deg_sum = a.dsplit;
    io.n = a.n;
    io.seg = a.seg;
    io.S = a.S;
    io.nnz = a.nnz;
    io.dec0 = r == 0;
    if (r == 1 && a.gen0 && !a.masked && !a.batch.voff && !a.abl && a.near) {
        io.dec1 = true;
        io.near = a.near;
    }
    return io;
}

// Sizes of worklist1 / worklist2 at the start of round r (wavefront 0; the
// identity start has n of each, a masked start its active count in slot 0).
__device__ __forceinline__ void round_sizes(const RoundsArgs &a, int r, uint32_t &c1,
                                            uint32_t &c2) {
    if (r == 0 && !a.masked) {
        c1 = c2 = (uint32_t)a.n;
        return;
    }
    const uint32_t *slot = a.ctr + (size_t)(r % kCtrRing) * kCtrSlot;
    c1 = ctr_sum(slot);
    c2 = r == 0 ? c1 : ctr_sum(slot + kCtrList);
}

// Refresh Column of round r.  Workgroup 0 records the round's sizes and
// reports (r, |worklist1|) to the host, with bit 31 of the low word set from
// round 1 on when round 0 met rows long enough for the cooperative pass.
// RD / WR: read / write the compacted rows.
__device__ __forceinline__ void round_start(const RoundsArgs &a, int r) {
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        uint32_t c1, c2;
        round_sizes(a, r, c1, c2);
        const uint32_t longs = (r >= 1 && !a.masked && a.lflag) ? ctr_sum(a.lflag) : 0u;
        if (threadIdx.x == 0) {
            a.rt[(size_t)r * kRoundStride] = c1;
            a.rt[(size_t)r * kRoundStride + 1] = c2;
            if (a.rt_host) {
                // the host reads the sizes after the call without a copy
                a.rt_host[(size_t)r * kRoundStride] = c1;
                a.rt_host[(size_t)r * kRoundStride + 1] = c2;
            }
            if (a.alive_host) {
                // word 1: (round, |worklist2|), stored before word 0 so that a
                // host that reads word 0 of round r finds word 1 of round r
                __hip_atomic_store(a.alive_host + 1, host_word(a.epoch, r, c2), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(a.alive_host,
                                   host_word(a.epoch, r, c1 | (longs ? kLongRowsBit : 0u)),
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
    clear_slot(a.ctr, r);
}

// GEN: the kernel that may compute the tuples of rounds 0 and 1
// (k_col_round0); the others never do, so the code that would is compiled
// out of them.
template <int L, bool RD, bool WR, bool GEN = false>
__device__ __forceinline__ void col_round(const int64_t *__restrict__ row_ptr,
                                          const int32_t *__restrict__ col,
                                          const uint32_t *__restrict__ T, uint32_t *__restrict__ M,
                                          const RoundsArgs &a, int r) {
    round_start(a, r);
    SegIO io = round_col_io(a, r);
    if (!GEN) io.gen0 = 0;
    if (RD) {
        io.ccol_in = a.colc;
        io.lenc_in = a.lenc;
    }
    if (WR) {
        io.ccol_out = a.colc;
        io.lenc_out = a.lenc;
    }
    const int64_t w = wave_id();
    const Seg sg = seg_of(io, w);
    const uint32_t kept = any_column<L, RD, WR>(row_ptr, col, T, M, io, sg);
    seg_finish(io, w, kept);
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_col_round(const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const uint32_t *__restrict__ T,
                                                      uint32_t *__restrict__ M, RoundsArgs a,
                                                      int r) {
    col_round<L, false, false>(row_ptr, col, T, M, a, r);
}

// Rounds 0 and 1: computes the neighbours' tuples where that is exact
// (unmasked, one graph; round 1 after k_push_in), else gathers them as
// k_col_round does.
template <int L>
__global__ __launch_bounds__(kBlock) void k_col_round0(const int64_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col,
                                                       const uint32_t *__restrict__ T,
                                                       uint32_t *__restrict__ M, RoundsArgs a,
                                                       int r) {
    col_round<L, false, false, true>(row_ptr, col, T, M, a, r);
}

// The first compacting round: reads the CSR's rows, writes compacted ones.
template <int L>
__global__ __launch_bounds__(kBlock) void k_col_round_w(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const uint32_t *__restrict__ T,
                                                        uint32_t *__restrict__ M, RoundsArgs a,
                                                        int r) {
    col_round<L, false, true>(row_ptr, col, T, M, a, r);
}

// Later compacting rounds: read compacted rows and rewrite the long ones.
template <int L>
__global__ __launch_bounds__(kBlock) void k_col_round_rw(const int64_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const uint32_t *__restrict__ T,
                                                         uint32_t *__restrict__ M, RoundsArgs a,
                                                         int r) {
    col_round<L, true, true>(row_ptr, col, T, M, a, r);
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_dec_round(const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      uint32_t *__restrict__ T,
                                                      const uint32_t *__restrict__ M,
                                                      RoundsArgs a, int r) {
    const SegIO io = round_dec_io(a, r);
    const TupleParams next{xs64star((a.seed << 32) ^ (uint64_t)(r + 1)), a.pmask, a.b, a.batch};
    const int64_t w = wave_id();
    const Seg sg = seg_of(io, w);
    const uint32_t kept = any_decide<L>(row_ptr, col, T, M, next, io, sg);
    seg_finish(io, w, kept);
}

// ---------------------------------------------------------------------------
// Tail: the last rounds of a run in one workgroup.  Once both worklists hold
// at most kTailCap vertices, the round kernels would spend their time on
// dispatching a full grid for a few thousand rows, and the host on issuing
// them; one workgroup instead copies the per-wavefront lists into LDS and
// runs Refresh Column, Decide Set and the compaction of both lists round
// after round, with workgroup barriers between the phases (every wavefront
// is on one compute unit, so the barriers order the global stores too),
// until worklist1 is empty.  The arithmetic per row is that of the round
// kernels: long rows (beyond kTailRowCap entries) go to a whole wavefront,
// and rows longer than the plan's cooperative threshold are read and
// rewritten in compacted form exactly as the launched rounds would.
// ---------------------------------------------------------------------------
constexpr int kTailThreads = 1024;
constexpr int kTailWaves = kTailThreads / 64;
constexpr int kTailRowCap = 32;  // longer rows: a whole wavefront each

struct TailLds {
    int32_t l1[kTailCap];
    int32_t l2[kTailCap];
    uint16_t off[kMaxBlocks];  // tail_gather: first list position of each workgroup's entries
    uint8_t keep[kTailCap];
    uint32_t wtot[kTailWaves];
    unsigned long long wsum[kTailWaves][3];
    uint32_t n1, n2;
};

// Exclusive prefix of x over the workgroup (in thread order); *total gets the
// sum.  All threads call it; it ends with a barrier.
__device__ __forceinline__ uint32_t tail_scan(TailLds &sh, uint32_t x, uint32_t *total) {
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    const uint32_t inc = wave_incl_scan(x);
    if (lane == 63) sh.wtot[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int q = 0; q < kTailWaves; q++) {
        const uint32_t c = sh.wtot[q];
        before += q < w ? c : 0u;
        all += c;
    }
    *total = all;
    __syncthreads();
    return before + inc - x;
}

// Sums over the workgroup of three counters (thread 0 gets them).
__device__ __forceinline__ void tail_sum3(TailLds &sh, unsigned long long a, unsigned long long b,
                                          unsigned long long c, unsigned long long *out) {
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
        c += __shfl_xor(c, off, 64);
    }
    if (lane == 0) {
        sh.wsum[w][0] = a;
        sh.wsum[w][1] = b;
        sh.wsum[w][2] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = out[1] = out[2] = 0;
        for (int q = 0; q < kTailWaves; q++)
            for (int k = 0; k < 3; k++) out[k] += sh.wsum[q][k];
    }
    __syncthreads();
}

// Copies the per-wavefront segments of a worklist (S = 4 B segments of seg
// slots, counts cnt; wavefronts 4b .. 4b + 3 belong to workgroup b) into dst
// in segment order; returns the size (at most kTailCap, which the host
// checked; more returns 0xFFFFFFFF).  Thread t first adds the counts of
// workgroups tJ .. tJ + J - 1 (16-byte loads, all in flight at once), a
// workgroup scan gives each workgroup its first position (kept in LDS as 16
// bits), and then every thread copies up to kTailCap / kTailThreads entries:
// a binary search in those positions finds an entry's workgroup, its four
// counts its wavefront.  Only positions below the size are searched and
// copied, and with copy false only the size is taken (a run that has ended
// needs no list).
__device__ uint32_t tail_gather(TailLds &sh, const int32_t *wl, const uint32_t *cnt, int64_t S,
                                int64_t seg, int32_t *dst, bool copy = true) {
    constexpr int kJ = kMaxBlocks / kTailThreads;  // workgroups per thread, at most
    const int B = (int)(S / 4);
    const int J = (B + kTailThreads - 1) / kTailThreads;
    const int tid = (int)threadIdx.x;
    uint32_t tot[kJ];
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < kJ; j++) {
        const int b = tid * J + j;
        const bool ok = j < J && b < B;
        const uint4 c = *(const uint4 *)(cnt + 4 * (size_t)(ok ? b : 0));
        tot[j] = ok ? c.x + c.y + c.z + c.w : 0u;
        mine += tot[j];
    }
    uint32_t total = 0;
    uint32_t at = tail_scan(sh, mine, &total);
    if (total > (uint32_t)kTailCap) return 0xFFFFFFFFu;  // the same in every thread
    if (!copy || total == 0u) return total;
#pragma unroll
    for (int j = 0; j < kJ; j++) {
        const int b = tid * J + j;
        if (j < J && b < B) sh.off[b] = (uint16_t)at;
        at += tot[j];
    }
    __syncthreads();
    constexpr int kPer = kTailCap / kTailThreads;
    int32_t val[kPer];
#pragma unroll
    for (int i = 0; i < kPer; i++) {
        const uint32_t p = (uint32_t)(tid + i * kTailThreads);
        val[i] = 0;
        if (p < total) {
            // the last workgroup whose first position is <= p (a workgroup
            // after an empty one starts where it starts, so this one holds
            // entry p)
            int lo = 0, hi = B - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((uint32_t)sh.off[mid] <= p) lo = mid; else hi = mid - 1;
            }
            const uint4 c = *(const uint4 *)(cnt + 4 * (size_t)lo);
            uint32_t q = p - (uint32_t)sh.off[lo];
            int w = 0;
            if (q >= c.x) { q -= c.x; w = 1;
                if (q >= c.y) { q -= c.y; w = 2;
                    if (q >= c.z) { q -= c.z; w = 3; } } }
            val[i] = wl[(4 * (int64_t)lo + w) * seg + q];
        }
    }
#pragma unroll
    for (int i = 0; i < kPer; i++) {
        const uint32_t p = (uint32_t)(tid + i * kTailThreads);
        if (p < total) dst[p] = val[i];
    }
    __syncthreads();
    return total;
}

// Keeps the entries of list[0, n) whose sh.keep flag is set, in order and in
// place: entries are taken kTailThreads at a time, and each chunk is read
// before any slot of it is written.  Returns the new size.
__device__ uint32_t tail_compact(TailLds &sh, int32_t *list, uint32_t n) {
    uint32_t kept = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += kTailThreads) {
        const uint32_t i = i0 + threadIdx.x;
        const bool keep = i < n && sh.keep[i] != 0;
        const int32_t v = i < n ? list[i] : 0;
        uint32_t total = 0;
        const uint32_t pos = tail_scan(sh, keep ? 1u : 0u, &total);  // ends with a barrier
        if (keep) list[kept + pos] = v;
        kept += total;
        __syncthreads();
    }
    return kept;
}

// Device wall clock (constant rate) into two round-table words.
__device__ __forceinline__ void stamp(uint32_t *p) {
    const uint64_t t = wall_clock64();
    p[0] = (uint32_t)t;
    p[1] = (uint32_t)(t >> 32);
}

struct TailArgs {
    int r0;          // first round run here
    int cstart;      // first compacting round (mode 1), later rounds mode 2; < 0: no compaction
    int64_t thr;     // cooperative threshold of the launched plan (rows longer are compacted)
    uint32_t *rt_host;               // host-pinned round table of this phase (rows >= r0)
    unsigned long long *end_host;    // host-pinned: rounds + 1 of the run, written at the end
};

__global__ __launch_bounds__(kTailThreads) void k_tail(const int64_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col,
                                                       uint32_t *__restrict__ T,
                                                       uint32_t *__restrict__ M, RoundsArgs a,
                                                       TailArgs ta) {
    __shared__ TailLds sh;
    const int lane = (int)(threadIdx.x & 63u);
    const int tid = (int)threadIdx.x;
    int r = ta.r0;
    {
        const int cur = r & 1;
        const uint32_t c1 = tail_gather(sh, a.wl1[cur], a.cnt1[cur], a.S, a.seg, sh.l1);
        // an empty worklist1 ends the run at once: worklist2's size is still
        // recorded, its entries are not needed
        const uint32_t c2 = tail_gather(sh, a.wl2[cur], a.cnt2[cur], a.S, a.seg, sh.l2, c1 != 0u);
        if (tid == 0) {
            sh.n1 = c1;
            sh.n2 = c2;
        }
        __syncthreads();
    }
    for (;;) {
        const uint32_t n1 = sh.n1, n2 = sh.n2;
        uint32_t *rth = ta.rt_host + (size_t)r * kRoundStride;
        if (tid == 0) {
            a.rt[(size_t)r * kRoundStride] = n1;
            a.rt[(size_t)r * kRoundStride + 1] = n2;
            rth[0] = n1;
            rth[1] = n2;
            stamp(rth + kRtStamp0);  // wall-clock stamps of the round's phases
        }
        if (n1 == 0u || n1 == 0xFFFFFFFFu || n2 == 0xFFFFFFFFu || r + 2 >= a.max_rounds) break;
        const bool rd = ta.cstart >= 0 && r > ta.cstart && a.colc;
        const bool wr = ta.cstart >= 0 && r >= ta.cstart && a.colc;
        // Refresh Column over worklist2
        unsigned long long dcol = 0, dwr = 0;
        for (uint32_t i0 = 0; i0 < n2; i0 += kTailThreads) {
            const bool has = i0 + (uint32_t)tid < n2;
            const int32_t v = has ? sh.l2[i0 + tid] : 0;
            int64_t s = row_ptr[v], e = has ? row_ptr[v + 1] : s;
            const bool cf = rd && e - s > ta.thr;
            if (cf) e = s + a.lenc[v];
            const int32_t *src = cf ? a.colc : col;
            uint32_t m = T[v];
            dcol += (unsigned long long)(e - s);
            uint32_t wc = 0;
            bool wrote = false;
            uint64_t heavy = __ballot(e - s > kTailRowCap);
            while (heavy) {
                const int q = __ffsll((unsigned long long)heavy) - 1;
                heavy &= heavy - 1;
                const int64_t hs = __shfl(s, q, 64), he = __shfl(e, q, 64);
                const bool hcf = __shfl((int)cf, q, 64) != 0;
                // rewritten only where the launched rounds would rewrite it
                const bool hw = wr && he - hs > ta.thr;
                uint32_t hwc = 0;
                const uint32_t hm = coop_min_T(hcf ? a.colc : col, T, hs, he,
                                               hw ? a.colc : nullptr, hw ? &hwc : nullptr);
                if (lane == 0) dwr += hwc;
                if (lane == q) {
                    m = min(m, hm);
                    e = s;
                    wc = hwc;
                    wrote = hw;
                }
            }
            {
                // a short row's entries all load at once, from clamped valid
                // addresses (entry 0 exists: the host runs the tail only when
                // nnz > 0); slots past the row's end gather v itself
                const int64_t hi = e > s ? e - 1 : 0;
                int32_t x[kTailRowCap];
#pragma unroll
                for (int k = 0; k < kTailRowCap; k++) {
                    const int32_t y = src[min(s + k, hi)];
                    x[k] = s + k < e ? y : v;
                }
                uint32_t t[kTailRowCap];
#pragma unroll
                for (int k = 0; k < kTailRowCap; k++) t[k] = T[x[k]];
#pragma unroll
                for (int k = 0; k < kTailRowCap; k++) m = min(m, t[k]);
            }
            if (has) {
                if (m == kIn) m = kOut;
                M[v] = m;
                sh.keep[i0 + tid] = m != kOut;
                if (wrote && m != kOut) a.lenc[v] = (int32_t)wc;
            }
        }
        __syncthreads();  // M of this round is complete
        const uint32_t kept2 = tail_compact(sh, sh.l2, n2);
        if (tid == 0) stamp(rth + kRtStamp1);
        // Decide Set over worklist1, with the next round's tuples
        const TupleParams next{xs64star((a.seed << 32) ^ (uint64_t)(r + 1)), a.pmask, a.b, a.batch};
        unsigned long long ddec = 0;
        for (uint32_t i0 = 0; i0 < n1; i0 += kTailThreads) {
            const bool has = i0 + (uint32_t)tid < n1;
            const int32_t v = has ? sh.l1[i0 + tid] : 0;
            int64_t s = row_ptr[v], e = has ? row_ptr[v + 1] : s;
            const uint32_t t0 = T[v], mv = M[v];
            ddec += (unsigned long long)(e - s);
            int any_out = mv == kOut, all_eq = mv == t0;
            if (mv == kOut) e = s;
            uint64_t heavy = __ballot(e - s > kTailRowCap);
            while (heavy) {
                const int q = __ffsll((unsigned long long)heavy) - 1;
                heavy &= heavy - 1;
                const int64_t hs = __shfl(s, q, 64), he = __shfl(e, q, 64);
                const uint32_t ht0 = __shfl(t0, q, 64);
                int hao, hae;
                coop_decide(col, M, hs, he, ht0, hao, hae);
                if (lane == q) {
                    any_out |= hao;
                    all_eq &= hae;
                    e = s;
                }
            }
            {
                const int64_t hi = e > s ? e - 1 : 0;
                int32_t x[kTailRowCap];
#pragma unroll
                for (int k = 0; k < kTailRowCap; k++) {
                    const int32_t y = col[min(s + k, hi)];
                    x[k] = s + k < e ? y : v;
                }
                uint32_t mw[kTailRowCap];
#pragma unroll
                for (int k = 0; k < kTailRowCap; k++) mw[k] = M[x[k]];
#pragma unroll
                for (int k = 0; k < kTailRowCap; k++) {
                    if (s + k < e) {
                        any_out |= (mw[k] == kOut);
                        all_eq &= (mw[k] == t0) | (mw[k] == kAbsent);
                    }
                }
            }
            if (has) {
                uint32_t nt;
                bool keep = false;
                if (any_out) {
                    nt = kOut;
                } else if (all_eq) {
                    nt = kIn;
                } else {
                    nt = make_tuple(next, (uint32_t)v);
                    keep = true;
                }
                T[v] = nt;
                sh.keep[i0 + tid] = keep;
            }
        }
        __syncthreads();
        const uint32_t kept1 = tail_compact(sh, sh.l1, n1);
        if (tid == 0) stamp(rth + kRtStamp2);
        if (a.degs) {
            unsigned long long tot[3];
            tail_sum3(sh, ddec, dcol, dwr, tot);
            if (tid == 0) {
                a.degs[kDegStride * r] = tot[0];
                a.degs[kDegStride * r + 1] = tot[1];
                a.degs[kDegStride * r + 2] = tot[2];
            }
        }
        if (tid == 0) {
            sh.n1 = kept1;
            sh.n2 = kept2;
        }
        __syncthreads();  // T of this round and the new sizes are complete
        r++;
    }
    if (tid == 0)
        __hip_atomic_store(ta.end_host, (unsigned long long)(r + 1), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---------------------------------------------------------------------------
// Persistent form: one cooperative launch runs every round of Algorithm 1.
// The grid synchronises twice per round (after Refresh Column and after
// Decide Set) with an epoch barrier: each workgroup publishes its epoch in
// its own flag word, workgroup 0 waits for all flags and publishes the epoch,
// and everyone waits for that.  Writes are released and acquired at device
// (agent) scope around the flags, so M and T written before a barrier are
// seen after it.  Every wait is bounded by a wall-clock limit; a timeout sets
// an abort word that makes every later wait return at once, so all
// wavefronts always leave the kernel.
// ---------------------------------------------------------------------------
constexpr uint64_t kBarrierTimeoutTicks = 2000000000ull;  // wall clock ticks (about 20 s at 100 MHz)

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// Returns false if the barrier timed out (or had timed out before).
__device__ bool grid_barrier(uint32_t *flags, uint32_t *gen, uint32_t *abort_word,
                             uint32_t epoch) {
    __shared__ uint32_t ok_s;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();  // release this workgroup's writes
        st_agent(&flags[blockIdx.x], epoch);
    }
    if (blockIdx.x == 0) {
        const uint64_t t0 = wall_clock64();
        for (uint32_t b = threadIdx.x; b < gridDim.x; b += blockDim.x) {
            while (ld_agent(&flags[b]) < epoch) {
                if (ld_agent(abort_word) || wall_clock64() - t0 > kBarrierTimeoutTicks) {
                    st_agent(abort_word, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) st_agent(gen, epoch);
    }
    if (threadIdx.x == 0) {
        const uint64_t t0 = wall_clock64();
        while (ld_agent(gen) < epoch) {
            if (ld_agent(abort_word) || wall_clock64() - t0 > kBarrierTimeoutTicks) {
                st_agent(abort_word, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __threadfence();  // acquire everyone's writes
        ok_s = ld_agent(abort_word) == 0u;
    }
    __syncthreads();
    return ok_s != 0u;
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_rounds(const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col,
                                                   uint32_t *__restrict__ T,
                                                   uint32_t *__restrict__ M, RoundsArgs a) {
    __shared__ uint32_t alive_s;
    const int64_t w = wave_id();
    uint32_t *flags = a.bar;
    uint32_t *gen = a.bar + kMaxBlocks;
    uint32_t *abort_word = a.bar + kMaxBlocks + 16;
    uint32_t epoch = 0;
    int r = 0;
    // round 0 sizes: the masked start's counters (slot 0); the host wrote
    // them for the identity start
    if (blockIdx.x == 0 && threadIdx.x < 64 && a.masked) {
        const uint32_t c = ctr_sum(a.ctr);
        if (threadIdx.x == 0) {
            a.rt[0] = c;
            a.rt[1] = c;
        }
    }
    for (;;) {
        uint32_t *slot_next = a.ctr + (size_t)((r + 1) % kCtrRing) * kCtrSlot;
        SegIO cio = round_col_io(a, r);
        cio.gen0 = 0;  // the persistent kernel gathers in every round
        clear_slot(a.ctr, r);
        uint32_t *row_cur = a.rt + (size_t)r * kRoundStride;
        if (blockIdx.x == 0 && threadIdx.x == 0) stamp(row_cur + kRtStamp0);
        Seg sg = seg_of(cio, w);
        uint32_t kept = any_column<L>(row_ptr, col, T, M, cio, sg);
        seg_finish(cio, w, kept);
        if (!grid_barrier(flags, gen, abort_word, ++epoch)) break;
        if (blockIdx.x == 0 && threadIdx.x == 0) stamp(row_cur + kRtStamp1);
        if (a.dsplit && blockIdx.x == 0 && threadIdx.x < 64)
            fold_deg(a.dsplit + (size_t)kSplit * kDegLine, a.degs + kDegStride * r + 1,
                     a.degs + kDegStride * r + 2);
        SegIO dio = round_dec_io(a, r);
        dio.dec1 = false;  // the persistent kernel runs no k_push_near
        const TupleParams next{xs64star((a.seed << 32) ^ (uint64_t)(r + 1)), a.pmask, a.b, a.batch};
        sg = seg_of(dio, w);
        kept = any_decide<L>(row_ptr, col, T, M, next, dio, sg);
        seg_finish(dio, w, kept);
        if (!grid_barrier(flags, gen, abort_word, ++epoch)) break;
        if (blockIdx.x == 0 && threadIdx.x == 0) stamp(row_cur + kRtStamp2);
        if (a.dsplit && blockIdx.x == 0 && threadIdx.x < 64)
            fold_deg(a.dsplit, a.degs + kDegStride * r, nullptr);
        r++;
        // sizes at the start of round r; every workgroup needs worklist1's
        if (threadIdx.x < 64) {
            const uint32_t c1 = ctr_sum(slot_next);
            const uint32_t c2 = ctr_sum(slot_next + kCtrList);
            if (threadIdx.x == 0) {
                alive_s = c1;
                if (blockIdx.x == 0) {
                    a.rt[(size_t)r * kRoundStride] = c1;
                    a.rt[(size_t)r * kRoundStride + 1] = c2;
                }
            }
        }
        __syncthreads();
        const uint32_t alive = alive_s;
        __syncthreads();
        if (alive == 0u || r + 2 >= a.max_rounds) break;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st_agent(a.bar + kMaxBlocks + 32, (uint32_t)r);
}

__global__ __launch_bounds__(64) void k_fold_deg(unsigned long long *split,
                                                 unsigned long long *target,
                                                 unsigned long long *target_w) {
    fold_deg(split, target, target_w);
}

// Round-0 tuples for every vertex, and the round loop's start-up fills
// (words no other part of this launch touches).
__global__ __launch_bounds__(kBlock) void k_init_tuples(TupleParams tp, int64_t n,
                                                        uint32_t *__restrict__ T, FillSpans f) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        T[v] = make_tuple(tp, (uint32_t)v);
    fill_span_words(f);
}

// Induced-subgraph start: vertices with label -1 take part; the others read
// as OUT in T (neutral for the minimum) and as absent in M.  Each wavefront
// also lists the active vertices of its own range, in order, as its segment
// of both round-0 worklists.  The launch also does the round loop's
// start-up fills f (words this launch does not otherwise touch).
__global__ __launch_bounds__(kBlock) void k_init_masked(TupleParams tp, int64_t n,
                                                        const int32_t *__restrict__ label,
                                                        uint32_t *__restrict__ T,
                                                        uint32_t *__restrict__ M, SegIO io,
                                                        FillSpans f) {
    fill_span_words(f);
    const int64_t w = wave_id();
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t lo = w * io.seg, hi = min(n, lo + io.seg);
    uint32_t kept = 0;
    Seg sg{lo, 0};
    for (int64_t v0 = lo; v0 < hi; v0 += 64) {
        const int64_t v = v0 + lane;
        bool act = false;
        if (v < hi) {
            act = label[v] == -1;
            T[v] = act ? make_tuple(tp, (uint32_t)v) : kOut;
            M[v] = act ? kOut : kAbsent;
        }
        seg_append(io, sg, act, (int32_t)v, kept);
    }
    seg_finish(io, w, kept);
}

// M[v] = OUT for every v with T_v = IN and for its neighbours: one lane per
// vertex, which walks the row of an IN vertex (IN vertices are few).  Writes
// that meet store the same value.
__global__ __launch_bounds__(kBlock) void k_push_in(int64_t n, const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const uint32_t *__restrict__ T,
                                                    uint32_t *__restrict__ M) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
        if (T[v] != kIn) continue;
        M[v] = kOut;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) M[col[e]] = kOut;
    }
}

// near = 1 on every vertex whose M is OUT and on its neighbours.  A
// wavefront takes 64 vertices at a time and writes the rows of the marked
// ones, one after another, 64 entries per step, so a long row (a hub next to
// an IN vertex) costs its length / 64 steps and is walked once.
__global__ __launch_bounds__(kBlock) void k_push_near(int64_t n, const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const uint32_t *__restrict__ M,
                                                      uint8_t *__restrict__ near) {
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t W = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t base = ((int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * 64; base < n;
         base += W * 64) {
        const int64_t v = base + lane;
        const bool mark = v < n && M[v] == kOut;
        if (mark) near[v] = 1;
        uint64_t todo = __ballot(mark);
        while (todo) {
            const int j = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int64_t u = base + j;
            const int64_t s = row_ptr[u], e = row_ptr[u + 1];
            for (int64_t k = s + lane; k < e; k += 64) near[col[k]] = 1;
        }
    }
}

// status[v] = (T_v == IN); the tile's IN count goes to blocksum[tile] (tiles
// of kCountTile vertices, one per workgroup).
constexpr int kCountTile = kBlock * 8;

__global__ __launch_bounds__(kBlock) void k_status(int64_t n, const uint32_t *__restrict__ T,
                                                   uint8_t *__restrict__ status,
                                                   uint32_t *__restrict__ blocksum) {
    __shared__ uint32_t part[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kCountTile;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < kCountTile / kBlock; j++) {
        const int64_t v = base + (int64_t)j * kBlock + threadIdx.x;
        if (v < n) {
            const uint8_t in = T[v] == kIn;
            status[v] = in;
            c += in;
        }
    }
    for (int off = 32; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off, 64);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kBlock / 64; k++) t += part[k];
        blocksum[blockIdx.x] = t;
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_fill(V *__restrict__ p, V value, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = value;
}

// Up to kFillSpans fills of 32-bit words in one launch (one dispatch instead
// of one per array at the start of a run).
__global__ __launch_bounds__(kBlock) void k_fill_spans(FillSpans f) { fill_span_words(f); }

// CSR checks: bit 0 row_ptr[0] != 0, bit 1 decreasing or out-of-range
// row_ptr, bit 2 row_ptr[n] != nnz, bit 3 column out of range, bit 4
// self-loop.
__global__ __launch_bounds__(kBlock) void k_validate(int64_t n, int64_t nnz,
                                                     const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     uint32_t *__restrict__ err) {
    uint32_t bits = 0;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (tid == 0) {
        if (row_ptr[0] != 0) bits |= 1u;
        if (row_ptr[n] != nnz) bits |= 4u;
    }
    for (int64_t v = tid; v < n; v += (int64_t)gridDim.x * kBlock) {
        const int64_t s = row_ptr[v], e = row_ptr[v + 1];
        if (e < s || s < 0 || e > nnz) {
            bits |= 2u;
            continue;
        }
        for (int64_t k = s; k < e; k++) {
            const int32_t c = col[k];
            if (c < 0 || (int64_t)c >= n) bits |= 8u;
            if ((int64_t)c == v) bits |= 16u;
        }
    }
    if (bits) atomicOr(err, bits);
}

int grid_for(int64_t work, int per_block, int cap) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}


// ---------------------------------------------------------------------------
// Ablation kernels (Section V, Fig. 2 and Table I): Algorithm 1 with the
// optimizations of Section V taken away, one lane per CSR row and plain
// loops over each row.
//   UNPACKED: three-field tuples (status, priority, id) in three arrays
//             (status 0 = IN, 1 = undecided, 2 = OUT; Section V-C's
//             alternative) instead of one packed 32-bit word
//   ALL:      every round sweeps every vertex (Bell et al.; no worklists);
//             Decide Set leaves decided vertices as they are
//   a.abl:    kAblFixed = priorities drawn once (round 0's hash in every
//             round), kAblXorshift = f is xorshift*'s first stage (no
//             multiplication) instead of xorshift*
// The priority field holds the same low 32 - b bits of the hash as the
// packed tuple, so the two forms order vertices alike.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t xs64(uint64_t x) {
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    return x;
}

__device__ __forceinline__ uint64_t abl_f(uint64_t x, int abl) {
    return (abl & kAblXorshift) ? xs64(x) : xs64star(x);
}

// Priority bits of vertex v in round r.
__device__ __forceinline__ uint32_t abl_prio(const RoundsArgs &a, int r, uint32_t v) {
    const uint64_t it = (a.abl & kAblFixed) ? 0ull : (uint64_t)r;
    const uint64_t h = abl_f(abl_f((a.seed << 32) ^ it, a.abl) ^ abl_f((uint64_t)v, a.abl), a.abl);
    return (uint32_t)(h & a.pmask);
}

struct Tup3 {
    uint32_t s, p, i;
};
constexpr uint32_t kSt3In = 0, kSt3Und = 1, kSt3Out = 2;

template <bool UNPACKED>
struct AblTuple;

template <>
struct AblTuple<false> {  // packed: (priority << b) | (id + 1), IN = 0, OUT = UINT_MAX
    using T = uint32_t;
    static __device__ __forceinline__ T load(const AblTuples &t, int64_t v) { return t.s[v]; }
    static __device__ __forceinline__ void store(const AblTuples &t, int64_t v, T x) { t.s[v] = x; }
    static __device__ __forceinline__ bool less(T x, T y) { return x < y; }
    static __device__ __forceinline__ bool eq(T x, T y) { return x == y; }
    static __device__ __forceinline__ bool is_in(T x) { return x == kIn; }
    static __device__ __forceinline__ bool is_out(T x) { return x == kOut; }
    static __device__ __forceinline__ T in() { return kIn; }
    static __device__ __forceinline__ T out() { return kOut; }
    static __device__ __forceinline__ T fresh(const RoundsArgs &a, int r, uint32_t v) {
        return (uint32_t)(((uint64_t)abl_prio(a, r, v) << a.b) | (uint64_t)(v + 1u));
    }
};

template <>
struct AblTuple<true> {  // (status, priority, id) compared in that order
    using T = Tup3;
    static __device__ __forceinline__ T load(const AblTuples &t, int64_t v) {
        return Tup3{t.s[v], t.p[v], t.i[v]};
    }
    static __device__ __forceinline__ void store(const AblTuples &t, int64_t v, T x) {
        t.s[v] = x.s;
        t.p[v] = x.p;
        t.i[v] = x.i;
    }
    static __device__ __forceinline__ bool less(T x, T y) {
        if (x.s != y.s) return x.s < y.s;
        if (x.p != y.p) return x.p < y.p;
        return x.i < y.i;
    }
    static __device__ __forceinline__ bool eq(T x, T y) {
        return x.s == y.s && x.p == y.p && x.i == y.i;
    }
    static __device__ __forceinline__ bool is_in(T x) { return x.s == kSt3In; }
    static __device__ __forceinline__ bool is_out(T x) { return x.s == kSt3Out; }
    static __device__ __forceinline__ T in() { return Tup3{kSt3In, 0u, 0u}; }
    static __device__ __forceinline__ T out() { return Tup3{kSt3Out, 0u, 0u}; }
    static __device__ __forceinline__ T fresh(const RoundsArgs &a, int r, uint32_t v) {
        return Tup3{kSt3Und, abl_prio(a, r, v), v};
    }
};

// Round 0's tuples for every vertex.
template <bool UNPACKED>
__global__ __launch_bounds__(kBlock) void k_abl_init(AblTuples t, RoundsArgs a) {
    using Tu = AblTuple<UNPACKED>;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < a.n;
         v += (int64_t)gridDim.x * kBlock)
        Tu::store(t, v, Tu::fresh(a, 0, (uint32_t)v));
}

// Row v of the wavefront's rows i0 + lane (the identity range or the list
// segment); count >= 1.
__device__ __forceinline__ int32_t abl_row(const SegIO &io, const Seg &sg, int64_t i) {
    const int64_t ic = i < sg.count ? i : sg.count - 1;
    return io.wl_in ? io.wl_in[sg.base + ic] : (int32_t)(sg.base + ic);
}

// Longest row length over the wavefront: the loop over a row runs this many
// steps in every lane (a wave-uniform trip count).
__device__ __forceinline__ int64_t abl_wave_max(int64_t len) {
    for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
    return len;
}

template <bool UNPACKED, bool ALL>
__global__ __launch_bounds__(kBlock) void k_abl_col(const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, AblTuples T,
                                                    AblTuples M, RoundsArgs a, int r) {
    using Tu = AblTuple<UNPACKED>;
    round_start(a, r);
    SegIO io = round_col_io(a, r);
    if (ALL) {
        io.wl_in = nullptr;
        io.cnt_in = nullptr;
    }
    const int64_t w = wave_id();
    const Seg sg = seg_of(io, w);
    const int lane = (int)(threadIdx.x & 63u);
    uint32_t kept = 0;
    for (int64_t i0 = 0; i0 < sg.count; i0 += 64) {
        const int64_t i = i0 + lane;
        const bool ok = i < sg.count;
        const int32_t v = abl_row(io, sg, i);
        const int64_t s = row_ptr[v], e = ok ? row_ptr[v + 1] : s;
        typename Tu::T m = Tu::load(T, v);
        const int64_t steps = abl_wave_max(e - s);
        for (int64_t c = 0; c < steps; c++) {
            const int64_t j = s + c;
            const typename Tu::T t = Tu::load(T, col[j < e ? j : 0]);
            if (j < e && Tu::less(t, m)) m = t;
        }
        if (Tu::is_in(m)) m = Tu::out();
        if (ok) Tu::store(M, v, m);
        seg_append(io, sg, ok && !Tu::is_out(m), v, kept);
    }
    seg_finish(io, w, kept);
}

template <bool UNPACKED, bool ALL>
__global__ __launch_bounds__(kBlock) void k_abl_dec(const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, AblTuples T,
                                                    AblTuples M, RoundsArgs a, int r) {
    using Tu = AblTuple<UNPACKED>;
    SegIO io = round_dec_io(a, r);
    if (ALL) {
        io.wl_in = nullptr;
        io.cnt_in = nullptr;
    }
    const int64_t w = wave_id();
    const Seg sg = seg_of(io, w);
    const int lane = (int)(threadIdx.x & 63u);
    uint32_t kept = 0;
    for (int64_t i0 = 0; i0 < sg.count; i0 += 64) {
        const int64_t i = i0 + lane;
        const int32_t v = abl_row(io, sg, i);
        const typename Tu::T t0 = Tu::load(T, v);
        const bool act = i < sg.count && !(ALL && (Tu::is_in(t0) || Tu::is_out(t0)));
        const typename Tu::T mv = Tu::load(M, v);
        bool any_out = Tu::is_out(mv), all_eq = Tu::eq(mv, t0);
        const int64_t s = row_ptr[v], e = act ? row_ptr[v + 1] : s;
        const int64_t steps = abl_wave_max(e - s);
        for (int64_t c = 0; c < steps; c++) {
            const int64_t j = s + c;
            const typename Tu::T mw = Tu::load(M, col[j < e ? j : 0]);
            if (j < e) {
                any_out |= Tu::is_out(mw);
                all_eq &= Tu::eq(mw, t0);
            }
        }
        bool keep = false;
        if (act) {
            if (any_out) {
                Tu::store(T, v, Tu::out());
            } else if (all_eq) {
                Tu::store(T, v, Tu::in());
            } else {
                Tu::store(T, v, Tu::fresh(a, r + 1, (uint32_t)v));
                keep = true;
            }
        }
        seg_append(io, sg, keep, v, kept);
    }
    seg_finish(io, w, kept);
}

}  // namespace

int id_bits(int64_t n) {
    int b = 0;
    while (b < 63 && (int64_t{1} << b) < n + 2) b++;
    return b;
}

TupleParams tuple_params(int64_t n, uint64_t seed, uint64_t iter) {
    TupleParams p{};
    p.b = (uint32_t)id_bits(n);
    const int pb = 32 - (int)p.b;
    p.pmask = pb <= 0 ? 0ull : ((1ull << pb) - 1ull);
    p.f_iter = xs64star((seed << 32) ^ iter);
    return p;
}

#define MIS2_LANE_DISPATCH(L, KERNEL, ...)                                              \
    switch (L) {                                                                        \
        case 0: hipLaunchKernelGGL(KERNEL<0>, __VA_ARGS__); break;                      \
        case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                      \
        case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                      \
        case 4: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                      \
        case 8: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                      \
        case 16: hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__); break;                    \
        case 32: hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__); break;                    \
        case 64: hipLaunchKernelGGL(KERNEL<64>, __VA_ARGS__); break;                    \
        case kStagedLanes: hipLaunchKernelGGL(KERNEL<kStagedLanes>, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                           \
    }

// With e0 / e1 the launch records its own start and end (the events time
// the kernel alone, not the gap before it).
#define MIS2_LANE_DISPATCH_TIMED(L, KERNEL, GRID, BLOCK, S, E0, E1, ...)                 \
    if (E0) {                                                                           \
        switch (L) {                                                                    \
            case 0: hipExtLaunchKernelGGL(KERNEL<0>, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); break;  \
            case 1: hipExtLaunchKernelGGL(KERNEL<1>, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); break;  \
            case 2: hipExtLaunchKernelGGL(KERNEL<2>, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); break;  \
            case 4: hipExtLaunchKernelGGL(KERNEL<4>, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); break;  \
            case 8: hipExtLaunchKernelGGL(KERNEL<8>, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); break;  \
            case 16: hipExtLaunchKernelGGL(KERNEL<16>, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); break; \
            case 32: hipExtLaunchKernelGGL(KERNEL<32>, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); break; \
            case 64: hipExtLaunchKernelGGL(KERNEL<64>, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); break; \
            case kStagedLanes: hipExtLaunchKernelGGL(KERNEL<kStagedLanes>, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); break; \
            default: return hipErrorInvalidValue;                                       \
        }                                                                               \
    } else {                                                                            \
        MIS2_LANE_DISPATCH(L, KERNEL, GRID, BLOCK, 0, S, __VA_ARGS__);                  \
    }

hipError_t launch_push_in(int64_t n, const int64_t *row_ptr, const int32_t *col, const uint32_t *T,
                          uint32_t *M, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_push_in, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, row_ptr,
                       col, T, M);
    return hipGetLastError();
}

hipError_t launch_push_near(int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const uint32_t *M, uint8_t *near, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_push_near, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n,
                       row_ptr, col, M, near);
    return hipGetLastError();
}

hipError_t launch_col_round(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                            const uint32_t *T, uint32_t *M, const RoundsArgs &a, int r, int mode,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (mode != 0 && (lanes <= 0 || !a.colc || !a.lenc)) return hipErrorInvalidValue;
    if (mode == 1) {
        MIS2_LANE_DISPATCH_TIMED(lanes, k_col_round_w, dim3(blocks), dim3(kBlock), s, e0, e1,
                                 row_ptr, col, T, M, a, r);
    } else if (mode == 2) {
        MIS2_LANE_DISPATCH_TIMED(lanes, k_col_round_rw, dim3(blocks), dim3(kBlock), s, e0, e1,
                                 row_ptr, col, T, M, a, r);
    } else if (r <= 1) {
        MIS2_LANE_DISPATCH_TIMED(lanes, k_col_round0, dim3(blocks), dim3(kBlock), s, e0, e1,
                                 row_ptr, col, T, M, a, r);
    } else {
        MIS2_LANE_DISPATCH_TIMED(lanes, k_col_round, dim3(blocks), dim3(kBlock), s, e0, e1,
                                 row_ptr, col, T, M, a, r);
    }
    if (a.dsplit) {
        hipLaunchKernelGGL(k_fold_deg, dim3(1), dim3(64), 0, s, a.dsplit + (size_t)kSplit * kDegLine,
                           a.degs + kDegStride * r + 1, a.degs + kDegStride * r + 2);
    }
    return hipGetLastError();
}

hipError_t launch_dec_round(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                            uint32_t *T, const uint32_t *M, const RoundsArgs &a, int r,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    MIS2_LANE_DISPATCH_TIMED(lanes, k_dec_round, dim3(blocks), dim3(kBlock), s, e0, e1, row_ptr,
                             col, T, M, a, r);
    if (a.dsplit)
        hipLaunchKernelGGL(k_fold_deg, dim3(1), dim3(64), 0, s, a.dsplit, a.degs + kDegStride * r,
                           (unsigned long long *)nullptr);
    return hipGetLastError();
}

hipError_t launch_tail(const int64_t *row_ptr, const int32_t *col, uint32_t *T, uint32_t *M,
                       const RoundsArgs &a, int r0, int cstart, int64_t thr, uint32_t *rt_host,
                       unsigned long long *end_host, hipStream_t s, hipEvent_t e0,
                       hipEvent_t e1) {
    TailArgs ta{r0, cstart, thr, rt_host, end_host};
    if (e0)
        hipExtLaunchKernelGGL(k_tail, dim3(1), dim3(kTailThreads), 0, s, e0, e1, 0, row_ptr, col, T,
                              M, a, ta);
    else
        hipLaunchKernelGGL(k_tail, dim3(1), dim3(kTailThreads), 0, s, row_ptr, col, T, M, a, ta);
    return hipGetLastError();
}

int64_t coop_threshold(int lanes) {
    if (lanes == kStagedLanes) return kStagedCap;
    return lanes >= 64 ? 1024 : (int64_t)32 * std::max(lanes, 1);
}

hipError_t launch_init_tuples(const TupleParams &tp, int64_t n, uint32_t *T, const FillSpans &f,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_init_tuples, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, tp, n,
                       T, f);
    return hipGetLastError();
}

hipError_t launch_init_masked(int blocks, const TupleParams &tp, int64_t n, const int32_t *label,
                              uint32_t *T, uint32_t *M, const SegIO &io, const FillSpans &f,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_init_masked, dim3(blocks), dim3(kBlock), 0, s, tp, n, label, T, M, io,
                       f);
    return hipGetLastError();
}

template <int L>
hipError_t launch_rounds_t(int blocks, const int64_t *row_ptr, const int32_t *col, uint32_t *T,
                           uint32_t *M, const RoundsArgs &a, hipStream_t s) {
    const int64_t *rp = row_ptr;
    const int32_t *cl = col;
    uint32_t *t = T, *m = M;
    RoundsArgs aa = a;
    void *args[] = {(void *)&rp, (void *)&cl, (void *)&t, (void *)&m, (void *)&aa};
    return hipLaunchCooperativeKernel((const void *)k_rounds<L>, dim3(blocks), dim3(kBlock), args,
                                      0, s);
}

int sweep_resident_blocks(int lanes, int num_cus) {
    int per_cu = 0, per_cu2 = 0;
    hipError_t e = hipErrorInvalidValue, e2 = hipErrorInvalidValue;
    if (lanes == kStagedLanes) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_col_round<kStagedLanes>, kBlock, 0);
        e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, k_dec_round<kStagedLanes>, kBlock, 0);
    }
    if (e != hipSuccess || e2 != hipSuccess || per_cu <= 0 || per_cu2 <= 0) return 0;
    return std::min(per_cu, per_cu2) * num_cus;
}

int rounds_max_blocks(int lanes, int num_cus) {
    int per_cu = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (lanes) {
        case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<0>, kBlock, 0); break;
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<1>, kBlock, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<2>, kBlock, 0); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<4>, kBlock, 0); break;
        case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<8>, kBlock, 0); break;
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<16>, kBlock, 0); break;
        case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<32>, kBlock, 0); break;
        case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<64>, kBlock, 0); break;
        case kStagedLanes:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<kStagedLanes>, kBlock, 0);
            break;
        default: break;
    }
    if (e != hipSuccess || per_cu <= 0) return 0;
    return per_cu * num_cus;
}

hipError_t launch_rounds(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                         uint32_t *T, uint32_t *M, const RoundsArgs &a, hipStream_t s) {
    switch (lanes) {
        case 0: return launch_rounds_t<0>(blocks, row_ptr, col, T, M, a, s);
        case 1: return launch_rounds_t<1>(blocks, row_ptr, col, T, M, a, s);
        case 2: return launch_rounds_t<2>(blocks, row_ptr, col, T, M, a, s);
        case 4: return launch_rounds_t<4>(blocks, row_ptr, col, T, M, a, s);
        case 8: return launch_rounds_t<8>(blocks, row_ptr, col, T, M, a, s);
        case 16: return launch_rounds_t<16>(blocks, row_ptr, col, T, M, a, s);
        case 32: return launch_rounds_t<32>(blocks, row_ptr, col, T, M, a, s);
        case 64: return launch_rounds_t<64>(blocks, row_ptr, col, T, M, a, s);
        case kStagedLanes: return launch_rounds_t<kStagedLanes>(blocks, row_ptr, col, T, M, a, s);
        default: return hipErrorInvalidValue;
    }
}

int64_t status_blocks(int64_t n) { return n <= 0 ? 0 : (n + kCountTile - 1) / kCountTile; }

hipError_t launch_status(int64_t n, const uint32_t *T, uint8_t *status, uint32_t *blocksum,
                         uint32_t *d_total, hipStream_t s) {
    const int64_t nb = status_blocks(n);
    if (nb > 0)
        hipLaunchKernelGGL(k_status, dim3((unsigned)nb), dim3(kBlock), 0, s, n, T, status,
                           blocksum);
    return launch_scan_tiles(blocksum, nb, d_total, s);
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(count, kBlock, 8192)), dim3(kBlock), 0, s,
                       p, value, count);
    return hipGetLastError();
}

hipError_t launch_fill_spans(const FillSpans &f, hipStream_t s) {
    int64_t total = 0;
    for (int k = 0; k < f.k; k++) total += f.n[k];
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_spans, dim3(grid_for(total, kBlock, 8192)), dim3(kBlock), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(count, kBlock, 8192)), dim3(kBlock), 0, s,
                       p, value, count);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, uint8_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_for(count, kBlock, 8192)), dim3(kBlock), 0, s,
                       p, value, count);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long value, int64_t count,
                           hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(grid_for(count, kBlock, 8192)),
                       dim3(kBlock), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_validate(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                           uint32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(n > 0 ? n : 1, kBlock, 4096)), dim3(kBlock), 0,
                       s, n, nnz, row_ptr, col, err);
    return hipGetLastError();
}


hipError_t launch_abl_init(bool unpacked, const AblTuples &t, const RoundsArgs &a,
                           hipStream_t s) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((a.n + kBlock - 1) / kBlock, 8192));
    if (unpacked)
        hipLaunchKernelGGL(k_abl_init<true>, dim3(grid), dim3(kBlock), 0, s, t, a);
    else
        hipLaunchKernelGGL(k_abl_init<false>, dim3(grid), dim3(kBlock), 0, s, t, a);
    return hipGetLastError();
}

template <bool U, bool A>
void abl_round_t(int kind, int blocks, const int64_t *row_ptr, const int32_t *col,
                 const AblTuples &T, const AblTuples &M, const RoundsArgs &a, int r,
                 hipStream_t s) {
    if (kind == 0)
        k_abl_col<U, A><<<dim3(blocks), dim3(kBlock), 0, s>>>(row_ptr, col, T, M, a, r);
    else
        k_abl_dec<U, A><<<dim3(blocks), dim3(kBlock), 0, s>>>(row_ptr, col, T, M, a, r);
}

hipError_t launch_abl_round(int kind, bool unpacked, bool all, int blocks,
                            const int64_t *row_ptr, const int32_t *col, const AblTuples &T,
                            const AblTuples &M, const RoundsArgs &a, int r, hipStream_t s,
                            hipEvent_t e0, hipEvent_t e1) {
    if (e0) {
        const hipError_t er = hipEventRecord(e0, s);
        if (er != hipSuccess) return er;
    }
    if (unpacked) {
        if (all) abl_round_t<true, true>(kind, blocks, row_ptr, col, T, M, a, r, s);
        else abl_round_t<true, false>(kind, blocks, row_ptr, col, T, M, a, r, s);
    } else {
        if (all) abl_round_t<false, true>(kind, blocks, row_ptr, col, T, M, a, r, s);
        else abl_round_t<false, false>(kind, blocks, row_ptr, col, T, M, a, r, s);
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (e1) return hipEventRecord(e1, s);
    return hipSuccess;
}

}  // namespace mis2
