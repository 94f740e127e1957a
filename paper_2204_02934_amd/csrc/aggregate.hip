// aggregate.hip -- the labelling phases of Algorithm 3 (Section III-B) for gfx950.
//
// Phase 1 / phase 2 labelling push a root's aggregate id to its neighbours:
// the roots of an MIS-2 are at least three edges apart, so the written sets
// are disjoint and the order of the writes cannot matter.  The same pass
// knows each aggregate's size (the root plus the neighbours it labelled), so
// aggsize needs no histogram.  Phase 3 reads only the labels frozen after
// phase 2 (the "tentative" labels) and writes a separate output array, so
// every row is decided independently.
#include "internal.h"
#include "lanes.h"

namespace mis2 {

namespace {

constexpr int kLabelLanes = 16;  // lanes per root in the labelling push

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ int64_t wave_id() {
    const int64_t B = gridDim.x;
    const int64_t b = blockIdx.x;
    const int64_t lb = (B % 8 == 0) ? (b % 8) * (B / 8) + b / 8 : b;
    return lb * (kBlock / 64) + (threadIdx.x >> 6);
}

constexpr int kCoopLoads = 8;      // loads per lane per cooperative step
constexpr int64_t kHeavyRoot = 256;  // roots longer than this are pushed by the whole wavefront

// Labels the neighbours in [s, e) of a root with id (all of them, or only
// those still at -1), by the whole wavefront; returns the number labelled.
__device__ __forceinline__ int coop_label(const int32_t *__restrict__ col,
                                          int32_t *__restrict__ label, int64_t s, int64_t e,
                                          int32_t id, int only_unlabelled) {
    const int lane = (int)(threadIdx.x & 63u);
    int took = 0;
    for (int64_t b = s; b < e; b += 64 * kCoopLoads) {
        int32_t x[kCoopLoads];
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++) {
            const int64_t j = b + (int64_t)k * 64 + lane;
            x[k] = col[j < e ? j : s];
        }
        int32_t old[kCoopLoads];
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++) old[k] = only_unlabelled ? label[x[k]] : -1;
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++) {
            if (b + (int64_t)k * 64 + lane < e && old[k] == -1) {
                label[x[k]] = id;
                took++;
            }
        }
    }
    return group_sum_i<64>(took);
}

// roots[0..*d_count) get ids base + k; their neighbours (all of them, or only
// those still at -1 when only_unlabelled) get the same id, and aggsize[id]
// becomes 1 + the number of neighbours labelled.  Groups of kLabelLanes
// lanes push ordinary roots; long rows are pushed by the whole wavefront.
__global__ __launch_bounds__(kBlock) void k_label_roots(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ roots,
                                                        const uint32_t *__restrict__ d_count,
                                                        const uint32_t *__restrict__ d_base,
                                                        int only_unlabelled,
                                                        int32_t *__restrict__ label,
                                                        int32_t *__restrict__ aggsize,
                                                        uint8_t *__restrict__ root_mark,
                                                        uint8_t mark) {
    constexpr int L = kLabelLanes, G = kBlock / L;
    const int64_t count = *d_count;
    const int32_t base = d_base ? (int32_t)*d_base : 0;
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = (int)(threadIdx.x & (L - 1));
    // the loop bound is the same for the whole wavefront, so the shuffles
    // below always run with all lanes active
    const int64_t step = (int64_t)gridDim.x * G;
    const int64_t k0 = (int64_t)blockIdx.x * G + (threadIdx.x & ~63u) / L;
    for (int64_t kw = k0; kw < count; kw += step) {
        const int64_t k = kw + lane / L;
        const bool ok = k < count;
        const int32_t r = roots[ok ? k : count - 1];
        const int32_t id = base + (int32_t)k;
        int64_t s = row_ptr[r], e = row_ptr[r + 1];
        if (!ok) e = s;
        int took = 0;
        int heavy_took = 0;
        uint64_t heavy = __ballot(sub == 0 && e - s > kHeavyRoot);
        while (heavy) {
            const int src = __ffsll((unsigned long long)heavy) - 1;
            heavy &= heavy - 1;
            const int64_t hs = __shfl(s, src, 64), he = __shfl(e, src, 64);
            const int32_t hid = __shfl(id, src, 64);
            const int t = coop_label(col, label, hs, he, hid, only_unlabelled);
            if ((lane & ~(L - 1)) == (src & ~(L - 1))) {
                heavy_took = t;
                e = s;  // its group skips the row below
            }
        }
        for (int64_t j = s + sub; j < e; j += L) {
            const int32_t w = col[j];
            if (!only_unlabelled || label[w] == -1) {
                label[w] = id;
                took++;
            }
        }
        took = group_sum_i<L>(took);
        if (ok && sub == 0) {
            label[r] = id;
            aggsize[id] = 1 + took + heavy_took;
            if (root_mark) root_mark[r] = mark;
        }
    }
}

// flag[v] = 1 iff v is a root of the phase-2 MIS-2 (T_v = IN in the masked
// run) with at least two neighbours that are unlabelled after phase 1.  Each
// wavefront scans 64 vertices at a time; a candidate's row of up to
// kAcceptLane entries is counted by its own lane, longer ones by the whole
// wavefront, one row at a time.
constexpr int64_t kAcceptLane = 32;  // rows a lane counts alone in k_accept_phase2

// Buffer resource over n labels: a load whose byte offset is at or past
// 4n returns 0 without a memory access (the range check of raw buffer
// loads), which predicates a load per lane without a branch.  Word 3 is the
// gfx9 data-format word (32-bit elements).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t label_rsrc(const int32_t *label, int64_t n) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)label, (short)0, (int)(uint32_t)(4 * n),
                                             0x00020000);
}

// BUF: 4n < 2^32, so every label is reachable by a 32-bit buffer offset.
template <bool BUF>
__global__ __launch_bounds__(kBlock) void k_accept_phase2(int64_t n,
                                                          const int64_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col,
                                                          const uint32_t *__restrict__ T,
                                                          const int32_t *__restrict__ label,
                                                          uint8_t *__restrict__ flag) {
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t base = ((int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * 64; base < n;
         base += waves * 64) {
        const int64_t v = base + lane;
        const bool cand = v < n && label[v] == -1 && T[v] == kIn;
        // a candidate with a row of up to kAcceptLane entries counts its own
        // row; longer rows go to the whole wavefront one at a time
        int64_t rs = 0, re = 0;
        if (cand) {
            rs = row_ptr[v];
            re = row_ptr[v + 1];
        }
        const bool own = cand && re - rs <= kAcceptLane;
        uint8_t f = 0;
        if (own) {
            // every entry of the row loads at once, then every label: two
            // dependent steps for the whole row; each load is issued only for
            // the entries the lane's row has
            const int len = (int)(re - rs);
            int32_t x[kAcceptLane];
#pragma unroll
            for (int k = 0; k < (int)kAcceptLane; k++) {
                x[k] = 0;
                if (k < len) x[k] = col[rs + k];
            }
            if constexpr (BUF) {
                const __amdgpu_buffer_rsrc_t rl = label_rsrc(label, n);
#pragma unroll
                for (int k = 0; k < (int)kAcceptLane; k++)
                    x[k] = __builtin_amdgcn_raw_buffer_load_b32(
                        rl, k < len ? (int)(4u * (uint32_t)x[k]) : (int)0xFFFFFFFCu, 0, 0);
            } else {
                // entries past the row all read label 0: one line for the wavefront
#pragma unroll
                for (int k = 0; k < (int)kAcceptLane; k++) x[k] = label[k < len ? x[k] : 0];
            }
            int cnt = 0;
#pragma unroll
            for (int k = 0; k < (int)kAcceptLane; k++) cnt += (k < len) & (x[k] == -1);
            f = cnt >= 2;
        }
        uint64_t mask = __ballot(cand && !own);
        while (mask) {
            const int t = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            const int64_t u = base + t;
            const int64_t s = row_ptr[u], e = row_ptr[u + 1];
            int cnt = 0;
            for (int64_t b = s; b < e; b += 64 * kCoopLoads) {
                int32_t x[kCoopLoads];
#pragma unroll
                for (int k = 0; k < kCoopLoads; k++) {
                    const int64_t j = b + (int64_t)k * 64 + lane;
                    x[k] = col[j < e ? j : s];
                }
                int32_t lb[kCoopLoads];
#pragma unroll
                for (int k = 0; k < kCoopLoads; k++) lb[k] = label[x[k]];
#pragma unroll
                for (int k = 0; k < kCoopLoads; k++)
                    cnt += (b + (int64_t)k * 64 + lane < e) & (lb[k] == -1);
            }
            cnt = group_sum_i<64>(cnt);
            if (lane == t) f = cnt >= 2;
        }
        if (v < n) flag[v] = f;
    }
}

// Each wavefront lists, in order, the vertices of its own range still
// unlabelled after phase 2, as its segment of io.wl_out, and copies the
// labels of its range to copy_to (the segments cover every vertex).
__global__ __launch_bounds__(kBlock) void k_list_unlabelled(int64_t n,
                                                            const int32_t *__restrict__ label,
                                                            int32_t *__restrict__ copy_to,
                                                            SegIO io) {
    const int64_t w = wave_id();
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t lo = w * io.seg, hi = min(n, lo + io.seg);
    uint32_t kept = 0;
    for (int64_t v0 = lo; v0 < hi; v0 += 64) {
        const int64_t v = v0 + lane;
        const int32_t lv = v < hi ? label[v] : 0;
        if (v < hi) copy_to[v] = lv;
        const bool keep = v < hi && lv == -1;
        const uint64_t mask = __ballot(keep);
        if (keep) io.wl_out[lo + kept + (uint32_t)__popcll(mask & lanes_below(lane))] = (int32_t)v;
        kept += (uint32_t)__popcll(mask);
    }
    if (lane == 0 && w < io.S) io.cnt_out[w] = kept;
}

__device__ __forceinline__ uint64_t lanes_below_p3(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Orders the wavefront's LDS accesses before and after it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Candidate order of phase 3: larger coupling first, then smaller aggsize,
// then smaller aggregate id.  Returns true if (c1, s1, a1) beats (c2, s2, a2).
__device__ __forceinline__ bool better(int c1, int s1, int a1, int c2, int s2, int a2) {
    if (c1 != c2) return c1 > c2;
    if (s1 != s2) return s1 < s2;
    return a1 < a2;
}

// The best (coupling, size, id) candidate over each aligned group of L lanes,
// in every lane of the group.
template <int J>
__device__ __forceinline__ void p3_best_step(int &bc, int &bs, int &ba) {
    const int oc = lane_xor_i<J>(bc), os = lane_xor_i<J>(bs), oa = lane_xor_i<J>(ba);
    if (better(oc, os, oa, bc, bs, ba)) {
        bc = oc;
        bs = os;
        ba = oa;
    }
}

template <int L>
__device__ __forceinline__ void p3_group_best(int &bc, int &bs, int &ba) {
    if constexpr (L >= 64) p3_best_step<32>(bc, bs, ba);
    if constexpr (L >= 32) p3_best_step<16>(bc, bs, ba);
    if constexpr (L >= 16) p3_best_step<8>(bc, bs, ba);
    if constexpr (L >= 8) p3_best_step<4>(bc, bs, ba);
    if constexpr (L >= 4) p3_best_step<2>(bc, bs, ba);
    if constexpr (L >= 2) p3_best_step<1>(bc, bs, ba);
}

constexpr int32_t kPad = -2;  // label of a padding lane; never equals an aggregate id

// Short rows: lane j of the group holds the tent labels of neighbours
// k*L + j for k < K, and the sizes of their aggregates, all loaded before any
// is used.  Every lane broadcasts its K labels to the group once; each lane
// counts, for each of its own labels, the equal ones among all L*K (its
// coupling), and keeps its best candidate in the order above.  (Counting
// only the chunks that the wavefront's longest row reaches was measured on
// gfx950 and changed nothing: 30.7 us on the 27-point 100^3 graph, 217 us
// on Chung-Lu 4M, either way.)
template <int L, int K>
__device__ __forceinline__ void p3_count(const int32_t (&a)[K], const int32_t (&sz)[K], int &bc,
                                         int &bs, int &ba) {
    int cnt[K];
#pragma unroll
    for (int k = 0; k < K; k++) cnt[k] = 0;
#pragma unroll
    for (int t = 0; t < L; t++) {
#pragma unroll
        for (int k2 = 0; k2 < K; k2++) {
            const int32_t b = __shfl(a[k2], t, L);
#pragma unroll
            for (int k = 0; k < K; k++) cnt[k] += (b == a[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (a[k] >= 0 && better(cnt[k], sz[k], a[k], bc, bs, ba)) {
            bc = cnt[k];
            bs = sz[k];
            ba = a[k];
        }
    }
}

// One group of L lanes per unaggregated row of the wavefront's segment.  Rows
// of at most K chunks of L entries are counted in registers; longer rows are
// listed, in order, in the wavefront's segment of io.wl_out for
// k_phase3_long.  The group's best candidate is reduced with the candidate
// order above.
template <int L>
__global__ __launch_bounds__(kBlock) void k_phase3(const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col,
                                                   const int32_t *__restrict__ label,
                                                   const int32_t *__restrict__ aggsize,
                                                   SegIO io, int32_t *__restrict__ agg_out,
                                                   uint32_t *__restrict__ err) {
    constexpr int K = L >= 32 ? 1 : (32 / L > 8 ? 8 : 32 / L);
    const int64_t w = wave_id();
    if (w >= io.S) return;
    const int64_t count = io.cnt_in[w];
    const int64_t sbase = w * io.seg;
    constexpr int G = 64 / L;
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & (L - 1);
    uint32_t kept = 0;
    for (int64_t i0 = 0; i0 < count; i0 += G) {
        const int64_t i = i0 + lane / L;
        const bool valid = i < count;
        int32_t v = 0;
        int64_t s = 0, e = 0;
        if (valid) {
            v = io.wl_in[sbase + i];
            s = row_ptr[v];
            e = row_ptr[v + 1];
        }
        const bool is_long = e - s > (int64_t)K * L;
        const int64_t es = is_long ? s : e;  // long rows are left to k_phase3_long
        const int64_t wmax = group_max64<64>((es - s + L - 1) / L);
        int bc = 0, bs = 0x7FFFFFFF, ba = 0x7FFFFFFF;
        if (wmax > 0) {
            int32_t a[K], sz[K];
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int64_t j = s + k * L + sub;
                a[k] = col[j < es ? j : 0];
            }
#pragma unroll
            for (int k = 0; k < K; k++) a[k] = label[a[k]];
#pragma unroll
            for (int k = 0; k < K; k++) {
                if (s + k * L + sub >= es) a[k] = kPad;
                sz[k] = aggsize[a[k] >= 0 ? a[k] : 0];
            }
            p3_count<L, K>(a, sz, bc, bs, ba);
        }
        p3_group_best<L>(bc, bs, ba);
        if (valid && sub == 0 && !is_long) {
            if (bc > 0)
                agg_out[v] = ba;
            else
                atomicOr(err, 1u);
        }
        const bool keep = valid && sub == 0 && is_long;
        const uint64_t mask = __ballot(keep);
        if (keep) io.wl_out[sbase + kept + (uint32_t)__popcll(mask & lanes_below_p3(lane))] = v;
        kept += (uint32_t)__popcll(mask);
    }
    if (lane == 0) io.cnt_out[w] = kept;
}

// Long unaggregated rows, one at a time per wavefront: the couplings are
// counted in an LDS hash map (aggregate id -> count) of cap slots, cap the
// power of two >= 2 * len between 64 and kP3Slots, so that clearing and
// reading the map cost in proportion to the row (every row of up to
// kP3Slots entries fits: it has at most len distinct ids); then the
// wavefront reduces its entries with the candidate order.  Rows longer than
// kP3Slots count each label against the whole row, 64 labels at a time.
// The grid is small enough to be resident at once (the map takes 64 KiB per
// workgroup): wavefront w takes the list segments w, w + W, w + 2W, ... (W
// wavefronts in the grid), reading 64 segment sizes in one load.  Measured on
// gfx950 (Chung-Lu 4M, 22 791 rows of 33-291 entries): one wavefront per
// segment with the whole 2048-slot map for every row took 288 us.
constexpr int kP3Slots = 2048;
constexpr int kP3LongBlocks = 512;  // 2 resident workgroups on each of 256 compute units

__device__ __forceinline__ void p3_reduce(int &bc, int &bs, int &ba) {
    p3_group_best<64>(bc, bs, ba);
}

__global__ __launch_bounds__(kBlock) void k_phase3_long(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ label,
                                                        const int32_t *__restrict__ aggsize,
                                                        SegIO io, int32_t *__restrict__ agg_out,
                                                        uint32_t *__restrict__ err) {
    constexpr uint32_t kEmpty = 0xFFFFFFFFu;
    __shared__ uint32_t keys_s[kBlock / 64][kP3Slots];
    __shared__ uint32_t cnts_s[kBlock / 64][kP3Slots];
    uint32_t *keys = keys_s[threadIdx.x >> 6];
    uint32_t *cnts = cnts_s[threadIdx.x >> 6];
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t W = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t w = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    for (int64_t w0 = w; w0 < io.S; w0 += 64 * W) {
        const int64_t mine = w0 + (int64_t)lane * W;  // the segment this lane reads the size of
        const uint32_t my_count = mine < io.S ? io.cnt_in[mine] : 0u;
        uint64_t todo = __ballot(my_count != 0u);
        while (todo) {
            const int j = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int64_t count = __shfl((int)my_count, j, 64);
            const int64_t sbase = (w0 + (int64_t)j * W) * io.seg;
            for (int64_t i = 0; i < count; i++) {
                const int32_t v = io.wl_in[sbase + i];
                const int64_t s = row_ptr[v], e = row_ptr[v + 1];
                int bc = 0, bs = 0x7FFFFFFF, ba = 0x7FFFFFFF;
                if (e - s <= kP3Slots) {
                    int lg = 6;
                    while ((int64_t)1 << lg < 2 * (e - s) && lg < 11) lg++;
                    const uint32_t cap = 1u << lg;
                    for (uint32_t k = (uint32_t)lane; k < cap; k += 64) {
                        keys[k] = kEmpty;
                        cnts[k] = 0u;
                    }
                    wave_lds_sync();
                    for (int64_t j0 = s; j0 < e; j0 += 64 * kCoopLoads) {
                        int32_t x[kCoopLoads];
#pragma unroll
                        for (int k = 0; k < kCoopLoads; k++) {
                            const int64_t jj = j0 + (int64_t)k * 64 + lane;
                            x[k] = col[jj < e ? jj : s];
                        }
                        int32_t a[kCoopLoads];
#pragma unroll
                        for (int k = 0; k < kCoopLoads; k++) a[k] = label[x[k]];
#pragma unroll
                        for (int k = 0; k < kCoopLoads; k++) {
                            if (j0 + (int64_t)k * 64 + lane < e && a[k] >= 0) {
                                const uint32_t key = (uint32_t)a[k];
                                uint32_t h = (key * 2654435761u) >> (32 - lg);
                                for (;;) {  // the map has a slot for every entry of the row
                                    const uint32_t prev = atomicCAS(&keys[h], kEmpty, key);
                                    if (prev == kEmpty || prev == key) break;
                                    h = (h + 1) & (cap - 1);
                                }
                                atomicAdd(&cnts[h], 1u);
                            }
                        }
                    }
                    wave_lds_sync();
                    for (uint32_t k = (uint32_t)lane; k < cap; k += 64) {
                        const uint32_t key = keys[k];
                        if (key != kEmpty) {
                            const int c = (int)cnts[k], sz = aggsize[key];
                            if (better(c, sz, (int)key, bc, bs, ba)) {
                                bc = c;
                                bs = sz;
                                ba = (int)key;
                            }
                        }
                    }
                    wave_lds_sync();
                } else {
                    for (int64_t c1 = s; c1 < e; c1 += 64) {
                        const int64_t jj = c1 + lane;
                        const int32_t a = jj < e ? label[col[jj]] : kPad;
                        int cnt = 0;
                        for (int64_t c2 = s; c2 < e; c2 += 64) {
                            const int64_t j2 = c2 + lane;
                            const int32_t a2 = j2 < e ? label[col[j2]] : kPad;
                            for (int t = 0; t < 64; t++)
                                cnt += (__builtin_amdgcn_readlane(a2, t) == a);
                        }
                        if (a >= 0) {
                            const int sz = aggsize[a];
                            if (better(cnt, sz, a, bc, bs, ba)) {
                                bc = cnt;
                                bs = sz;
                                ba = a;
                            }
                        }
                    }
                }
                p3_reduce(bc, bs, ba);
                if (lane == 0) {
                    if (bc > 0)
                        agg_out[v] = ba;
                    else
                        atomicOr(err, 1u);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Algorithm 2's second loop: every vertex left unaggregated by the first loop
// joins the aggregate of a neighbour -- the smallest aggregate id among its
// neighbours' first-loop labels.  The labels are read as unsigned, so -1
// (unaggregated) is above every id and never wins.  The labels read are
// the frozen first-loop ones (label); the result goes to agg_out, so rows
// are independent.
// ---------------------------------------------------------------------------

// Smallest label (as unsigned) over the column indices [s, e), by the whole
// wavefront.
__device__ __forceinline__ uint32_t coop_min_label(const int32_t *__restrict__ col,
                                                   const int32_t *__restrict__ label, int64_t s,
                                                   int64_t e) {
    const int lane = (int)(threadIdx.x & 63u);
    uint32_t m = 0xFFFFFFFFu;
    for (int64_t b = s; b < e; b += 64 * kCoopLoads) {
        int32_t x[kCoopLoads];
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++) {
            const int64_t j = b + (int64_t)k * 64 + lane;
            x[k] = col[j < e ? j : s];
        }
        uint32_t a[kCoopLoads];
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++) a[k] = (uint32_t)label[x[k]];
#pragma unroll
        for (int k = 0; k < kCoopLoads; k++)
            if (b + (int64_t)k * 64 + lane < e) m = min(m, a[k]);
    }
    return group_min<64>(m);
}

// One group of L lanes per row of the wavefront's segment of io.wl_in (the
// unaggregated vertices), K chunks of L column indices loaded before their
// labels are gathered; rows longer than 32 * L go to the whole wavefront.
// A vertex with no aggregated neighbour sets bit 1 of *err.
template <int L>
__global__ __launch_bounds__(kBlock) void k_join_min(const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ label,
                                                     SegIO io, int32_t *__restrict__ agg_out,
                                                     uint32_t *__restrict__ err) {
    constexpr int K = L >= 32 ? 1 : (32 / L > 8 ? 8 : 32 / L);
    constexpr int G = 64 / L;
    constexpr int64_t kLong = L >= 64 ? 1024 : (int64_t)32 * L;
    const int64_t w = wave_id();
    if (w >= io.S) return;
    const int64_t count = io.cnt_in[w];
    const int64_t sbase = w * io.seg;
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & (L - 1);
    for (int64_t i0 = 0; i0 < count; i0 += G) {
        const int64_t i = i0 + lane / L;
        const bool valid = i < count;
        const int32_t v = io.wl_in[sbase + (valid ? i : count - 1)];
        const int64_t s = row_ptr[v];
        int64_t e = valid ? row_ptr[v + 1] : s;
        uint32_t m = 0xFFFFFFFFu;
        uint64_t heavy = __ballot(sub == 0 && e - s > kLong);
        while (heavy) {
            const int src = __ffsll((unsigned long long)heavy) - 1;
            heavy &= heavy - 1;
            const uint32_t hm =
                coop_min_label(col, label, __shfl(s, src, 64), __shfl(e, src, 64));
            if ((lane & ~(L - 1)) == (src & ~(L - 1))) {
                m = min(m, hm);
                e = s;  // its group skips the row below
            }
        }
        const int64_t wmax = group_max64<64>(e - s);
        for (int64_t c0 = 0; c0 < wmax; c0 += (int64_t)L * K) {
            int32_t x[K];
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int64_t j = s + c0 + k * L + sub;
                x[k] = col[j < e ? j : 0];
            }
            uint32_t a[K];
#pragma unroll
            for (int k = 0; k < K; k++) a[k] = (uint32_t)label[x[k]];
#pragma unroll
            for (int k = 0; k < K; k++)
                if (s + c0 + k * L + sub < e) m = min(m, a[k]);
        }
        m = group_min<L>(m);
        if (valid && sub == 0) {
            if (m == 0xFFFFFFFFu)
                atomicOr(err, 2u);
            else
                agg_out[v] = (int32_t)m;
        }
    }
}

int grid_for(int64_t work, int per_block, int cap) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace

hipError_t launch_label_roots(int64_t n, const int64_t *row_ptr, const int32_t *col,
                              const int32_t *roots, const uint32_t *d_count,
                              const uint32_t *d_base, bool only_unlabelled, int32_t *label,
                              int32_t *aggsize, uint8_t *root_mark, uint8_t mark, hipStream_t s) {
    hipLaunchKernelGGL(k_label_roots, dim3(grid_for(n / 8 + 1, kBlock / kLabelLanes, 4096)),
                       dim3(kBlock), 0, s, row_ptr, col, roots, d_count, d_base,
                       (int)only_unlabelled, label, aggsize, root_mark, mark);
    return hipGetLastError();
}

hipError_t launch_accept_phase2(int64_t n, const int64_t *row_ptr, const int32_t *col,
                                const uint32_t *T, const int32_t *label, uint8_t *flag,
                                hipStream_t s) {
    if (4 * n < ((int64_t)1 << 32))
        hipLaunchKernelGGL(k_accept_phase2<true>, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0,
                           s, n, row_ptr, col, T, label, flag);
    else
        hipLaunchKernelGGL(k_accept_phase2<false>, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock),
                           0, s, n, row_ptr, col, T, label, flag);
    return hipGetLastError();
}

hipError_t launch_list_unlabelled(int blocks, int64_t n, const int32_t *label, int32_t *copy_to,
                                  const SegIO &io, hipStream_t s) {
    hipLaunchKernelGGL(k_list_unlabelled, dim3(blocks), dim3(kBlock), 0, s, n, label, copy_to, io);
    return hipGetLastError();
}

#define MIS2_P3_DISPATCH(L, ...)                                                       \
    switch (L) {                                                                       \
        case 1: hipLaunchKernelGGL(k_phase3<1>, __VA_ARGS__); break;                   \
        case 2: hipLaunchKernelGGL(k_phase3<2>, __VA_ARGS__); break;                   \
        case 4: hipLaunchKernelGGL(k_phase3<4>, __VA_ARGS__); break;                   \
        case 8: hipLaunchKernelGGL(k_phase3<8>, __VA_ARGS__); break;                   \
        case 16: hipLaunchKernelGGL(k_phase3<16>, __VA_ARGS__); break;                 \
        case 32: hipLaunchKernelGGL(k_phase3<32>, __VA_ARGS__); break;                 \
        case 64: hipLaunchKernelGGL(k_phase3<64>, __VA_ARGS__); break;                 \
        default: return hipErrorInvalidValue;                                          \
    }

#define MIS2_JOIN_DISPATCH(L, ...)                                                     \
    switch (L) {                                                                       \
        case 1: hipLaunchKernelGGL(k_join_min<1>, __VA_ARGS__); break;                 \
        case 2: hipLaunchKernelGGL(k_join_min<2>, __VA_ARGS__); break;                 \
        case 4: hipLaunchKernelGGL(k_join_min<4>, __VA_ARGS__); break;                 \
        case 8: hipLaunchKernelGGL(k_join_min<8>, __VA_ARGS__); break;                 \
        case 16: hipLaunchKernelGGL(k_join_min<16>, __VA_ARGS__); break;               \
        case 32: hipLaunchKernelGGL(k_join_min<32>, __VA_ARGS__); break;               \
        case 64: hipLaunchKernelGGL(k_join_min<64>, __VA_ARGS__); break;               \
        default: return hipErrorInvalidValue;                                          \
    }

hipError_t launch_join_min(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                           const int32_t *label, const SegIO &io, int32_t *agg_out,
                           uint32_t *err, hipStream_t s) {
    MIS2_JOIN_DISPATCH(lanes, dim3(blocks), dim3(kBlock), 0, s, row_ptr, col, label, io, agg_out,
                       err);
    return hipGetLastError();
}

hipError_t launch_phase3(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                         const int32_t *label, const int32_t *aggsize, const SegIO &io,
                         const SegIO &io_long, int32_t *agg_out, uint32_t *err, hipStream_t s) {
    MIS2_P3_DISPATCH(lanes, dim3(blocks), dim3(kBlock), 0, s, row_ptr, col, label, aggsize, io,
                     agg_out, err);
    hipLaunchKernelGGL(k_phase3_long, dim3(std::min(blocks, kP3LongBlocks)), dim3(kBlock), 0, s,
                       row_ptr, col, label, aggsize, io_long, agg_out, err);
    return hipGetLastError();
}

}  // namespace mis2
