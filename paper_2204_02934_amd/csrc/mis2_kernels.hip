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
#include "internal.h"

namespace mis2 {

namespace {

constexpr int kUnroll = 4;  // rows per lane group in flight

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

// Sum of the L-lane groups' row lengths over the wavefront, added to *sum by
// lane 0 (accounting runs only).
__device__ __forceinline__ void wave_degsum(unsigned long long *sum, unsigned long long d) {
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
    if ((threadIdx.x & 63u) == 0 && d) atomicAdd(sum, d);
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

// Ends a sweep: the wavefront's count, the alive flag, and the workgroup's
// total added to one of 8 trace counters (spread so that same-address
// atomics do not serialise the whole grid).  All threads must call it.
__device__ __forceinline__ void seg_finish(const SegIO &io, int64_t w, uint32_t kept) {
    __shared__ uint32_t part[kBlock / 64];
    if ((threadIdx.x & 63u) == 0) {
        if (w < io.S) io.cnt_out[w] = kept;
        if (kept && io.alive_out) *io.alive_out = 1u;
        part[threadIdx.x >> 6] = kept;
    }
    if (!io.trace_out) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kBlock / 64; k++) t += part[k];
        if (t) atomicAdd(&io.trace_out[blockIdx.x % kTraceSplit], t);
    }
}

// Largest row length among the rows this lane's group holds, over the
// wavefront (so every lane runs the same number of chunk steps).
template <int U>
__device__ __forceinline__ int64_t wave_max_len(const int64_t (&s)[U], const int64_t (&e)[U]) {
    int64_t m = 0;
#pragma unroll
    for (int u = 0; u < U; u++) m = max(m, e[u] - s[u]);
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    return m;
}

// The U rows of this lane group for the step starting at row i0 of the
// segment; rows past the end repeat the last row (a valid address) with
// ok = false.
template <int L, int U>
__device__ __forceinline__ void load_rows(const SegIO &io, const Seg &sg, int64_t i0,
                                          int32_t (&v)[U], bool (&ok)[U]) {
    constexpr int G = 64 / L;
    const int lane = (int)(threadIdx.x & 63u);
    int64_t ic[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int64_t i = i0 + u * G + lane / L;
        ok[u] = i < sg.count;
        ic[u] = ok[u] ? i : sg.count - 1;
    }
    if (io.wl_in) {
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = io.wl_in[sg.base + ic[u]];
    } else {
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = (int32_t)(sg.base + ic[u]);
    }
}

// Refresh Column over the wavefront's segment: U rows per lane group per
// step, so that U independent row streams are in flight.  Loads are issued
// unconditionally from clamped, always valid addresses and their results
// selected afterwards: a predicated load would become a branch with a full
// wait after it and serialise the U streams.
template <int L, int U>
__device__ __forceinline__ uint32_t sweep_column(const int64_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col,
                                                 const uint32_t *__restrict__ T,
                                                 uint32_t *__restrict__ M, const SegIO &io,
                                                 const Seg &sg) {
    constexpr int G = 64 / L;  // rows per wavefront per unrolled slot
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & (L - 1);
    uint32_t kept = 0;
    unsigned long long dsum = 0;
    for (int64_t i0 = 0; i0 < sg.count; i0 += G * U) {
        int32_t v[U];
        bool ok[U];
        int64_t s[U], e[U];
        uint32_t m[U];
        load_rows<L, U>(io, sg, i0, v, ok);
#pragma unroll
        for (int u = 0; u < U; u++) {
            s[u] = row_ptr[v[u]];
            e[u] = row_ptr[v[u] + 1];
            m[u] = T[v[u]];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (!ok[u]) e[u] = s[u];
            if (sub != 0) m[u] = kOut;
            if (sub == 0) dsum += (unsigned long long)(e[u] - s[u]);
        }
        const int64_t steps = wave_max_len<U>(s, e);
        for (int64_t c0 = 0; c0 < steps; c0 += L) {
            const int64_t c = c0 + sub;
            int32_t x[U];
#pragma unroll
            for (int u = 0; u < U; u++) x[u] = col[(s[u] + c < e[u]) ? s[u] + c : 0];
            uint32_t t[U];
#pragma unroll
            for (int u = 0; u < U; u++) t[u] = T[x[u]];
#pragma unroll
            for (int u = 0; u < U; u++)
                if (s[u] + c < e[u]) m[u] = min(m[u], t[u]);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
#pragma unroll
            for (int off = L / 2; off > 0; off >>= 1)
                m[u] = min(m[u], (uint32_t)__shfl_xor((int)m[u], off, L));
            bool keep = false;
            if (ok[u] && sub == 0) {
                if (m[u] == kIn) m[u] = kOut;
                M[v[u]] = m[u];
                keep = (m[u] != kOut);
            }
            seg_append(io, sg, keep, v[u], kept);
        }
    }
    if (io.deg_sum) wave_degsum(io.deg_sum, dsum);
    return kept;
}

// Decide Set over the wavefront's segment, with the next round's Refresh Row
// for the vertices that stay undecided (loads as in sweep_column).
template <int L, int U>
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
    for (int64_t i0 = 0; i0 < sg.count; i0 += G * U) {
        int32_t v[U];
        bool ok[U];
        int64_t s[U], e[U];
        uint32_t t0[U], mv[U];
        int any_out[U], all_eq[U];
        load_rows<L, U>(io, sg, i0, v, ok);
#pragma unroll
        for (int u = 0; u < U; u++) {
            s[u] = row_ptr[v[u]];
            e[u] = row_ptr[v[u] + 1];
            t0[u] = T[v[u]];
            mv[u] = M[v[u]];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (!ok[u]) e[u] = s[u];
            any_out[u] = (sub == 0) & (mv[u] == kOut);
            all_eq[u] = (sub != 0) | (mv[u] == t0[u]);
            if (sub == 0) dsum += (unsigned long long)(e[u] - s[u]);
        }
        const int64_t steps = wave_max_len<U>(s, e);
        for (int64_t c0 = 0; c0 < steps; c0 += L) {
            const int64_t c = c0 + sub;
            int32_t x[U];
#pragma unroll
            for (int u = 0; u < U; u++) x[u] = col[(s[u] + c < e[u]) ? s[u] + c : 0];
            uint32_t mw[U];
#pragma unroll
            for (int u = 0; u < U; u++) mw[u] = M[x[u]];
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (s[u] + c < e[u]) {
                    any_out[u] |= (mw[u] == kOut);
                    all_eq[u] &= (mw[u] == t0[u]) | (mw[u] == kAbsent);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
#pragma unroll
            for (int off = L / 2; off > 0; off >>= 1) {
                any_out[u] |= __shfl_xor(any_out[u], off, L);
                all_eq[u] &= __shfl_xor(all_eq[u], off, L);
            }
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
    }
    if (io.deg_sum) wave_degsum(io.deg_sum, dsum);
    return kept;
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_refresh_column(const int64_t *__restrict__ row_ptr,
                                                           const int32_t *__restrict__ col,
                                                           const uint32_t *__restrict__ T,
                                                           uint32_t *__restrict__ M, SegIO io) {
    const int64_t w = wave_id();
    if (blockIdx.x == 0 && threadIdx.x < kRoundStride && io.round_zero)
        io.round_zero[threadIdx.x] = 0u;
    const Seg sg = seg_of(io, w);
    const uint32_t kept = sweep_column<L, kUnroll>(row_ptr, col, T, M, io, sg);
    seg_finish(io, w, kept);
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_decide(const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col,
                                                   uint32_t *__restrict__ T,
                                                   const uint32_t *__restrict__ M,
                                                   TupleParams next, SegIO io) {
    const int64_t w = wave_id();
    const Seg sg = seg_of(io, w);
    const uint32_t kept = sweep_decide<L, kUnroll>(row_ptr, col, T, M, next, io, sg);
    seg_finish(io, w, kept);
}

// Round-0 tuples for every vertex.
__global__ __launch_bounds__(kBlock) void k_init_tuples(TupleParams tp, int64_t n,
                                                        uint32_t *__restrict__ T) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        T[v] = make_tuple(tp, (uint32_t)v);
}

// Induced-subgraph start: vertices with label -1 take part; the others read
// as OUT in T (neutral for the minimum) and as absent in M.  Each wavefront
// also lists the active vertices of its own range, in order, as its segment
// of both round-0 worklists.
__global__ __launch_bounds__(kBlock) void k_init_masked(TupleParams tp, int64_t n,
                                                        const int32_t *__restrict__ label,
                                                        uint32_t *__restrict__ T,
                                                        uint32_t *__restrict__ M, SegIO io) {
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

}  // namespace

int id_bits(int64_t n) {
    int b = 0;
    while (b < 63 && (int64_t{1} << b) < n + 2) b++;
    return b;
}

TupleParams tuple_params(int64_t n, uint64_t seed, uint64_t iter) {
    TupleParams p;
    p.b = (uint32_t)id_bits(n);
    const int pb = 32 - (int)p.b;
    p.pmask = pb <= 0 ? 0ull : ((1ull << pb) - 1ull);
    p.f_iter = xs64star((seed << 32) ^ iter);
    return p;
}

#define MIS2_LANE_DISPATCH(L, KERNEL, ...)                                              \
    switch (L) {                                                                        \
        case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                      \
        case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                      \
        case 4: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                      \
        case 8: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                      \
        case 16: hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__); break;                    \
        case 32: hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__); break;                    \
        case 64: hipLaunchKernelGGL(KERNEL<64>, __VA_ARGS__); break;                    \
        default: return hipErrorInvalidValue;                                           \
    }

hipError_t launch_refresh_column(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                                 const uint32_t *T, uint32_t *M, const SegIO &io,
                                 hipStream_t s) {
    MIS2_LANE_DISPATCH(lanes, k_refresh_column, dim3(blocks), dim3(kBlock), 0, s, row_ptr, col, T,
                       M, io);
    return hipGetLastError();
}

hipError_t launch_decide(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                         uint32_t *T, const uint32_t *M, const TupleParams &next, const SegIO &io,
                         hipStream_t s) {
    MIS2_LANE_DISPATCH(lanes, k_decide, dim3(blocks), dim3(kBlock), 0, s, row_ptr, col, T, M,
                       next, io);
    return hipGetLastError();
}

hipError_t launch_init_tuples(const TupleParams &tp, int64_t n, uint32_t *T, hipStream_t s) {
    hipLaunchKernelGGL(k_init_tuples, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, tp, n,
                       T);
    return hipGetLastError();
}

hipError_t launch_init_masked(int blocks, const TupleParams &tp, int64_t n, const int32_t *label,
                              uint32_t *T, uint32_t *M, const SegIO &io, hipStream_t s) {
    hipLaunchKernelGGL(k_init_masked, dim3(blocks), dim3(kBlock), 0, s, tp, n, label, T, M, io);
    return hipGetLastError();
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

}  // namespace mis2
