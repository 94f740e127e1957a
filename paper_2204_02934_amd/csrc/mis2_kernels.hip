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
// Decide Set reads only M and writes only T_v, so rows are independent; the
// per-row reductions are min / any / all and the worklist appends change only
// the order of the lists, never their contents, so results do not depend on
// scheduling.  A group of L lanes (a power of two up to a wave of 64) streams
// one row's column indices with coalesced loads (Section V-D uses SIMD lanes
// for the same reason) and combines its partial results with cross-lane
// shuffles.
#include "internal.h"

namespace mis2 {

namespace {

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Append v (for lanes with keep) to out[*cnt ...]: one atomic per wavefront,
// lane order preserved inside the wavefront.
__device__ __forceinline__ void wave_append(bool keep, int32_t v, int32_t *out, uint32_t *cnt) {
    const int lane = (int)(threadIdx.x & 63u);
    const uint64_t mask = __ballot(keep);
    if (mask == 0ull) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(mask));
    base = (uint32_t)__shfl((int)base, leader);
    if (keep) out[base + (uint32_t)__popcll(mask & lanes_below(lane))] = v;
}

__device__ __forceinline__ int64_t sweep_count(const SweepIO &io) {
    return io.cnt_in ? (int64_t)(*io.cnt_in) : io.identity_n;
}

__device__ __forceinline__ void sweep_bookkeeping(const SweepIO &io, int64_t count) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (io.cnt_zero) *io.cnt_zero = 0u;
        if (io.trace_slot) *io.trace_slot = (uint32_t)count;
    }
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_refresh_column(const int64_t *__restrict__ row_ptr,
                                                           const int32_t *__restrict__ col,
                                                           const uint32_t *__restrict__ T,
                                                           uint32_t *__restrict__ M, SweepIO io) {
    const int64_t count = sweep_count(io);
    sweep_bookkeeping(io, count);
    constexpr int G = kBlock / L;  // rows per workgroup per step
    const int sub = (int)(threadIdx.x & (L - 1));
    const int64_t step = (int64_t)gridDim.x * G;
    for (int64_t base = (int64_t)blockIdx.x * G; base < count; base += step) {
        const int64_t i = base + threadIdx.x / L;
        const bool valid = i < count;
        int32_t v = 0;
        uint32_t m = kOut;
        if (valid) {
            v = io.wl_in ? io.wl_in[i] : (int32_t)i;
            const int64_t s = row_ptr[v], e = row_ptr[v + 1];
            if (sub == 0) m = T[v];
            for (int64_t k = s + sub; k < e; k += L) m = min(m, T[col[k]]);
        }
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1)
            m = min(m, (uint32_t)__shfl_xor((int)m, off, L));
        bool keep = false;
        if (valid && sub == 0) {
            if (m == kIn) m = kOut;
            M[v] = m;
            keep = (m != kOut);
        }
        wave_append(keep, v, io.wl_out, io.cnt_out);
    }
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_decide(const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col,
                                                   uint32_t *__restrict__ T,
                                                   const uint32_t *__restrict__ M,
                                                   TupleParams next, SweepIO io) {
    const int64_t count = sweep_count(io);
    sweep_bookkeeping(io, count);
    constexpr int G = kBlock / L;
    const int sub = (int)(threadIdx.x & (L - 1));
    const int64_t step = (int64_t)gridDim.x * G;
    for (int64_t base = (int64_t)blockIdx.x * G; base < count; base += step) {
        const int64_t i = base + threadIdx.x / L;
        const bool valid = i < count;
        int32_t v = 0;
        int any_out = 0, all_eq = 1;
        if (valid) {
            v = io.wl_in ? io.wl_in[i] : (int32_t)i;
            const uint32_t t0 = T[v];
            const int64_t s = row_ptr[v], e = row_ptr[v + 1];
            if (sub == 0) {
                const uint32_t mv = M[v];
                any_out = (mv == kOut);
                all_eq = (mv == t0);
            }
            for (int64_t k = s + sub; k < e; k += L) {
                const uint32_t mw = M[col[k]];
                any_out |= (mw == kOut);
                all_eq &= (mw == t0) | (mw == kAbsent);
            }
        }
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) {
            any_out |= __shfl_xor(any_out, off, L);
            all_eq &= __shfl_xor(all_eq, off, L);
        }
        bool keep = false;
        if (valid && sub == 0) {
            if (any_out) {
                T[v] = kOut;
            } else if (all_eq) {
                T[v] = kIn;
            } else {
                T[v] = make_tuple(next, (uint32_t)v);
                keep = true;
            }
        }
        wave_append(keep, v, io.wl_out, io.cnt_out);
    }
}

// Round-0 tuples for every vertex; clears the per-round counters.
__global__ __launch_bounds__(kBlock) void k_init_tuples(TupleParams tp, int64_t n,
                                                        uint32_t *__restrict__ T,
                                                        uint32_t *__restrict__ ring) {
    if (blockIdx.x == 0 && threadIdx.x < 2 * kRing) ring[threadIdx.x] = 0u;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        T[v] = make_tuple(tp, (uint32_t)v);
}

// Induced-subgraph start: vertices with label -1 take part; the others read
// as OUT in T (neutral for the minimum) and as absent in M.
__global__ __launch_bounds__(kBlock) void k_init_masked(TupleParams tp, int64_t n,
                                                        const int32_t *__restrict__ label,
                                                        uint32_t *__restrict__ T,
                                                        uint32_t *__restrict__ M,
                                                        uint32_t *__restrict__ ring) {
    if (blockIdx.x == 0 && threadIdx.x < 2 * kRing) ring[threadIdx.x] = 0u;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const bool act = label[v] == -1;
        T[v] = act ? make_tuple(tp, (uint32_t)v) : kOut;
        M[v] = act ? kOut : kAbsent;
    }
}

__global__ __launch_bounds__(kBlock) void k_status(int64_t n, const uint32_t *__restrict__ T,
                                                   uint8_t *__restrict__ status,
                                                   uint32_t *__restrict__ count) {
    __shared__ uint32_t part[kBlock / 64];
    uint32_t c = 0;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const uint8_t in = T[v] == kIn;
        status[v] = in;
        c += in;
    }
    for (int off = 32; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off, 64);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kBlock / 64; w++) t += part[w];
        if (t) atomicAdd(count, t);
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_fill(V *__restrict__ p, V value, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = value;
}

// CSR checks: bit 0 row_ptr[0] != 0, bit 1 decreasing row_ptr, bit 2
// row_ptr[n] != nnz, bit 3 column out of range, bit 4 self-loop.
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
                                 const uint32_t *T, uint32_t *M, const SweepIO &io,
                                 hipStream_t s) {
    MIS2_LANE_DISPATCH(lanes, k_refresh_column, dim3(blocks), dim3(kBlock), 0, s, row_ptr, col, T,
                       M, io);
    return hipGetLastError();
}

hipError_t launch_decide(int lanes, int blocks, const int64_t *row_ptr, const int32_t *col,
                         uint32_t *T, const uint32_t *M, const TupleParams &next,
                         const SweepIO &io, hipStream_t s) {
    MIS2_LANE_DISPATCH(lanes, k_decide, dim3(blocks), dim3(kBlock), 0, s, row_ptr, col, T, M,
                       next, io);
    return hipGetLastError();
}

hipError_t launch_init_tuples(const TupleParams &tp, int64_t n, uint32_t *T, uint32_t *ring,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_init_tuples, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, tp, n,
                       T, ring);
    return hipGetLastError();
}

hipError_t launch_init_masked(const TupleParams &tp, int64_t n, const int32_t *label, uint32_t *T,
                              uint32_t *M, uint32_t *ring, hipStream_t s) {
    hipLaunchKernelGGL(k_init_masked, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, tp, n,
                       label, T, M, ring);
    return hipGetLastError();
}

hipError_t launch_status(int64_t n, const uint32_t *T, uint8_t *status, uint32_t *count,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_status, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, n, T,
                       status, count);
    return hipGetLastError();
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

hipError_t launch_validate(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                           uint32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(n > 0 ? n : 1, kBlock, 4096)), dim3(kBlock), 0,
                       s, n, nnz, row_ptr, col, err);
    return hipGetLastError();
}

}  // namespace mis2
