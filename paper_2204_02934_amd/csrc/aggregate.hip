// aggregate.hip -- the labelling phases of Algorithm 3 (Section III-B) for gfx950.
//
// Phase 1 / phase 2 labelling push a root's aggregate id to its neighbours:
// the roots of an MIS-2 are at least three edges apart, so the written sets
// are disjoint and the order of the writes cannot matter.  Phase 3 reads only
// the labels frozen after phase 2 (the "tentative" labels) and writes a
// separate output array, so every row is decided independently.
#include "internal.h"

namespace mis2 {

namespace {

constexpr int kLabelLanes = 16;  // lanes per root in the labelling push

// roots[0..*d_count) get ids base + k; their neighbours (all of them, or only
// those still at -1 when only_unlabelled) get the same id.
__global__ __launch_bounds__(kBlock) void k_label_roots(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ roots,
                                                        const uint32_t *__restrict__ d_count,
                                                        const uint32_t *__restrict__ d_base,
                                                        int only_unlabelled,
                                                        int32_t *__restrict__ label,
                                                        uint8_t *__restrict__ root_mark,
                                                        uint8_t mark) {
    constexpr int L = kLabelLanes, G = kBlock / L;
    const int64_t count = *d_count;
    const int32_t base = d_base ? (int32_t)*d_base : 0;
    const int sub = (int)(threadIdx.x & (L - 1));
    for (int64_t k = (int64_t)blockIdx.x * G + threadIdx.x / L; k < count;
         k += (int64_t)gridDim.x * G) {
        const int32_t r = roots[k];
        const int32_t id = base + (int32_t)k;
        const int64_t s = row_ptr[r], e = row_ptr[r + 1];
        for (int64_t j = s + sub; j < e; j += L) {
            const int32_t w = col[j];
            if (!only_unlabelled || label[w] == -1) label[w] = id;
        }
        if (sub == 0) {
            label[r] = id;
            if (root_mark) root_mark[r] = mark;
        }
    }
}

// flag[v] = 1 iff v is a root of the phase-2 MIS-2 (T_v = IN in the masked
// run) with at least two neighbours that are unlabelled after phase 1.
__global__ __launch_bounds__(kBlock) void k_accept_phase2(int64_t n,
                                                          const int64_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col,
                                                          const uint32_t *__restrict__ T,
                                                          const int32_t *__restrict__ label,
                                                          uint8_t *__restrict__ flag) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        uint8_t f = 0;
        if (label[v] == -1 && T[v] == kIn) {
            // The whole row is counted: this toolchain miscompiles a loop whose
            // exit test depends on the count when the count is used after it.
            int cnt = 0;
            const int64_t e = row_ptr[v + 1];
            for (int64_t j = row_ptr[v]; j < e; j++) cnt += label[col[j]] == -1;
            f = cnt >= 2;
        }
        flag[v] = f;
    }
}

__global__ __launch_bounds__(kBlock) void k_aggsize(int64_t n, const int32_t *__restrict__ label,
                                                    int32_t *__restrict__ aggsize) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const int32_t a = label[v];
        if (a >= 0) atomicAdd(&aggsize[a], 1);
    }
}

__global__ __launch_bounds__(kBlock) void k_copy_i32(const int32_t *__restrict__ src,
                                                     int32_t *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        dst[i] = src[i];
}

// Candidate order of phase 3: larger coupling first, then smaller aggsize,
// then smaller aggregate id.  Returns true if (c1, s1, a1) beats (c2, s2, a2).
__device__ __forceinline__ bool better(int c1, int s1, int a1, int c2, int s2, int a2) {
    if (c1 != c2) return c1 > c2;
    if (s1 != s2) return s1 < s2;
    return a1 < a2;
}

// One wavefront per unaggregated row.  Lane j of chunk c1 holds the tent
// label of neighbour c1*64 + j; its coupling is the number of equal labels
// over all chunks, counted with broadcasts.  A lane-wise best is reduced
// across the wavefront with the candidate order above.
__global__ __launch_bounds__(kBlock) void k_phase3(const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col,
                                                   const int32_t *__restrict__ label,
                                                   const int32_t *__restrict__ aggsize,
                                                   const int32_t *__restrict__ rows,
                                                   const uint32_t *__restrict__ d_rows,
                                                   int32_t *__restrict__ agg_out,
                                                   uint32_t *__restrict__ err) {
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t nrows = *d_rows;
    const int64_t wstep = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t k = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); k < nrows;
         k += wstep) {
        const int32_t v = rows[k];
        const int64_t s = row_ptr[v], e = row_ptr[v + 1];
        int bc = 0, bs = 0x7FFFFFFF, ba = 0x7FFFFFFF;  // best (coupling, size, id)
        for (int64_t c1 = s; c1 < e; c1 += 64) {
            const int64_t j = c1 + lane;
            const int32_t a = j < e ? label[col[j]] : -1;
            int cnt = 0;
            for (int64_t c2 = s; c2 < e; c2 += 64) {
                const int64_t j2 = c2 + lane;
                const int32_t a2 = j2 < e ? label[col[j2]] : -1;
                const int lim = (int)min<int64_t>(64, e - c2);
                for (int t = 0; t < lim; t++) cnt += (__shfl(a2, t, 64) == a);
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
        for (int off = 32; off > 0; off >>= 1) {
            const int oc = __shfl_xor(bc, off, 64);
            const int os = __shfl_xor(bs, off, 64);
            const int oa = __shfl_xor(ba, off, 64);
            if (better(oc, os, oa, bc, bs, ba)) {
                bc = oc;
                bs = os;
                ba = oa;
            }
        }
        if (lane == 0) {
            if (bc > 0)
                agg_out[v] = ba;
            else
                atomicOr(err, 1u);
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
                              uint8_t *root_mark, uint8_t mark, hipStream_t s) {
    hipLaunchKernelGGL(k_label_roots, dim3(grid_for(n / 4 + 1, kBlock / kLabelLanes, 4096)),
                       dim3(kBlock), 0, s, row_ptr, col, roots, d_count, d_base,
                       (int)only_unlabelled, label, root_mark, mark);
    return hipGetLastError();
}

hipError_t launch_accept_phase2(int64_t n, const int64_t *row_ptr, const int32_t *col,
                                const uint32_t *T, const int32_t *label, uint8_t *flag,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_accept_phase2, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n,
                       row_ptr, col, T, label, flag);
    return hipGetLastError();
}

hipError_t launch_aggsize(int64_t n, const int32_t *label, int32_t *aggsize, hipStream_t s) {
    hipLaunchKernelGGL(k_aggsize, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, label,
                       aggsize);
    return hipGetLastError();
}

hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, src, dst,
                       n);
    return hipGetLastError();
}

hipError_t launch_phase3(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const int32_t *label, const int32_t *aggsize, const int32_t *rows,
                         const uint32_t *d_rows, int32_t *agg_out, uint32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(k_phase3, dim3(grid_for(n / 8 + 1, kBlock / 64, 4096)), dim3(kBlock), 0, s,
                       row_ptr, col, label, aggsize, rows, d_rows, agg_out, err);
    return hipGetLastError();
}

}  // namespace mis2
