// cgs.hip -- cluster multicolor Gauss-Seidel (Algorithm 4, Section III-C) on gfx950.
//
// Setup colours a graph (the coarse graph of an aggregation, or the graph
// itself for point multicolor Gauss-Seidel) and orders the rows by colour,
// then by cluster, then by row id.  Apply runs, for each colour in turn, one
// lane per cluster: the lane updates its cluster's rows one after the other.
// Clusters of one colour share no edge, so no lane reads a value another
// lane of the same launch writes, and the result is that of the sequential
// sweep in the same order.
//
// Colouring (the paper takes it from other work): Jones-Plassmann with fixed
// priorities, the packed tuple of h(seed, 0, v) (Sections V-A, V-C).  Each
// round every uncoloured vertex whose tuple is below those of its uncoloured
// neighbours takes the smallest colour no coloured neighbour has.  Two
// vertices picked in one round are never adjacent (each would be below the
// other), so a round reads only colours fixed in earlier rounds.
#include "internal.h"

namespace mis2 {

namespace {

__global__ __launch_bounds__(kBlock) void k_jp_init(int64_t n, TupleParams tp,
                                                    uint32_t *__restrict__ pr,
                                                    int32_t *__restrict__ cround,
                                                    int32_t *__restrict__ color) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        pr[v] = make_tuple(tp, (uint32_t)v);
        cround[v] = -1;
        color[v] = -1;
    }
}

// Round r.  cround[w] is the round w was coloured in (-1: not yet); a
// neighbour coloured in this very round reads as -1 or r, both "uncoloured
// when the round started", and its colour is never read.  *d_left gets the
// vertices still uncoloured after the round, *d_maxc the largest colour.
__global__ __launch_bounds__(kBlock) void k_jp_round(int64_t n, const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const uint32_t *__restrict__ pr,
                                                     int32_t *cround, int32_t *color, int r,
                                                     uint32_t *__restrict__ d_left,
                                                     uint32_t *__restrict__ d_maxc) {
    __shared__ uint32_t s_left, s_max;
    if (threadIdx.x == 0) {
        s_left = 0;
        s_max = 0;
    }
    __syncthreads();
    uint32_t left = 0;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        if (cround[v] != -1) continue;
        const int64_t s = row_ptr[v], e = row_ptr[v + 1];
        const uint32_t pv = pr[v];
        bool local_min = true;
        for (int64_t j = s; j < e; j++) {
            const int32_t w = col[j];
            const int32_t cw = cround[w];
            if ((cw == -1 || cw == r) && pr[w] < pv) local_min = false;
        }
        if (!local_min) {
            left++;
            continue;
        }
        // smallest colour not on a neighbour coloured in an earlier round,
        // 64 colours at a time; stored inside the loop
        for (int32_t base = 0;; base += 64) {
            uint64_t used = 0;
            for (int64_t j = s; j < e; j++) {
                const int32_t w = col[j];
                const int32_t cw = cround[w];
                if (cw >= 0 && cw < r) {
                    const int32_t c = color[w] - base;
                    if (c >= 0 && c < 64) used |= 1ull << c;
                }
            }
            if (used != ~0ull) {
                const int32_t c = base + __ffsll((unsigned long long)~used) - 1;
                color[v] = c;
                cround[v] = r;
                atomicMax(&s_max, (uint32_t)c);
                break;
            }
        }
    }
    if (left) atomicAdd(&s_left, left);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_left) atomicAdd(d_left, s_left);
        atomicMax(d_maxc, s_max);
    }
}

__global__ __launch_bounds__(kBlock) void k_iota(int64_t n, int32_t *__restrict__ out) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        out[v] = (int32_t)v;
}

__global__ __launch_bounds__(kBlock) void k_count_of(int64_t n, const int32_t *__restrict__ key,
                                                     uint32_t *__restrict__ cnt) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        atomicAdd(&cnt[key[v]], 1u);
}

// Colour histogram through a workgroup-local table (colours < kHistBins).
constexpr int kHistBins = 2048;
__global__ __launch_bounds__(kBlock) void k_color_hist(int64_t n, const int32_t *__restrict__ color,
                                                       int32_t n_colors, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[kHistBins];
    for (int k = threadIdx.x; k < n_colors; k += kBlock) h[k] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        atomicAdd(&h[color[v]], 1u);
    __syncthreads();
    for (int k = threadIdx.x; k < n_colors; k += kBlock)
        if (h[k]) atomicAdd(&hist[k], h[k]);
}

// members of cluster a at [moff[a], moff[a+1]) in any order.
__global__ __launch_bounds__(kBlock) void k_scatter_members(int64_t n,
                                                            const int32_t *__restrict__ cluster,
                                                            const int64_t *__restrict__ moff,
                                                            uint32_t *__restrict__ cursor,
                                                            int32_t *__restrict__ members) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const int32_t a = cluster[v];
        members[moff[a] + atomicAdd(&cursor[a], 1u)] = (int32_t)v;
    }
}

constexpr int64_t kSmallCluster = 64;

// Each cluster of at most kSmallCluster members: insertion sort by its lane
// (position by counting, then a shift: no loop leaves on a value it computes).
__global__ __launch_bounds__(kBlock) void k_sort_small(int64_t nc, const int64_t *__restrict__ moff,
                                                       int32_t *__restrict__ members) {
    for (int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x; a < nc;
         a += (int64_t)gridDim.x * kBlock) {
        const int64_t s = moff[a], e = moff[a + 1];
        if (e - s > kSmallCluster) continue;
        for (int64_t i = s + 1; i < e; i++) {
            const int32_t x = members[i];
            int64_t above = 0;  // sorted members before i that are larger than x
            for (int64_t t = s; t < i; t++) above += members[t] > x;
            for (int64_t t = i; t > i - above; t--) members[t] = members[t - 1];
            members[i - above] = x;
        }
    }
}

// Each larger cluster: one workgroup sorts it in place with a bitonic
// network on the next power of two, positions past the end reading as +inf.
// The network's first step of every merge compares i with i ^ (k - 1) and
// the later ones i with i ^ j, always the smaller value to the lower index,
// so no real value ever moves past the end.
__global__ __launch_bounds__(kBlock) void k_sort_large(int64_t nc, const int64_t *__restrict__ moff,
                                                       int32_t *__restrict__ members) {
    for (int64_t a = blockIdx.x; a < nc; a += gridDim.x) {
        const int64_t s = moff[a], size = moff[a + 1] - s;
        if (size <= kSmallCluster) continue;
        int64_t P = 1;
        while (P < size) P <<= 1;
        int32_t *m = members + s;
        for (int64_t k = 2; k <= P; k <<= 1) {
            for (int64_t j = k >> 1; j > 0; j >>= 1) {
                for (int64_t i = threadIdx.x; i < P; i += kBlock) {
                    const int64_t p = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
                    if (p > i && p < size) {
                        const int32_t x = m[i], y = m[p];
                        if (x > y) {
                            m[i] = y;
                            m[p] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_gather_sizes(int64_t nk, const int32_t *__restrict__ order,
                                                         const uint32_t *__restrict__ cnt,
                                                         uint32_t *__restrict__ out) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nk;
         k += (int64_t)gridDim.x * kBlock)
        out[k] = cnt[order[k]];
}

// rows[cluster_off[k] ...] = the sorted members of the k-th cluster of the
// sweep order.
__global__ __launch_bounds__(kBlock) void k_place_rows(int64_t nk, const int32_t *__restrict__ order,
                                                       const int64_t *__restrict__ moff,
                                                       const int32_t *__restrict__ members,
                                                       const int64_t *__restrict__ cluster_off,
                                                       int32_t *__restrict__ rows) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nk;
         k += (int64_t)gridDim.x * kBlock) {
        const int32_t a = order[k];
        const int64_t s = moff[a], e = moff[a + 1], o = cluster_off[k];
        for (int64_t t = s; t < e; t++) rows[o + t - s] = members[t];
    }
}

// One colour of a sweep: the sweep-order clusters [k0, k1), one lane each,
// rows in order (or reversed).  The update of row i is
// x_i = (b_i - sum over its off-diagonal entries of a_ij x_j) / d_i, summed
// in CSR order with separate roundings (no fused multiply-add), as the
// sequential sweep does it.
__global__ __launch_bounds__(kBlock) void k_cgs_sweep(const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ diag,
                                                      const double *__restrict__ b, double *x,
                                                      const int32_t *__restrict__ rows,
                                                      const int64_t *__restrict__ cluster_off,
                                                      int64_t k0, int64_t k1, int backward) {
#pragma clang fp contract(off)
    const int64_t k = k0 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= k1) return;
    const int64_t s = cluster_off[k], e = cluster_off[k + 1];
    for (int64_t u = 0; u < e - s; u++) {
        const int32_t i = rows[backward ? e - 1 - u : s + u];
        double r = b[i];
        for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; j++) {
            const double p = val[j] * x[col[j]];
            r = r - p;
        }
        x[i] = r / diag[i];
    }
}

int grid_of(int64_t work, int cap) {
    int64_t g = (work + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

hipError_t launch_jp_init(int64_t n, const TupleParams &tp, uint32_t *pr, int32_t *cround,
                          int32_t *color, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jp_init, dim3(grid_of(n, 8192)), dim3(kBlock), 0, s, n, tp, pr, cround,
                       color);
    return hipGetLastError();
}

hipError_t launch_jp_round(int64_t n, const int64_t *row_ptr, const int32_t *col,
                           const uint32_t *pr, int32_t *cround, int32_t *color, int r,
                           uint32_t *d_left, uint32_t *d_maxc, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jp_round, dim3(grid_of(n, 4096)), dim3(kBlock), 0, s, n, row_ptr, col,
                       pr, cround, color, r, d_left, d_maxc);
    return hipGetLastError();
}

hipError_t launch_iota(int64_t n, int32_t *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(grid_of(n, 8192)), dim3(kBlock), 0, s, n, out);
    return hipGetLastError();
}

hipError_t launch_count_of(int64_t n, const int32_t *key, uint32_t *cnt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_of, dim3(grid_of(n, 8192)), dim3(kBlock), 0, s, n, key, cnt);
    return hipGetLastError();
}

hipError_t launch_color_hist(int64_t n, const int32_t *color, int32_t n_colors, uint32_t *hist,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n_colors > kHistBins) return launch_count_of(n, color, hist, s);
    hipLaunchKernelGGL(k_color_hist, dim3(grid_of(n, 1024)), dim3(kBlock), 0, s, n, color,
                       n_colors, hist);
    return hipGetLastError();
}

hipError_t launch_sorted_members(int64_t n, const int32_t *cluster, int64_t nc,
                                 const int64_t *moff, uint32_t *cursor, int32_t *members,
                                 hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_members, dim3(grid_of(n, 8192)), dim3(kBlock), 0, s, n, cluster,
                       moff, cursor, members);
    hipLaunchKernelGGL(k_sort_small, dim3(grid_of(nc, 8192)), dim3(kBlock), 0, s, nc, moff,
                       members);
    hipLaunchKernelGGL(k_sort_large, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(nc, 1024))),
                       dim3(kBlock), 0, s, nc, moff, members);
    return hipGetLastError();
}

hipError_t launch_gather_sizes(int64_t nk, const int32_t *order, const uint32_t *cnt,
                               uint32_t *out, hipStream_t s) {
    if (nk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_sizes, dim3(grid_of(nk, 8192)), dim3(kBlock), 0, s, nk, order,
                       cnt, out);
    return hipGetLastError();
}

hipError_t launch_place_rows(int64_t nk, const int32_t *order, const int64_t *moff,
                             const int32_t *members, const int64_t *cluster_off, int32_t *rows,
                             hipStream_t s) {
    if (nk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_place_rows, dim3(grid_of(nk, 8192)), dim3(kBlock), 0, s, nk, order, moff,
                       members, cluster_off, rows);
    return hipGetLastError();
}

hipError_t launch_cgs_sweep(const int64_t *row_ptr, const int32_t *col, const double *val,
                            const double *diag, const double *b, double *x, const int32_t *rows,
                            const int64_t *cluster_off, int64_t k0, int64_t k1, bool backward,
                            hipStream_t s) {
    if (k1 <= k0) return hipSuccess;
    hipLaunchKernelGGL(k_cgs_sweep, dim3((unsigned)((k1 - k0 + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, row_ptr, col, val, diag, b, x, rows, cluster_off, k0,
                       k1, backward ? 1 : 0);
    return hipGetLastError();
}

}  // namespace mis2
