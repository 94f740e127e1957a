// batch.hip -- many graphs in one run: the disjoint union of the graphs goes
// through the same MIS-2 and aggregation kernels, and these kernels turn the
// union's aggregate numbering back into each graph's own.
//
// In the union, phase-1 roots are numbered 0..N1-1 in increasing union id and
// phase-2 roots N1..N1+N2-1 the same way (Algorithm 3's numbering applied to
// the union).  Restricted to one graph g this order is the graph's own order
// (its phase-1 roots by id, then its phase-2 roots by id), so every phase-3
// tie-break (smallest aggregate) picks the same aggregate as a run on g alone.
// Graph g's own ids are then
//   a - P1[g]                        for a phase-1 aggregate a < N1,
//   (a - N1) - P2[g] + n1[g]         for a phase-2 aggregate,
// where P1[g] / P2[g] count the union's phase-1 / phase-2 roots below g's
// first vertex and n1[g] = P1[g+1] - P1[g].
#include "internal.h"

namespace mis2 {

namespace {

// P[g] = number of entries of the increasing list[0..*d_count) below voff[g],
// for g = 0..G (P[G] = *d_count).
__global__ __launch_bounds__(kBlock) void k_graph_bounds(const int32_t *__restrict__ list,
                                                         const uint32_t *__restrict__ d_count,
                                                         const int64_t *__restrict__ voff,
                                                         int32_t G, uint32_t *__restrict__ P) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g > G) return;
    const uint32_t cnt = *d_count;
    if (g == G) {
        P[g] = cnt;
        return;
    }
    const int64_t key = voff[g];
    uint32_t lo = 0, hi = cnt;  // first index with list[idx] >= key
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)list[mid] < key) lo = mid + 1; else hi = mid;
    }
    P[g] = lo;
}

// Union aggregate ids -> graph-local ids (in place), or -1 for the vertices
// of graphs with live[g] == 0 (graphs that take no part in this level);
// map[v] (if not null) = the coarse union id of v's aggregate for graphs that
// go on to the next level (newoff[g] + local), -1 for the others.
__global__ __launch_bounds__(kBlock) void k_batch_local(int64_t n, BatchInfo bt,
                                                        const uint32_t *__restrict__ P1,
                                                        const uint32_t *__restrict__ P2,
                                                        int32_t *__restrict__ agg,
                                                        const uint8_t *__restrict__ live,
                                                        const uint8_t *__restrict__ cont,
                                                        const int64_t *__restrict__ newoff,
                                                        int32_t *__restrict__ map) {
    const uint32_t N1 = P1[bt.G];
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const int32_t g = graph_of(bt, v);
        const uint32_t a = (uint32_t)agg[v];
        const uint32_t local =
            a < N1 ? a - P1[g] : (a - N1) - P2[g] + (P1[g + 1] - P1[g]);
        // an aggregate outside g (only possible with edges between graphs)
        // is dropped rather than numbered out of range
        const bool ok = live[g] && local < (P1[g + 1] - P1[g]) + (P2[g + 1] - P2[g]);
        agg[v] = ok ? (int32_t)local : -1;
        if (map) map[v] = ok && cont[g] ? (int32_t)(newoff[g] + (int64_t)local) : -1;
    }
}

// gid[v] = graph of union vertex v (by binary search over the offsets).
__global__ __launch_bounds__(kBlock) void k_graph_ids(int64_t n, BatchInfo bt,
                                                      int32_t *__restrict__ gid) {
    bt.gid = nullptr;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        gid[v] = graph_of(bt, v);
}

// out[i] = src[idx[i]], i < count.
__global__ __launch_bounds__(kBlock) void k_gather_i64(const int64_t *__restrict__ src,
                                                       const int64_t *__restrict__ idx,
                                                       int64_t count, int64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) out[i] = src[idx[i]];
}

int grid_of(int64_t work, int cap) {
    int64_t b = (work + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace

hipError_t launch_graph_bounds(const int32_t *list, const uint32_t *d_count, const int64_t *voff,
                               int32_t G, uint32_t *P, hipStream_t s) {
    hipLaunchKernelGGL(k_graph_bounds, dim3(grid_of((int64_t)G + 1, 1 << 20)), dim3(kBlock), 0, s,
                       list, d_count, voff, G, P);
    return hipGetLastError();
}

hipError_t launch_batch_local(int64_t n, const BatchInfo &bt, const uint32_t *P1,
                              const uint32_t *P2, int32_t *agg, const uint8_t *live,
                              const uint8_t *cont, const int64_t *newoff, int32_t *map,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_local, dim3(grid_of(n, 8192)), dim3(kBlock), 0, s, n, bt, P1, P2,
                       agg, live, cont, newoff, map);
    return hipGetLastError();
}

hipError_t launch_graph_ids(int64_t n, const BatchInfo &bt, int32_t *gid, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_graph_ids, dim3(grid_of(n, 8192)), dim3(kBlock), 0, s, n, bt, gid);
    return hipGetLastError();
}

hipError_t launch_gather_i64(const int64_t *src, const int64_t *idx, int64_t count, int64_t *out,
                             hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_i64, dim3(grid_of(count, 1 << 20)), dim3(kBlock), 0, s, src, idx,
                       count, out);
    return hipGetLastError();
}

}  // namespace mis2
