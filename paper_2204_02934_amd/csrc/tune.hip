// tune.hip -- the degree histogram that classifies a graph for the plan
// tuner: how many rows have a degree in each of kDegBins ranges, and the
// largest degree.  Each of kHistBlocks workgroups writes its own partial
// counts (no atomics); the host adds them.
#include "internal.h"
#include "lanes.h"

namespace mis2 {

namespace {

// Bin of a row of d entries: 0 for d = 0, then [1,2], [3,4], [5,8], [9,16],
// [17,32], [33,128], [129,1024], above 1024.
__device__ __forceinline__ int deg_bin(int64_t d) {
    if (d <= 0) return 0;
    if (d <= 2) return 1;
    if (d <= 4) return 2;
    if (d <= 8) return 3;
    if (d <= 16) return 4;
    if (d <= 32) return 5;
    if (d <= 128) return 6;
    if (d <= 1024) return 7;
    return 8;
}

__global__ __launch_bounds__(kBlock) void k_degree_hist(int64_t n, const int64_t *__restrict__ row_ptr,
                                                        unsigned long long *__restrict__ part) {
    __shared__ unsigned long long acc[kBlock / 64][kHistWords];
    uint32_t c[kDegBins] = {};
    uint32_t mx = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
        const int64_t d = row_ptr[v + 1] - row_ptr[v];
        const int b = deg_bin(d);
#pragma unroll
        for (int k = 0; k < kDegBins; k++) c[k] += (b == k);
        mx = max(mx, (uint32_t)min(d, (int64_t)0xFFFFFFFF));
    }
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
#pragma unroll
    for (int k = 0; k < kDegBins; k++) {
        const uint32_t t = group_sum<64>(c[k]);
        if (lane == 0) acc[w][k] = t;
    }
    mx = group_max<64>(mx);
    if (lane == 0) acc[w][kDegBins] = mx;
    __syncthreads();
    if (threadIdx.x < kHistWords) {
        unsigned long long t = 0;
        for (int q = 0; q < kBlock / 64; q++) {
            const unsigned long long x = acc[q][threadIdx.x];
            t = threadIdx.x == kDegBins ? (x > t ? x : t) : t + x;
        }
        part[(size_t)blockIdx.x * kHistWords + threadIdx.x] = t;
    }
}

}  // namespace

hipError_t launch_degree_hist(int64_t n, const int64_t *row_ptr, unsigned long long *part,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_degree_hist, dim3(kHistBlocks), dim3(kBlock), 0, s, n, row_ptr, part);
    return hipGetLastError();
}

}  // namespace mis2
