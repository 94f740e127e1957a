// compact.hip -- order-preserving stream compaction for gfx950.
//
// out = [v in 0..n-1 : pred(v)] in increasing v.  Used wherever a numbering
// must be deterministic: aggregate ids are ranks of roots in increasing
// vertex id, so the positions here are exact prefix sums (no atomics).
// Up to 4096 tiles: per-tile counts, then one scatter launch in which each
// workgroup sums the counts of the tiles before its own and scans its tile
// with wave64 ballots.  Past that: counts, a one-workgroup scan of the
// counts, then the per-tile scatter.
#include "internal.h"

namespace mis2 {

namespace {

constexpr int kItems = 8;                  // elements per thread per tile
constexpr int kTile = kBlock * kItems;     // 2048 elements per tile
constexpr int kWaves = kBlock / 64;
static_assert(kTile == kCompactTile, "one tile size for every compaction");
constexpr int64_t kOnePassTiles = 4096;    // one-launch scatter up to this many tiles

struct PredU32Eq {
    const uint32_t *a;
    uint32_t value;
    __device__ bool operator()(int64_t i) const { return a[i] == value; }
};
struct PredU8Nz {
    const uint8_t *a;
    __device__ bool operator()(int64_t i) const { return a[i] != 0; }
};

__global__ void k_fill_first_i64(int64_t *out) {
    if (threadIdx.x == 0) out[0] = 0;
}

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

template <class P>
__global__ __launch_bounds__(kBlock) void k_tile_count(P pred, int64_t n,
                                                       uint32_t *__restrict__ blocksum) {
    __shared__ uint32_t part[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if (i < n && pred(i)) c++;
    }
    for (int off = 32; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off, 64);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; w++) t += part[w];
        blocksum[blockIdx.x] = t;
    }
}

// Exclusive scan of blocksum[0..nb) in place; the total goes to
// blocksum[nb] and *d_count.  One workgroup, chunks of kBlock with a carry.
__global__ __launch_bounds__(kBlock) void k_scan_tiles(uint32_t *__restrict__ blocksum, int64_t nb,
                                                       uint32_t *__restrict__ d_count) {
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    for (int64_t c0 = 0; c0 < nb; c0 += kBlock) {
        const int64_t i = c0 + threadIdx.x;
        const uint32_t x = i < nb ? blocksum[i] : 0u;
        // inclusive scan inside the wavefront
        uint32_t incl = x;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = carry_s;
        for (int w = 0; w < wave; w++) before += wsum[w];
        if (i < nb) blocksum[i] = before + incl - x;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry_s = before + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        blocksum[nb] = carry_s;
        *d_count = carry_s;
    }
}

template <class P>
__global__ __launch_bounds__(kBlock) void k_tile_scatter(P pred, int64_t n,
                                                         const uint32_t *__restrict__ blocksum,
                                                         int32_t *__restrict__ out) {
    __shared__ uint32_t wcount[kItems][kWaves];
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint64_t masks[kItems];
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        const bool p = i < n && pred(i);
        masks[j] = __ballot(p);
        if (lane == 0) wcount[j][wave] = (uint32_t)__popcll(masks[j]);
    }
    __syncthreads();
    uint32_t run = blocksum[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        uint32_t before = run;
        for (int w = 0; w < wave; w++) before += wcount[j][w];
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if ((masks[j] >> lane) & 1ull)
            out[before + (uint32_t)__popcll(masks[j] & lanes_below(lane))] = (int32_t)i;
        for (int w = 0; w < kWaves; w++) run += wcount[j][w];
    }
}

// k_tile_count with fills beside it: zero_u8 over the tile (when not null)
// and the spans of f over the grid.
template <class P>
__global__ __launch_bounds__(kBlock) void k_tile_count_fill(P pred, int64_t n,
                                                            uint32_t *__restrict__ blocksum,
                                                            FillSpans f, uint8_t *zero_u8) {
    __shared__ uint32_t part[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if (i < n && pred(i)) c++;
        if (zero_u8 && i < n) zero_u8[i] = 0;
    }
    for (int off = 32; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off, 64);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; w++) t += part[w];
        blocksum[blockIdx.x] = t;
    }
    fill_span_words(f);
}

// k_tile_scatter with its own scan: workgroup b sums the counts of tiles
// 0 .. b-1 itself (blocksum holds every tile's count, as k_tile_count wrote
// it), and the last workgroup writes the total to *d_count.
template <class P>
__global__ __launch_bounds__(kBlock) void k_scan_scatter(P pred, int64_t n,
                                                         const uint32_t *__restrict__ blocksum,
                                                         int32_t *__restrict__ out,
                                                         uint32_t *__restrict__ d_count) {
    __shared__ uint32_t wcount[kItems][kWaves];
    __shared__ uint32_t red[kWaves];
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    uint32_t pre = 0;
    for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += kBlock) pre += blocksum[t];
    for (int off = 32; off > 0; off >>= 1) pre += (uint32_t)__shfl_xor((int)pre, off, 64);
    if (lane == 0) red[wave] = pre;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint64_t masks[kItems];
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        const bool p = i < n && pred(i);
        masks[j] = __ballot(p);
        if (lane == 0) wcount[j][wave] = (uint32_t)__popcll(masks[j]);
    }
    __syncthreads();
    uint32_t run = 0;
    for (int w = 0; w < kWaves; w++) run += red[w];
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        uint32_t before = run;
        for (int w = 0; w < wave; w++) before += wcount[j][w];
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if ((masks[j] >> lane) & 1ull)
            out[before + (uint32_t)__popcll(masks[j] & lanes_below(lane))] = (int32_t)i;
        for (int w = 0; w < kWaves; w++) run += wcount[j][w];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *d_count = run;
}

template <class P>
hipError_t scatter_counted(P pred, int64_t n, int32_t *out, uint32_t *d_count,
                           uint32_t *blocksum, hipStream_t s) {
    const int64_t nb = compact_blocks(n);
    if (nb > 0 && nb <= kOnePassTiles) {
        hipLaunchKernelGGL(k_scan_scatter<P>, dim3((unsigned)nb), dim3(kBlock), 0, s, pred, n,
                           (const uint32_t *)blocksum, out, d_count);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, s, blocksum, nb, d_count);
    if (nb > 0) {
        hipLaunchKernelGGL(k_tile_scatter<P>, dim3((unsigned)nb), dim3(kBlock), 0, s, pred, n,
                           (const uint32_t *)blocksum, out);
    }
    return hipGetLastError();
}

template <class P>
hipError_t compact(P pred, int64_t n, int32_t *out, uint32_t *d_count, uint32_t *blocksum,
                   hipStream_t s) {
    const int64_t nb = compact_blocks(n);
    if (nb > 0) {
        hipLaunchKernelGGL(k_tile_count<P>, dim3((unsigned)nb), dim3(kBlock), 0, s, pred, n,
                           blocksum);
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, s, blocksum, nb, d_count);
    if (nb > 0) {
        hipLaunchKernelGGL(k_tile_scatter<P>, dim3((unsigned)nb), dim3(kBlock), 0, s, pred, n,
                           blocksum, out);
    }
    return hipGetLastError();
}

}  // namespace

int64_t compact_blocks(int64_t n) { return n <= 0 ? 0 : (n + kTile - 1) / kTile; }

hipError_t compact_u32_eq(const uint32_t *a, uint32_t value, int64_t n, int32_t *out,
                          uint32_t *d_count, uint32_t *blocksum, hipStream_t s) {
    return compact(PredU32Eq{a, value}, n, out, d_count, blocksum, s);
}

hipError_t count_in_with_fills(const uint32_t *T, int64_t n, const FillSpans &f, uint8_t *zero_u8,
                               uint32_t *blocksum, hipStream_t s) {
    const int64_t nb = compact_blocks(n);
    if (nb <= 0) return launch_fill_spans(f, s);
    hipLaunchKernelGGL(k_tile_count_fill<PredU32Eq>, dim3((unsigned)nb), dim3(kBlock), 0, s,
                       PredU32Eq{T, kIn}, n, blocksum, f, zero_u8);
    return hipGetLastError();
}

hipError_t scatter_counted_u32_eq(const uint32_t *a, uint32_t value, int64_t n, int32_t *out,
                                  uint32_t *d_count, uint32_t *blocksum, hipStream_t s) {
    return scatter_counted(PredU32Eq{a, value}, n, out, d_count, blocksum, s);
}

hipError_t scatter_counted_u8_nz(const uint8_t *a8, int64_t n, int32_t *out, uint32_t *d_count,
                                 uint32_t *blocksum, hipStream_t s) {
    return scatter_counted(PredU8Nz{a8}, n, out, d_count, blocksum, s);
}

hipError_t count_u8_nz(const uint8_t *a8, int64_t n, uint32_t *blocksum, hipStream_t s) {
    const int64_t nb = compact_blocks(n);
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_count<PredU8Nz>, dim3((unsigned)nb), dim3(kBlock), 0, s,
                       PredU8Nz{a8}, n, blocksum);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum of u32 counts into int64 offsets: out[i] = sum of
// in[0..i), out[n] = total.  Tile sums, a one-workgroup scan of the tile sums
// (64-bit), then a per-tile scan that writes the offsets.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_tile_sum_u32(const uint32_t *__restrict__ in, int64_t n,
                                                         unsigned long long *__restrict__ part) {
    __shared__ unsigned long long ws[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    unsigned long long c = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        if (i < n) c += in[i];
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63u) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kWaves; w++) t += ws[w];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_parts_u64(unsigned long long *__restrict__ part,
                                                           int64_t nb) {
    __shared__ unsigned long long wsum[kWaves];
    __shared__ unsigned long long carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    for (int64_t c0 = 0; c0 < nb; c0 += kBlock) {
        const int64_t i = c0 + threadIdx.x;
        const unsigned long long x = i < nb ? part[i] : 0ull;
        unsigned long long incl = x;
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned long long y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        unsigned long long before = carry_s;
        for (int w = 0; w < wave; w++) before += wsum[w];
        if (i < nb) part[i] = before + incl - x;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry_s = before + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) part[nb] = carry_s;
}

__global__ __launch_bounds__(kBlock) void k_tile_scan_u32(const uint32_t *__restrict__ in, int64_t n,
                                                          const unsigned long long *__restrict__ part,
                                                          int64_t *__restrict__ out, int64_t nb) {
    __shared__ unsigned long long wsum[kWaves];
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    unsigned long long run = part[blockIdx.x];
    for (int j = 0; j < kItems; j++) {
        const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
        const unsigned long long x = i < n ? in[i] : 0ull;
        unsigned long long incl = x;
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned long long y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        unsigned long long before = run;
        for (int w = 0; w < wave; w++) before += wsum[w];
        if (i < n) out[i] = (int64_t)(before + incl - x);
        unsigned long long tot = 0;
        for (int w = 0; w < kWaves; w++) tot += wsum[w];
        __syncthreads();
        run += tot;
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = (int64_t)part[nb];
}

hipError_t launch_scan_tiles(uint32_t *blocksum, int64_t nb, uint32_t *d_total, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, s, blocksum, nb, d_total);
    return hipGetLastError();
}

int64_t scan_parts(int64_t n) { return compact_blocks(n) + 1; }

hipError_t exclusive_scan_u32_i64(const uint32_t *in, int64_t n, int64_t *out,
                                  unsigned long long *part, hipStream_t s) {
    const int64_t nb = compact_blocks(n);
    if (nb == 0) {
        hipLaunchKernelGGL(k_fill_first_i64, dim3(1), dim3(64), 0, s, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_tile_sum_u32, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_parts_u64, dim3(1), dim3(kBlock), 0, s, part, nb);
    hipLaunchKernelGGL(k_tile_scan_u32, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, part, out, nb);
    return hipGetLastError();
}

hipError_t compact_u8_nz(const uint8_t *a, int64_t n, int32_t *out, uint32_t *d_count,
                         uint32_t *blocksum, hipStream_t s) {
    return compact(PredU8Nz{a}, n, out, d_count, blocksum, s);
}

}  // namespace mis2
