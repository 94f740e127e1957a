// quotient.hip -- coarse graph of an aggregation, for multilevel coarsening on gfx950.
//
// The paper coarsens recursively (Sections I and II) without saying how the
// next graph is formed.  Here it is the quotient graph: vertices are the
// aggregates, and a is adjacent to c iff some edge (u, w) has agg u = a,
// agg w = c and a != c.  Rows come out with ascending, distinct columns.
//
// A vertex with agg < 0 belongs to no coarse vertex (a batched run uses this
// for graphs that stop coarsening) and edges to it are dropped.
//
// Member lists are built by a counting sort (their order does not matter:
// every coarse row is a sorted set).  A coarse row whose members have at most
// kWCap stored entries in all is handled by one wavefront: it puts the
// aggregate ids of the members' neighbours into an LDS hash set and sorts the
// distinct ones.  Larger rows
// are listed and handled by a whole workgroup each: the same gather and sort
// for up to kQCap candidates, else a sweep over the coarse id space in
// windows of 32*kQCap ids with an LDS bitmap, which emits ids in increasing
// order.  Both kernels run twice: once to count each row, once (after a
// prefix sum) to write it.
#include "internal.h"

namespace mis2 {

namespace {

constexpr int kQCap = 4096;                  // candidates sorted in LDS per coarse row
constexpr int64_t kQWindow = 32 * kQCap;     // coarse ids per bitmap window
constexpr int kWaves = kBlock / 64;
constexpr int kWCap = 1024;                  // candidates of a row handled by one wavefront
constexpr int kWEdges = 8;                   // entries per lane loaded together
constexpr int kShortRow = 64;                // member rows read by one thread (bitmap path)
constexpr uint32_t kLongCap = 1024;          // long member rows listed in LDS (bitmap path)

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Coarse rows with at most kWCap candidates, one wavefront each (the others
// are appended to big[] by the counting pass).  The candidates go into a
// per-wavefront LDS hash set (open addressing, kWCap slots, so it never
// fills); each id that enters it is also appended to a list.  The distinct
// ids are then sorted -- in registers with a 64-lane bitonic network when
// there are at most 64, in LDS otherwise -- and the set is emptied by
// clearing just their slots.  FILL = false: ccnt[a]; FILL = true:
// ccol[crow[a] ...].
__device__ __forceinline__ uint32_t qhash(uint32_t c) { return (c * 2654435761u) >> 22; }

template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_coarse_rows_wave(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ agg, int64_t n_agg, const int64_t *__restrict__ moff,
    const int32_t *__restrict__ members, uint32_t *__restrict__ ccnt,
    const int64_t *__restrict__ crow, int32_t *__restrict__ ccol, int32_t *__restrict__ big,
    uint32_t *__restrict__ big_count) {
    static_assert(kWCap == 1024, "qhash yields 10 bits");
    constexpr uint32_t kEmpty = 0xFFFFFFFFu;
    __shared__ uint32_t tabs[kWaves][kWCap];
    __shared__ uint32_t lists[kWaves][kWCap];
    __shared__ uint32_t nums[kWaves];
    const int wv = (int)(threadIdx.x >> 6);
    uint32_t *tab = tabs[wv];
    uint32_t *list = lists[wv];
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int i = lane; i < kWCap; i += 64) tab[i] = kEmpty;
    if (lane == 0) nums[wv] = 0u;
    wave_sync();
    for (int64_t a = (int64_t)blockIdx.x * kWaves + wv; a < n_agg; a += nw) {
        const int64_t m0 = moff[a], m1 = moff[a + 1];
        // candidates: stored entries of all members
        unsigned long long cand = 0;
        for (int64_t i = m0 + lane; i < m1; i += 64) {
            const int32_t v = members[i];
            cand += (unsigned long long)(row_ptr[v + 1] - row_ptr[v]);
        }
        for (int off = 32; off > 0; off >>= 1) cand += __shfl_xor(cand, off, 64);
        if (cand > (unsigned long long)kWCap) {
            if (!FILL && lane == 0) big[atomicAdd(big_count, 1u)] = (int32_t)a;
            continue;
        }
        // gather into the set: each lane takes one member at a time and
        // loads kWEdges of its entries together
        for (int64_t i0 = m0; i0 < m1; i0 += 64) {
            const int64_t i = i0 + lane;
            int64_t s = 0, e = 0;
            if (i < m1) {
                const int32_t v = members[i];
                s = row_ptr[v];
                e = row_ptr[v + 1];
            }
            int64_t len = e - s, lmax = len;
            for (int off = 32; off > 0; off >>= 1) lmax = max(lmax, __shfl_xor(lmax, off, 64));
            for (int64_t c0 = 0; c0 < lmax; c0 += kWEdges) {
                int32_t x[kWEdges];
#pragma unroll
                for (int k = 0; k < kWEdges; k++) x[k] = col[c0 + k < len ? s + c0 + k : 0];
                int32_t c[kWEdges];
#pragma unroll
                for (int k = 0; k < kWEdges; k++) c[k] = agg[x[k]];
#pragma unroll
                for (int k = 0; k < kWEdges; k++) {
                    if (c0 + k < len && c[k] >= 0 && (int64_t)c[k] != a) {
                        const uint32_t key = (uint32_t)c[k];
                        uint32_t h = qhash(key);
                        for (;;) {  // the set has room for every candidate, so this ends
                            const uint32_t prev = atomicCAS(&tab[h], kEmpty, key);
                            if (prev == kEmpty) {
                                list[atomicAdd(&nums[wv], 1u)] = key;
                                break;
                            }
                            if (prev == key) break;
                            h = (h + 1) & (kWCap - 1);
                        }
                    }
                }
            }
        }
        wave_sync();
        const uint32_t m = nums[wv];
        // empty the set again: clear the slot of each distinct id (its probe
        // run holds it exactly once; other lanes' clears only leave holes)
        for (uint32_t i = lane; i < m; i += 64) {
            const uint32_t key = list[i];
            uint32_t h = qhash(key);
            while (tab[h] != key) h = (h + 1) & (kWCap - 1);
            tab[h] = kEmpty;
        }
        if (m <= 64) {
            // one id per lane; bitonic network over lane order with shuffles
            uint32_t x = (uint32_t)lane < m ? list[lane] : kEmpty;
            for (int k = 2; k <= 64; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    const uint32_t y = (uint32_t)__shfl_xor((int)x, j, 64);
                    const bool lower = (lane & j) == 0;
                    const bool up = (lane & k) == 0;
                    x = (lower == up) ? min(x, y) : max(x, y);
                }
            }
            if (FILL && (uint32_t)lane < m) ccol[crow[a] + lane] = (int32_t)x;
        } else {
            uint32_t P = 1;
            while (P < m) P <<= 1;
            for (uint32_t i = m + lane; i < P; i += 64) list[i] = kEmpty;
            wave_sync();
            for (uint32_t k = 2; k <= P; k <<= 1) {
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    for (uint32_t i = lane; i < P; i += 64) {
                        const uint32_t ixj = i ^ j;
                        if (ixj > i) {
                            const uint32_t x = list[i], y = list[ixj];
                            const bool up = (i & k) == 0;
                            if ((x > y) == up) {
                                list[i] = y;
                                list[ixj] = x;
                            }
                        }
                    }
                    wave_sync();
                }
            }
            if (FILL)
                for (uint32_t i = lane; i < m; i += 64) ccol[crow[a] + i] = (int32_t)list[i];
        }
        if (!FILL && lane == 0) ccnt[a] = m;
        wave_sync();
        if (lane == 0) nums[wv] = 0u;
        wave_sync();
    }
}

__global__ __launch_bounds__(kBlock) void k_member_count(int64_t n, const int32_t *__restrict__ agg,
                                                         uint32_t *__restrict__ cnt) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const int32_t a = agg[v];
        if (a >= 0) atomicAdd(&cnt[a], 1u);
    }
}

__global__ __launch_bounds__(kBlock) void k_member_scatter(int64_t n, const int32_t *__restrict__ agg,
                                                           const int64_t *__restrict__ moff,
                                                           uint32_t *__restrict__ cursor,
                                                           int32_t *__restrict__ members) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const int32_t a = agg[v];
        if (a < 0) continue;
        const uint32_t pos = atomicAdd(&cursor[a], 1u);
        members[moff[a] + pos] = (int32_t)v;
    }
}

// Sum over the workgroup (all threads must call it; result in every thread).
__device__ __forceinline__ unsigned long long block_sum(unsigned long long x,
                                                        unsigned long long *scratch) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) scratch[threadIdx.x >> 6] = x;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < kWaves; w++) t += scratch[w];
    return t;
}

// Exclusive prefix of x over the workgroup in thread order; *total gets the
// sum.  All threads must call it.
__device__ __forceinline__ uint32_t block_excl(uint32_t x, uint32_t *scratch, uint32_t *total) {
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    uint32_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, off, 64);
        if (lane >= off) incl += y;
    }
    __syncthreads();
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    uint32_t before = 0, t = 0;
    for (int w = 0; w < kWaves; w++) {
        if (w < wave) before += scratch[w];
        t += scratch[w];
    }
    *total = t;
    return before + incl - x;
}

// FILL = false: ccnt[a] = number of distinct coarse neighbours of row a.
// FILL = true:  ccol[crow[a] ...] = those neighbours in increasing order.
// The listed (large) coarse rows big[0 .. *big_count), one workgroup each.
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_coarse_rows(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ agg,
                                                        int64_t n_agg,
                                                        const int64_t *__restrict__ moff,
                                                        const int32_t *__restrict__ members,
                                                        uint32_t *__restrict__ ccnt,
                                                        const int64_t *__restrict__ crow,
                                                        int32_t *__restrict__ ccol,
                                                        const int32_t *__restrict__ big,
                                                        const uint32_t *__restrict__ big_count) {
    __shared__ uint32_t buf[kQCap];
    __shared__ unsigned long long red[kWaves];
    __shared__ uint32_t scan_s[kWaves];
    __shared__ uint32_t fill_s;
    __shared__ uint32_t longm[kLongCap];
    __shared__ uint32_t nlong_s;
    const int tid = (int)threadIdx.x;
    const int64_t nbig = *big_count;
    for (int64_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const int64_t a = big[bi];
        const int64_t m0 = moff[a], m1 = moff[a + 1];
        unsigned long long cand = 0;
        for (int64_t i = m0 + tid; i < m1; i += kBlock) {
            const int32_t v = members[i];
            cand += (unsigned long long)(row_ptr[v + 1] - row_ptr[v]);
        }
        cand = block_sum(cand, red);
        uint32_t distinct = 0;
        if (cand <= (unsigned long long)kQCap) {
            // gather the candidate ids (self excluded) into LDS
            if (tid == 0) fill_s = 0;
            __syncthreads();
            for (int64_t i = m0 + tid; i < m1; i += kBlock) {
                const int32_t v = members[i];
                for (int64_t j = row_ptr[v], e = row_ptr[v + 1]; j < e; j++) {
                    const int32_t c = agg[col[j]];
                    if (c >= 0 && (int64_t)c != a) buf[atomicAdd(&fill_s, 1u)] = (uint32_t)c;
                }
            }
            __syncthreads();
            const uint32_t m = fill_s;
            uint32_t P = 1;
            while (P < m) P <<= 1;
            for (uint32_t i = m + tid; i < P; i += kBlock) buf[i] = 0xFFFFFFFFu;
            __syncthreads();
            // bitonic sort of buf[0..P)
            for (uint32_t k = 2; k <= P; k <<= 1) {
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    for (uint32_t i = tid; i < P; i += kBlock) {
                        const uint32_t ixj = i ^ j;
                        if (ixj > i) {
                            const uint32_t x = buf[i], y = buf[ixj];
                            const bool up = (i & k) == 0;
                            if ((x > y) == up) {
                                buf[i] = y;
                                buf[ixj] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            // distinct values, in order
            uint32_t run = 0;
            for (uint32_t c0 = 0; c0 < m; c0 += kBlock) {
                const uint32_t i = c0 + tid;
                const bool first = i < m && (i == 0 || buf[i] != buf[i - 1]);
                uint32_t tot;
                const uint32_t pos = block_excl(first ? 1u : 0u, scan_s, &tot);
                if (FILL && first) ccol[crow[a] + run + pos] = (int32_t)buf[i];
                run += tot;
            }
            distinct = run;
        } else {
            // bitmap windows over the coarse id space.  Members with short
            // rows are read one per thread; members with long rows (listed
            // once, in LDS) by the whole workgroup each.
            if (tid == 0) nlong_s = 0u;
            __syncthreads();
            for (int64_t i = m0 + tid; i < m1; i += kBlock) {
                const int32_t v = members[i];
                if (row_ptr[v + 1] - row_ptr[v] > kShortRow) {
                    const uint32_t k = atomicAdd(&nlong_s, 1u);
                    if (k < kLongCap) longm[k] = (uint32_t)(i - m0);
                }
            }
            __syncthreads();
            const uint32_t nlong = nlong_s;
            uint32_t run = 0;
            for (int64_t lo = 0; lo < n_agg; lo += kQWindow) {
                for (int i = tid; i < kQCap; i += kBlock) buf[i] = 0u;
                __syncthreads();
                for (int64_t i = m0 + tid; i < m1; i += kBlock) {
                    const int32_t v = members[i];
                    const int64_t rs = row_ptr[v], len = row_ptr[v + 1] - rs;
                    if (len > kShortRow) continue;
                    for (int64_t c0 = 0; c0 < len; c0 += kWEdges) {
                        int32_t x[kWEdges];
#pragma unroll
                        for (int k = 0; k < kWEdges; k++) x[k] = col[c0 + k < len ? rs + c0 + k : rs];
                        int32_t c[kWEdges];
#pragma unroll
                        for (int k = 0; k < kWEdges; k++) c[k] = agg[x[k]];
#pragma unroll
                        for (int k = 0; k < kWEdges; k++) {
                            const int64_t ck = c[k];
                            if (c0 + k < len && ck != a && ck >= lo && ck < lo + kQWindow) {
                                const int64_t o = ck - lo;
                                atomicOr(&buf[o >> 5], 1u << (o & 31));
                            }
                        }
                    }
                }
                for (uint32_t t = 0; t < (nlong <= kLongCap ? nlong : 0u); t++) {
                    const int32_t v = members[m0 + longm[t]];
                    for (int64_t j = row_ptr[v] + tid, e = row_ptr[v + 1]; j < e; j += kBlock) {
                        const int64_t c = agg[col[j]];
                        if (c != a && c >= lo && c < lo + kQWindow) {
                            const int64_t o = c - lo;
                            atomicOr(&buf[o >> 5], 1u << (o & 31));
                        }
                    }
                }
                if (nlong > kLongCap) {  // too many long members to list: scan them all
                    for (int64_t i = m0; i < m1; i++) {
                        const int32_t v = members[i];
                        if (row_ptr[v + 1] - row_ptr[v] <= kShortRow) continue;
                        for (int64_t j = row_ptr[v] + tid, e = row_ptr[v + 1]; j < e;
                             j += kBlock) {
                            const int64_t c = agg[col[j]];
                            if (c != a && c >= lo && c < lo + kQWindow) {
                                const int64_t o = c - lo;
                                atomicOr(&buf[o >> 5], 1u << (o & 31));
                            }
                        }
                    }
                }
                __syncthreads();
                for (int c0 = 0; c0 < kQCap; c0 += kBlock) {
                    const int wi = c0 + tid;
                    const uint32_t word = buf[wi];
                    uint32_t tot;
                    const uint32_t pos = block_excl((uint32_t)__popc(word), scan_s, &tot);
                    if (FILL) {
                        uint32_t wv = word, k = 0;
                        while (wv) {
                            const int bit = __ffs(wv) - 1;
                            wv &= wv - 1;
                            ccol[crow[a] + run + pos + k] = (int32_t)(lo + (int64_t)wi * 32 + bit);
                            k++;
                        }
                    }
                    run += tot;
                }
                __syncthreads();
            }
            distinct = run;
        }
        if (!FILL && tid == 0) ccnt[a] = distinct;
        __syncthreads();
    }
}

int grid_for(int64_t work, int per_block, int cap) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace

hipError_t quotient_graph(const int64_t *row_ptr, const int32_t *col, int64_t n, const int32_t *agg,
                          int64_t n_agg, int64_t *crow, int32_t *ccol, const QuotientWs &q,
                          hipStream_t s) {
    hipError_t e;
    if ((e = launch_fill_u32(q.cnt, 0u, n_agg, s)) != hipSuccess) return e;
    if (n > 0)
        hipLaunchKernelGGL(k_member_count, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n,
                           agg, q.cnt);
    if ((e = exclusive_scan_u32_i64(q.cnt, n_agg, q.moff, q.part, s)) != hipSuccess) return e;
    if ((e = launch_fill_u32(q.cnt, 0u, n_agg, s)) != hipSuccess) return e;
    if (n > 0)
        hipLaunchKernelGGL(k_member_scatter, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s,
                           n, agg, q.moff, q.cnt, q.members);
    const int wblocks = grid_for(n_agg, kWaves, 8192);
    const int bblocks = 1024;
    if ((e = launch_fill_u32(q.big_count, 0u, 1, s)) != hipSuccess) return e;
    if (n_agg > 0) {
        hipLaunchKernelGGL(k_coarse_rows_wave<false>, dim3(wblocks), dim3(kBlock), 0, s, row_ptr,
                           col, agg, n_agg, q.moff, q.members, q.cnt, (const int64_t *)nullptr,
                           (int32_t *)nullptr, q.big, q.big_count);
        hipLaunchKernelGGL(k_coarse_rows<false>, dim3(bblocks), dim3(kBlock), 0, s, row_ptr, col,
                           agg, n_agg, q.moff, q.members, q.cnt, (const int64_t *)nullptr,
                           (int32_t *)nullptr, (const int32_t *)q.big,
                           (const uint32_t *)q.big_count);
    }
    if ((e = exclusive_scan_u32_i64(q.cnt, n_agg, crow, q.part, s)) != hipSuccess) return e;
    if (n_agg > 0) {
        hipLaunchKernelGGL(k_coarse_rows_wave<true>, dim3(wblocks), dim3(kBlock), 0, s, row_ptr,
                           col, agg, n_agg, q.moff, q.members, q.cnt, crow, ccol, q.big,
                           q.big_count);
        hipLaunchKernelGGL(k_coarse_rows<true>, dim3(bblocks), dim3(kBlock), 0, s, row_ptr, col,
                           agg, n_agg, q.moff, q.members, q.cnt, crow, ccol,
                           (const int32_t *)q.big, (const uint32_t *)q.big_count);
    }
    return hipGetLastError();
}

}  // namespace mis2
