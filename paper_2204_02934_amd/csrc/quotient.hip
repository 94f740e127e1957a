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
// every coarse row is a sorted set).  Rows go to one of four paths by their
// candidate count (the members' stored entries): up to kWSmall and up to
// kWCap, one wavefront each (two passes; the first, with a small LDS hash
// set, keeps many rows in flight and marks the rows it leaves to the
// second); up to kGiantCand, one workgroup each; beyond, a bitmap slot that
// the whole grid fills.  A wavefront puts the aggregate ids of the members'
// neighbours into its LDS hash set and ranks the distinct ones; a workgroup
// sorts them in LDS or sweeps windows of 32*kBitWords coarse ids with an LDS
// bitmap, which emits ids in increasing order and, after the first window,
// visits only the range the row's candidates span.  Every path deals the
// members' entries out evenly over its lanes.  Each kernel runs twice: once
// to count each row, once (after a prefix sum) to write it.
#include "internal.h"
#include "lanes.h"

namespace mis2 {

namespace {

constexpr int kQCap = 4096;                  // candidates sorted in LDS per coarse row
constexpr int kBitWords = 12288;             // LDS bitmap words (48 KiB)
constexpr int64_t kQWindow = 32 * (int64_t)kBitWords;  // coarse ids per bitmap window
constexpr int kWaves = kBlock / 64;
constexpr int kWCap = 1024;                  // candidates of a row handled by one wavefront
constexpr int kWSmall = 128;                 // rows a wavefront takes in the first pass
constexpr int kWEdges = 8;                   // entries per lane loaded together

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Coarse rows with at most CAP candidates, one wavefront each.  kRowsMark:
// every coarse row; the count pass marks in cls[a] whether row a has more
// than CAP candidates (1) or not (0), and the fill pass skips the marked
// rows.  kRowsMarked: the rows marked 1; the count pass marks 2 on those with
// more than CAP candidates and lists them in next[] for the workgroup kernel.
// kRowsList: every coarse row, listing those with more than CAP in next[].  The candidates go into a per-wavefront LDS hash set
// (open addressing, CAP slots, so it never fills); each id that enters it is
// also appended to a list.  The distinct ids are then ranked -- by counting,
// each against all the others, when there are at most 64, else by a bitonic
// sort in LDS -- and the set is emptied by clearing just their slots.  A
// small CAP keeps the LDS per wavefront small, so that many rows are in
// flight at once: the rows of a fine mesh's aggregates are a few dozen
// candidates each.  FILL = false: ccnt[a]; FILL = true: ccol[crow[a] ...].
template <int CAP>
__device__ __forceinline__ uint32_t qhash(uint32_t c) {
    static_assert((CAP & (CAP - 1)) == 0 && CAP >= 64 && CAP <= 65536, "CAP: a power of two");
    constexpr int bits = __builtin_ctz(CAP);
    return (c * 2654435761u) >> (32 - bits);
}

// MODE: which rows a pass takes and what it does with the rows of more
// than CAP candidates.
enum { kRowsMark = 0, kRowsMarked = 1, kRowsList = 2 };

template <bool FILL, int CAP, int MODE>
__global__ __launch_bounds__(kBlock) void k_coarse_rows_wave(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ agg, int64_t n_agg, const int64_t *__restrict__ moff,
    const int32_t *__restrict__ members, uint32_t *__restrict__ ccnt,
    const int64_t *__restrict__ crow, int32_t *__restrict__ ccol, uint8_t *__restrict__ cls,
    int32_t *__restrict__ next, uint32_t *__restrict__ next_count) {
    constexpr uint32_t kEmpty = 0xFFFFFFFFu;
    __shared__ uint32_t tabs[kWaves][CAP];
    __shared__ uint32_t lists[kWaves][CAP];
    __shared__ uint32_t nums[kWaves];
    __shared__ uint32_t woffs[kWaves][65];
    __shared__ int64_t wsts[kWaves][64];
    const int wv = (int)(threadIdx.x >> 6);
    uint32_t *tab = tabs[wv];
    uint32_t *list = lists[wv];
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int i = lane; i < CAP; i += 64) tab[i] = kEmpty;
    if (lane == 0) nums[wv] = 0u;
    wave_sync();
    auto row = [&](const int64_t a) {
        const int64_t m0 = moff[a], m1 = moff[a + 1];
        // candidates: stored entries of all members (each lane's part
        // clamped: only "more than CAP" matters)
        uint32_t cand = 0;
        for (int64_t i = m0 + lane; i < m1; i += 64) {
            const int32_t v = members[i];
            const int64_t d = row_ptr[v + 1] - row_ptr[v];
            cand = (uint32_t)min((int64_t)cand + d, (int64_t)1 << 24);
        }
        cand = group_sum<64>(cand);
        if (!FILL && lane == 0) {
            if (MODE == kRowsMark) {
                cls[a] = cand > (uint32_t)CAP ? 1 : 0;
            } else if (cand > (uint32_t)CAP) {
                if (MODE == kRowsMarked) cls[a] = 2;
                next[atomicAdd(next_count, 1u)] = (int32_t)a;
            }
        }
        if (cand > (uint32_t)CAP) return;
        // gather into the set: the members go 64 at a time; their entries
        // are numbered by a wave scan of the row lengths and dealt out
        // evenly, kWEdges per lane loaded together, each lane finding its
        // row by binary search over the offsets
        auto put = [&](int32_t cv) {
            if (cv < 0 || (int64_t)cv == a) return;
            const uint32_t key = (uint32_t)cv;
            uint32_t h = qhash<CAP>(key);
            for (;;) {  // the set has room for every candidate, so this ends
                const uint32_t prev = atomicCAS(&tab[h], kEmpty, key);
                if (prev == kEmpty) {
                    list[atomicAdd(&nums[wv], 1u)] = key;
                    break;
                }
                if (prev == key) break;
                h = (h + 1) & (CAP - 1);
            }
        };
        uint32_t *woff = woffs[wv];
        int64_t *wst = wsts[wv];
        for (int64_t c0 = m0; c0 < m1; c0 += 64) {
            const int64_t i = c0 + lane;
            int64_t rs = 0;
            uint32_t len = 0;  // a row of this path has at most CAP entries
            if (i < m1) {
                const int32_t v = members[i];
                rs = row_ptr[v];
                len = (uint32_t)(row_ptr[v + 1] - rs);
            }
            const uint32_t incl = wave_incl_scan(len);
            const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            woff[lane + 1] = incl;
            wst[lane] = rs;
            if (lane == 0) woff[0] = 0u;
            wave_sync();
            for (uint32_t q0 = (uint32_t)lane; q0 < tot; q0 += 64u * kWEdges) {
                int32_t x[kWEdges];
#pragma unroll
                for (int k = 0; k < kWEdges; k++) {
                    uint32_t q = q0 + 64u * (uint32_t)k;
                    if (q >= tot) q = tot - 1;  // a valid entry; its result is not used
                    int r = 0;  // the last row with woff[r] <= q (it is not empty)
#pragma unroll
                    for (int st = 32; st > 0; st >>= 1)
                        if (woff[r + st] <= q) r += st;
                    x[k] = col[wst[r] + (int64_t)(q - woff[r])];
                }
                int32_t c[kWEdges];
#pragma unroll
                for (int k = 0; k < kWEdges; k++) c[k] = agg[x[k]];
#pragma unroll
                for (int k = 0; k < kWEdges; k++)
                    if (q0 + 64u * (uint32_t)k < tot) put(c[k]);
            }
            wave_sync();  // the offsets are rewritten by the next chunk
        }
        wave_sync();
        const uint32_t m = nums[wv];
        if (m <= 64) {
            // rank each id by counting the smaller ones (ids are distinct)
            if (FILL && (uint32_t)lane < m) {
                const uint32_t x = list[lane];
                uint32_t rank = 0;
                for (uint32_t y = 0; y < m; y++) rank += list[y] < x ? 1u : 0u;
                ccol[crow[a] + rank] = (int32_t)x;
            }
        } else if (FILL) {
            // bitonic sort of a copy in the set's table, then the table
            // is cleared whole
            uint32_t P = 1;
            while (P < m) P <<= 1;
            for (uint32_t i = lane; i < P; i += 64) tab[i] = i < m ? list[i] : kEmpty;
            wave_sync();
            for (uint32_t k = 2; k <= P; k <<= 1) {
                for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                    for (uint32_t i = lane; i < P; i += 64) {
                        const uint32_t ixj = i ^ jj;
                        if (ixj > i) {
                            const uint32_t x = tab[i], y = tab[ixj];
                            const bool up = (i & k) == 0;
                            if ((x > y) == up) {
                                tab[i] = y;
                                tab[ixj] = x;
                            }
                        }
                    }
                    wave_sync();
                }
            }
            for (uint32_t i = lane; i < m; i += 64) ccol[crow[a] + i] = (int32_t)tab[i];
        }
        wave_sync();
        // empty the set again
        if (FILL && m > 64) {
            for (int i = lane; i < CAP; i += 64) tab[i] = kEmpty;
        } else {
            // clear the slot of each distinct id (its probe run holds it
            // exactly once; other lanes' clears only leave holes)
            for (uint32_t i = lane; i < m; i += 64) {
                const uint32_t key = list[i];
                uint32_t h = qhash<CAP>(key);
                while (tab[h] != key) h = (h + 1) & (CAP - 1);
                tab[h] = kEmpty;
            }
        }
        if (!FILL && lane == 0) ccnt[a] = m;
        wave_sync();
        if (lane == 0) nums[wv] = 0u;
        wave_sync();
    };
    const int64_t w0 = (int64_t)blockIdx.x * kWaves + wv;
    if (MODE != kRowsMarked) {
        for (int64_t a = w0; a < n_agg; a += nw) row(a);
    } else {
        // the wavefront's rows w0, w0 + nw, ...: 64 marks read at once (2:
        // marked by this kernel's count pass), so the marked rows stay
        // spread over all wavefronts
        for (int64_t j0 = 0; w0 + j0 * nw < n_agg; j0 += 64) {
            const int64_t v = w0 + (j0 + lane) * nw;
            const bool mine = v < n_agg && cls[v] >= 1;
            uint64_t mask = __ballot(mine);
            while (mask) {
                const int r = __ffsll((unsigned long long)mask) - 1;
                mask &= mask - 1;
                row(w0 + (j0 + r) * nw);
            }
        }
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

// Minimum of *mn and maximum of *mx over the workgroup, in every thread (all
// threads must call it).
__device__ __forceinline__ void block_minmax(int32_t *mn, int32_t *mx, int32_t *scratch) {
    int32_t a = *mn, b = *mx;
    for (int off = 32; off > 0; off >>= 1) {
        a = min(a, __shfl_xor(a, off, 64));
        b = max(b, __shfl_xor(b, off, 64));
    }
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) {
        scratch[threadIdx.x >> 6] = a;
        scratch[kWaves + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    for (int w = 0; w < kWaves; w++) {
        a = min(a, scratch[w]);
        b = max(b, scratch[kWaves + w]);
    }
    *mn = a;
    *mx = b;
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

// Exclusive prefix of x over the workgroup in thread order (64-bit); *total
// gets the sum.  All threads must call it.
__device__ __forceinline__ unsigned long long block_excl64(unsigned long long x,
                                                           unsigned long long *scratch,
                                                           unsigned long long *total) {
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    unsigned long long incl = x;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    __syncthreads();
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    unsigned long long before = 0, t = 0;
    for (int w = 0; w < kWaves; w++) {
        if (w < wave) before += scratch[w];
        t += scratch[w];
    }
    *total = t;
    return before + incl - x;
}

// LDS of walk_members: the entry offsets and row starts of one chunk of
// kBlock members.
struct WalkLds {
    unsigned long long off[kBlock + 1];
    int64_t start[kBlock];
    unsigned long long scan[kWaves];
};

// f(c) for the coarse id c = agg[col[j]] of every entry j of every member of
// an aggregate (members[m0 .. m1)).  The members go in chunks of kBlock; the
// chunk's entries are numbered through a prefix sum of the row lengths and
// dealt out evenly, kWEdges per thread loaded together, each finding its
// row by binary search over the offsets.  Rows of any length mix keep every
// thread equally busy.  All threads must call it.
template <typename F>
__device__ __forceinline__ void walk_members(const int64_t *__restrict__ row_ptr,
                                             const int32_t *__restrict__ col,
                                             const int32_t *__restrict__ agg,
                                             const int32_t *__restrict__ members, int64_t m0,
                                             int64_t m1, WalkLds &w, F f) {
    const int tid = (int)threadIdx.x;
    for (int64_t c0 = m0; c0 < m1; c0 += kBlock) {
        const int64_t i = c0 + tid;
        int64_t rs = 0;
        unsigned long long len = 0;
        if (i < m1) {
            const int32_t v = members[i];
            rs = row_ptr[v];
            len = (unsigned long long)(row_ptr[v + 1] - rs);
        }
        unsigned long long tot;
        const unsigned long long ex = block_excl64(len, w.scan, &tot);
        w.off[tid] = ex;
        w.start[tid] = rs;
        if (tid == 0) w.off[kBlock] = tot;
        __syncthreads();
        for (unsigned long long q0 = tid; q0 < tot; q0 += (unsigned long long)kBlock * kWEdges) {
            int32_t x[kWEdges];
#pragma unroll
            for (int k = 0; k < kWEdges; k++) {
                unsigned long long q = q0 + (unsigned long long)k * kBlock;
                if (q >= tot) q = tot - 1;  // a valid entry; its result is not used
                // the last row r with off[r] <= q (it is not empty: off[r + 1] > q)
                int lo = 0, hi = kBlock;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (w.off[mid] <= q) lo = mid;
                    else hi = mid;
                }
                x[k] = col[w.start[lo] + (int64_t)(q - w.off[lo])];
            }
            int32_t c[kWEdges];
#pragma unroll
            for (int k = 0; k < kWEdges; k++) c[k] = agg[x[k]];
#pragma unroll
            for (int k = 0; k < kWEdges; k++)
                if (q0 + (unsigned long long)k * kBlock < tot) f(c[k]);
        }
        __syncthreads();  // the offsets are rewritten by the next chunk
    }
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
                                                        const uint32_t *__restrict__ big_count,
                                                        uint32_t *__restrict__ gmeta) {
    static_assert(kBitWords >= kQCap, "the sort buffer is the bitmap");
    __shared__ uint32_t buf[kBitWords];
    __shared__ unsigned long long red[kWaves];
    __shared__ uint32_t scan_s[kWaves];
    __shared__ uint32_t fill_s;
    __shared__ WalkLds walk;
    __shared__ int32_t range_s[2 * kWaves];
    __shared__ uint32_t giant_s;
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
        if (gmeta && cand > (unsigned long long)kGiantCand) {
            // a giant row: the count pass claims a bitmap slot for it (the
            // slot kernels then count and write it); without a free slot it
            // stays here
            if (tid == 0) {
                uint32_t taken = 0;
                if (!FILL) {
                    const uint32_t k = atomicAdd(&gmeta[3 * kGiantSlots], 1u);
                    if (k < (uint32_t)kGiantSlots) {
                        gmeta[k] = (uint32_t)a;
                        taken = 1;
                    }
                } else {
                    const uint32_t cnt = min(gmeta[3 * kGiantSlots], (uint32_t)kGiantSlots);
                    for (uint32_t k = 0; k < cnt; k++) taken |= gmeta[k] == (uint32_t)a ? 1u : 0u;
                }
                giant_s = taken;
            }
            __syncthreads();
            if (giant_s) continue;  // uniform; the next block_sum synchronises first
        }
        uint32_t distinct = 0;
        if (cand <= (unsigned long long)kQCap) {
            // gather the candidate ids (self excluded) into LDS
            if (tid == 0) fill_s = 0;
            __syncthreads();
            walk_members(row_ptr, col, agg, members, m0, m1, walk, [&](int32_t c) {
                if (c >= 0 && (int64_t)c != a) buf[atomicAdd(&fill_s, 1u)] = (uint32_t)c;
            });
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
            // bitmap windows over the coarse id space
            uint32_t run = 0;
            // The first window also finds the smallest and largest candidate;
            // later windows cover only that range, and each window emits
            // only the words inside it.  In a disjoint union the candidates
            // lie in the row's own graph, so a big row never sweeps the
            // coarse ids of the other graphs.
            int64_t hi = n_agg;
            int32_t tmin = INT32_MAX, tmax = -1;
            bool first = true;
            for (int64_t lo = 0; lo < hi;) {
                for (int i = tid; i < kBitWords; i += kBlock) buf[i] = 0u;
                __syncthreads();
                walk_members(row_ptr, col, agg, members, m0, m1, walk, [&](int32_t c) {
                    if (c < 0 || (int64_t)c == a) return;
                    if (first) {
                        tmin = min(tmin, c);
                        tmax = max(tmax, c);
                    }
                    const int64_t o = (int64_t)c - lo;
                    if (o >= 0 && o < kQWindow) atomicOr(&buf[o >> 5], 1u << (o & 31));
                });
                __syncthreads();
                if (first) {
                    block_minmax(&tmin, &tmax, range_s);
                    hi = (int64_t)tmax + 1;  // no candidate at all: tmax = -1 ends the sweep
                }
                // emit the set ids of this window in increasing order
                const int64_t e_lo = max(lo, (int64_t)tmin);
                const int64_t e_hi = min(lo + kQWindow, hi);
                if (e_lo < e_hi) {
                    const int w0 = (int)((e_lo - lo) >> 5), w1 = (int)((e_hi - lo + 31) >> 5);
                    for (int c0 = w0; c0 < w1; c0 += kBlock) {
                        const int wi = c0 + tid;
                        const uint32_t word = wi < w1 ? buf[wi] : 0u;
                        uint32_t tot;
                        const uint32_t pos = block_excl((uint32_t)__popc(word), scan_s, &tot);
                        if (FILL) {
                            uint32_t wv = word, k = 0;
                            while (wv) {
                                const int bit = __ffs(wv) - 1;
                                wv &= wv - 1;
                                ccol[crow[a] + run + pos + k] =
                                    (int32_t)(lo + (int64_t)wi * 32 + bit);
                                k++;
                            }
                        }
                        run += tot;
                    }
                }
                __syncthreads();
                int64_t next = lo + kQWindow;
                if (first) {
                    if ((int64_t)tmin > next) next = tmin;
                    first = false;
                }
                lo = next;
            }
            distinct = run;
        }
        if (!FILL && tid == 0) ccnt[a] = distinct;
        __syncthreads();
    }
}

// Giant rows, one bitmap slot each (gmeta: rows [0, S), smallest ids
// [S, 2S), largest ids [2S, 3S), rows claimed [3S]).  Slot blockIdx.y; the
// workgroups of a slot share its members in chunks of kBlock and set the bit
// of every candidate (a plain read first skips bits already set: most
// candidates of a giant row repeat).
__global__ __launch_bounds__(kBlock) void k_giant_set(const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const int32_t *__restrict__ agg,
                                                      const int64_t *__restrict__ moff,
                                                      const int32_t *__restrict__ members,
                                                      uint32_t *__restrict__ gbits, int64_t words,
                                                      uint32_t *__restrict__ gmeta) {
    __shared__ WalkLds walk;
    __shared__ int32_t range_s[2 * kWaves];
    const int slot = (int)blockIdx.y;
    if ((uint32_t)slot >= min(gmeta[3 * kGiantSlots], (uint32_t)kGiantSlots)) return;
    const int64_t a = gmeta[slot];
    const int64_t m0 = moff[a], m1 = moff[a + 1];
    uint32_t *bits = gbits + (int64_t)slot * words;
    int32_t tmin = INT32_MAX, tmax = -1;
    for (int64_t c0 = m0 + (int64_t)blockIdx.x * kBlock; c0 < m1;
         c0 += (int64_t)gridDim.x * kBlock) {
        walk_members(row_ptr, col, agg, members, c0, min(c0 + kBlock, m1), walk, [&](int32_t c) {
            if (c < 0 || (int64_t)c == a) return;
            tmin = min(tmin, c);
            tmax = max(tmax, c);
            const uint32_t bit = 1u << (c & 31);
            if (!(bits[c >> 5] & bit)) atomicOr(&bits[c >> 5], bit);
        });
    }
    block_minmax(&tmin, &tmax, range_s);
    if (threadIdx.x == 0 && tmax >= 0) {
        atomicMin((int32_t *)&gmeta[kGiantSlots + slot], tmin);
        atomicMax((int32_t *)&gmeta[2 * kGiantSlots + slot], tmax);
    }
}

// One workgroup per giant slot: FILL = false: ccnt[a] = the bits set;
// FILL = true: their ids in increasing order to ccol[crow[a] ...].
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_giant_emit(const uint32_t *__restrict__ gbits,
                                                       int64_t words,
                                                       const uint32_t *__restrict__ gmeta,
                                                       uint32_t *__restrict__ ccnt,
                                                       const int64_t *__restrict__ crow,
                                                       int32_t *__restrict__ ccol) {
    __shared__ uint32_t scan_s[kWaves];
    const int slot = (int)blockIdx.x;
    if ((uint32_t)slot >= min(gmeta[3 * kGiantSlots], (uint32_t)kGiantSlots)) return;
    const int64_t a = gmeta[slot];
    const int32_t lo = (int32_t)gmeta[kGiantSlots + slot];
    const int32_t hi = (int32_t)gmeta[2 * kGiantSlots + slot];
    const uint32_t *bits = gbits + (int64_t)slot * words;
    uint32_t run = 0;
    if (hi >= 0) {
        const int64_t w0 = lo >> 5, w1 = ((int64_t)hi >> 5) + 1;
        for (int64_t c0 = w0; c0 < w1; c0 += kBlock) {
            const int64_t wi = c0 + (int64_t)threadIdx.x;
            const uint32_t word = wi < w1 ? bits[wi] : 0u;
            uint32_t tot;
            const uint32_t pos = block_excl((uint32_t)__popc(word), scan_s, &tot);
            if (FILL) {
                uint32_t wv = word, k = 0;
                while (wv) {
                    const int bit = __ffs(wv) - 1;
                    wv &= wv - 1;
                    ccol[crow[a] + run + pos + k] = (int32_t)(wi * 32 + bit);
                    k++;
                }
            }
            run += tot;
        }
    }
    if (!FILL && threadIdx.x == 0) ccnt[a] = run;
}

// gmeta before a count pass: no rows, empty ranges.
__global__ void k_giant_init(uint32_t *__restrict__ gmeta) {
    const int i = (int)threadIdx.x;
    if (i < kGiantMeta)
        gmeta[i] = (i >= kGiantSlots && i < 2 * kGiantSlots) ? (uint32_t)INT32_MAX
                   : (i >= 2 * kGiantSlots && i < 3 * kGiantSlots) ? 0xFFFFFFFFu
                   : 0u;
}

int grid_for(int64_t work, int per_block, int cap) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace

hipError_t quotient_graph(const int64_t *row_ptr, const int32_t *col, int64_t n, int64_t nnz,
                          const int32_t *agg, int64_t n_agg, int64_t *crow, int32_t *ccol,
                          const QuotientWs &q, hipStream_t s) {
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
    // no coarse row has more candidates than the fine graph has entries
    const bool giant = nnz > kGiantCand && n_agg > 0;
    const int64_t words = (int64_t)giant_words(n_agg);
    uint32_t *gmeta = giant ? q.gmeta : nullptr;
    if ((e = launch_fill_u32(q.big_count, 0u, 1, s)) != hipSuccess) return e;
    if (giant) {
        hipLaunchKernelGGL(k_giant_init, dim3(1), dim3(64), 0, s, q.gmeta);
        if ((e = launch_fill_u32(q.gbits, 0u, kGiantSlots * words, s)) != hipSuccess) return e;
    }
    // two wavefront passes (rows of up to kWSmall candidates first) when
    // rows are small on average and many; else one
    const bool two = n_agg >= 16384 && nnz <= (int64_t)kWSmall * 2 * n_agg;
    if (n_agg > 0) {
        if (two) {
            hipLaunchKernelGGL((k_coarse_rows_wave<false, kWSmall, kRowsMark>), dim3(wblocks),
                               dim3(kBlock), 0, s, row_ptr, col, agg, n_agg, q.moff, q.members,
                               q.cnt, (const int64_t *)nullptr, (int32_t *)nullptr, q.cls, q.big,
                               q.big_count);
            hipLaunchKernelGGL((k_coarse_rows_wave<false, kWCap, kRowsMarked>), dim3(wblocks),
                               dim3(kBlock), 0, s, row_ptr, col, agg, n_agg, q.moff, q.members,
                               q.cnt, (const int64_t *)nullptr, (int32_t *)nullptr, q.cls, q.big,
                               q.big_count);
        } else {
            hipLaunchKernelGGL((k_coarse_rows_wave<false, kWCap, kRowsList>), dim3(wblocks),
                               dim3(kBlock), 0, s, row_ptr, col, agg, n_agg, q.moff, q.members,
                               q.cnt, (const int64_t *)nullptr, (int32_t *)nullptr, q.cls, q.big,
                               q.big_count);
        }
        hipLaunchKernelGGL(k_coarse_rows<false>, dim3(bblocks), dim3(kBlock), 0, s, row_ptr, col,
                           agg, n_agg, q.moff, q.members, q.cnt, (const int64_t *)nullptr,
                           (int32_t *)nullptr, (const int32_t *)q.big,
                           (const uint32_t *)q.big_count, gmeta);
    }
    if (giant) {
        hipLaunchKernelGGL(k_giant_set, dim3(256, kGiantSlots), dim3(kBlock), 0, s, row_ptr, col,
                           agg, q.moff, q.members, q.gbits, words, q.gmeta);
        hipLaunchKernelGGL(k_giant_emit<false>, dim3(kGiantSlots), dim3(kBlock), 0, s,
                           (const uint32_t *)q.gbits, words, (const uint32_t *)q.gmeta, q.cnt,
                           (const int64_t *)nullptr, (int32_t *)nullptr);
    }
    if ((e = exclusive_scan_u32_i64(q.cnt, n_agg, crow, q.part, s)) != hipSuccess) return e;
    if (n_agg > 0) {
        if (two) {
            hipLaunchKernelGGL((k_coarse_rows_wave<true, kWSmall, kRowsMark>), dim3(wblocks),
                               dim3(kBlock), 0, s, row_ptr, col, agg, n_agg, q.moff, q.members,
                               q.cnt, crow, ccol, q.cls, q.big, q.big_count);
            hipLaunchKernelGGL((k_coarse_rows_wave<true, kWCap, kRowsMarked>), dim3(wblocks),
                               dim3(kBlock), 0, s, row_ptr, col, agg, n_agg, q.moff, q.members,
                               q.cnt, crow, ccol, q.cls, q.big, q.big_count);
        } else {
            hipLaunchKernelGGL((k_coarse_rows_wave<true, kWCap, kRowsList>), dim3(wblocks),
                               dim3(kBlock), 0, s, row_ptr, col, agg, n_agg, q.moff, q.members,
                               q.cnt, crow, ccol, q.cls, q.big, q.big_count);
        }
        hipLaunchKernelGGL(k_coarse_rows<true>, dim3(bblocks), dim3(kBlock), 0, s, row_ptr, col,
                           agg, n_agg, q.moff, q.members, q.cnt, crow, ccol,
                           (const int32_t *)q.big, (const uint32_t *)q.big_count, gmeta);
    }
    if (giant)
        hipLaunchKernelGGL(k_giant_emit<true>, dim3(kGiantSlots), dim3(kBlock), 0, s,
                           (const uint32_t *)q.gbits, words, (const uint32_t *)q.gmeta, q.cnt, crow,
                           ccol);
    return hipGetLastError();
}

}  // namespace mis2
