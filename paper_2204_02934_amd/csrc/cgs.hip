// cgs.hip -- cluster multicolor Gauss-Seidel (Algorithm 4, Section III-C) on gfx950.
//
// Setup colours a graph (the coarse graph of an aggregation, or the graph
// itself for point multicolor Gauss-Seidel) and orders the rows by colour,
// then by cluster, then by row id.  Apply runs, for each colour in turn, one
// wavefront per cluster: the wave updates its cluster's rows one after the
// other.  Clusters of one colour share no edge, so no wave reads a value
// another wave of the same launch writes, and the result is that of the
// sequential sweep in the same order.
//
// Colouring (the paper takes it from other work): Jones-Plassmann with fixed
// priorities, the packed tuple of h(seed, 0, v) (Sections V-A, V-C).  Each
// round every uncoloured vertex whose tuple is below those of its uncoloured
// neighbours takes the smallest colour no coloured neighbour has.  Two
// vertices picked in one round are never adjacent (each would be below the
// other), so a round reads only colours fixed in earlier rounds.
#include "internal.h"
#include "lanes.h"

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

// Each cluster of 2 .. kSmallCluster members: one wavefront, one member per
// lane; a member's place is the number of smaller ones (ids are distinct),
// counted across the lanes.  Every lane has its member in a register before
// any is written back.
__global__ __launch_bounds__(kBlock) void k_sort_small(int64_t nc, const int64_t *__restrict__ moff,
                                                       int32_t *__restrict__ members) {
    const int lane = threadIdx.x & 63;
    const int64_t a = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (a >= nc) return;
    const int64_t s = moff[a], m = moff[a + 1] - s;
    if (m < 2 || m > kSmallCluster) return;
    const int32_t x = lane < m ? members[s + lane] : 0x7fffffff;
    int rank = 0;
    for (int w = 0; w < (int)m; w++) rank += __builtin_amdgcn_readlane(x, w) < x;
    if (lane < m) members[s + rank] = x;
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
__global__ __launch_bounds__(kBlock) void k_scatter_pos(int64_t n, const int32_t *__restrict__ rows,
                                                        int32_t *__restrict__ pos) {
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock)
        pos[rows[t]] = (int32_t)t;
}

// ---- apply ----------------------------------------------------------------
//
// One wavefront per cluster.  The cluster's rows are taken in batches of at
// most 64 rows of at most 64 entries each and Cap entries in all; lane k
// holds the batch's k-th row.  The batch is staged in LDS in parallel: for
// each entry (row order, then CSR order) either the product a_ij * x_j with
// index kOne (x_j is final for this pass when j is not a row of the batch:
// another colour's x, a row of this cluster updated in an earlier batch, or
// one not yet reached, whose old value Gauss-Seidel uses), or a_ij with the
// batch index of j.  xb holds the batch's x, current as rows finish, and
// xb[kOne] = 1 (an exact product).  The chain then runs the rows in order:
// lane q forms the row's q-th term v * xb[index], and the terms are
// subtracted from b_i one by one in CSR order, read across lanes; a row of
// at most 8, 16, 32 (else 64) entries subtracts that many terms, the
// missing ones +0.0, which leaves every value unchanged, so every rounding
// is the sequential sweep's.  A row's LDS reads are issued while the row before it
// runs (its indices and values two rows ahead); the one x they cannot see,
// the previous row's, is taken from the chain directly.  A row longer than
// 64 entries is a batch of its own, read from global memory in pieces of 64
// (no row of its batch but itself, and it has no self-loop).
constexpr int kCgsWaves = kBlock / 64;
constexpr int kOne = 64;
// 256 entries per batch and 8 waves per SIMD (the most a SIMD holds): on the
// 27-point and 7-point 100^3 plans, 384, 512, 768 and 1024 entries at the
// occupancy their LDS allows (7, 6, 4, 3 waves) all sweep slower
constexpr int kCgsLaunchCap = 256;
constexpr int kCgsLaunchWaves = 8;

template <int Cap>
struct CgsStage {
    double v[Cap + 64];  // 64 spare entries: reads past a batch's end stay inside
    uint8_t tag[Cap + 64];
    double xb[65];
    int64_t rs[64];
    int32_t off[65];
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double lane_bcast(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int64_t lane_bcast64(int64_t v, int l) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// acc minus the terms of lanes 0 .. W-1, in lane order; the lanes' values
// are read eight at a time ahead of their eight subtractions
template <int W>
__device__ __forceinline__ double chain_w(double acc, double term) {
#pragma clang fp contract(off)
#pragma unroll
    for (int g = 0; g < W; g += 8) {
        double t[8];
#pragma unroll
        for (int z = 0; z < 8; z++) t[z] = lane_bcast(term, g + z);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int z = 0; z < 8; z++) acc = acc - t[z];
        __builtin_amdgcn_sched_barrier(0);
    }
    return acc;
}

// Cap: LDS entries per batch; MinW: waves per SIMD that the LDS of a wave
// (about 9 bytes per entry) still allows
template <int Cap, int MinW>
__global__ __launch_bounds__(kBlock, MinW) void k_cgs_cluster(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ diag,
                                                        const double *__restrict__ b, double *x,
                                                        const int32_t *__restrict__ rows,
                                                        const int32_t *__restrict__ pos,
                                                        const int64_t *__restrict__ cluster_off,
                                                        int64_t k0, int64_t k1, int backward) {
#pragma clang fp contract(off)
    constexpr int kCgsCap = Cap, kCgsU = Cap / 64;
    __shared__ CgsStage<Cap> stage[kCgsWaves];
    const int lane = threadIdx.x & 63;
    CgsStage<Cap> &S = stage[threadIdx.x >> 6];
    const int64_t k = k0 + (int64_t)blockIdx.x * kCgsWaves + (threadIdx.x >> 6);
    if (k >= k1) return;
    const int64_t r0 = cluster_off[k], r1 = cluster_off[k + 1], m = r1 - r0;
    if (lane == 0) S.xb[kOne] = 1.0;
    S.v[kCgsCap + lane] = 0.0;
    S.tag[kCgsCap + lane] = kOne;
    for (int64_t u = 0; u < m;) {
        // the next (up to) 64 rows in visiting order, one per lane
        const int64_t cand = u + lane;
        const bool valid = cand < m;
        const int64_t t = backward ? r1 - 1 - cand : r0 + cand;
        const int32_t i = valid ? rows[t] : 0;
        const int64_t rs = valid ? row_ptr[i] : 0;
        const int64_t len = valid ? row_ptr[i + 1] - rs : 0;
        const double bi = valid ? b[i] : 0.0;
        const double di = valid ? diag[i] : 1.0;
        const double xo = valid ? x[i] : 0.0;
        // prefix of the lengths, each clamped to kCgsCap + 1: only prefixes up
        // to kCgsCap are used, and those are exact
        const int64_t incl =
            (int64_t)wave_incl_scan((uint32_t)(len < kCgsCap + 1 ? len : kCgsCap + 1));
        // rows before the first one longer than 64, within Cap entries
        const uint64_t longm = __ballot(valid && len > 64);
        const int first_long = longm ? __ffsll((unsigned long long)longm) - 1 : 64;
        int nb = __popcll(__ballot(valid && incl <= kCgsCap));
        nb = nb < first_long ? nb : first_long;
        if (nb == 0) {
            // lane 0's row alone, longer than 64 entries
            const int32_t i0 = __builtin_amdgcn_readfirstlane(i);
            const int64_t s0 = lane_bcast64(rs, 0), l0 = lane_bcast64(len, 0);
            double acc = lane_bcast(bi, 0);
            for (int64_t pc = 0; pc < l0; pc += 64) {
                const int64_t q = pc + lane;
                double term = 0.0;
                if (q < l0) {
                    const int64_t pe = s0 + q;
                    term = val[pe] * x[col[pe]];
                }
                acc = chain_w<64>(acc, term);
            }
            const double xn = acc / lane_bcast(di, 0);
            if (lane == 0) x[i0] = xn;
            wave_sync();
            u += 1;
            continue;
        }
        const int tot = (int)lane_bcast64(incl, nb - 1);
        // sweep positions of the batch: [lo, lo + nb)
        const int64_t lo = backward ? r1 - u - nb : r0 + u;
        if (lane < nb) {
            S.off[lane + 1] = (int32_t)incl;
            S.rs[lane] = rs;
            S.xb[lane] = xo;
        }
        if (lane == 0) S.off[0] = 0;
        wave_sync();
        // stage the batch's entries, all of a lane's loads in flight at once
        // (slots past tot re-read entry 0 and store nothing).  A batch with no
        // entries (rows without off-diagonal entries) loads nothing: its rows'
        // CSR starts may equal nnz, one past the last entry
        if (tot > 0) {
            int64_t pp[kCgsU];
#pragma unroll
            for (int c = 0; c < kCgsU; c++) {
                const int q = lane + 64 * c < tot ? lane + 64 * c : 0;
                int kr = 0;
                for (int st = 32; st > 0; st >>= 1)
                    if (kr + st < nb && S.off[kr + st] <= q) kr += st;
                pp[c] = S.rs[kr] + (q - S.off[kr]);
            }
            int32_t jj[kCgsU];
            double aa[kCgsU];
#pragma unroll
            for (int c = 0; c < kCgsU; c++) {
                jj[c] = col[pp[c]];
                aa[c] = val[pp[c]];
            }
#pragma unroll
            for (int c = 0; c < kCgsU; c++) {
                const int q = lane + 64 * c;
                const int64_t pj = pos[jj[c]];
                const double xj = x[jj[c]];
                const bool inb = pj >= lo && pj < lo + nb;
                if (q < tot) {
                    S.tag[q] = inb ? (uint8_t)(backward ? lo + nb - 1 - pj : pj - lo) : kOne;
                    S.v[q] = inb ? aa[c] : aa[c] * xj;
                }
            }
        }
        wave_sync();
        // the chain.  Row r's entries are [incl(r) - len(r), incl(r)); lane q
        // reads entry q of a row (past its end: a spare zero entry, or the
        // next row's, both masked out of the term)
        auto start = [&](int r) { return r == 0 ? 0 : (int)lane_bcast64(incl, r - 1); };
        const int s1 = start(1 < nb ? 1 : nb - 1);
        // (an index read past a row's end may be stale: clamp it into xb)
        double v0 = S.v[lane], v1 = S.v[s1 + lane];
        int g0 = min((int)S.tag[lane], kOne), g1 = min((int)S.tag[s1 + lane], kOne);
        double x0 = S.xb[g0];
        double xs = 0.0;  // x of the previous row
        for (int kk = 0; kk < nb; kk++) {
            const int ln = (int)lane_bcast64(incl, kk) - start(kk);
            // row kk's term; xb[kk - 1] was not yet written when x0 was read
            const double xf = g0 == kk - 1 ? xs : x0;
            const double term = lane < ln ? v0 * xf : 0.0;
            // reads for rows kk + 1 (x) and kk + 2 (values, indices)
            const double x1 = S.xb[g1];
            const int s2 = start(kk + 2 < nb ? kk + 2 : nb - 1);
            const double v2 = S.v[s2 + lane];
            const int g2 = min((int)S.tag[s2 + lane], kOne);
            double acc = lane_bcast(bi, kk);
            acc = ln <= 8    ? chain_w<8>(acc, term)
                  : ln <= 16 ? chain_w<16>(acc, term)
                  : ln <= 32 ? chain_w<32>(acc, term)
                             : chain_w<64>(acc, term);
            const double xn = acc / lane_bcast(di, kk);
            if (lane == 0) S.xb[kk] = xn;
            if (lane == kk) x[i] = xn;
            xs = xn;
            v0 = v1;
            g0 = g1;
            x0 = x1;
            v1 = v2;
            g1 = g2;
        }
        wave_sync();
        u += nb;
    }
}

// Point form (every cluster one row): the rows of one colour share no edge,
// so each reads only x of other colours and their order does not matter.
// One lane per row, R consecutive sweep positions per wavefront (fewer rows
// per wave give a small colour more waves): the wave stages the products
// a_ij * x_j of its rows' entries in LDS, kPtCap at a time, and each lane
// subtracts its own row's products in CSR order.
constexpr int kPtCap = 1024;

struct PointStage {
    double v[kPtCap];
    int64_t off[65];  // entry offsets of the wave's rows (off[64] = total)
    int64_t rs[64];
};

template <int R>
__global__ __launch_bounds__(kBlock) void k_cgs_point(const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ diag,
                                                      const double *__restrict__ b, double *x,
                                                      const int32_t *__restrict__ rows,
                                                      int64_t t0, int64_t t1) {
#pragma clang fp contract(off)
    __shared__ PointStage stage[kCgsWaves];
    const int lane = threadIdx.x & 63;
    PointStage &S = stage[threadIdx.x >> 6];
    const int64_t base = t0 + ((int64_t)blockIdx.x * kCgsWaves + (threadIdx.x >> 6)) * R;
    if (base >= t1) return;
    const int64_t t = base + lane;
    const bool valid = lane < R && t < t1;
    const int32_t i = valid ? rows[t] : 0;
    const int64_t rs = valid ? row_ptr[i] : 0;
    const int64_t len = valid ? row_ptr[i + 1] - rs : 0;
    double acc = valid ? b[i] : 0.0;
    int64_t incl = len;
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    const int64_t excl = incl - len;
    S.off[lane + 1] = incl;
    S.rs[lane] = rs;
    if (lane == 0) S.off[0] = 0;
    const int64_t tot = lane_bcast64(incl, 63);
    wave_sync();
    for (int64_t E = 0; E < tot; E += kPtCap) {
        const int64_t cnt = tot - E < kPtCap ? tot - E : kPtCap;
        constexpr int U = kPtCap / 64;
        int64_t pp[U];
#pragma unroll
        for (int c = 0; c < U; c++) {
            const int64_t e = E + (lane + 64 * c < cnt ? lane + 64 * c : 0);
            int kr = 0;
            for (int st = 32; st > 0; st >>= 1)
                if (S.off[kr + st] <= e) kr += st;
            pp[c] = S.rs[kr] + (e - S.off[kr]);
        }
        int32_t jj[U];
        double aa[U];
#pragma unroll
        for (int c = 0; c < U; c++) {
            jj[c] = col[pp[c]];
            aa[c] = val[pp[c]];
        }
#pragma unroll
        for (int c = 0; c < U; c++) {
            const double pr = aa[c] * x[jj[c]];
            if (lane + 64 * c < cnt) S.v[lane + 64 * c] = pr;
        }
        wave_sync();
        const int64_t lo = (excl > E ? excl : E) - E;
        const int64_t hi = (incl < E + cnt ? incl : E + cnt) - E;
        int64_t e = lo;
        for (; e + 4 <= hi; e += 4) {
            const double p0 = S.v[e], p1 = S.v[e + 1], p2 = S.v[e + 2], p3 = S.v[e + 3];
            acc = acc - p0;
            acc = acc - p1;
            acc = acc - p2;
            acc = acc - p3;
        }
        for (; e < hi; e++) acc = acc - S.v[e];
        wave_sync();
    }
    if (valid) x[i] = acc / diag[i];
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
    if (n <= 0 || nc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_members, dim3(grid_of(n, 8192)), dim3(kBlock), 0, s, n, cluster,
                       moff, cursor, members);
    const int64_t sblocks = (nc + kBlock / 64 - 1) / (kBlock / 64);
    if (sblocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sort_small, dim3((unsigned)sblocks), dim3(kBlock), 0, s, nc, moff,
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

hipError_t launch_scatter_pos(int64_t n, const int32_t *rows, int32_t *pos, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_pos, dim3(grid_of(n, 8192)), dim3(kBlock), 0, s, n, rows, pos);
    return hipGetLastError();
}

hipError_t launch_cgs_sweep(const int64_t *row_ptr, const int32_t *col, const double *val,
                            const double *diag, const double *b, double *x, const int32_t *rows,
                            const int32_t *pos, const int64_t *cluster_off, int64_t k0, int64_t k1,
                            bool backward, hipStream_t s) {
    if (k1 <= k0) return hipSuccess;
    const int64_t blocks = (k1 - k0 + kCgsWaves - 1) / kCgsWaves;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_cgs_cluster<kCgsLaunchCap, kCgsLaunchWaves>), dim3((unsigned)blocks),
                       dim3(kBlock), 0, s, row_ptr, col, val, diag, b, x, rows, pos, cluster_off,
                       k0, k1, backward ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_cgs_point(const int64_t *row_ptr, const int32_t *col, const double *val,
                            const double *diag, const double *b, double *x, const int32_t *rows,
                            int64_t t0, int64_t t1, hipStream_t s) {
    if (t1 <= t0) return hipSuccess;
    // rows per wave: the most that still leaves 4 waves per SIMD (1024 SIMDs)
    const int64_t nr = t1 - t0;
    const int R = nr >= 64 * 4096 ? 64 : nr >= 32 * 4096 ? 32 : 16;
    const int64_t per = (int64_t)R * kCgsWaves;
    const int64_t blocks = (nr + per - 1) / per;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (R == 64)
        hipLaunchKernelGGL(k_cgs_point<64>, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr,
                           col, val, diag, b, x, rows, t0, t1);
    else if (R == 32)
        hipLaunchKernelGGL(k_cgs_point<32>, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr,
                           col, val, diag, b, x, rows, t0, t1);
    else
        hipLaunchKernelGGL(k_cgs_point<16>, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr,
                           col, val, diag, b, x, rows, t0, t1);
    return hipGetLastError();
}

}  // namespace mis2
