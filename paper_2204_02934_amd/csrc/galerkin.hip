// galerkin.hip -- Galerkin coarse operator of an aggregation on gfx950, the
// multigrid hookup of the aggregates (Section VI-E sets up smoothed-aggregation
// multigrid on them).
//
// With the tentative prolongator for the constant near-null space,
// P[i][a] = 1/sqrt(n_a) when row i is in aggregate a (n_a members), the coarse
// operator is A_c = P^T A P:
//     (A_c)[a][b] = (sum of A[i][j] over i in a, j in b) / sqrt(n_a * n_b).
// Its off-diagonal part lives on the quotient graph (rows by aggregate,
// ascending columns, no self); its diagonal takes the fine diagonal and every
// coupling inside an aggregate.  Every sum runs over the fine rows in
// increasing id -- within a row, its diagonal first, then its entries in CSR
// order -- from 0.0, and is divided once by sqrt(n_a * n_b) (the product is
// exact), so the result is one fixed sequence of roundings.
//
// One wavefront per coarse row a.  Its members (counting-sorted by id) are
// walked in order, 64 at a time; their items (a member's diagonal, then its
// entries), in that order, are taken 64 at a time, one per lane.  Each lane
// finds the coarse column of its item (binary search in the coarse row; the
// member holding the item by binary search over the batch's item offsets),
// and the chunk is folded into the row's
// accumulators in item order: the chunk is sorted by (column, lane) with a
// 64-lane bitonic network, and the first lane of each column's run adds the
// run's items one after the other.  Accumulators (and
// the coarse row's columns) live in LDS for rows of at most kGCap columns,
// else in the output arrays themselves.  A final pass does the division.
#include "internal.h"
#include "lanes.h"

namespace mis2 {

namespace {

// coarse columns of a row held in LDS: 17 KB per 4-wave block, so registers
// (69 VGPRs, 7 waves per SIMD) rather than LDS set the occupancy; 511 columns
// (30 KB, 5 waves) took 9% longer on the 27-point 100^3 aggregation, whose
// coarse rows have at most 29 columns
constexpr int kGCap = 255;
constexpr int kGWaves = kBlock / 64;

struct GStage {
    double acc[kGCap + 1];  // [0, d): the row's columns, [d]: its diagonal
    int32_t cols[kGCap];
    int64_t off[65];        // item offsets of a batch of 64 members
    int64_t rs[64];         // their CSR starts
    int32_t mi[64];         // their ids
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t lane_bcast64(int64_t v, int l) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// flag[0] |= 1 when an aggregate id is outside [0, n_agg); flag[0] |= 2 when a
// coarse column is.
__global__ __launch_bounds__(kBlock) void k_check_ids(int64_t n, const int32_t *__restrict__ agg,
                                                      int64_t cnnz,
                                                      const int32_t *__restrict__ ccol,
                                                      int64_t n_agg, uint32_t *flag) {
    uint32_t bad = 0;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n || v < cnnz;
         v += (int64_t)gridDim.x * kBlock) {
        if (v < n && (agg[v] < 0 || agg[v] >= n_agg)) bad |= 1u;
        if (v < cnnz && (ccol[v] < 0 || ccol[v] >= n_agg)) bad |= 2u;
    }
    if (bad) atomicOr(flag, bad);
}

// The slot of coarse column b in the ascending cs[0 .. d) (top: the largest
// power of two <= d); -1, and *missing = 4, when b is not there.
__device__ __forceinline__ int coarse_slot(const int32_t *cs, int d, int top, int32_t b,
                                           uint32_t *missing) {
    int lo = 0;  // entries of cs below b
    for (int st = top; st > 0; st >>= 1)
        if (lo + st <= d && cs[lo + st - 1] < b) lo += st;
    if (lo < d && cs[lo] == b) return lo;
    *missing = 4u;
    return -1;
}

template <int K, int J>
__device__ __forceinline__ uint32_t bitonic_step(uint32_t key, int lane) {
    const uint32_t other = lane_xor<J>(key);
    const bool keep_min = ((lane & J) == 0) == ((lane & K) == 0);
    return keep_min ? (key < other ? key : other) : (key > other ? key : other);
}

template <int K, int J>
__device__ __forceinline__ uint32_t bitonic_merge(uint32_t key, int lane) {
    key = bitonic_step<K, J>(key, lane);
    if constexpr (J > 1) key = bitonic_merge<K, J / 2>(key, lane);
    return key;
}

// The 32-bit form of fold_chunk below, with register cross-lane moves.
__device__ __forceinline__ void fold_chunk32(int p, double v, int d, double *acc, double *accd,
                                             int lane) {
#pragma clang fp contract(off)
    uint32_t key = p >= 0 ? ((uint32_t)p << 6) | (uint32_t)lane : ~0u;
    key = bitonic_merge<2, 1>(key, lane);
    key = bitonic_merge<4, 2>(key, lane);
    key = bitonic_merge<8, 4>(key, lane);
    key = bitonic_merge<16, 8>(key, lane);
    key = bitonic_merge<32, 16>(key, lane);
    key = bitonic_merge<64, 32>(key, lane);
    const bool valid = key != ~0u;
    const int sp = valid ? (int)(key >> 6) : -1;
    const double sv = __shfl(v, (int)(key & 63), 64);
    const int prev = (int)from_prev((uint32_t)sp);
    const bool head = valid && (lane == 0 || prev != sp);
    const uint64_t heads = __ballot(head) | __ballot(!valid);
    const uint64_t after = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
    const int run = head ? (after ? __ffsll((unsigned long long)after) - 1 : 64) - lane : 0;
    const int longest = (int)__builtin_amdgcn_readfirstlane(group_max<64>((uint32_t)run));
    double my = head ? (sp == d ? *accd : acc[sp]) : 0.0;
    uint32_t lo = __double2loint(sv), hi = __double2hiint(sv);  // lane l: item l + j
    for (int j = 0; j < longest; j++) {
        const double sum = my + __hiloint2double((int)hi, (int)lo);
        my = j < run ? sum : my;
        lo = from_next(lo);
        hi = from_next(hi);
    }
    if (head) {
        if (sp == d) *accd = my;
        else acc[sp] = my;
    }
}

// Folds a chunk (lane q: slot p, -1 for none, d for the diagonal; value v) into
// the accumulators in lane order.  The chunk is sorted by (slot, lane) with a
// 64-lane bitonic network, so each slot's items form one run of lanes, still
// in lane order, and the run's first lane adds them one after the other.
// Key = slot * 64 + lane in a K-bit word (32 bits while d < 2^25).
template <typename K>
__device__ __forceinline__ void fold_chunk(int p, double v, int d, double *acc, double *accd,
                                           int lane) {
#pragma clang fp contract(off)
    const K none = ~(K)0;
    K key = p >= 0 ? ((K)(uint32_t)p << 6) | (K)(uint32_t)lane : none;
    for (int k = 2; k <= 64; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            const K other = __shfl_xor(key, j, 64);
            const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
            key = keep_min ? (key < other ? key : other) : (key > other ? key : other);
        }
    const bool valid = key != none;
    const int sp = valid ? (int)(key >> 6) : -1;
    const double sv = __shfl(v, (int)(key & 63), 64);
    const int prev = __shfl_up(sp, 1, 64);
    const bool head = valid && (lane == 0 || prev != sp);
    // the run of the head at lane r ends at the next head (or the first
    // invalid lane)
    const uint64_t heads = __ballot(head) | __ballot(!valid);
    const uint64_t after = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
    const int run = head ? (after ? __ffsll((unsigned long long)after) - 1 : 64) - lane : 0;
    int longest = run;
    for (int o = 32; o > 0; o >>= 1) longest = max(longest, __shfl_xor(longest, o, 64));
    double my = head ? (sp == d ? *accd : acc[sp]) : 0.0;
    for (int j = 0; j < longest; j++) {
        const double vj = __shfl(sv, lane + j < 64 ? lane + j : 63, 64);
        const double sum = my + vj;
        my = j < run ? sum : my;
    }
    if (head) {
        if (sp == d) *accd = my;
        else acc[sp] = my;
    }
}

// flag[0] |= 4 when an entry's aggregate pair is missing from the coarse row.
__global__ __launch_bounds__(kBlock) void k_galerkin(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ diag,
    const int32_t *__restrict__ agg, int64_t n_agg, const int64_t *__restrict__ moff,
    const int32_t *__restrict__ members, const int64_t *__restrict__ crow,
    const int32_t *__restrict__ ccol, double *cval, double *cdiag, uint32_t *flag, int64_t nnz) {
#pragma clang fp contract(off)
    __shared__ GStage stage[kGWaves];
    const int lane = threadIdx.x & 63;
    GStage &S = stage[threadIdx.x >> 6];
    const int64_t a = (int64_t)blockIdx.x * kGWaves + (threadIdx.x >> 6);
    if (a >= n_agg) return;
    const int64_t c0 = crow[a], c1 = crow[a + 1];
    const int d = (int)(c1 - c0);
    const int64_t m0 = moff[a], m1 = moff[a + 1];
    const bool small = d <= kGCap;
    double *acc = small ? S.acc : cval + c0;
    double *accd = small ? &S.acc[d] : cdiag + a;
    const int32_t *cs = small ? S.cols : ccol + c0;
    for (int p = lane; p < d; p += 64) {
        if (small) S.cols[p] = ccol[c0 + p];
        acc[p] = 0.0;
    }
    if (lane == 0) *accd = 0.0;
    const int top = d > 0 ? 1 << (31 - __builtin_clz((unsigned)d)) : 0;
    const bool narrow = d < (1 << 25);  // slot * 64 + lane fits 31 bits
    wave_sync();
    uint32_t missing = 0;
    // members 64 at a time (lane j: member k0 + j); their items, in member
    // order, 64 at a time (lane q: item t0 + q of the batch)
    for (int64_t k0 = m0; k0 < m1; k0 += 64) {
        const bool mv = k0 + lane < m1;
        const int32_t mi = mv ? members[k0 + lane] : 0;
        const int64_t rs = mv ? row_ptr[mi] : 0;
        const int64_t cnt_i = mv ? 1 + (row_ptr[mi + 1] - rs) : 0;
        int64_t incl = cnt_i;
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int64_t o = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += o;
        }
        S.off[lane + 1] = incl;
        S.rs[lane] = rs;
        S.mi[lane] = mi;
        if (lane == 0) S.off[0] = 0;
        const int64_t total = lane_bcast64(incl, 63);
        wave_sync();
        // two chunks per step, A = items t0 .. t0+63 and B = the next 64: their
        // loads are issued together from clamped valid addresses, then A is
        // folded and B after it
        for (int64_t t0 = 0; t0 < total; t0 += 128) {
            const int64_t ta = t0 + lane, tb = t0 + 64 + lane;
            const bool ina = ta < total, inb = tb < total;
            const int64_t tac = ina ? ta : 0, tbc = inb ? tb : 0;
            int kra = 0, krb = 0;  // the members holding the items
            for (int st = 32; st > 0; st >>= 1) {
                if (S.off[kra + st] <= tac) kra += st;
                if (S.off[krb + st] <= tbc) krb += st;
            }
            const int64_t oa = tac - S.off[kra], ob = tbc - S.off[krb];
            const bool da = oa == 0, db = ob == 0;  // the member's diagonal
            const double dga = diag[S.mi[kra]], dgb = diag[S.mi[krb]];
            int pa = ina ? d : -1, pb = inb ? d : -1;  // -1: no item; d: the diagonal
            double va = dga, vb = dgb;
            if (nnz > 0) {
                const int64_t ea = ina && !da ? S.rs[kra] + oa - 1 : 0;
                const int64_t eb = inb && !db ? S.rs[krb] + ob - 1 : 0;
                const int32_t ca = col[ea], cb = col[eb];
                const double xa = val[ea], xb = val[eb];
                const int32_t ba = agg[ca], bb = agg[cb];
                if (ina && !da) {
                    va = xa;
                    if (ba != (int32_t)a) pa = coarse_slot(cs, d, top, ba, &missing);
                }
                if (inb && !db) {
                    vb = xb;
                    if (bb != (int32_t)a) pb = coarse_slot(cs, d, top, bb, &missing);
                }
            }
            if (narrow) fold_chunk32(pa, va, d, acc, accd, lane);
            else fold_chunk<uint64_t>(pa, va, d, acc, accd, lane);
            wave_sync();
            if (t0 + 64 < total) {
                if (narrow) fold_chunk32(pb, vb, d, acc, accd, lane);
                else fold_chunk<uint64_t>(pb, vb, d, acc, accd, lane);
                wave_sync();
            }
        }
    }
    // the division by sqrt(n_a * n_b)
    const double na = (double)(m1 - m0);
    for (int p = lane; p < d; p += 64) {
        const int32_t b = cs[p];
        const double nb = (double)(moff[b + 1] - moff[b]);
        cval[c0 + p] = acc[p] / sqrt(na * nb);
    }
    if (lane == 0) cdiag[a] = m1 > m0 ? *accd / sqrt(na * na) : *accd;
    if (missing) atomicOr(flag, missing);
}

int grid_for(int64_t work, int cap) {
    const int64_t g = (work + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

hipError_t launch_check_ids(int64_t n, const int32_t *agg, int64_t cnnz, const int32_t *ccol,
                            int64_t n_agg, uint32_t *flag, hipStream_t s) {
    if (n <= 0 && cnnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_ids, dim3(grid_for(std::max(n, cnnz), 4096)), dim3(kBlock), 0, s,
                       n, agg, cnnz, ccol, n_agg, flag);
    return hipGetLastError();
}

hipError_t launch_galerkin(const int64_t *row_ptr, const int32_t *col, const double *val,
                           const double *diag, const int32_t *agg, int64_t n_agg,
                           const int64_t *moff, const int32_t *members, const int64_t *crow,
                           const int32_t *ccol, double *cval, double *cdiag, uint32_t *flag,
                           int64_t nnz, hipStream_t s) {
    if (n_agg <= 0) return hipSuccess;
    const int64_t blocks = (n_agg + kGWaves - 1) / kGWaves;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_galerkin, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr, col, val,
                       diag, agg, n_agg, moff, members, crow, ccol, cval, cdiag, flag, nnz);
    return hipGetLastError();
}

}  // namespace mis2
