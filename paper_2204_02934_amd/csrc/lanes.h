// lanes.h -- cross-lane moves and reductions over lane groups, in registers.
//
// On gfx950 __shfl_xor and __shfl compile to ds_bpermute_b32, an LDS round
// trip per step; a reduction or a sorting network built on them is a chain
// of LDS latencies.  The moves here use DPP where the pattern allows: quad
// permutes for xor 1 and 2, a pair of row shifts (lane l reads l + J, or
// l - J) for xor 4 and 8, wave shifts by one lane; a swizzle within 32 lanes
// for xor 16, and a permute only for xor 32.  Every lane of the wavefront
// must be active where they are called.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mis2 {

// lane l's view of lane l ^ J
template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t x) {
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
    } else if constexpr (J == 4 || J == 8) {
        const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x100 + J, 0xF, 0xF, false);
        const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x110 + J, 0xF, 0xF, false);
        return (threadIdx.x & J) ? dn : up;
    } else if constexpr (J == 16) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (16 << 10) | 0x1F);
    } else {
        static_assert(J == 32, "lane_xor: J is a power of two below 64");
        return (uint32_t)__shfl_xor((int)x, 32, 64);
    }
}

template <int J>
__device__ __forceinline__ int32_t lane_xor_i(int32_t x) {
    return (int32_t)lane_xor<J>((uint32_t)x);
}

template <int J>
__device__ __forceinline__ int64_t lane_xor64(int64_t x) {
    const uint32_t lo = lane_xor<J>((uint32_t)(uint64_t)x);
    const uint32_t hi = lane_xor<J>((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// lane l's view of lane l + 1 (wave_shl1) and of lane l - 1 (wave_shr1)
__device__ __forceinline__ uint32_t from_next(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_prev(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x138, 0xF, 0xF, false);
}

// Inclusive prefix sum over the 64 lanes: sums within each row of 16 lanes by
// row shifts (lanes shifted in from outside the row read 0), then the totals
// of rows 0 and 2 broadcast into rows 1 and 3, and that of rows 0-1 into 2-3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}

// Reductions over aligned groups of L lanes (L a power of two <= 64); every
// lane of a group gets the group's result.
#define MIS2_GROUP_REDUCE(NAME, T, XOR, OP)                    \
    template <int L>                                           \
    __device__ __forceinline__ T NAME(T x) {                   \
        if constexpr (L >= 64) x = OP(x, XOR<32>(x));          \
        if constexpr (L >= 32) x = OP(x, XOR<16>(x));          \
        if constexpr (L >= 16) x = OP(x, XOR<8>(x));           \
        if constexpr (L >= 8) x = OP(x, XOR<4>(x));            \
        if constexpr (L >= 4) x = OP(x, XOR<2>(x));            \
        if constexpr (L >= 2) x = OP(x, XOR<1>(x));            \
        return x;                                              \
    }

__device__ __forceinline__ uint32_t op_min_u(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t op_or_u(uint32_t a, uint32_t b) { return a | b; }
__device__ __forceinline__ uint32_t op_and_u(uint32_t a, uint32_t b) { return a & b; }
__device__ __forceinline__ uint32_t op_add_u(uint32_t a, uint32_t b) { return a + b; }
__device__ __forceinline__ int32_t op_add_i(int32_t a, int32_t b) { return a + b; }
__device__ __forceinline__ uint32_t op_max_u(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ __forceinline__ int64_t op_max_l(int64_t a, int64_t b) { return a > b ? a : b; }

MIS2_GROUP_REDUCE(group_min, uint32_t, lane_xor, op_min_u)
MIS2_GROUP_REDUCE(group_or, uint32_t, lane_xor, op_or_u)
MIS2_GROUP_REDUCE(group_and, uint32_t, lane_xor, op_and_u)
MIS2_GROUP_REDUCE(group_sum, uint32_t, lane_xor, op_add_u)
MIS2_GROUP_REDUCE(group_sum_i, int32_t, lane_xor_i, op_add_i)
MIS2_GROUP_REDUCE(group_max, uint32_t, lane_xor, op_max_u)
MIS2_GROUP_REDUCE(group_max64, int64_t, lane_xor64, op_max_l)

#undef MIS2_GROUP_REDUCE

}  // namespace mis2
