// Lane exchanges within a wave64 on the vector ALU (DPP row shifts, the
// gfx950 permlane swaps, lane reads) for the pairwise trees and prefix sums of
// the device library, instead of LDS permutes.  All lanes of the wave must be
// active where these are called.
#ifndef HTREE_WAVE_OPS_H
#define HTREE_WAVE_OPS_H

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wave_ops {

// The value of the lane OFF places above (OFF = 1, 2, ..., 32), for the lanes
// 0..OFF-1 of the wave; other lanes get unspecified values.  OFF < 16 is a DPP
// row shift (lanes 0..OFF-1 and their partners share a 16-lane row); 16 and 32
// are the swaps of 16-lane rows and 32-lane halves, whose second result holds
// the upper row (half) in the lower one.
template <int OFF>
__device__ __forceinline__ uint32_t above_u32(uint32_t v) {
    static_assert(OFF >= 1 && OFF <= 32 && (OFF & (OFF - 1)) == 0, "power-of-two lane offset");
    if constexpr (OFF == 32) return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
    else if constexpr (OFF == 16) return __builtin_amdgcn_permlane16_swap(v, v, false, false)[1];
    else return __builtin_amdgcn_update_dpp(0u, v, 0x100 + OFF, 0xf, 0xf, true);   // row_shl:OFF
}

// The value of the lane OFF places below in the same 16-lane row (OFF = 1, 2,
// 4, 8); the first OFF lanes of each row get 0.
template <int OFF>
__device__ __forceinline__ uint32_t below_in_row_u32(uint32_t v) {
    static_assert(OFF >= 1 && OFF <= 8 && (OFF & (OFF - 1)) == 0, "power-of-two lane offset below 16");
    return __builtin_amdgcn_update_dpp(0u, v, 0x110 + OFF, 0xf, 0xf, true);   // row_shr:OFF
}

// 32- and 64-bit values move as 32-bit halves.
template <class V, class F>
__device__ __forceinline__ V by_halves(V v, F f) {
    static_assert(sizeof(V) == 4 || sizeof(V) == 8, "32- or 64-bit values");
    if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, f(__builtin_bit_cast(uint32_t, v)));
    } else {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = f(static_cast<uint32_t>(b));
        const uint32_t hi = f(static_cast<uint32_t>(b >> 32));
        return __builtin_bit_cast(V, (static_cast<uint64_t>(hi) << 32) | lo);
    }
}

template <int OFF, class V>
__device__ __forceinline__ V above(V v) {
    return by_halves(v, [](uint32_t u) { return above_u32<OFF>(u); });
}

template <int OFF, class V>
__device__ __forceinline__ V below_in_row(V v) {
    return by_halves(v, [](uint32_t u) { return below_in_row_u32<OFF>(u); });
}

// Lane l's value, the same in every lane.
template <class V>
__device__ __forceinline__ V read_lane(V v, int l) {
    return by_halves(v, [l](uint32_t u) { return static_cast<uint32_t>(__builtin_amdgcn_readlane(u, l)); });
}

// Pairwise tree over a wave, lane k combining with lane k + OFF for OFF =
// FIRST, FIRST / 2, ..., LAST: with FIRST = 32 and LAST = 1 lane 0 ends with
// the whole wave's reduction.
template <int FIRST, int LAST, class V, class Op>
__device__ __forceinline__ V tree(V v, Op op) {
    if constexpr (FIRST >= LAST) {
        v = op(v, above<FIRST>(v));
        return tree<FIRST / 2, LAST>(v, op);
    } else {
        return v;
    }
}

// Inclusive prefix sum over the wave (lane l: lanes 0..l) for integers, or
// for doubles whose partial sums are exact (whole numbers): a scan within each
// 16-lane row by row shifts, then the lower rows' totals read from lanes 15,
// 31 and 47.
template <class V>
__device__ __forceinline__ V scan_inclusive(V x) {
    x += below_in_row<1>(x);
    x += below_in_row<2>(x);
    x += below_in_row<4>(x);
    x += below_in_row<8>(x);
    const V r0 = read_lane(x, 15), r1 = read_lane(x, 31), r2 = read_lane(x, 47);
    const int row = (threadIdx.x & 63) >> 4;
    if (row >= 1) x += r0;
    if (row >= 2) x += r1;
    if (row >= 3) x += r2;
    return x;
}

}  // namespace wave_ops

#endif
