// ra_dpp.hpp — DPP row operations of gfx950 used by the pair and HI kernels:
// masked lane moves, 16-lane row sums and the whole-wave inclusive scan.
#pragma once
#include "ra_device.hpp"

namespace ra {

// DPP lane exchanges (GFX9 controls). Lanes whose source is outside the row,
// or whose row is not in ROW_MASK, read 0.
constexpr int DPP_QUAD_1032 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int DPP_ROW_MIRROR = 0x140;      // lane i of a row reads lane 15 - i
constexpr int DPP_ROW_HALF_MIRROR = 0x141; // lane i of a half-row reads lane 7 - i
constexpr int DPP_ROW_SHR = 0x110;         // + n: lane i reads lane i - n of its row
constexpr int DPP_ROW_BCAST15 = 0x142;     // lane 15 of each row to the next row
constexpr int DPP_ROW_BCAST31 = 0x143;     // lane 31 to rows 2 and 3

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_or0(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, false));
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_or0(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 16 lanes of each row, the same value in every lane (pairs,
// quads, half-rows, rows; every step is a commutative pairwise add).
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
    v += dpp_or0<DPP_QUAD_1032>(v);
    v += dpp_or0<DPP_QUAD_2301>(v);
    v += dpp_or0<DPP_ROW_HALF_MIRROR>(v);
    v += dpp_or0<DPP_ROW_MIRROR>(v);
    return v;
}

// Inclusive prefix sum over the 64 lanes: within rows by shifts 1, 2, 4, 8,
// then the row totals carried by the row broadcasts.
template <typename T>
__device__ __forceinline__ T wave_scan_incl(T v) {
    v += dpp_or0<DPP_ROW_SHR + 1>(v);
    v += dpp_or0<DPP_ROW_SHR + 2>(v);
    v += dpp_or0<DPP_ROW_SHR + 4>(v);
    v += dpp_or0<DPP_ROW_SHR + 8>(v);
    v += dpp_or0<DPP_ROW_BCAST15, 0xA>(v);
    v += dpp_or0<DPP_ROW_BCAST31, 0xC>(v);
    return v;
}

}  // namespace ra
