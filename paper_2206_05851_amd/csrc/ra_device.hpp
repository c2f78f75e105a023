// ra_device.hpp — gfx950 device building blocks: counter-based noise,
// lane-neighbour exchange, spring law. Shared by every kernel of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ra {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). The paper fixes only
// zero mean and covariance 2 D dt for the random displacement (Eq. 1 text);
// a counter-based generator gives every (step, bead, replica, group) its own
// draw with no stored state, so any tile layout and any replay (adjoint
// recompute, graph replay) reproduces the same noise.
// Counter words c0 (step) and c3 (tag|group) are wave-uniform and stay in
// SGPRs; the compiler then keeps the first round's c0 product on the scalar
// unit.
// ---------------------------------------------------------------------------
struct Words {
    uint32_t x, y, z, w;
};

// Round keys of one seed: key + r * (Weyl increments), r = 0..9. Built once
// per kernel so the step loop does not redo the key schedule. They are pinned
// to VGPRs (the empty asm only constrains the register class): with a scalar
// key the compiler splits each three-way XOR back into two v_xor_b32, with
// vector keys it selects one v_bitop3_b32, and the per-step scalar work of
// the first rounds disappears from the single instruction stream.
struct RoundKeys {
    uint32_t k0[10], k1[10];
};

// PIN_VGPR = false keeps the keys in scalar registers (20 fewer VGPRs, two
// v_xor_b32 per three-way XOR): for kernels where occupancy matters more.
template <bool PIN_VGPR = true>
__device__ __forceinline__ RoundKeys round_keys(uint32_t key0, uint32_t key1) {
    RoundKeys k;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        k.k0[r] = key0 + (uint32_t)r * 0x9E3779B9u;
        k.k1[r] = key1 + (uint32_t)r * 0xBB67AE85u;
        if constexpr (PIN_VGPR) {
            asm volatile("" : "+v"(k.k0[r]));
            asm volatile("" : "+v"(k.k1[r]));
        }
    }
    return k;
}

// Three-input XOR as one gfx950 v_bitop3_b32 (truth table 0x96 = a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          const RoundKeys& k) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k.k0[round]);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k.k1[round]);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return Words{c0, c1, c2, c3};
}

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t key0, uint32_t key1) {
    return philox10(c0, c1, c2, c3, round_keys(key0, key1));
}

// Uniform in (0,1): the top 23 bits j of a word give (2j + 1) 2^-24 — an odd
// integer below 2^24 times a power of two, hence exact in binary32 and binary64.
// FP32: one v_alignbit_b32 forms the binary32 word of 1 + j 2^-23 (exponent
// bits 0x7F above the top 23 bits of x); subtracting 1 - 2^-24 is exact
// (Sterbenz) and leaves (2j + 1) 2^-24.
__device__ __forceinline__ float u01_f32(uint32_t x) {
    const uint32_t one_plus = __builtin_amdgcn_alignbit(0x7Fu, x, 9u);
    return __builtin_bit_cast(float, one_plus) - 0x1.fffffep-1f;
}
__device__ __forceinline__ double u01_f64(uint32_t x) {
    return (double)((x >> 8) | 1u) * 0x1p-24;
}
// Unfolding-event uniform from two words: the top 52 bits m of hi:lo give
// (2m + 1) 2^-53, exact in binary64; event probabilities per window reach
// 1e-7 and below, under the 2^-24 grid of the one-word map.
__device__ __forceinline__ double u01_f64_53(uint32_t hi, uint32_t lo) {
    const uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return (double)(2 * m + 1) * 0x1p-53;
}

// Box-Muller, three normals from one Philox block: (r0 cos 2pi u1, r0 sin 2pi u1,
// r1 cos 2pi u3), r = sqrt(-2 ln u). FP32 uses the hardware transcendentals:
// v_log_f32 is log2, so -2 ln u = (-2 ln 2) log2 u; v_sin_f32/v_cos_f32 take
// their argument in revolutions, so sin(2 pi u) is one instruction on u.
__device__ __forceinline__ void normals3(const Words& w, float& a, float& b, float& c) {
    const float m2ln2 = -1.3862943611198906f;
    const float u0 = u01_f32(w.x), u1 = u01_f32(w.y), u2 = u01_f32(w.z), u3 = u01_f32(w.w);
    const float r0 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
    const float r1 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u2));
    a = r0 * __builtin_amdgcn_cosf(u1);
    b = r0 * __builtin_amdgcn_sinf(u1);
    c = r1 * __builtin_amdgcn_cosf(u3);
}
// The same with the second pair's other output, d = r1 sin 2 pi u3 (noise map 1).
__device__ __forceinline__ void normals4(const Words& w, float& a, float& b, float& c, float& d) {
    const float m2ln2 = -1.3862943611198906f;
    const float u0 = u01_f32(w.x), u1 = u01_f32(w.y), u2 = u01_f32(w.z), u3 = u01_f32(w.w);
    const float r0 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
    const float r1 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u2));
    a = r0 * __builtin_amdgcn_cosf(u1);
    b = r0 * __builtin_amdgcn_sinf(u1);
    c = r1 * __builtin_amdgcn_cosf(u3);
    d = r1 * __builtin_amdgcn_sinf(u3);
}
__device__ __forceinline__ void normals4(const Words& w, double& a, double& b, double& c, double& d) {
    const double u0 = u01_f64(w.x), u1 = u01_f64(w.y), u2 = u01_f64(w.z), u3 = u01_f64(w.w);
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    double s1, c1, s3, c3;
    sincospi(2.0 * u1, &s1, &c1);
    sincospi(2.0 * u3, &s3, &c3);
    a = r0 * c1;
    b = r0 * s1;
    c = r1 * c3;
    d = r1 * s3;
}

__device__ __forceinline__ void normals3(const Words& w, double& a, double& b, double& c) {
    const double u0 = u01_f64(w.x), u1 = u01_f64(w.y), u2 = u01_f64(w.z), u3 = u01_f64(w.w);
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    double s1, c1, s3, c3;
    sincospi(2.0 * u1, &s1, &c1);
    sincospi(2.0 * u3, &s3, &c3);
    (void)s3;
    a = r0 * c1;
    b = r0 * s1;
    c = r1 * c3;
}

// ---------------------------------------------------------------------------
// Whole-wavefront lane shifts by DPP (GFX9 wave_shr:1 / wave_shl:1). Lanes
// whose source is outside the wave read 0 (bound_ctrl).
// ---------------------------------------------------------------------------
constexpr int DPP_WAVE_SHL1 = 0x130;   // lane l reads lane l+1
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane l reads lane l-1

// mov_dpp with bound_ctrl writes 0 where the source lane is outside the wave
// and leaves the old value undefined, which lets the compiler fold the shift
// into the consuming VOP2 instruction.
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <typename T> __device__ __forceinline__ T from_prev_lane(T v) { return dpp_shift<DPP_WAVE_SHR1>(v); }
template <typename T> __device__ __forceinline__ T from_next_lane(T v) { return dpp_shift<DPP_WAVE_SHL1>(v); }

// ---------------------------------------------------------------------------
// Numeric helpers per precision.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }

constexpr double FENE_DELTA = 1.0e-3;   // guard: s = |Q|^2/Q0^2 is clamped at 1 - delta
constexpr float FENE_FP64_BAND = 0.9f;  // FP32 path recomputes s and 1/(1-s) in FP64 above this

// FENE factor g = 1/(1 - min(s, 1 - delta)) from a bond of squared length q2.
// The FP32 path keeps g in FP32 except near full extension, where 1 - s loses
// digits: there s is recomputed in FP64 from the FP32 components (their
// products are exact in FP64). Returns the clamp flag through `clamped`.
__device__ __forceinline__ float fene_g(float qx, float qy, float qz, float q2, float inv_q0sq,
                                        double inv_q0sq_d, int& clamped) {
    const float s = q2 * inv_q0sq;
    float g = fast_rcp(1.0f - s);
    // wave vote: the common case (no lane near full extension) costs one
    // compare and a scalar branch instead of an exec-mask save/restore
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(s > FENE_FP64_BAND) != 0, 0)) {
        if (s > FENE_FP64_BAND) {
            const double dx = qx, dy = qy, dz = qz;
            double sd = (dx * dx + dy * dy + dz * dz) * inv_q0sq_d;
            if (sd > 1.0 - FENE_DELTA) { sd = 1.0 - FENE_DELTA; clamped += 1; }
            g = (float)(1.0 / (1.0 - sd));
        }
    }
    return g;
}
__device__ __forceinline__ double fene_g(double qx, double qy, double qz, double q2, double,
                                         double inv_q0sq_d, int& clamped) {
    (void)qx; (void)qy; (void)qz;
    double s = q2 * inv_q0sq_d;
    if (s > 1.0 - FENE_DELTA) { s = 1.0 - FENE_DELTA; clamped += 1; }
    return 1.0 / (1.0 - s);
}

}  // namespace ra
