// device_common.h -- gfx950 device helpers shared by the sweep kernels:
// counter-based uniforms, the Gibbs weight quantisation and wave64 cross-lane
// primitives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdit {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round multiplies
// words 0 and 2 by the two round multipliers, mixes the high halves with the
// other two words and the round key, and the key advances by the two Weyl
// increments between rounds.  Only word 0 is used by the sweeps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one 32 x 32 -> 64-bit product per word (v_mad_u64_u32)
        const uint64_t pA = (uint64_t)kMulA * c0, pB = (uint64_t)kMulB * c2;
        const uint32_t n0 = (uint32_t)(pB >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pA >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)pB;
        c2 = n2;
        c3 = (uint32_t)pA;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return c0;
}

// 24-bit uniform of the update of location r in global sweep g of replica
// `rep` of instance `inst`.
__device__ __forceinline__ uint32_t uniform24(uint64_t seed, uint32_t r, uint32_t g, uint32_t rep,
                                              uint32_t inst) {
    return philox_word0(r, g, rep, inst, (uint32_t)seed, (uint32_t)(seed >> 32)) >> 8;
}

// ---------------------------------------------------------------------------
// Gibbs weights.  The weight of a candidate whose energy change exceeds the
// row minimum by d >= 0 is q = rint(expf(-fl32(beta * fl32(d))) * 2^25), an
// integer in [0, 2^25]; sums of q are exact (32 bits for up to 64 candidates,
// 64 bits beyond) and the draw is the first candidate whose running sum C
// satisfies C * 2^24 > u24 * Z.
// ---------------------------------------------------------------------------
constexpr uint32_t kWeightOne = 1u << 25;  // weight of the row minimum

__device__ __forceinline__ uint32_t gibbs_weight(float beta, float d) {
    const float x = __fmul_rn(beta, d);
    const float w = expf(-x);
    return (uint32_t)rintf(w * 33554432.0f);
}

// Smallest integer distance above which every weight is provably 0:
// fl32(beta * fl32(d)) >= 19.5 for all d >= the returned value
// (e^-19.5 * 2^25 < 0.12 rounds to 0).  The hardware reciprocal (error
// within 1 ulp) and the rounding of beta * d are covered by the 1e-4 margin
// and the +2.  Returns INT32_MAX when no such integer is in range: only for
// kernels whose distances stay below 2^31 - 1.
__device__ __forceinline__ int32_t zero_weight_distance(float beta) {
    if (!(beta > 0.0f)) return INT32_MAX;
    const float t = (19.5f * 1.0001f) * __builtin_amdgcn_rcpf(beta) + 2.0f;
    if (!(t < 2.0e9f)) return INT32_MAX;
    return (int32_t)t;
}

// The same bound for kernels whose distances are int64 (they may pass 2^31):
// INT64_MAX when beta is 0 or so small that no int64 distance reaches it, so
// that a distance is never cut that the weight formula does not round to 0.
__device__ __forceinline__ int64_t zero_weight_distance64(float beta) {
    if (!(beta > 0.0f)) return INT64_MAX;
    const float t = (19.5f * 1.0001f) * __builtin_amdgcn_rcpf(beta) + 2.0f;
    if (!(t < 9.0e18f)) return INT64_MAX;
    return (int64_t)t;
}

// Tie test shared by the kernels: the threshold u24*Z lies within Z*2^4 of a
// CDF boundary between two candidates of nonzero weight.
__device__ __forceinline__ bool is_tie(uint64_t c_prev, uint64_t c_sel, uint64_t Z,
                                       uint32_t u24) {
    const uint64_t target = (uint64_t)u24 * Z;
    const uint64_t band = Z << 4;
    const bool lo = c_prev > 0 && (target - (c_prev << 24)) < band;
    const bool hi = c_sel < Z && ((c_sel << 24) - target) <= band;
    return lo || hi;
}

// ---------------------------------------------------------------------------
// wave64 cross-lane primitives (GFX9 DPP row shifts within 16-lane rows, then
// readlane to combine the four rows).
// ---------------------------------------------------------------------------
template <int kShift>
__device__ __forceinline__ int32_t dpp_row_shr(int32_t fill, int32_t v) {
    return __builtin_amdgcn_update_dpp(fill, v, 0x110 + kShift, 0xF, 0xF, false);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Minimum over the wave, returned in every lane (uniform).
__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
    v = min(v, dpp_row_shr<1>(INT32_MAX, v));
    v = min(v, dpp_row_shr<2>(INT32_MAX, v));
    v = min(v, dpp_row_shr<4>(INT32_MAX, v));
    v = min(v, dpp_row_shr<8>(INT32_MAX, v));
    const int32_t a = __builtin_amdgcn_readlane(v, 15), b = __builtin_amdgcn_readlane(v, 31);
    const int32_t c = __builtin_amdgcn_readlane(v, 47), d = __builtin_amdgcn_readlane(v, 63);
    return min(min(a, b), min(c, d));
}

// Inclusive prefix sum of a 64-bit value across the wave (lane order).
__device__ __forceinline__ uint64_t wave_scan_u64(uint64_t v) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#define PDIT_SCAN_STEP(K)                                                  \
    {                                                                      \
        const uint32_t tl = (uint32_t)dpp_row_shr<K>(0, (int32_t)lo);      \
        const uint32_t th = (uint32_t)dpp_row_shr<K>(0, (int32_t)hi);      \
        const uint64_t s = ((uint64_t)hi << 32 | lo) + ((uint64_t)th << 32 | tl); \
        lo = (uint32_t)s;                                                  \
        hi = (uint32_t)(s >> 32);                                          \
    }
    PDIT_SCAN_STEP(1)
    PDIT_SCAN_STEP(2)
    PDIT_SCAN_STEP(4)
    PDIT_SCAN_STEP(8)
#undef PDIT_SCAN_STEP
    uint64_t x = (uint64_t)hi << 32 | lo;
    const uint64_t r0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)hi, 15) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int32_t)lo, 15);
    const uint64_t r1 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)hi, 31) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int32_t)lo, 31);
    const uint64_t r2 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)hi, 47) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int32_t)lo, 47);
    const int row = lane_id() >> 4;
    const uint64_t add = row == 0 ? 0 : row == 1 ? r0 : row == 2 ? r0 + r1 : r0 + r1 + r2;
    return x + add;
}

// Inclusive prefix sum of a 32-bit value across the wave (lane order).
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t v) {
    v += (uint32_t)dpp_row_shr<1>(0, (int32_t)v);
    v += (uint32_t)dpp_row_shr<2>(0, (int32_t)v);
    v += (uint32_t)dpp_row_shr<4>(0, (int32_t)v);
    v += (uint32_t)dpp_row_shr<8>(0, (int32_t)v);
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int32_t)v, 15);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int32_t)v, 31);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int32_t)v, 47);
    const int row = lane_id() >> 4;
    return v + (row == 0 ? 0u : row == 1 ? r0 : row == 2 ? r0 + r1 : r0 + r1 + r2);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(v >> 32), lane);
    return (uint64_t)hi << 32 | lo;
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int lane) {
    return (int64_t)readlane_u64((uint64_t)v, lane);
}

// ---------------------------------------------------------------------------
// Quad (4-lane) exchanges by DPP quad_perm: lane i of each quad reads lane
// sel[i] of the same quad.
// ---------------------------------------------------------------------------
constexpr int kQuadXor1 = 0xB1;   // [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;   // [2,3,0,1]
constexpr int kQuadPrev1 = 0x90;  // [0,0,1,2]
constexpr int kQuadPrev2 = 0x40;  // [0,0,0,1]
constexpr int kQuadPrev3 = 0x00;  // [0,0,0,0]
constexpr int kQuadLast = 0xFF;   // [3,3,3,3]

template <int CTRL>
__device__ __forceinline__ int32_t quad(int32_t v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint32_t quadu(uint32_t v) {
    return (uint32_t)quad<CTRL>((int32_t)v);
}
template <int CTRL>
__device__ __forceinline__ uint64_t quadu(uint64_t v) {
    const uint32_t lo = quadu<CTRL>((uint32_t)v), hi = quadu<CTRL>((uint32_t)(v >> 32));
    return (uint64_t)hi << 32 | lo;
}

}  // namespace pdit
