// Device-side integer core shared by all kernels: float conversion (Sec. 2.1, Alg. 1),
// the nested uniform scramble and shifts (Sec. 2.1, 2.3), lattice points (Sec. 2.4) and
// the per-pixel hash.  Everything stays in 32-bit integers until the final conversion.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qmc {
namespace dev {

__device__ __forceinline__ uint32_t brev(uint32_t x) { return __builtin_bitreverse32(x); }

// u * 2^-32 rounded down to binary32, times 2^32: u with every bit below its 24 leading
// significant bits cleared, as a float (exact, at most 24 significant bits).  With z the count
// of leading zeros, keep = 0xFFFFFF00 >> z selects bits 31-z .. 8-z; v_ffbh_u32 returns
// 0xFFFFFFFF for u = 0 and the shift reads the low five bits of its count, so u = 0 gives
// keep = 1 and the result 0.  Four VALU instructions (find-first-bit, shift, and, convert).
__device__ __forceinline__ float u32_to_unifloat_x32(uint32_t u) {
    uint32_t keep;
    asm("v_ffbh_u32 %0, %1\n\tv_lshrrev_b32_e64 %0, %0, %2" : "=&v"(keep) : "v"(u), "s"(0xFFFFFF00u));
    return static_cast<float>(u & keep);
}

// Largest binary32 not above u * 2^-32 (never 1): the value above scaled exactly by 2^-32.
__device__ __forceinline__ float u32_to_unifloat(uint32_t u) { return u32_to_unifloat_x32(u) * 0x1p-32f; }

// Switches this wavefront's FP32 rounding to round-toward-zero (MODE register, single-precision
// round field = 3).  The mode is per-wavefront state initialised at wave launch, so it only
// affects the calling kernel, which must perform no other FP32 arithmetic that relies on
// round-to-nearest.
__device__ __forceinline__ void set_fp32_round_toward_zero() { __builtin_amdgcn_s_setreg(0x801, 3); }

// Same result as u32_to_unifloat, valid only after set_fp32_round_toward_zero(): the
// conversion truncates u to 24 significant bits and the scaling by 2^-32 is exact (the product
// of 0 or a value >= 1 and a power of two stays normal), done as a multiply, which issues at
// twice the rate of ldexp.
__device__ __forceinline__ float u32_to_unifloat_rtz(uint32_t u) {
    return static_cast<float>(u) * 0x1p-32f;
}

// The low-to-high mixing P_s of the nested uniform scramble, applied to the mirrored value.
// sm = (s >> 8) & 0xFFFFFE is the seed-dependent even multiplier, precomputed per seed.
// __umul24 multiplies the low 24 bits of both operands (every multiplier is below 2^24).
__device__ __forceinline__ uint32_t nus_permute(uint32_t v, uint32_t s, uint32_t sm) {
    v += s;
    v = __umul24(v, 0x612362u) + v;
    v ^= v << 8;
    v = __umul24(v, sm) + v;
    v = __umul24(v, 0x934C76u) + v;
    v ^= v << 9;
    v ^= v * 0xFA8F38AAu;
    return v;
}

__device__ __forceinline__ uint32_t seed_multiplier(uint32_t s) { return (s >> 8) & 0xFFFFFEu; }

// Nested uniform scramble of a value already given in mirrored (bit-reversed) form.
__device__ __forceinline__ uint32_t nus_from_mirrored(uint32_t vr, uint32_t s, uint32_t sm) {
    return brev(nus_permute(vr, s, sm));
}

template <bool XOR>
__device__ __forceinline__ uint32_t apply_shift(uint32_t v, uint32_t d) {
    return XOR ? (v ^ d) : (v + d);
}

// Integer hash "pcg" (Jarzynski and Olano, JCGT 2020): a PCG state step followed by the
// RXS-M-XS output permutation.
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

}  // namespace dev
}  // namespace qmc
