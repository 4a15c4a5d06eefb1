// Lanes of a wave whose 8-bit digit equals this lane's: the ranking step of
// the stable radix passes (device-wide scatter and the per-bucket LDS sort).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ifgp {

// Mask of the valid lanes of this wave whose g agrees with this lane's in the
// low `bits` bits (at most 8, the same on every lane; callers whose digits
// differ only there pass fewer).  Per bit b: the lanes whose bit b is set (one
// compare), kept as is where this lane's bit is set and inverted where it is
// clear.  The inversion is an XOR with this lane's bit b sign-extended from
// ~g (all ones where the bit is clear), so each bit costs one bit-field
// extract, one compare and one three-input bitwise operation per 32-lane half.
__device__ __forceinline__ uint64_t match_digit8(unsigned g, bool valid, int bits = 8) {
    constexpr int ICMP_EQ = 32;  // integer-compare predicate "equal"
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    const int ng = (int)~g;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if (b < bits) {
            const uint32_t clear = (uint32_t)__builtin_amdgcn_sbfe(ng, b, 1);  // ~0: bit b is 0
            const uint64_t set = __builtin_amdgcn_uicmp((int)clear, 0, ICMP_EQ);  // bit b set
            lo &= (uint32_t)set ^ clear;
            hi &= (uint32_t)(set >> 32) ^ clear;
        }
    }
    return ((uint64_t)hi << 32) | lo;
}

}  // namespace ifgp
