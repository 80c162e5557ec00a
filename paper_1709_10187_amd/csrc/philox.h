// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw, SC'11), written from
// the published round definition: ten rounds of two 32x32->64 multiplies with the
// multipliers 0xD2511F53 and 0xCD9E8D57, key increments 0x9E3779B9 and 0xBB67AE85.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rddmc {

struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c0;
        const uint64_t p1 = (uint64_t)M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        // three-input xors as single gfx950 bitop3 instructions (truth table 0x96)
        c0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
        c1 = lo1;
        c2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return {c0, c1, c2, c3};
}

}  // namespace rddmc
