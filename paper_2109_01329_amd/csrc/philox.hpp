// Philox4x32-10 bijection for gfx950 device code (library-internal):
// Salmon et al. (SC'11), ten rounds, Weyl key bumps between rounds.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "transforms.hpp"

namespace mirng {

// a ^ b ^ c in one gfx950 v_bitop3_b32 (truth table 0x96; XOR3 is symmetric
// in its inputs, so the table does not depend on operand order).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2,
                                          uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t rk0 = k0 + (uint32_t)r * kPhiloxW0;
        const uint32_t rk1 = k1 + (uint32_t)r * kPhiloxW1;
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, rk0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, rk1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    u32x4 w;
    w.x = c0; w.y = c1; w.z = c2; w.w = c3;
    return w;
}

// Block base + j as a 128-bit counter.
__device__ __forceinline__ u32x4 block_at(const uint32_t base[4], uint32_t k0, uint32_t k1,
                                          uint32_t j)
{
    const uint64_t lo0 = ((uint64_t)base[1] << 32) | base[0];
    const uint64_t hi0 = ((uint64_t)base[3] << 32) | base[2];
    const uint64_t lo = lo0 + j;
    const uint64_t hi = hi0 + (lo < lo0 ? 1u : 0u);
    return philox10((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32),
                    k0, k1);
}

}  // namespace mirng
