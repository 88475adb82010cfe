// Counter-based random numbers of the engine: Philox4x32-10 (Salmon et al.
// 2011, "Parallel random numbers: as easy as 1, 2, 3") and the map of a
// 32-bit output to a uniform in (0, 1).  Every draw of a history is keyed by
// the run seed and addressed by (uid, step index, tag), so results do not
// depend on which lane or launch takes the history.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pmc {

// Philox4x32-10 (Salmon et al. 2011); key = run seed, counter = (uid, k, tag)
template <bool kScalarKey = false>
__host__ __device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
            // a key shared by the wave stays a pair of per-round scalar adds
            // (precomputed and hoisted out of the step loop, the ten round
            // keys only spill to VGPR lanes)
            if constexpr (kScalarKey) asm volatile("" : "+s"(k0), "+s"(k1));
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return make_uint4(c0, c1, c2, c3);
}

// strictly inside (0,1), exactly representable in float
__host__ __device__ __forceinline__ float u01(uint32_t x) { return ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f); }

}  // namespace pmc
