// Workgroup LDS deposit cache of the transport kernel: the slot lookup
// shared by the transport and the roofline replay (device code only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pmc {

// Deposit cache lookup: the slot of a workgroup's LDS cache that holds key,
// claiming a free one on the way (compare-and-swap), trying `probes`
// consecutive slots from the key's hash position; -1 when all are taken by
// other keys.  h: the key's 32-bit hash, reduced to [0, n_slots) by a high
// product.
template <typename Key>
__device__ __forceinline__ int cache_slot(Key* ckey, Key key, uint32_t h, uint32_t n_slots, int probes)
{
    constexpr Key kEmpty = ~Key(0);
    uint32_t slot = __umulhi(h, n_slots);
    auto take = [&](uint32_t sl) {
        Key held = ckey[sl];
        if (held == kEmpty) {
            held = atomicCAS(&ckey[sl], kEmpty, key);
            if (held == kEmpty) held = key;
        }
        return held == key;
    };
    bool hit = take(slot);
    // further slots by linear probing (written out for the second, a loop
    // beyond it)
    for (int probe = 1; !hit && probe < probes; ++probe) {
        slot = slot + 1u == n_slots ? 0u : slot + 1u;
        hit = take(slot);
    }
    return hit ? (int)slot : -1;
}

}  // namespace pmc
