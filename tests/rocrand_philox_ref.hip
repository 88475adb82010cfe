// Host-side access to rocRAND's Philox4x32-10 engine, used only to pin the
// CPU oracle's independent Philox implementation (built by the test-suite).
#include <rocrand/rocrand_kernel.h>

extern "C" void rocrand_ref_block(const unsigned int key[2], const unsigned int ctr[4],
                                  unsigned int out[4])
{
    // rocRAND's counter is (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi)
    const unsigned long long seed = (unsigned long long)key[0] | ((unsigned long long)key[1] << 32);
    const unsigned long long sub = (unsigned long long)ctr[2] | ((unsigned long long)ctr[3] << 32);
    const unsigned long long c01 = (unsigned long long)ctr[0] | ((unsigned long long)ctr[1] << 32);
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, 0ull, &st);
    // the offset counts 32-bit outputs (4 per counter step): advance in
    // pieces of 2^60 counter steps so that no offset overflows 64 bits
    const unsigned long long low = c01 & ((1ull << 60) - 1);
    if (low) skipahead(4ull * low, &st);
    for (unsigned long long q = c01 >> 60; q > 0; --q) skipahead(1ull << 62, &st);
    for (int i = 0; i < 4; ++i) out[i] = rocrand(&st);
}
