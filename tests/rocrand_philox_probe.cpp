// Host-only probe used by the oracle tests: evaluates rocRAND's Philox4x32-10
// engine (header-only, host-callable) so the oracle's own Philox can be
// checked against an independent implementation.  Reads lines
// "seed c0 c1 c2 c3" on stdin and prints the four output words of the block
// at counter (c0, c1, c2, c3) under key (seed lo, seed hi).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        // subsequence selects counter words 2..3, offset (in words) words 0..1
        unsigned long long subsequence = c2 | (c3 << 32);
        // offset (in words) = 4 * (c0 + 2^32 c1), applied in pieces that fit
        // in 64 bits: 4 c0, then 2^34 (c1 mod 2^29), then 2^63 per 2^29 of c1
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 4ull * c0);
        eng.discard((c1 & ((1ull << 29) - 1)) << 34);
        for (unsigned long long h = 0; h < (c1 >> 29); ++h)
            eng.discard(1ull << 63);
        uint4 w = eng.next4();
        std::printf("%u %u %u %u\n", w.x, w.y, w.z, w.w);
    }
    return 0;
}
