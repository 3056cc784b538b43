// Test helper: prints rocRAND's host-side Philox4x32-10 output for the
// counters and keys read from stdin, one "key_lo key_hi c0 c1 c2 c3" line per
// query.  rocRAND's engine keys Philox with the seed and starts its counter at
// (offset/4 as a 64-bit word, subsequence as a 64-bit word), so every counter
// can be reached through rocrand_init's arguments.
#include <cstdio>
#include <cstdint>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long klo, khi, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &klo, &khi, &c0, &c1, &c2, &c3) == 6) {
        const unsigned long long seed = klo | (khi << 32);
        const unsigned long long subsequence = c2 | (c3 << 32);
        const unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, offset, &st);
        uint4 v = rocrand4(&st);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
