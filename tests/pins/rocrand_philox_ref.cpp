// Test helper: raw Philox4x32-10 words from rocRAND's header-only engine, run
// on the host.  Reads lines "key0 key1 c0 c1 c2 c3" (decimal) from stdin and
// prints the four output words of that (key, counter) block.  rocRAND seeds
// key = (lo32 seed, hi32 seed); skipping k numbers advances the 64-bit counter
// word pair (c0, c1) by k/4, and the subsequence index sets (c2, c3).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subsequence = c2 | (c3 << 32);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 4ull * c0);
        for (int i = 0; i < 4; ++i) // four skips of c1 * 2^32 numbers add c1 to word c1
            eng.discard(c1 << 32);
        uint4 v = eng.next4();
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
