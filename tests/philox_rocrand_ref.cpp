// Host-side reference for the Philox4x32-10 pin: evaluates rocRAND's own
// philox4x32_10 engine (an independent, published implementation) at
// arbitrary (key, counter) pairs read from stdin, one "k0 k1 c0 c1 c2 c3"
// line per query, and prints the four output words.  Runs on the CPU only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>

int main()
{
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        const unsigned long long seed = k0 | (k1 << 32);
        // The engine's counter starts at zero; a subsequence advances the
        // upper two counter words, a discard of 4*n outputs the lower two.
        rocrand_device::philox4x32_10_engine e(seed, c2 | (c3 << 32), 4ull * c0);
        // Advance the second counter word in chunks that keep 4*n in range.
        unsigned long long hi = c1;
        while (hi > 0) {
            unsigned long long chunk = hi > (1ull << 29) ? (1ull << 29) : hi;
            e.discard(4ull * (chunk << 32));
            hi -= chunk;
        }
        unsigned int w0 = e(), w1 = e(), w2 = e(), w3 = e();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
