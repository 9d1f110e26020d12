// Test helper: prints Philox4x32-10 words computed by rocRAND's open-source engine
// (public API only), one line per "c0 c1 c2 c3 k0 k1" line read from stdin.
// rocRAND's engine(seed, subsequence, offset) puts the key at (seed lo, seed hi), the
// subsequence in counter words 2..3 and offset/4 in counter words 0..1.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long pos = ((unsigned long long)c1 << 32) | c0;
        rocrand_device::philox4x32_10_engine eng(seed, 0ull, 0ull);
        eng.discard_subsequence(sub);
        eng.discard(4ull * pos);
        unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
