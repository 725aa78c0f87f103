// Known-answer source for the oracle's Philox4x32-10: rocRAND's Philox4x32-10 engine, run on the host.
// Test infrastructure only.  Reads lines "seed subsequence block" (decimal, 64-bit) from stdin and prints
// the four 32-bit outputs the engine returns after skipping `block` blocks of four numbers in
// `subsequence`, as "w0 w1 w2 w3" per line.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long seed, subsequence, block;
    while (std::scanf("%llu %llu %llu", &seed, &subsequence, &block) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, subsequence, 4ull * block);
        unsigned int w[4];
        for (int i = 0; i < 4; ++i) w[i] = e.next();
        std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
