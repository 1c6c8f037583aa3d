// Known-answer helper for the Philox4x32-10 pin: prints rocRAND's host-side
// Philox4x32-10 block for each (key0 key1 x0 x1 x2 x3) line read from stdin.
// rocRAND's engine maps seed -> key, subsequence -> (x2, x3) and
// offset / 4 -> (x0, x1), and its first four outputs are one block.
#include <cstdio>
#include <cstdlib>
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned k0, k1, x0, x1, x2, x3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &x0, &x1, &x2, &x3) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subsequence = (unsigned long long)x2 | ((unsigned long long)x3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)x0 | ((unsigned long long)x1 << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, offset, &st);
        for (int i = 0; i < 4; ++i) std::printf("%u%c", rocrand(&st), i == 3 ? '\n' : ' ');
    }
    return 0;
}
