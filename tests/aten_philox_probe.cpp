// Test helper: prints Philox4x32-10 blocks computed by PyTorch's independent
// header-only implementation (ATen/core/PhiloxRNGEngine.h), one line per input
// line "seed c0 c1 c2 c3". Used only to pin the oracle's generator.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        const unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        const unsigned long long offset = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        at::philox_engine e(seed, subsequence, offset);
        const unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
