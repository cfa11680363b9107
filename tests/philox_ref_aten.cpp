// Test helper: prints ATen's Philox4x32-10 block for (counter, key) lines
// read from stdin ("c0 c1 c2 c3 k0 k1", decimal).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>

int main()
{
    unsigned c[4], k[2];
    while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        uint64_t seed = (uint64_t)k[0] | ((uint64_t)k[1] << 32);
        uint64_t subseq = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
        at::Philox4_32 e(seed, subseq, 0);
        e.set_offset((uint64_t)c[0] | ((uint64_t)c[1] << 32));
        unsigned r0 = e(), r1 = e(), r2 = e(), r3 = e();
        std::printf("%u %u %u %u\n", r0, r1, r2, r3);
    }
    return 0;
}
