// Test helper: prints rocRAND's Philox4x32-10 block for (counter, key) lines
// read from stdin ("c0 c1 c2 c3 k0 k1", decimal).  Host code only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c[4], k[2];
    while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = (unsigned long long)k[0] | ((unsigned long long)k[1] << 32);
        unsigned long long subseq = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
        rocrand_device::philox4x32_10_engine e(seed, subseq, 0);
        // Move the low 64 counter bits to (c0, c1) in steps that do not overflow.
        unsigned long long lo = (unsigned long long)c[0] | ((unsigned long long)c[1] << 32);
        for (int part = 0; part < 4; ++part) e.discard(lo);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
