// Prints Philox4x32-10 output blocks computed by rocRAND's own engine (host
// side of its header), for counters and keys read from stdin:
//   c0 c1 c2 c3 k0 k1   (decimal, one block per line)
// rocRAND's engine maps seed -> key, subsequence -> counter words 2..3 and
// offset/4 -> counter words 0..1, so the first next4() is philox(ctr, key).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long c[4], k[2];
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = k[0] | (k[1] << 32);
        unsigned long long subseq = c[2] | (c[3] << 32);
        unsigned long long offset = 4ull * (c[0] | (c[1] << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
