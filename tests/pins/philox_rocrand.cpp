// Independent Philox4x32-10 for pinning the oracle: runs rocRAND's engine
// (a third-party implementation of the same SC'11 generator) on the host.
// Reads lines "x y z w k0 k1" (decimal counter words and key words) and
// prints the four output words of that block.  The engine is positioned at
// counter (x, y, z, w) through its documented seeding interface: the seed
// is the key (low word first), the subsequence fills counter words z, w and
// the offset (4 draws per block) fills counter words x, y.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long x, y, z, w, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &x, &y, &z, &w, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subsequence = z | (w << 32);
        unsigned long long block = x | (y << 32);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 4ull * block);
        unsigned int a = eng.next(), b = eng.next(), c = eng.next(), d = eng.next();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
