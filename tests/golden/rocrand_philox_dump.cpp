// Host-side dump of rocRAND's Philox4x32-10 for the counter/key scheme of the Z4
// noise: counter (n, alpha, t, 0), key (m, 0x4C415048).  An independent library
// implementation used to pin the oracle's generator.  Output: one line per element,
// "t alpha n word0".
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_philox4x32_10.h>

int main(int argc, char** argv)
{
    unsigned m = (unsigned)strtoul(argv[1], nullptr, 0);
    int nt = atoi(argv[2]), nv = atoi(argv[3]);
    unsigned long long seed = (unsigned long long)m | (0x4C415048ull << 32);
    for (int t = 0; t < nt; t++)
        for (int a = 0; a < 4; a++)
            for (int n = 0; n < nv; n++) {
                // counter words (x,y) = offset/4 as 64 bits, (z,w) = subsequence
                unsigned long long offset = 4ull * ((unsigned long long)n | ((unsigned long long)a << 32));
                rocrand_device::philox4x32_10_engine eng(seed, (unsigned long long)t, offset);
                uint4 r = eng.next4();
                printf("%d %d %d %u\n", t, a, n, r.x);
            }
    return 0;
}
