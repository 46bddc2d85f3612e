// Host-only reference for Philox4x32-10 taken from rocRAND's engine
// (rocrand/rocrand_philox4x32_10.h), an implementation independent of the
// oracle's.  Reads groups of six numbers from argv:
//   key_lo key_hi c0 c1 c2 c3
// and prints the four output words of Philox4x32-10(counter=c, key=key).
// The engine's counter is set through its public API: the subsequence sets
// words (c2, c3); four discards of (c1<<32 | c0) add exactly that value to
// words (c0, c1) without touching the sub-word position.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>
#include <cstdlib>

int main(int argc, char **argv)
{
    for (int i = 1; i + 5 < argc; i += 6) {
        const unsigned long long k0 = strtoull(argv[i], 0, 0), k1 = strtoull(argv[i + 1], 0, 0);
        const unsigned long long c0 = strtoull(argv[i + 2], 0, 0), c1 = strtoull(argv[i + 3], 0, 0);
        const unsigned long long c2 = strtoull(argv[i + 4], 0, 0), c3 = strtoull(argv[i + 5], 0, 0);
        rocrand_device::philox4x32_10_engine e((k1 << 32) | k0, (c3 << 32) | c2, 0);
        for (int q = 0; q < 4; ++q) e.discard((c1 << 32) | c0);
        const uint4 r = e.next4();
        printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
