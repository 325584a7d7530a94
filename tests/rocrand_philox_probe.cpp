// Host-only probe: prints Philox4x32-10 of (counter, key) as computed by the
// installed rocRAND engine.  Used by the oracle's RNG pin as an independent
// implementation; counter words map to rocRAND's (offset/4, subsequence).
// Arguments: key64 c0 c1 c2 c3 (c1 < 2^30 so that 4 * offset fits 64 bits).
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv)
{
    if (argc != 6) return 2;
    unsigned long long key = strtoull(argv[1], nullptr, 0);
    unsigned c0 = strtoul(argv[2], nullptr, 0), c1 = strtoul(argv[3], nullptr, 0);
    unsigned c2 = strtoul(argv[4], nullptr, 0), c3 = strtoul(argv[5], nullptr, 0);
    rocrand_state_philox4x32_10 st;
    unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
    unsigned long long offset = ((((unsigned long long)c1) << 32) | c0) * 4ull;
    rocrand_init(key, subsequence, offset, &st);
    uint4 v = rocrand4(&st);
    printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
    return 0;
}
