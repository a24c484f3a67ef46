// Independent Philox4x32-10 reference: runs rocRAND's own engine (a
// third-party implementation of the SC'11 definition) so that the oracle's
// Philox can be checked against it.  Reads lines "k0 k1 c0 c1 c2 c3" (hex)
// on stdin and prints the four output words of the block function.
//
// rocRAND seeds its engine as key = seed, counter words 2-3 = subsequence and
// counter words 0-1 = offset / 4, and the first value it returns is word 0 of
// the block function at that counter.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = (((unsigned long long)c1 << 32) | c0) * 4ull;
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        unsigned a = eng(), b = eng(), c = eng(), d = eng();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
