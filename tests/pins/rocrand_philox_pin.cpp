// Host-side known-answer generator for Philox4x32-10 using rocRAND's engine header.
// Test infrastructure: pins the CPU oracle's Philox against an independent library
// implementation of the same published generator (Salmon et al., SC'11).
// stdin: lines "c0 c1 c2 c3 k0 k1" (decimal); stdout: the four output words per line.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        // rocRAND: key = seed, counter words (z, w) = subsequence, (x, y) = offset / 4
        const unsigned long long seed = k0 | (k1 << 32);
        const unsigned long long subsequence = c2 | (c3 << 32);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 0);
        // skip (c0 | c1 << 32) blocks of four words in parts of at most 2^61 blocks, so
        // that the word offset 4 * part never overflows 64 bits
        unsigned long long blocks = c0 | (c1 << 32);
        while (blocks > 0) {
            const unsigned long long part = blocks < (1ull << 61) ? blocks : (1ull << 61);
            eng.discard(4ull * part);
            blocks -= part;
        }
        const uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
