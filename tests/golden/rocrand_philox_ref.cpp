// Reference Philox4x32-10 outputs from AMD's rocRAND headers (host-compiled).
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin and prints the four output
// words. rocRAND's state maps (seed, subsequence, offset) to counter
// (offset/4 low, offset/4 high, subsequence low, subsequence high) and key
// (seed low, seed high); rocrand4 returns the block for the current counter.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdint>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long block = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        // offset is in 32-bit outputs: 4 per counter block; blocks >= 2^62 are not
        // reachable this way, so the caller keeps c1 < 2^30.
        rocrand_init(seed, subseq, block * 4ULL, &st);
        uint4 v = rocrand4(&st);
        std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
