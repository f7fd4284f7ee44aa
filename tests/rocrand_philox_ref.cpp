// Independent reference for the oracle's Philox4x32-10: the open-source
// rocRAND engine, run on the host.  Reads "key0 key1 c0 c1 c2 c3" lines
// (decimal) and prints the four output words of Philox4x32-10(counter, key).
// rocRAND keys its engine with the 64-bit seed (low word first) and starts
// the counter at (offset/4 low, offset/4 high, subsequence low, subsequence
// high), so an arbitrary counter is reached through subsequence and skip-ahead.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subsequence = c2 | (c3 << 32);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, 4ull * c0, &st);
        // advance the counter by c1 << 32 in four steps (each offset < 2^64)
        for (int i = 0; i < 4; ++i) skipahead(4ull * (c1 << 30), &st);
        uint4 v = rocrand4(&st);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
