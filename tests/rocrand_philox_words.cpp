// Raw Philox4x32-10 words from rocRAND's host/device engine header, for the
// known-answer comparison of the oracle's generator (built and run on the
// host by tests/test_oracle_philox.py; no GPU code is executed).
//
// rocRAND's engine keys the block function with (seed mod 2^32, seed / 2^32)
// and starts its 128-bit counter at (offset / 4 as words 0-1, subsequence as
// words 2-3).  Counter block (g, j, s, 0) is therefore reached with
// subsequence = s and an offset of 4 * (g + 2^32 j) numbers (applied in
// parts that each fit in 64 bits); four draws return its words.
//
// stdin: lines "seed stream g j"; stdout: the four words in hex per line.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
    unsigned long long seed, stream, g, j;
    while (std::scanf("%llu %llu %llu %llu", &seed, &stream, &g, &j) == 4) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, stream, 4ull * g, &st);
        for (int part = 0; part < 4; ++part) skipahead(4ull * (j << 30), &st);   // 4 x j 2^30 blocks
        unsigned w[4];
        for (int e = 0; e < 4; ++e) w[e] = rocrand(&st);
        std::printf("%08x %08x %08x %08x\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
