// Host-side reference for Philox4x32-10 that runs rocRAND's own engine
// (header-only, host-callable) -- an implementation independent of the
// project's.  Reads lines "seed c0 c1 c2 c3" on stdin, prints the four
// output words of the block at that counter.
//
// rocRAND's engine starts from counter 0 and advances by (offset / 4) in
// words 0-1 and by `subsequence` in words 2-3, so counter (c0,c1,c2,c3) is
// reached with offset = 4*(c0 + 2^32 c1) and subsequence = c2 + 2^32 c3.
#include <cstdio>
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        rocrand_state_philox4x32_10 st;
        unsigned long long offset = 4ull * (c0 + (c1 << 32));
        unsigned long long subseq = c2 + (c3 << 32);
        rocrand_init(seed, subseq, offset, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
