// Independent Philox4x32-10 reference for the oracle's pin test: prints the
// first block of rocRAND's host-compiled philox4x32_10 engine for each
// (counter, key) read from stdin as six hex words "c0 c1 c2 c3 k0 k1".
// rocRAND keys the engine with the 64-bit seed (k0 low word), puts the
// subsequence in counter words 2-3 and offset/4 in counter words 0-1.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
    unsigned c[4], k[2];
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
        unsigned long long subseq = ((unsigned long long)c[3] << 32) | c[2];
        unsigned long long offset = 4ull * (((unsigned long long)c[1] << 32) | c[0]);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, offset, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), d = rocrand(&st), e = rocrand(&st);
        std::printf("%08x %08x %08x %08x\n", a, b, d, e);
    }
    return 0;
}
