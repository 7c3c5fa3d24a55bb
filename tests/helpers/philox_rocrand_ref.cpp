// Independent Philox4x32-10 reference for the oracle's pin test: rocRAND's
// host-callable engine (a separate implementation of the Salmon et al.
// SC'11 generator) evaluated at an arbitrary (counter, key).  rocRAND keeps
// counter = (64-bit low words advanced by discard(4 k), subsequence as the
// 64-bit high words) and key = (lo32 seed, hi32 seed); next4() returns the
// block at the current counter.  The low words are reached in chunks below
// 2^62 blocks (discard takes a 64-bit count of 32-bit numbers).
// Reads lines "seed c0 c1 c2 c3", prints "w0 w1 w2 w3".
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned int c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long lo = (static_cast<unsigned long long>(c1) << 32) | c0;
        unsigned long long subseq = (static_cast<unsigned long long>(c3) << 32) | c2;
        rocrand_device::philox4x32_10_engine e(seed, subseq, 0ULL);
        const unsigned long long chunk = (1ULL << 62) - 1;
        while (lo > 0) {
            unsigned long long k = lo < chunk ? lo : chunk;
            e.discard(4ULL * k);
            lo -= k;
        }
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
