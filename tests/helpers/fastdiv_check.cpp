// Exhaustive-by-sampling check of the library's division by a precomputed
// multiplier against the hardware division, on the host build of the same
// inline functions the kernels use.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <random>

#include "asd_device.h"

int main()
{
    std::mt19937_64 g(12345);
    long bad = 0, checked = 0;
    const uint32_t fixed[] = {1u, 2u, 3u, 5u, 7u, 16u, 33u, 62u, 200u, 40000u, 1320000u,
                              65537u, 2147483647u, 4294967295u};
    for (uint32_t d : fixed) {
        asd::FastDiv f = asd::make_fastdiv(d);
        for (uint32_t i = 0; i < 200000; ++i) {
            uint32_t n = i < 1000 ? i : (i < 2000 ? 0xFFFFFFFFu - (i - 1000) : (uint32_t)g());
            bad += asd::fdiv(n, f) != n / d;
            ++checked;
        }
    }
    for (int k = 0; k < 100000; ++k) {
        uint32_t d = (uint32_t)(g() % 0xFFFFFFFFull) + 1u;
        asd::FastDiv f = asd::make_fastdiv(d);
        for (int j = 0; j < 20; ++j) {
            uint32_t n = (uint32_t)g();
            bad += asd::fdiv(n, f) != n / d;
            ++checked;
        }
    }
    std::printf("%ld %ld\n", checked, bad);
    return bad != 0;
}
