// asd_device.h -- device-side building blocks of the sLLG Heun step.
//
// Counter-based noise: Philox4x32-R (Salmon, Moraes, Dror, Shaw, SC'11):
// per round two 32x32->64 products of the S-box, xor with the key and the
// other words, key bumped by the Weyl constants between rounds.
//
// FP64 noise and temperature use this library's fixed-order evaluations of
// ln, sin/cos(2 pi u) and exp built only from IEEE + - * / and exact
// scalings (compiled without FMA contraction), so that FP64 results depend
// on the definitions alone:
//   ln u : u = m 2^e, m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(z),
//          z = (m-1)/(m+1), series through z^21 (Horner in z^2),
//          result e*ln2_hi + (e*ln2_lo + ln m);
//   sin/cos(2 pi u), u in [0,1): q = floor(4u + 1/2), th = (4u - q) pi/2,
//          sin th = th - th^3 P(th^2) (through th^21), cos th = 1 - th^2 C(th^2)
//          (through th^20), rotated by quadrant q mod 4;
//   exp x (x <= 0): k = floor(x/ln2 + 1/2), r = (x - k ln2_hi) - k ln2_lo,
//          Taylor through r^13 (Horner), scaled by 2^k; 0 below -700.
// FP32 uses the hardware transcendentals (v_log_f32, v_exp_f32, v_sin_f32,
// v_cos_f32, v_sqrt_f32) and folds sigma into the Box-Muller radius.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asd {

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ void philox_round(uint32_t k0, uint32_t k1, uint32_t &c0, uint32_t &c1,
                                             uint32_t &c2, uint32_t &c3)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    // three-way xor in one v_bitop3_b32 (truth table 0x96)
    uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
}

// rounds is 7 or 10 (or 1..10 for the raw export); the key schedule is
// uniform across the wavefront, so the bumps stay on the scalar unit
__device__ __forceinline__ Words4 philox4x32(int rounds, uint32_t k0, uint32_t k1, uint32_t c0,
                                             uint32_t c1, uint32_t c2, uint32_t c3)
{
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    if (rounds == 10) {
#pragma unroll
        for (int r = 0; r < 10; ++r) philox_round(k0 + r * W0, k1 + r * W1, c0, c1, c2, c3);
    } else if (rounds == 7) {
#pragma unroll
        for (int r = 0; r < 7; ++r) philox_round(k0 + r * W0, k1 + r * W1, c0, c1, c2, c3);
    } else {
        for (int r = 0; r < rounds; ++r) philox_round(k0 + r * W0, k1 + r * W1, c0, c1, c2, c3);
    }
    return Words4{c0, c1, c2, c3};
}

// The step kernels run 10 rounds (the generator's standard count) or 7; the
// first seven are shared, so there is one uniform branch and no loop.
__device__ __forceinline__ Words4 philox4x32_7or10(int rounds, uint32_t k0, uint32_t k1,
                                                   uint32_t c0, uint32_t c1, uint32_t c2,
                                                   uint32_t c3)
{
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 7; ++r) philox_round(k0 + r * W0, k1 + r * W1, c0, c1, c2, c3);
    if (rounds != 7) {
#pragma unroll
        for (int r = 7; r < 10; ++r) philox_round(k0 + r * W0, k1 + r * W1, c0, c1, c2, c3);
    }
    return Words4{c0, c1, c2, c3};
}

// Division by a run-time divisor d >= 1 for 32-bit unsigned dividends with a
// precomputed multiplier (Granlund and Montgomery, PLDI 1994, Fig. 4.1):
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
// q = (t + ((n - t) >> 1)) >> (l - 1), t = mulhi(m, n); d = 1 handled by l = 0.
struct FastDiv {
    uint32_t d, m, l;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while (l < 32 && ((uint64_t)1 << l) < d) ++l;
    f.l = l;
    f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
    return f;
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, FastDiv f)
{
    if (f.l == 0) return n;
#ifdef __HIP_DEVICE_COMPILE__
    uint32_t t = __umulhi(f.m, n);
#else
    uint32_t t = (uint32_t)(((uint64_t)f.m * n) >> 32);
#endif
    return (t + ((n - t) >> 1)) >> (f.l - 1);
}

// ---------------------------------------------------------------- FP64
namespace f64 {

__device__ __forceinline__ double ln(double u)
{
    const double LN2_HI = 6.93147180369123816490e-01;
    const double LN2_LO = 1.90821492927058770002e-10;
    const double SQRT_HALF = 0.70710678118654752440;
    int e;
    double m = frexp(u, &e);
    if (m < SQRT_HALF) {
        m = m * 2.0;
        e = e - 1;
    }
    double z = (m - 1.0) / (m + 1.0);
    double z2 = z * z;
    double p = 1.0 / 21.0;
    p = 1.0 / 19.0 + z2 * p;
    p = 1.0 / 17.0 + z2 * p;
    p = 1.0 / 15.0 + z2 * p;
    p = 1.0 / 13.0 + z2 * p;
    p = 1.0 / 11.0 + z2 * p;
    p = 1.0 / 9.0 + z2 * p;
    p = 1.0 / 7.0 + z2 * p;
    p = 1.0 / 5.0 + z2 * p;
    p = 1.0 / 3.0 + z2 * p;
    p = 1.0 + z2 * p;
    double lm = (2.0 * z) * p;
    double de = (double)e;
    return de * LN2_HI + (de * LN2_LO + lm);
}

__device__ __forceinline__ void sincos2pi(double u, double &s_out, double &c_out)
{
    const double PIO2 = 1.57079632679489661923;
    double t = 4.0 * u;
    double q = floor(t + 0.5);
    double th = (t - q) * PIO2;
    double t2 = th * th;
    double ps = -1.0 / 51090942171709440000.0;
    ps = 1.0 / 121645100408832000.0 + t2 * ps;
    ps = -1.0 / 355687428096000.0 + t2 * ps;
    ps = 1.0 / 1307674368000.0 + t2 * ps;
    ps = -1.0 / 6227020800.0 + t2 * ps;
    ps = 1.0 / 39916800.0 + t2 * ps;
    ps = -1.0 / 362880.0 + t2 * ps;
    ps = 1.0 / 5040.0 + t2 * ps;
    ps = -1.0 / 120.0 + t2 * ps;
    ps = 1.0 / 6.0 + t2 * ps;
    double s = th - (th * t2) * ps;
    double pc = -1.0 / 2432902008176640000.0;
    pc = 1.0 / 6402373705728000.0 + t2 * pc;
    pc = -1.0 / 20922789888000.0 + t2 * pc;
    pc = 1.0 / 87178291200.0 + t2 * pc;
    pc = -1.0 / 479001600.0 + t2 * pc;
    pc = 1.0 / 3628800.0 + t2 * pc;
    pc = -1.0 / 40320.0 + t2 * pc;
    pc = 1.0 / 720.0 + t2 * pc;
    pc = -1.0 / 24.0 + t2 * pc;
    pc = 0.5 + t2 * pc;
    double c = 1.0 - t2 * pc;
    int quad = ((int)q) & 3;
    double rs = quad == 0 ? s : (quad == 1 ? c : (quad == 2 ? -s : -c));
    double rc = quad == 0 ? c : (quad == 1 ? -s : (quad == 2 ? -c : s));
    s_out = rs;
    c_out = rc;
}

__device__ __forceinline__ double expn(double x)
{
    const double LN2_HI = 6.93147180369123816490e-01;
    const double LN2_LO = 1.90821492927058770002e-10;
    const double INV_LN2 = 1.44269504088896340736;
    if (x < -700.0) return 0.0;
    double k = floor(x * INV_LN2 + 0.5);
    double r = (x - k * LN2_HI) - k * LN2_LO;
    double p = 1.0 / 6227020800.0;
    p = 1.0 / 479001600.0 + r * p;
    p = 1.0 / 39916800.0 + r * p;
    p = 1.0 / 3628800.0 + r * p;
    p = 1.0 / 362880.0 + r * p;
    p = 1.0 / 40320.0 + r * p;
    p = 1.0 / 5040.0 + r * p;
    p = 1.0 / 720.0 + r * p;
    p = 1.0 / 120.0 + r * p;
    p = 1.0 / 24.0 + r * p;
    p = 1.0 / 6.0 + r * p;
    p = 0.5 + r * p;
    p = 1.0 + r * p;
    p = 1.0 + r * p;
    return ldexp(p, (int)k);
}

// Box-Muller pair from two Philox words: radius word wr, angle word wt.
__device__ __forceinline__ void box_muller(uint32_t wr, uint32_t wt, double &gc, double &gs)
{
    const double TWO_M32 = 2.3283064365386962890625e-10;
    double ur = ((double)wr + 0.5) * TWO_M32;
    double ut = (double)wt * TWO_M32;
    double r = sqrt(-2.0 * ln(ur));
    double s, c;
    sincos2pi(ut, s, c);
    gc = r * c;
    gs = r * s;
}

}  // namespace f64

// ---------------------------------------------------------------- FP32
namespace f32 {

// Thermal-field Box-Muller pair in FP32 with sigma folded into the radius:
// sigma r = sqrt(sigma^2 (-2 ln u_r)) = sqrt(ns2 log2 u_r) with
// ns2 = -2 ln2 sigma^2; u_r = w 2^-32 + 2^-33 rounded to FP32; v_log_f32 is
// log2, v_sqrt_f32 the hardware square root (about 1 ulp), and v_sin_f32 /
// v_cos_f32 take their argument in revolutions.
__device__ __forceinline__ void box_muller_scaled(uint32_t wr, uint32_t wt, float ns2, float &gc,
                                                  float &gs)
{
    const float TWO_M32 = 2.3283064365386962890625e-10f;
    const float TWO_M33 = 1.16415321826934814453125e-10f;
    float ur = __builtin_fmaf((float)wr, TWO_M32, TWO_M33);
    float ut = (float)wt * TWO_M32;
    float r = __builtin_amdgcn_sqrtf(ns2 * __builtin_amdgcn_logf(ur));
    gc = r * __builtin_amdgcn_cosf(ut);
    gs = r * __builtin_amdgcn_sinf(ut);
}

__device__ __forceinline__ float box_muller_scaled_cos(uint32_t wr, uint32_t wt, float ns2)
{
    const float TWO_M32 = 2.3283064365386962890625e-10f;
    const float TWO_M33 = 1.16415321826934814453125e-10f;
    float ur = __builtin_fmaf((float)wr, TWO_M32, TWO_M33);
    float ut = (float)wt * TWO_M32;
    float r = __builtin_amdgcn_sqrtf(ns2 * __builtin_amdgcn_logf(ur));
    return r * __builtin_amdgcn_cosf(ut);
}

// -2 ln 2 sigma^2 with sigma^2 = cth T
__device__ __forceinline__ float neg2ln2_sigma2(float cth, float T)
{
    return -1.38629436111989061883f * (cth * T);
}

// exp(x) = 2^(x log2 e) on v_exp_f32
__device__ __forceinline__ float expn(float x)
{
    return __builtin_amdgcn_exp2f(x * 1.44269504088896340736f);
}

}  // namespace f32

}  // namespace asd
