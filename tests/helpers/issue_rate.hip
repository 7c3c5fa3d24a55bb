// issue_rate.hip -- VALU issue-rate calibration (measurement only; not part of
// the step library and not called by it).
//
// Each kernel runs CH independent dependency chains of one instruction class per
// lane for `iters` iterations, with enough waves per SIMD to hide every
// latency, so the time per instruction is the issue cost of that class alone.
// The benchmark turns the times into SIMD cycles per wave64 instruction; the
// ratios to an FP32 FMA are the weights of its VALU cost model (a 32 x 32 -> 64
// product of Philox, a transcendental of Box-Muller or of the Boltzmann test).
//
// Every lane writes one 32-bit word to out[global id]: out must hold
// blocks * 256 words.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kThreads = 256;
constexpr int CH = 8;

// v_fma_f32: a <- a * c1 + c2
__global__ __launch_bounds__(kThreads) void k_fma_f32(uint32_t *out, int iters, uint32_t seed)
{
    float a[CH];
    for (int c = 0; c < CH; ++c) a[c] = (float)(threadIdx.x + c + seed) * 1e-3f;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) a[c] = __builtin_fmaf(a[c], 0.999f, 1e-4f);
    float r = 0.0f;
    for (int c = 0; c < CH; ++c) r += a[c];
    out[blockIdx.x * kThreads + threadIdx.x] = __builtin_bit_cast(uint32_t, r);
}

// v_xor_b32: a <- a ^ a' (the next chain's value)
__global__ __launch_bounds__(kThreads) void k_xor_u32(uint32_t *out, int iters, uint32_t seed)
{
    uint32_t a[CH];
    for (int c = 0; c < CH; ++c) a[c] = threadIdx.x * 7u + c + seed;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) a[c] = a[c] ^ a[(c + 1) % CH];
    uint32_t r = 0;
    for (int c = 0; c < CH; ++c) r ^= a[c];
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// v_mad_u64_u32: p <- lo(p) * M + p, the full 32 x 32 -> 64 product of a
// Philox round with a 64-bit addend, one instruction per chain and iteration
__global__ __launch_bounds__(kThreads) void k_mad_u64_u32(uint32_t *out, int iters, uint32_t seed)
{
    uint64_t p[CH];
    for (int c = 0; c < CH; ++c) p[c] = threadIdx.x * 0x9E3779B9ull + c + seed;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) p[c] = (uint64_t)(uint32_t)p[c] * 0xD2511F53u + p[c];
    uint64_t r = 0;
    for (int c = 0; c < CH; ++c) r ^= p[c];
    out[blockIdx.x * kThreads + threadIdx.x] = (uint32_t)r ^ (uint32_t)(r >> 32);
}

// v_log_f32 (a quarter-rate class): a <- log2(a); the values run down to -inf
// and NaN, which the issue cost does not depend on
__global__ __launch_bounds__(kThreads) void k_log_f32(uint32_t *out, int iters, uint32_t seed)
{
    float a[CH];
    for (int c = 0; c < CH; ++c) a[c] = 2.0f + (float)(threadIdx.x + c + seed) * 1e-4f;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) a[c] = __builtin_amdgcn_logf(a[c]);
    float r = 0.0f;
    for (int c = 0; c < CH; ++c) r += a[c];
    out[blockIdx.x * kThreads + threadIdx.x] = __builtin_bit_cast(uint32_t, r);
}

// v_rsq_f32: a <- 1 / sqrt(a) (converges to 1)
__global__ __launch_bounds__(kThreads) void k_rsq_f32(uint32_t *out, int iters, uint32_t seed)
{
    float a[CH];
    for (int c = 0; c < CH; ++c) a[c] = 2.0f + (float)(threadIdx.x + c + seed) * 1e-4f;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) a[c] = __builtin_amdgcn_rsqf(a[c]);
    float r = 0.0f;
    for (int c = 0; c < CH; ++c) r += a[c];
    out[blockIdx.x * kThreads + threadIdx.x] = __builtin_bit_cast(uint32_t, r);
}

// v_fma_f64: a <- a * c1 + c2
__global__ __launch_bounds__(kThreads) void k_fma_f64(uint32_t *out, int iters, uint32_t seed)
{
    double a[CH];
    for (int c = 0; c < CH; ++c) a[c] = (double)(threadIdx.x + c + seed) * 1e-3;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CH; ++c) a[c] = __builtin_fma(a[c], 0.999, 1e-4);
    double r = 0.0;
    for (int c = 0; c < CH; ++c) r += a[c];
    float f = (float)r;
    out[blockIdx.x * kThreads + threadIdx.x] = __builtin_bit_cast(uint32_t, f);
}

using Kernel = void (*)(uint32_t *, int, uint32_t);
const Kernel kKernels[] = {k_fma_f32, k_xor_u32, k_mad_u64_u32, k_log_f32, k_rsq_f32, k_fma_f64};
const char *const kNames[] = {"v_fma_f32", "v_xor_b32", "v_mad_u64_u32", "v_log_f32", "v_rsq_f32",
                              "v_fma_f64"};
constexpr int kClasses = (int)(sizeof(kKernels) / sizeof(kKernels[0]));

}  // namespace

extern "C" {

// Number of instruction classes; names of class k.
int issue_rate_classes(void) { return kClasses; }
const char *issue_rate_name(int k) { return (k >= 0 && k < kClasses) ? kNames[k] : nullptr; }

// Time one launch of class k: `blocks` workgroups of 256 lanes, `iters`
// iterations of CH instructions per lane, after one untimed launch.  `out` is
// a device buffer of blocks * 256 words; the launch runs on the null stream.
// Returns 0, or -1 for bad arguments, or -2 for a HIP error; *ms = elapsed time.
int issue_rate_time(int k, void *out, int blocks, int iters, float *ms)
{
    if (k < 0 || k >= kClasses || !out || blocks <= 0 || iters <= 0 || !ms) return -1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -2;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -2;
    }
    auto *o = static_cast<uint32_t *>(out);
    kKernels[k]<<<blocks, kThreads>>>(o, iters, 0u);
    (void)hipEventRecord(e0, nullptr);
    kKernels[k]<<<blocks, kThreads>>>(o, iters, 1u);
    (void)hipEventRecord(e1, nullptr);
    int rc = 0;
    if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
        rc = -2;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// Instructions of the class per lane and iteration
int issue_rate_chains(void) { return CH; }

}  // extern "C"
