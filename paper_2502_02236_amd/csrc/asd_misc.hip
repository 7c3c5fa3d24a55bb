// asd_misc.hip -- Philox export, step-counter and window bookkeeping,
// column freezing for window shifts, the FP64 reductions, and the window-end
// transfer to and from a coarse (micromagnetic) grid.
#include "asd_device.h"
#include "asd_internal.h"
#include "asd.h"
#include "asd_pair.h"

namespace asd {

__global__ void k_philox_export(uint32_t k0, uint32_t k1, int rounds, const uint32_t *ctr,
                                uint32_t *out, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 c = reinterpret_cast<const uint4 *>(ctr)[i];
    Words4 w = philox4x32(rounds, k0, k1, c.x, c.y, c.z, c.w);
    reinterpret_cast<uint4 *>(out)[i] = make_uint4(w.w0, w.w1, w.w2, w.w3);
}

int launch_philox_export(uint64_t seed, int rounds, const uint32_t *ctr, uint32_t *out, int64_t n,
                         void *stream)
{
    if (n == 0) return 0;
    int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_philox_export, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t)seed, (uint32_t)(seed >> 32), rounds, ctr, out, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void k_advance(int64_t *step_base, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step_base += n;
}

int launch_advance_step(int64_t *step_base, int64_t n, void *stream)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, (hipStream_t)stream, step_base, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

struct I32x8 {
    int32_t v[8];
};

__global__ void k_set_i32(int32_t *dst, I32x8 vals, int n)
{
    int i = threadIdx.x;
    if (i < n) dst[i] = vals.v[i];
}

int launch_set_i32(int32_t *dst, const int32_t *vals, int n, void *stream)
{
    for (int off = 0; off < n; off += 8) {
        I32x8 v{};
        int m = n - off < 8 ? n - off : 8;
        for (int k = 0; k < m; ++k) v.v[k] = vals[off + k];
        hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, (hipStream_t)stream, dst + off, v, m);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// copy stored columns [x0, x0 + ncols) of one system from src to dst
template <typename T>
__global__ void k_copy_columns(T *dst, const T *src, int64_t ncs, int64_t base, int kind, int sx,
                               int ny, int nz, int x0, int ncols)
{
    int per_col = (kind == ASD_SC ? 1 : 2);
    int64_t m = (int64_t)ncols * ny * nz * per_col;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    int s = (int)(t % per_col);
    int64_t r = t / per_col;
    int xc = (int)(r % ncols);
    int64_t yz = r / ncols;
    int64_t cell = (x0 + xc) + (int64_t)sx * yz;
    int64_t i = base + cell * per_col + s;
    for (int k = 0; k < 3; ++k) dst[k * ncs + i] = src[k * ncs + i];
}

int launch_copy_columns(int prec, void *dst, const void *src, int64_t ncs, const SysDev &d, int x0,
                        int ncols, void *stream)
{
    int per_col = (d.kind == ASD_SC ? 1 : 2);
    int64_t m = (int64_t)ncols * d.ny * d.nz * per_col;
    if (m == 0) return 0;
    unsigned blocks = (unsigned)((m + 255) / 256);
    if (prec == ASD_FP64)
        hipLaunchKernelGGL(k_copy_columns<double>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (double *)dst, (const double *)src, ncs, d.base, d.kind, d.sx, d.ny, d.nz,
                           x0, ncols);
    else
        hipLaunchKernelGGL(k_copy_columns<float>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (float *)dst, (const float *)src, ncs, d.base, d.kind, d.sx, d.ny, d.nz,
                           x0, ncols);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
__global__ void k_mask(T *buf, int64_t ncs, const uint16_t *label, int64_t base, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int64_t i = base + t;
    if (label[i] == kNoGrain) {
        buf[i] = 0;
        buf[ncs + i] = 0;
        buf[2 * ncs + i] = 0;
    }
}

int launch_mask_spins(int prec, void *buf, int64_t ncs, const uint16_t *label, const SysDev &d,
                      void *stream)
{
    if (d.n_stored == 0) return 0;
    unsigned blocks = (unsigned)((d.n_stored + 255) / 256);
    if (prec == ASD_FP64)
        hipLaunchKernelGGL(k_mask<double>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (double *)buf, ncs, label, d.base, d.n_stored);
    else
        hipLaunchKernelGGL(k_mask<float>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (float *)buf, ncs, label, d.base, d.n_stored);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// A field per coarse cell of a window mesh ncx x ncy x ncz (dst [3][ncell]
// in the handle precision) from the cells [off, off + ncx) along x of a
// wider mesh of src_nx cells (src [3][src_nx ncy ncz], FP64)
template <typename T>
__global__ void k_cells_from_mesh(T *dst, const double *src, int src_nx, int src_off, int ncx,
                                  int ncy, int ncz)
{
    const int64_t ncell = (int64_t)ncx * ncy * ncz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * ncell) return;
    const int c = (int)(t / ncell);
    const int64_t q = t - c * ncell;
    const int i = (int)(q % ncx);
    const int64_t jk = q / ncx;
    dst[t] = (T)src[c * (int64_t)src_nx * ncy * ncz + (src_off + i) + (int64_t)src_nx * jk];
}

int launch_cells_from_mesh(int prec, void *dst, const double *src, int src_nx, int src_off, int ncx,
                           int ncy, int ncz, void *stream)
{
    const int64_t n = 3 * (int64_t)ncx * ncy * ncz;
    const int blocks = (int)((n + 255) / 256);
    if (prec == ASD_FP64)
        hipLaunchKernelGGL(k_cells_from_mesh<double>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (double *)dst, src, src_nx, src_off, ncx, ncy, ncz);
    else
        hipLaunchKernelGGL(k_cells_from_mesh<float>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (float *)dst, src, src_nx, src_off, ncx, ncy, ncz);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------- reductions
// One block per grain walks the grain's site list (ascending site index),
// keeps the sites inside the window, accumulates in FP64 per thread, and
// reduces the block in a fixed tree order: deterministic, no atomics.
constexpr int kRedBlock = 1024;
constexpr int kRedUnroll = 4;  // sites per thread and pass (independent loads)

__device__ __forceinline__ bool site_in_window(const SysDev &d, int org, int32_t local)
{
    if (!d.track) return true;
    const uint32_t cell = d.kind == ASD_SC ? (uint32_t)local : ((uint32_t)local >> 1);
    const int32_t X = (int32_t)(cell % (uint32_t)d.sx);
    return X >= org && X < org + d.nx;
}

// One workgroup per grain.  Each pass covers kRedUnroll * kRedBlock sites of
// the grain's list: thread t takes sites t, t + kRedBlock, ... (coalesced),
// loads them all, then adds them in that order; the workgroup then sums its
// threads in a fixed tree.  The order depends only on the site list, so the
// FP64 result is the same in every run.
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_reduce_grains(RedArgs a)
{
    const int g = blockIdx.x;
    const int s = a.grain_sys[g];
    const SysDev d = a.sys[s];
    const int org = d.track ? a.origin[s] : 0;
    const T *S = (const T *)a.S;
    const int64_t k0 = a.grain_ptr[g], k1 = a.grain_ptr[g + 1];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t base = k0; base < k1; base += (int64_t)kRedUnroll * kRedBlock) {
        int32_t loc[kRedUnroll];
        bool ok[kRedUnroll];
#pragma unroll
        for (int j = 0; j < kRedUnroll; ++j) {
            const int64_t k = base + threadIdx.x + (int64_t)j * kRedBlock;
            ok[j] = k < k1;
            loc[j] = ok[j] ? a.grain_sites[k] : 0;
        }
        T v[kRedUnroll][3];
#pragma unroll
        for (int j = 0; j < kRedUnroll; ++j) {
            ok[j] = ok[j] && site_in_window(d, org, loc[j]);
            const int64_t i = d.base + loc[j];
            v[j][0] = ok[j] ? S[i] : T(0);
            v[j][1] = ok[j] ? S[a.ncs + i] : T(0);
            v[j][2] = ok[j] ? S[2 * a.ncs + i] : T(0);
        }
#pragma unroll
        for (int j = 0; j < kRedUnroll; ++j)
            if (ok[j]) {
                acc[0] += (double)v[j][0];
                acc[1] += (double)v[j][1];
                acc[2] += (double)v[j][2];
                acc[3] += 1.0;
            }
    }
    __shared__ double red[4][kRedBlock];
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int off = kRedBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) a.grain_out[4 * (int64_t)g + k] = red[k][0];
}

int launch_reduce_grains(const RedArgs &a, void *stream)
{
    if (a.n_grains == 0) return 0;
    if (a.prec == ASD_FP64)
        hipLaunchKernelGGL(k_reduce_grains<double>, dim3(a.n_grains), dim3(kRedBlock), 0,
                           (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(k_reduce_grains<float>, dim3(a.n_grains), dim3(kRedBlock), 0,
                           (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// per system: ordered sum over its grains; optional moment statistics of
// m = |M| / N: samples, sum m, sum m^2, sum m^4
__global__ void k_reduce_systems(RedArgs a, int moments, int reset)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_sys) return;
    const SysDev d = a.sys[s];
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = d.grain_base; g < d.grain_base + d.n_grains; ++g)
        for (int k = 0; k < 4; ++k) t[k] += a.grain_out[4 * (int64_t)g + k];
    for (int k = 0; k < 4; ++k) a.sys_out[4 * (int64_t)s + k] = t[k];
    if (moments) {
        double *mo = a.moments + 5 * (int64_t)s;
        if (reset)
            for (int k = 0; k < 5; ++k) mo[k] = 0.0;
        double m = t[3] > 0.0 ? sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]) / t[3] : 0.0;
        double m2 = m * m;
        mo[0] += 1.0;
        mo[1] += m;
        mo[2] += m2;
        mo[3] += m2 * m2;
    }
}

int launch_reduce_systems(const RedArgs &a, int moments, int reset, void *stream)
{
    if (a.n_sys == 0) return 0;
    hipLaunchKernelGGL(k_reduce_systems, dim3((a.n_sys + 63) / 64), dim3(64), 0,
                       (hipStream_t)stream, a, moments, reset);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void k_energy_finish(const double *partial, const SysDev *sys, int n_sys, double *out)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sys) return;
    const SysDev d = sys[s];
    double t[3] = {0.0, 0.0, 0.0};
    for (int b = d.tile_base; b < d.tile_base + d.n_tiles; ++b)
        for (int k = 0; k < 3; ++k) t[k] += partial[3 * (int64_t)b + k];
    for (int k = 0; k < 3; ++k) out[4 * (int64_t)s + k] = t[k];
    out[4 * (int64_t)s + 3] = (t[0] + t[1]) + t[2];
}

int launch_energy_finish(const double *partial, const SysDev *sys, int n_sys, double *sys_out,
                         void *stream)
{
    hipLaunchKernelGGL(k_energy_finish, dim3((n_sys + 63) / 64), dim3(64), 0, (hipStream_t)stream,
                       partial, sys, n_sys, sys_out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------- transfer
// Eq. 6 read forwards (Sec. II).  A workgroup takes kCgX consecutive coarse
// cells (i, j) of one layer k, i fastest (neighbouring cells along x, or
// along y when the columns hold fewer than kCgX cells, as a strip of one
// coarse column does); thread (tx, tz) sums, for its cell, the lattice rows
// tz, tz + kCgZ, ... of the cell (rows numbered y fastest, each row's sites
// contiguous), then thread tz = 0 adds the kCgZ partial sums in order: the
// same FP64 result every run.  Non-magnetic sites hold S = 0, so only the
// count looks at the label and the loads of a row do not wait on it.
constexpr int kCgX = 32, kCgZ = 8;

template <typename T>
__device__ __forceinline__ void coarse_grain_block(const TransferArgs &a, int bx, int by)
{
    const int tx = threadIdx.x % kCgX, tz = threadIdx.x / kCgX;
    const int ij = bx * kCgX + tx;  // cell i + ncx j of layer k
    const bool live = ij < a.ncx * a.ncy;
    const int j = ij / a.ncx, i = ij - j * a.ncx, k = by;
    const int jk = j + a.ncy * k;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (live) {
        const int xb = a.x0 + i * a.cx, yb = j * a.cy, zb = k * a.cz;
        const int wx = min(a.cx, a.x0 + a.ncols - xb), wy = min(a.cy, a.d.ny - yb),
                  wz = min(a.cz, a.d.nz - zb);
        const T *S = (const T *)a.S[0];
        const int nq = a.per * wx;
        for (int r = tz; r < wy * wz; r += kCgZ) {
            const int zz = r / wy, yy = r - zz * wy;
            const int64_t row =
                a.d.base + a.per * ((int64_t)xb + (int64_t)a.d.sx *
                                                      ((yb + yy) + (int64_t)a.d.ny * (zb + zz)));
            for (int q = 0; q < nq; ++q) {
                const int64_t g = row + q;
                acc[0] += (double)S[g];
                acc[1] += (double)S[a.ncs + g];
                acc[2] += (double)S[2 * a.ncs + g];
                acc[3] += a.label[g] != kNoGrain ? 1.0 : 0.0;
            }
        }
    }
    __shared__ double red[4][kCgZ][kCgX];
    for (int m = 0; m < 4; ++m) red[m][tz][tx] = acc[m];
    __syncthreads();
    if (tz == 0 && live) {
        const int64_t c = i + (int64_t)a.ncx * jk;
        for (int m = 0; m < 4; ++m) {
            double t = red[m][0][tx];
            for (int z = 1; z < kCgZ; ++z) t += red[m][z][tx];
            a.out[4 * c + m] = t;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kCgX * kCgZ) void k_coarse_grain(TransferArgs a)
{
    coarse_grain_block<T>(a, blockIdx.x, blockIdx.y);
}

// two strips of the same shape in one launch: blocks [0, gx) of a layer take
// strip a0, the others strip a1
template <typename T>
__global__ __launch_bounds__(kCgX * kCgZ) void k_coarse_grain_pair(TransferArgs a0, TransferArgs a1,
                                                                   int gx)
{
    if ((int)blockIdx.x < gx)
        coarse_grain_block<T>(a0, blockIdx.x, blockIdx.y);
    else
        coarse_grain_block<T>(a1, blockIdx.x - gx, blockIdx.y);
}

int launch_coarse_grain_pair(const TransferArgs &a0, const TransferArgs &a1, void *stream)
{
    if (a0.ncx != a1.ncx || a0.ncy != a1.ncy || a0.ncell != a1.ncell || a0.prec != a1.prec) return -1;
    if (a0.ncell == 0) return 0;
    const int gx = (a0.ncx * a0.ncy + kCgX - 1) / kCgX;
    const dim3 grid(2 * gx, a0.ncell / (a0.ncx * a0.ncy));
    if (a0.prec == ASD_FP64)
        hipLaunchKernelGGL(k_coarse_grain_pair<double>, grid, dim3(kCgX * kCgZ), 0,
                           (hipStream_t)stream, a0, a1, gx);
    else
        hipLaunchKernelGGL(k_coarse_grain_pair<float>, grid, dim3(kCgX * kCgZ), 0,
                           (hipStream_t)stream, a0, a1, gx);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_coarse_grain(const TransferArgs &a, void *stream)
{
    if (a.ncell == 0) return 0;
    const int ncz = a.ncell / (a.ncx * a.ncy);
    const dim3 grid((a.ncx * a.ncy + kCgX - 1) / kCgX, ncz);
    if (a.prec == ASD_FP64)
        hipLaunchKernelGGL(k_coarse_grain<double>, grid, dim3(kCgX * kCgZ), 0, (hipStream_t)stream,
                           a);
    else
        hipLaunchKernelGGL(k_coarse_grain<float>, grid, dim3(kCgX * kCgZ), 0, (hipStream_t)stream,
                           a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Widest cone of the inverse transfer (Sec. II), as printed: (5 pi / 9)
// sqrt(1 - sqrt(1 + 6 (m - 1) / 5)) with m clamped to [1/6, 1].
__device__ __forceinline__ double cone_theta_max(double m)
{
    if (m > 1.0) m = 1.0;
    if (m < 1.0 / 6.0) m = 1.0 / 6.0;
    double t = 1.0 + (6.0 * (m - 1.0)) / 5.0;
    if (t < 0.0) t = 0.0;
    return 1.7453292519943295 * sqrt(1.0 - sqrt(t));
}

// Eq. 6 read backwards (Sec. II): each magnetic site of the columns takes a
// spin in the cone around its coarse cell's reduced magnetisation m: polar
// angle uniform on [0, theta_max] (the printed reading), or cos theta
// uniform on [2 m - 1, 1] (the cap reading, whose mean cos theta is m);
// azimuth uniform, measured in the orthonormal basis of Duff et al. (JCGT
// 2017) around the cell direction.  FP64 throughout; both spin buffers
// receive the result.
template <typename T>
__device__ __forceinline__ void cone_column_site(const TransferArgs &a, int64_t t)
{
    const int64_t n = (int64_t)a.per * a.ncols * a.d.ny * a.d.nz;
    if (t >= n) return;
    const int s = (int)(t % a.per);
    int64_t r = t / a.per;
    const int xx = (int)(r % a.ncols);
    r /= a.ncols;
    const int y = (int)(r % a.d.ny), z = (int)(r / a.d.ny);
    const int64_t site = a.per * ((int64_t)(a.x0 + xx) + (int64_t)a.d.sx * (y + (int64_t)a.d.ny * z)) + s;
    const int64_t g = a.d.base + site;
    if (a.label[g] == kNoGrain) return;
    const int c = xx / a.cx + a.ncx * (y / a.cy + a.ncy * (z / a.cz));
    const double mx = a.mcell[3 * (int64_t)c], my = a.mcell[3 * (int64_t)c + 1],
                 mz = a.mcell[3 * (int64_t)c + 2];
    const double m = sqrt((mx * mx + my * my) + mz * mz);
    double nx = 0.0, ny = 0.0, nz = 1.0;
    if (m > 0.0) {
        nx = mx / m;
        ny = my / m;
        nz = mz / m;
    }
    if (a.exact) {  // the coarse cell's direction itself
        T *S0 = (T *)a.S[0], *S1 = (T *)a.S[1];
        const T v[3] = {(T)nx, (T)ny, (T)nz};
        for (int k = 0; k < 3; ++k) {
            S0[k * a.ncs + g] = v[k];
            S1[k * a.ncs + g] = v[k];
        }
        return;
    }
    const Words4 w = philox4x32(a.rounds, a.k0, a.k1, (uint32_t)site, a.step, a.d.sys_id, 1u);
    const double TWO_M32 = 2.3283064365386962890625e-10;
    const double u1 = ((double)w.w0 + 0.5) * TWO_M32;
    const double u2 = (double)w.w1 * TWO_M32;
    double st, ct, sp, cp;
    if (a.cap) {
        const double mc = m > 1.0 ? 1.0 : m;
        ct = 1.0 - u1 * (2.0 - 2.0 * mc);
        st = sqrt((1.0 - ct) * (1.0 + ct));
    } else {
        const double th = u1 * cone_theta_max(m);
        f64::sincos2pi(th / 6.283185307179586, st, ct);
    }
    f64::sincos2pi(u2, sp, cp);
    const double sg = nz >= 0.0 ? 1.0 : -1.0;
    const double aa = -1.0 / (sg + nz);
    const double b = (nx * ny) * aa;
    const double b1x = 1.0 + ((sg * nx) * nx) * aa, b1y = sg * b, b1z = -sg * nx;
    const double b2x = b, b2y = sg + (ny * ny) * aa, b2z = -ny;
    const double ex = st * cp, ey = st * sp;
    double vx = (ex * b1x + ey * b2x) + ct * nx;
    double vy = (ex * b1y + ey * b2y) + ct * ny;
    double vz = (ex * b1z + ey * b2z) + ct * nz;
    const double nn = sqrt((vx * vx + vy * vy) + vz * vz);
    vx = vx / nn;
    vy = vy / nn;
    vz = vz / nn;
    for (int b2 = 0; b2 < 2; ++b2) {
        T *S = (T *)a.S[b2];
        S[g] = (T)vx;
        S[a.ncs + g] = (T)vy;
        S[2 * a.ncs + g] = (T)vz;
    }
}

template <typename T>
__global__ void k_cone_columns(TransferArgs a)
{
    cone_column_site<T>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// two strips of the same shape in one launch: blocks [0, b0) take strip a0
template <typename T>
__global__ void k_cone_columns_pair(TransferArgs a0, TransferArgs a1, int b0)
{
    if ((int)blockIdx.x < b0)
        cone_column_site<T>(a0, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    else
        cone_column_site<T>(a1, (int64_t)(blockIdx.x - b0) * blockDim.x + threadIdx.x);
}

int launch_cone_columns_pair(const TransferArgs &a0, const TransferArgs &a1, void *stream)
{
    const int64_t n = (int64_t)a0.per * a0.ncols * a0.d.ny * a0.d.nz;
    if (n != (int64_t)a1.per * a1.ncols * a1.d.ny * a1.d.nz || a0.prec != a1.prec) return -1;
    if (n == 0) return 0;
    const int64_t b0 = (n + 255) / 256;
    if (2 * b0 > INT32_MAX) return -1;
    if (a0.prec == ASD_FP64)
        hipLaunchKernelGGL(k_cone_columns_pair<double>, dim3((unsigned)(2 * b0)), dim3(256), 0,
                           (hipStream_t)stream, a0, a1, (int)b0);
    else
        hipLaunchKernelGGL(k_cone_columns_pair<float>, dim3((unsigned)(2 * b0)), dim3(256), 0,
                           (hipStream_t)stream, a0, a1, (int)b0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cone_columns(const TransferArgs &a, void *stream)
{
    const int64_t n = (int64_t)a.per * a.ncols * a.d.ny * a.d.nz;
    if (n == 0) return 0;
    const int64_t blocks = (n + 255) / 256;
    if (a.prec == ASD_FP64)
        hipLaunchKernelGGL(k_cone_columns<double>, dim3((unsigned)blocks), dim3(256), 0,
                           (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(k_cone_columns<float>, dim3((unsigned)blocks), dim3(256), 0,
                           (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace asd
