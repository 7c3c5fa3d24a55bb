// asd_demag.hip -- demagnetising field of the window (Eq. 7) on the coarse
// cells of Eq. 6, by zero-padded FFT convolution with the spectrum of
// Newell's cell-averaged tensor.
//
// Per evaluation, for every system of the handle (grid y):
//   gather_x  one workgroup per (y, z) row of coarse cells: sum the spins of
//             each cell (non-magnetic sites hold 0), FFT the three component
//             rows along x (zero-padded to Px)
//   y pass    FFT along y of the ncz planes that hold data (zero-padded to Py)
//   z pass    per (kx, ky): FFT along z, multiply by the 3x3 tensor
//             spectrum, inverse FFT along z, keep the ncz planes of the mesh
//   y pass    inverse FFT along y, keep the ncy rows of the mesh
//   x_out     inverse FFT along x, keep the ncx cells: the field per cell
// The spectrum carries -mu0 mu_s / (V Px Py Pz), so the result is the flux
// density mu0 H_d in tesla from plain spin sums.  Every transform is a
// radix-2 Stockham FFT over a batch of lines held in LDS (ping-pong
// buffers), one barrier per stage; the padded sizes are powers of two.
#include <hip/hip_runtime.h>

#include "asd.h"
#include "asd_device.h"
#include "asd_internal.h"

namespace asd {

namespace {

constexpr int kDmThreads = 256;

template <typename T>
struct Cx {
    T re, im;
};

// Stockham radix-2 over nl lines of length P = 2^lp stored line-major in
// x; y is the second buffer.  Stage s combines pairs (j, j + P/2) with the
// twiddle of index k = j mod 2^s and writes them to (j / 2^s) 2^(s+1) + k
// and + 2^s, which leaves the output in natural order.  Returns the buffer
// holding the result.  Callers synchronise before; the routine ends with a
// barrier.
template <typename T, bool INV>
__device__ Cx<T> *fft_lines(Cx<T> *x, Cx<T> *y, int nl, int lp, const Cx<T> *__restrict__ tw)
{
    if (lp == 0) return x;
    const int P = 1 << lp, half = P >> 1;
    const int nb = nl * half;
    for (int s = 0; s < lp; ++s) {
        const int Ns = 1 << s;
        for (int q = threadIdx.x; q < nb; q += blockDim.x) {
            const int line = q >> (lp - 1);
            const int j = q & (half - 1);
            const int k = j & (Ns - 1);
            Cx<T> w = tw[k << (lp - 1 - s)];
            if (INV) w.im = -w.im;
            const Cx<T> *xs = x + line * P;
            const Cx<T> a = xs[j], b = xs[j + half];
            const T br = b.re * w.re - b.im * w.im, bi = b.re * w.im + b.im * w.re;
            Cx<T> *yd = y + line * P + ((j >> s) << (s + 1)) + k;
            yd[0] = Cx<T>{a.re + br, a.im + bi};
            yd[Ns] = Cx<T>{a.re - br, a.im - bi};
        }
        __syncthreads();
        Cx<T> *t = x;
        x = y;
        y = t;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ Cx<T> *lds_base()
{
    extern __shared__ __align__(16) unsigned char dm_lds[];
    return (Cx<T> *)dm_lds;
}

// --- 1: cell sums of one (y, z) row of coarse cells, FFT along x
template <typename T>
__global__ __launch_bounds__(kDmThreads) void k_dm_gather_x(DemagDev dm, const T *__restrict__ S,
                                                            int64_t ncs, const SysDev *sys,
                                                            const int32_t *origin)
{
    const int Px = 1 << dm.lx;
    const int j = blockIdx.x % dm.ncy, k = blockIdx.x / dm.ncy, s = blockIdx.y;
    const SysDev d = sys[s];
    const int org = d.track ? origin[s] : 0;
    const int per = d.kind == ASD_SC ? 1 : 2;
    Cx<T> *x = lds_base<T>(), *y = x + 3 * Px;
    for (int q = threadIdx.x; q < 3 * Px; q += blockDim.x) x[q] = Cx<T>{T(0), T(0)};
    __syncthreads();
    const int yb = j * dm.cy, zb = k * dm.cz;
    const int wy = min(dm.cy, d.ny - yb), wz = min(dm.cz, d.nz - zb);
    for (int i = threadIdx.x; i < dm.ncx; i += blockDim.x) {
        const int xb = i * dm.cx;
        const int nq = per * min(dm.cx, d.nx - xb);
        T ax = T(0), ay = T(0), az = T(0);
        for (int zz = 0; zz < wz; ++zz)
            for (int yy = 0; yy < wy; ++yy) {
                const int64_t row =
                    d.base + per * ((int64_t)(org + xb) +
                                    (int64_t)d.sx * ((yb + yy) + (int64_t)d.ny * (zb + zz)));
                for (int q = 0; q < nq; ++q) {
                    ax += S[row + q];
                    ay += S[ncs + row + q];
                    az += S[2 * ncs + row + q];
                }
            }
        x[i].re = ax;
        x[Px + i].re = ay;
        x[2 * Px + i].re = az;
    }
    __syncthreads();
    const Cx<T> *r = fft_lines<T, false>(x, y, 3, dm.lx, (const Cx<T> *)dm.tw[0]);
    Cx<T> *out = (Cx<T> *)dm.wx;
    for (int q = threadIdx.x; q < 3 * Px; q += blockDim.x) {
        const int c = q >> dm.lx, kx = q & (Px - 1);
        out[((((int64_t)s * 3 + c) * dm.ncz + k) * dm.ncy + j) * Px + kx] = r[q];
    }
}

// --- 2 / 4: FFT along y of xb_y neighbouring x lines of one (c, z) plane.
// Forward: rows y < ncy of wx (zero-padded) -> all Py rows of wy.
// Inverse: all Py rows of wy -> rows y < ncy of wx.
template <typename T, bool INV>
__global__ __launch_bounds__(kDmThreads) void k_dm_y(DemagDev dm)
{
    const int Px = 1 << dm.lx, Py = 1 << dm.ly;
    const int XB = dm.xb_y, lxb = __ffs(XB) - 1;
    const int kx0 = blockIdx.x * XB;
    const int plane = blockIdx.y;  // c * ncz + z
    const int s = blockIdx.z;
    const Cx<T> *src = (const Cx<T> *)(INV ? dm.wy : dm.wx);
    Cx<T> *dst = (Cx<T> *)(INV ? dm.wx : dm.wy);
    const int rows_in = INV ? Py : dm.ncy, rows_out = INV ? dm.ncy : Py;
    const int64_t pin = ((int64_t)s * 3 * dm.ncz + plane) * rows_in * Px;
    const int64_t pout = ((int64_t)s * 3 * dm.ncz + plane) * rows_out * Px;
    Cx<T> *x = lds_base<T>(), *y = x + XB * Py;
    for (int q = threadIdx.x; q < XB * Py; q += blockDim.x) {
        const int yy = q >> lxb, xb = q & (XB - 1);
        x[xb * Py + yy] = yy < rows_in ? src[pin + (int64_t)yy * Px + kx0 + xb] : Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    const Cx<T> *r = fft_lines<T, INV>(x, y, XB, dm.ly, (const Cx<T> *)dm.tw[1]);
    for (int q = threadIdx.x; q < rows_out * XB; q += blockDim.x) {
        const int yy = q >> lxb, xb = q & (XB - 1);
        dst[pout + (int64_t)yy * Px + kx0 + xb] = r[xb * Py + yy];
    }
}

// --- 3: per (kx, ky) column: FFT along z, tensor product, inverse FFT
template <typename T>
__global__ __launch_bounds__(kDmThreads) void k_dm_z(DemagDev dm)
{
    const int Px = 1 << dm.lx, Py = 1 << dm.ly, Pz = 1 << dm.lz;
    const int XB = dm.xb_z;
    const int kx0 = blockIdx.x * XB, ky = blockIdx.y, s = blockIdx.z;
    Cx<T> *w = (Cx<T> *)dm.wy;
    const int64_t cstride = (int64_t)dm.ncz * Py * Px;  // component stride in wy
    const int64_t base = (int64_t)s * 3 * cstride + (int64_t)ky * Px + kx0;
    const int n = 3 * XB * Pz;
    Cx<T> *x = lds_base<T>(), *y = x + n;
    // line (c, xb) holds z = 0 .. Pz-1 of component c at kx0 + xb
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int z = q / (3 * XB), cxb = q - z * 3 * XB;
        const int c = cxb / XB, xb = cxb - c * XB;
        x[cxb * Pz + z] = z < dm.ncz ? w[base + c * cstride + (int64_t)z * Py * Px + xb]
                                     : Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    Cx<T> *r = fft_lines<T, false>(x, y, 3 * XB, dm.lz, (const Cx<T> *)dm.tw[2]);
    // tensor octant: components even in every wavenumber, or odd in the two
    // that appear in their name
    const int ox = (Px >> 1) + 1, oy = (Py >> 1) + 1, oz = (Pz >> 1) + 1;
    const int64_t ocomp = (int64_t)ox * oy * oz;
    const T *K = (const T *)dm.K;
    const int kyr = ky <= (Py >> 1) ? ky : Py - ky;
    const T sy = ky <= (Py >> 1) ? T(1) : T(-1);
    for (int q = threadIdx.x; q < XB * Pz; q += blockDim.x) {
        const int xb = q / Pz, kz = q - xb * Pz;
        const int kx = kx0 + xb;
        const int kxr = kx <= (Px >> 1) ? kx : Px - kx;
        const int kzr = kz <= (Pz >> 1) ? kz : Pz - kz;
        const T sx = kx <= (Px >> 1) ? T(1) : T(-1);
        const T sz = kz <= (Pz >> 1) ? T(1) : T(-1);
        const int64_t o = ((int64_t)kzr * oy + kyr) * ox + kxr;
        const T nxx = K[o], nyy = K[ocomp + o], nzz = K[2 * ocomp + o];
        const T nxy = sx * sy * K[3 * ocomp + o], nxz = sx * sz * K[4 * ocomp + o],
                nyz = sy * sz * K[5 * ocomp + o];
        Cx<T> *px = r + (0 * XB + xb) * Pz + kz;
        Cx<T> *py = r + (1 * XB + xb) * Pz + kz;
        Cx<T> *pz = r + (2 * XB + xb) * Pz + kz;
        const Cx<T> mx = *px, my = *py, mz = *pz;
        *px = Cx<T>{(nxx * mx.re + nxy * my.re) + nxz * mz.re, (nxx * mx.im + nxy * my.im) + nxz * mz.im};
        *py = Cx<T>{(nxy * mx.re + nyy * my.re) + nyz * mz.re, (nxy * mx.im + nyy * my.im) + nyz * mz.im};
        *pz = Cx<T>{(nxz * mx.re + nyz * my.re) + nzz * mz.re, (nxz * mx.im + nyz * my.im) + nzz * mz.im};
    }
    __syncthreads();
    Cx<T> *other = r == x ? y : x;
    const Cx<T> *h = fft_lines<T, true>(r, other, 3 * XB, dm.lz, (const Cx<T> *)dm.tw[2]);
    for (int q = threadIdx.x; q < 3 * XB * dm.ncz; q += blockDim.x) {
        const int z = q / (3 * XB), cxb = q - z * 3 * XB;
        const int c = cxb / XB, xb = cxb - c * XB;
        w[base + c * cstride + (int64_t)z * Py * Px + xb] = h[cxb * Pz + z];
    }
}

// --- 5: inverse FFT along x of one (y, z) row, the field of its ncx cells
template <typename T>
__global__ __launch_bounds__(kDmThreads) void k_dm_x_out(DemagDev dm, int stage)
{
    const int Px = 1 << dm.lx;
    const int j = blockIdx.x % dm.ncy, k = blockIdx.x / dm.ncy, s = blockIdx.y;
    const Cx<T> *in = (const Cx<T> *)dm.wx;
    Cx<T> *x = lds_base<T>(), *y = x + 3 * Px;
    for (int q = threadIdx.x; q < 3 * Px; q += blockDim.x) {
        const int c = q >> dm.lx, kx = q & (Px - 1);
        x[q] = in[((((int64_t)s * 3 + c) * dm.ncz + k) * dm.ncy + j) * Px + kx];
    }
    __syncthreads();
    const Cx<T> *r = fft_lines<T, true>(x, y, 3, dm.lx, (const Cx<T> *)dm.tw[0]);
    T *bd = (T *)dm.bd[stage];
    const int64_t cell0 = (int64_t)dm.ncx * (j + (int64_t)dm.ncy * k);
    for (int q = threadIdx.x; q < 3 * dm.ncx; q += blockDim.x) {
        const int c = q / dm.ncx, i = q - c * dm.ncx;
        bd[((int64_t)s * 3 + c) * dm.ncell + cell0 + i] = r[c * Px + i].re;
    }
}

template <typename T>
int run_demag(const DemagDev &dm, const T *S, int64_t ncs, const SysDev *sys,
                 const int32_t *origin, int stage, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const int Px = 1 << dm.lx, Py = 1 << dm.ly, Pz = 1 << dm.lz;
    const size_t cb = sizeof(Cx<T>);
    const dim3 blk(kDmThreads);
    const dim3 grows(dm.ncy * dm.ncz, dm.n_sys);
    hipLaunchKernelGGL(k_dm_gather_x<T>, grows, blk, 2 * 3 * Px * cb, st, dm, S, ncs, sys, origin);
    const dim3 gy(Px / dm.xb_y, 3 * dm.ncz, dm.n_sys);
    hipLaunchKernelGGL((k_dm_y<T, false>), gy, blk, 2 * dm.xb_y * Py * cb, st, dm);
    const dim3 gz(Px / dm.xb_z, Py, dm.n_sys);
    hipLaunchKernelGGL(k_dm_z<T>, gz, blk, 2 * 3 * dm.xb_z * Pz * cb, st, dm);
    hipLaunchKernelGGL((k_dm_y<T, true>), gy, blk, 2 * dm.xb_y * Py * cb, st, dm);
    hipLaunchKernelGGL(k_dm_x_out<T>, grows, blk, 2 * 3 * Px * cb, st, dm, stage);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int launch_demag_f64(const DemagDev &dm, const double *S, int64_t ncs, const SysDev *sys,
                     const int32_t *origin, int stage, void *stream)
{
    return run_demag<double>(dm, S, ncs, sys, origin, stage, stream);
}

int launch_demag_f32(const DemagDev &dm, const float *S, int64_t ncs, const SysDev *sys,
                     const int32_t *origin, int stage, void *stream)
{
    return run_demag<float>(dm, S, ncs, sys, origin, stage, stream);
}

}  // namespace asd
