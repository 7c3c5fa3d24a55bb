// asd_demag.hip -- demagnetising field of the window (Eq. 7) on the coarse
// cells of Eq. 6, by zero-padded FFT convolution with the spectrum of
// Newell's cell-averaged tensor.
//
// Per evaluation, for every system of the handle:
//   gather_x  one workgroup per (y, z) row of coarse cells: sum the spins of
//             each cell (non-magnetic sites hold 0), FFT the three component
//             rows along x (zero-padded to Px); or cells_x: the same from
//             cell sums the step kernels formed
//   yz        (ncz <= 16, 12 in FP64) one workgroup per kx column: FFT along
//             y, the convolution along z as direct sums over the planes with
//             the tensor transformed along x and y only, inverse FFT along y;
//   or, for thicker meshes, three passes:
//     y pass  FFT along y of the ncz planes that hold data (zero-padded to Py)
//     z pass  per (kx, ky): FFT along z, multiply by the 3x3 tensor
//             spectrum, inverse FFT along z, keep the ncz planes of the mesh
//     y pass  inverse FFT along y, keep the ncy rows of the mesh
//   x_out     inverse FFT along x, keep the ncx cells: the field per cell
// The x transform of the real cell sums is Hermitian, X(Px - k) = conj X(k),
// so only kx = 0 .. Px/2 (Pxh columns) is kept through the y and z passes and
// the full row is rebuilt before the inverse x transform.
// The spectrum carries -mu0 mu_s / (V Px Py Pz) (the mixed table of the yz
// pass -mu0 mu_s / (V Px Py)), so the result is the flux density mu0 H_d in
// tesla from plain spin sums.  Every transform is a
// Stockham FFT over a batch of lines held in LDS (ping-pong buffers): radix-4
// stages, after one radix-2 stage when log2 of the length is odd, one barrier
// per stage; the padded sizes are powers of two.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// twiddle exp(-+2 pi i t / P) for t < P from the half table tw (t < P/2)
template <typename T, bool INV>
__device__ __forceinline__ Cx<T> twiddle(const Cx<T> *__restrict__ tw, int t, int half)
{
    Cx<T> w = t < half ? tw[t] : Cx<T>{-tw[t - half].re, -tw[t - half].im};
    if (INV) w.im = -w.im;
    return w;
}

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b)
{
    return Cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// Stockham autosort FFT over nl lines of length P = 2^lp, line l at
// x + l * ls (ls >= P; an odd stride spreads lines written across lanes
// over the LDS banks); y is the second buffer.  With Ns the length of the
// sub-transforms done so far, a radix-R stage takes the R points
// j + r P/R (j < P/R), twiddles point r by exp(-2 pi i r k / (R Ns)) with
// k = j mod Ns, does an R-point DFT and writes output r to
// (j / Ns) R Ns + k + r Ns; the output ends in natural order.  One radix-2
// stage when lp is odd, radix-4 stages after it.  Returns the buffer
// holding the result.  Callers synchronise before; every stage ends with a
// barrier.  Between stages of lines of 64 points or more, point e of a line
// sits at e ^ ((e >> 2) & 31): the stages' strided writes (a lane's points
// 4 Ns apart) then fall on distinct LDS banks; the first stage reads and the
// last one writes the natural order, so callers never see the permutation.
__device__ __forceinline__ int fft_swz(int e, bool on) { return on ? e ^ ((e >> 2) & 31) : e; }

template <typename T, bool INV>
__device__ Cx<T> *fft_lines(Cx<T> *x, Cx<T> *y, int nl, int lp, int ls,
                            const Cx<T> *__restrict__ tw)
{
    if (lp == 0) return x;
    const int P = 1 << lp, half = P >> 1;
    const bool sw = lp >= 6;
    int Ns = 1;
    if (lp & 1) {
        const bool wsw = sw && lp > 1;
        for (int q = threadIdx.x; q < nl * half; q += blockDim.x) {
            const int line = q >> (lp - 1), j = q & (half - 1);
            const Cx<T> a = x[line * ls + j], b = x[line * ls + j + half];
            Cx<T> *yd = y + line * ls;
            yd[fft_swz(2 * j, wsw)] = Cx<T>{a.re + b.re, a.im + b.im};
            yd[fft_swz(2 * j + 1, wsw)] = Cx<T>{a.re - b.re, a.im - b.im};
        }
        __syncthreads();
        Cx<T> *t = x;
        x = y;
        y = t;
        Ns = 2;
    }
    const int quarter = P >> 2;
    for (; Ns < P; Ns <<= 2) {
        const int lns = __ffs(Ns) - 1;
        const int tstep = lp - 2 - lns;  // log2 of P / (4 Ns)
        const bool rsw = sw && Ns > 1, wsw = sw && 4 * Ns < P;
        for (int q = threadIdx.x; q < nl * quarter; q += blockDim.x) {
            const int line = q >> (lp - 2), j = q & (quarter - 1);
            const int k = j & (Ns - 1);
            const Cx<T> *xs = x + line * ls;
            const Cx<T> v0 = xs[fft_swz(j, rsw)];
            const Cx<T> v1 = cmul(xs[fft_swz(j + quarter, rsw)], twiddle<T, INV>(tw, k << tstep, half));
            const Cx<T> v2 =
                cmul(xs[fft_swz(j + 2 * quarter, rsw)], twiddle<T, INV>(tw, (2 * k) << tstep, half));
            const Cx<T> v3 =
                cmul(xs[fft_swz(j + 3 * quarter, rsw)], twiddle<T, INV>(tw, (3 * k) << tstep, half));
            const Cx<T> a0{v0.re + v2.re, v0.im + v2.im}, a1{v0.re - v2.re, v0.im - v2.im};
            const Cx<T> a2{v1.re + v3.re, v1.im + v3.im};
            const T dr = v1.re - v3.re, di = v1.im - v3.im;
            // (v1 - v3) times -i (forward) or +i (inverse)
            const Cx<T> a3 = INV ? Cx<T>{-di, dr} : Cx<T>{di, -dr};
            Cx<T> *yd = y + line * ls;
            const int e = ((j >> lns) << (lns + 2)) + k;
            yd[fft_swz(e, wsw)] = Cx<T>{a0.re + a2.re, a0.im + a2.im};
            yd[fft_swz(e + Ns, wsw)] = Cx<T>{a1.re + a3.re, a1.im + a3.im};
            yd[fft_swz(e + 2 * Ns, wsw)] = Cx<T>{a0.re - a2.re, a0.im - a2.im};
            yd[fft_swz(e + 3 * Ns, wsw)] = Cx<T>{a1.re - a3.re, a1.im - a3.im};
        }
        __syncthreads();
        Cx<T> *t = x;
        x = y;
        y = t;
    }
    return x;
}

// position of component c, plane k, row j, column kx of system s in wx
__device__ __forceinline__ int64_t wx_at(const DemagDev &dm, int s, int c, int k, int j, int kx,
                                         int Pxh)
{
    return ((((int64_t)s * 3 + c) * dm.ncz + k) * dm.ncy + j) * Pxh + kx;
}

template <typename T>
__device__ __forceinline__ Cx<T> *lds_base()
{
    extern __shared__ __align__(16) unsigned char dm_lds[];
    return (Cx<T> *)dm_lds;
}

// --- 1: cell sums of one (y, z) row of coarse cells, FFT along x.
// Thread t takes cell i = t mod ncx and the lattice rows g, g + G, ... of that
// cell (g = t / ncx, G = 256 / ncx row groups), so neighbouring lanes read
// neighbouring cells of one lattice row; the G partial sums of a cell are
// then added in group order.
template <typename T>
__global__ __launch_bounds__(kDmThreads) void k_dm_gather_x(DemagDev dm, const T *__restrict__ S,
                                                            int64_t ncs, const SysDev *sys,
                                                            const int32_t *origin)
{
    __shared__ T part[3][kDmThreads];
    const int Px = 1 << dm.lx;
    const int j = blockIdx.x % dm.ncy, k = blockIdx.x / dm.ncy, s = blockIdx.y;
    const SysDev d = sys[s];
    const int org = d.track ? origin[s] : 0;
    const int per = d.kind == ASD_SC ? 1 : 2;
    Cx<T> *x = lds_base<T>(), *y = x + 3 * Px;
    for (int q = threadIdx.x; q < 3 * Px; q += blockDim.x) x[q] = Cx<T>{T(0), T(0)};
    const int yb = j * dm.cy, zb = k * dm.cz;
    const int wy = min(dm.cy, d.ny - yb), wz = min(dm.cz, d.nz - zb);
    const int G = kDmThreads / dm.ncx;  // ncx <= 256
    const int i = threadIdx.x % dm.ncx, g = threadIdx.x / dm.ncx;
    T ax = T(0), ay = T(0), az = T(0);
    // window-frame columns [lo, hi) of cell i that hold sources
    int lo = i * dm.cx, hi = min(lo + dm.cx, d.nx);
    if (dm.stray) {
        lo = (i - (org + dm.cx - 1) / dm.cx) * dm.cx;
        hi = min(lo + dm.cx, d.sx - org);
        if (lo >= 0 && lo < d.nx) lo = d.nx;  // a window cell: only its columns past the window
        lo = max(lo, -org);
    }
    if (g < G && lo < hi) {
        const int nq = per * (hi - lo);
        for (int r = g; r < wy * wz; r += G) {
            const int zz = r / wy, yy = r - zz * wy;
            const int64_t row = d.base + per * ((int64_t)(org + lo) +
                                                (int64_t)d.sx * ((yb + yy) + (int64_t)d.ny * (zb + zz)));
            for (int q = 0; q < nq; ++q) {
                ax += S[row + q];
                ay += S[ncs + row + q];
                az += S[2 * ncs + row + q];
            }
        }
    }
    part[0][threadIdx.x] = ax;
    part[1][threadIdx.x] = ay;
    part[2][threadIdx.x] = az;
    __syncthreads();
    if (threadIdx.x < dm.ncx) {
        T sx = part[0][threadIdx.x], sy = part[1][threadIdx.x], sz = part[2][threadIdx.x];
        for (int gg = 1; gg < G; ++gg) {
            sx += part[0][gg * dm.ncx + threadIdx.x];
            sy += part[1][gg * dm.ncx + threadIdx.x];
            sz += part[2][gg * dm.ncx + threadIdx.x];
        }
        x[threadIdx.x].re = sx;
        x[Px + threadIdx.x].re = sy;
        x[2 * Px + threadIdx.x].re = sz;
    }
    __syncthreads();
    const Cx<T> *r = fft_lines<T, false>(x, y, 3, dm.lx, Px, (const Cx<T> *)dm.tw[0]);
    Cx<T> *out = (Cx<T> *)dm.wx;
    const int Pxh = (Px >> 1) + 1;
    for (int q = threadIdx.x; q < 3 * Pxh; q += blockDim.x) {
        const int c = q / Pxh, kx = q - c * Pxh;
        out[wx_at(dm, s, c, k, j, kx, Pxh)] = r[c * Px + kx];
    }
}

// --- 1': the same from given cell sums: src [S][3][ns][ncell] (cells x
// fastest, in units of the spin sums of a coarse cell; ns partial sums per
// cell, 1 when dm.ns is 0); FFT along x
template <typename T, typename U>
__global__ __launch_bounds__(kDmThreads) void k_dm_cells_x(DemagDev dm, const U *__restrict__ src)
{
    const int Px = 1 << dm.lx;
    const int j = blockIdx.x % dm.ncy, k = blockIdx.x / dm.ncy, s = blockIdx.y;
    Cx<T> *x = lds_base<T>(), *y = x + 3 * Px;
    const int ns = max(dm.ns, 1);  // partial sums per cell, added in slot order
    for (int q = threadIdx.x; q < 3 * Px; q += blockDim.x) {
        const int c = q >> dm.lx, i = q & (Px - 1);
        const int64_t cell = i + (int64_t)dm.ncx * (j + (int64_t)dm.ncy * k);
        T v = T(0);
        if (i < dm.ncx) {
            const U *p = src + ((int64_t)s * 3 + c) * ns * dm.ncell + cell;
            v = (T)p[0];
            for (int sl = 1; sl < ns; ++sl) v = v + (T)p[(int64_t)sl * dm.ncell];
        }
        x[q] = Cx<T>{v, T(0)};
    }
    __syncthreads();
    const Cx<T> *r = fft_lines<T, false>(x, y, 3, dm.lx, Px, (const Cx<T> *)dm.tw[0]);
    Cx<T> *out = (Cx<T> *)dm.wx;
    const int Pxh = (Px >> 1) + 1;
    for (int q = threadIdx.x; q < 3 * Pxh; q += blockDim.x) {
        const int c = q / Pxh, kx = q - c * Pxh;
        out[wx_at(dm, s, c, k, j, kx, Pxh)] = r[c * Px + kx];
    }
}

// --- 2 / 4: FFT along y of xb_y neighbouring x lines of one (c, z) plane.
// Forward: rows y < ncy of wx (zero-padded) -> all Py rows of wy.
// Inverse: all Py rows of wy -> rows y < ncy of wx.
template <typename T, bool INV>
__global__ __launch_bounds__(kDmThreads) void k_dm_y(DemagDev dm)
{
    const int Px = ((1 << dm.lx) >> 1) + 1, Py = 1 << dm.ly;  // Px: the kept columns
    const int XB = dm.xb_y, lxb = __ffs(XB) - 1;
    const int kx0 = blockIdx.x * XB;
    const int plane = blockIdx.y;  // c * ncz + z
    const int s = blockIdx.z;
    const Cx<T> *src = (const Cx<T> *)(INV ? dm.wy : dm.wx);
    Cx<T> *dst = (Cx<T> *)(INV ? dm.wx : dm.wy);
    const int rows_in = INV ? Py : dm.ncy, rows_out = INV ? dm.ncy : Py;
    const int64_t pin = ((int64_t)s * 3 * dm.ncz + plane) * rows_in * Px;
    const int64_t pout = ((int64_t)s * 3 * dm.ncz + plane) * rows_out * Px;
    const int ls = Py + 1;  // odd line stride: the transposed writes spread over the banks
    Cx<T> *x = lds_base<T>(), *y = x + XB * ls;
    for (int q = threadIdx.x; q < XB * Py; q += blockDim.x) {
        const int yy = q >> lxb, xb = q & (XB - 1);
        x[xb * ls + yy] = yy < rows_in && kx0 + xb < Px ? src[pin + (int64_t)yy * Px + kx0 + xb]
                                                        : Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    const Cx<T> *r = fft_lines<T, INV>(x, y, XB, dm.ly, ls, (const Cx<T> *)dm.tw[1]);
    for (int q = threadIdx.x; q < rows_out * XB; q += blockDim.x) {
        const int yy = q >> lxb, xb = q & (XB - 1);
        if (kx0 + xb < Px) dst[pout + (int64_t)yy * Px + kx0 + xb] = r[xb * ls + yy];
    }
}

// --- 3: per (kx, ky) column: FFT along z, tensor product, inverse FFT.
// Line (c, xb) holds z = 0 .. Pz-1 of component c at kx0 + xb, stride Pz + 1.
template <typename T>
__global__ __launch_bounds__(kDmThreads) void k_dm_z(DemagDev dm)
{
    const int Px = 1 << dm.lx, Py = 1 << dm.ly, Pz = 1 << dm.lz;
    const int Pxh = (Px >> 1) + 1;  // kept columns kx = 0 .. Px/2
    const int XB = dm.xb_z, lxb = __ffs(XB) - 1;
    const int kx0 = blockIdx.x * XB, ky = blockIdx.y, s = blockIdx.z;
    Cx<T> *w = (Cx<T> *)dm.wy;
    const int64_t plane = (int64_t)Py * Pxh;
    const int64_t cstride = (int64_t)dm.ncz * plane;  // component stride in wy
    const int64_t base = (int64_t)s * 3 * cstride + (int64_t)ky * Pxh + kx0;
    const int ls = Pz + 1;
    const int nl = 3 * XB;
    Cx<T> *x = lds_base<T>(), *y = x + nl * ls;
    // rows (c, z) of XB neighbouring kx: lanes read along kx
    for (int q = threadIdx.x; q < 3 * Pz * XB; q += blockDim.x) {
        const int xb = q & (XB - 1), row = q >> lxb;
        const int c = row >> dm.lz, z = row & (Pz - 1);
        x[(c * XB + xb) * ls + z] = z < dm.ncz && kx0 + xb < Pxh
                                        ? w[base + c * cstride + z * plane + xb]
                                        : Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    Cx<T> *r = fft_lines<T, false>(x, y, nl, dm.lz, ls, (const Cx<T> *)dm.tw[2]);
    // tensor spectrum octant [6][Py/2+1][Px/2+1][Pz/2+1] (kz fastest): the
    // components are even in every wavenumber, or odd in the two named ones
    const int ox = (Px >> 1) + 1, oy = (Py >> 1) + 1, oz = (Pz >> 1) + 1;
    const int64_t ocomp = (int64_t)ox * oy * oz;
    const T *K = (const T *)dm.K;
    const int kyr = ky <= (Py >> 1) ? ky : Py - ky;
    const T sy = ky <= (Py >> 1) ? T(1) : T(-1);
    for (int q = threadIdx.x; q < XB * Pz; q += blockDim.x) {
        const int kz = q & (Pz - 1), xb = q >> dm.lz;
        const int kx = min(kx0 + xb, Px >> 1);  // columns past Px/2 are never stored
        const int kxr = kx;
        const int kzr = kz <= (Pz >> 1) ? kz : Pz - kz;
        const T sx = T(1);
        const T sz = kz <= (Pz >> 1) ? T(1) : T(-1);
        const int64_t o = ((int64_t)kyr * ox + kxr) * oz + kzr;
        const T nxx = K[o], nyy = K[ocomp + o], nzz = K[2 * ocomp + o];
        const T nxy = sx * sy * K[3 * ocomp + o], nxz = sx * sz * K[4 * ocomp + o],
                nyz = sy * sz * K[5 * ocomp + o];
        Cx<T> *px = r + (0 * XB + xb) * ls + kz;
        Cx<T> *py = r + (1 * XB + xb) * ls + kz;
        Cx<T> *pz = r + (2 * XB + xb) * ls + kz;
        const Cx<T> mx = *px, my = *py, mz = *pz;
        *px = Cx<T>{(nxx * mx.re + nxy * my.re) + nxz * mz.re, (nxx * mx.im + nxy * my.im) + nxz * mz.im};
        *py = Cx<T>{(nxy * mx.re + nyy * my.re) + nyz * mz.re, (nxy * mx.im + nyy * my.im) + nyz * mz.im};
        *pz = Cx<T>{(nxz * mx.re + nyz * my.re) + nzz * mz.re, (nxz * mx.im + nyz * my.im) + nzz * mz.im};
    }
    __syncthreads();
    Cx<T> *other = r == x ? y : x;
    const Cx<T> *h = fft_lines<T, true>(r, other, nl, dm.lz, ls, (const Cx<T> *)dm.tw[2]);
    for (int q = threadIdx.x; q < 3 * Pz * XB; q += blockDim.x) {
        const int xb = q & (XB - 1), row = q >> lxb;
        const int c = row >> dm.lz, z = row & (Pz - 1);
        if (z < dm.ncz && kx0 + xb < Pxh) w[base + c * cstride + z * plane + xb] = h[(c * XB + xb) * ls + z];
    }
}

// --- 2-4 in one workgroup per (kx, system) when yzf: the 3 NCZ rows of
// column kx into LDS; FFT along y; per ky the field planes
// as direct sums over the source planes with the tensor transformed along x
// and y only, so the convolution along z needs neither padding nor
// transforms; inverse FFT along y; the ncy rows back.  Lanes: four groups of
// Py, group q computing the planes q, q + 4, ... (wavefront-uniform, so the
// unrolled sums need no divergent branches).
constexpr int kDmYzThreads = 512;

// one output component of the planes z = Q0, Q0 + 4, ... of one ky:
// H_c(z) = sum_zs [A(z - zs) Mx + B(z - zs) My + C(z - zs) Mz] with the three
// tensor components of row c (A, B, C; IA/IB/IC: the component is the
// imaginary one, odd in dz)
template <typename T, int NCZ, int Q0, bool IA, bool IB, bool IC>
__device__ __forceinline__ void yz_row(const T *__restrict__ ka, const T *__restrict__ kb,
                                       const T *__restrict__ kc, T sa, T sb, T sc, int oy,
                                       const Cx<T> (&m)[3][NCZ], Cx<T> *__restrict__ o, int ls,
                                       int ky, int c)
{
    constexpr int Q = 4;
    T ta[NCZ], tb[NCZ], tc[NCZ];
#pragma unroll
    for (int d = 0; d < NCZ; ++d) {
        ta[d] = sa * ka[d * (int64_t)oy];
        tb[d] = sb * kb[d * (int64_t)oy];
        tc[d] = sc * kc[d * (int64_t)oy];
    }
#pragma unroll
    for (int z = Q0; z < NCZ; z += Q) {
        T hr = T(0), hi = T(0);
#pragma unroll
        for (int zs = 0; zs < NCZ; ++zs) {
            const int d = z - zs, ad = d < 0 ? -d : d;
            const T sg = d < 0 ? T(-1) : T(1);
            // a real component adds t m; an imaginary one (i t, odd in dz) adds i sg t m
            const T A = IA ? sg * ta[ad] : ta[ad], Bv = IB ? sg * tb[ad] : tb[ad],
                    Cv = IC ? sg * tc[ad] : tc[ad];
            hr = hr + ((IA ? -A * m[0][zs].im : A * m[0][zs].re) +
                       (IB ? -Bv * m[1][zs].im : Bv * m[1][zs].re)) +
                 (IC ? -Cv * m[2][zs].im : Cv * m[2][zs].re);
            hi = hi + ((IA ? A * m[0][zs].re : A * m[0][zs].im) +
                       (IB ? Bv * m[1][zs].re : Bv * m[1][zs].im)) +
                 (IC ? Cv * m[2][zs].re : Cv * m[2][zs].im);
        }
        o[(c * NCZ + z) * ls + ky] = Cx<T>{hr, hi};
    }
}

// the three output components of one ky (tensor at kt + (comp NCZ + d) oy;
// xy and yz odd in ky, xz and yz imaginary and odd in dz)
template <typename T, int NCZ, int Q0>
__device__ __forceinline__ void yz_column(const T *__restrict__ kt, int oy, T sy,
                                          const Cx<T> *__restrict__ r, Cx<T> *__restrict__ o,
                                          int ls, int ky)
{
    // the sources of this ky (3 NCZ values) once
    Cx<T> m[3][NCZ];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int zs = 0; zs < NCZ; ++zs) m[c][zs] = r[(c * NCZ + zs) * ls + ky];
    const int64_t cs = (int64_t)NCZ * oy;  // component stride
    const T *kxx = kt, *kyy = kt + cs, *kzz = kt + 2 * cs, *kxy = kt + 3 * cs, *kxz = kt + 4 * cs,
            *kyz = kt + 5 * cs;
    yz_row<T, NCZ, Q0, false, false, true>(kxx, kxy, kxz, T(1), sy, T(1), oy, m, o, ls, ky, 0);
    yz_row<T, NCZ, Q0, false, false, true>(kxy, kyy, kyz, sy, T(1), sy, oy, m, o, ls, ky, 1);
    yz_row<T, NCZ, Q0, true, true, false>(kxz, kyz, kzz, T(1), sy, T(1), oy, m, o, ls, ky, 2);
}

template <typename T, int NCZ>
__global__ __launch_bounds__(kDmYzThreads, sizeof(T) == 4 && NCZ <= 11 ? 4 : 2) void k_dm_yz(DemagDev dm)
{
    constexpr int Q = 4, nl = 3 * NCZ;
    const int Px = 1 << dm.lx, Py = 1 << dm.ly;
    const int Pxh = (Px >> 1) + 1;
    // blocks go round-robin over the eight XCDs: give each XCD a contiguous
    // range of columns, so that the neighbouring columns that share the
    // cache lines of wx are read through the same L2
    const int nb = Pxh * dm.n_sys, per = gridDim.x >> 3;
    const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tile >= nb) return;
    const int kx = tile % Pxh, s = tile / Pxh;
    const int ncy = dm.ncy, ls = Py + 1;
    Cx<T> *bx = lds_base<T>(), *by = bx + nl * ls, *twy = by + nl * ls;
    // line (c, z) row y of column kx at ((s 3 ncz + line) ncy + y) Pxh + kx
    Cx<T> *w = (Cx<T> *)dm.wx + (int64_t)s * nl * ncy * Pxh + kx;
    for (int q = threadIdx.x; q < nl * Py; q += blockDim.x) {
        const int line = q >> dm.ly, yy = q & (Py - 1);
        bx[line * ls + yy] = yy < ncy ? w[((int64_t)line * ncy + yy) * Pxh] : Cx<T>{T(0), T(0)};
    }
    // the twiddles of the y transforms in LDS
    for (int q = threadIdx.x; q < max(Py >> 1, 1); q += blockDim.x) twy[q] = ((const Cx<T> *)dm.tw[1])[q];
    __syncthreads();
    Cx<T> *r = fft_lines<T, false>(bx, by, nl, dm.ly, ls, twy);
    Cx<T> *o = r == bx ? by : bx;
    const int oy = (Py >> 1) + 1;
    const T *kt0 = (const T *)dm.K + (int64_t)kx * 6 * NCZ * oy;
    for (int t = threadIdx.x; t < Py * Q; t += blockDim.x) {
        const int q = t >> dm.ly, ky = t & (Py - 1);
        const int kyr = ky <= (Py >> 1) ? ky : Py - ky;
        const T sy = ky <= (Py >> 1) ? T(1) : T(-1);
        const T *kt = kt0 + kyr;
        switch (q) {
        case 0: yz_column<T, NCZ, 0>(kt, oy, sy, r, o, ls, ky); break;
        case 1: yz_column<T, NCZ, 1>(kt, oy, sy, r, o, ls, ky); break;
        case 2: yz_column<T, NCZ, 2>(kt, oy, sy, r, o, ls, ky); break;
        default: yz_column<T, NCZ, 3>(kt, oy, sy, r, o, ls, ky); break;
        }
    }
    __syncthreads();
    const Cx<T> *h = fft_lines<T, true>(o, r, nl, dm.ly, ls, twy);
    for (int q = threadIdx.x; q < nl * ncy; q += blockDim.x) {
        const int line = q / ncy, yy = q - line * ncy;
        w[((int64_t)line * ncy + yy) * Pxh] = h[line * ls + yy];
    }
}

// --- 5: inverse FFT along x of one (y, z) row, the field of its ncx cells
template <typename T>
__global__ __launch_bounds__(kDmThreads) void k_dm_x_out(DemagDev dm, int stage,
                                                         const int32_t *origin)
{
    const int Px = 1 << dm.lx;
    const int j = blockIdx.x % dm.ncy, k = blockIdx.x / dm.ncy, s = blockIdx.y;
    const Cx<T> *in = (const Cx<T> *)dm.wx;
    Cx<T> *x = lds_base<T>(), *y = x + 3 * Px;
    const int Pxh = (Px >> 1) + 1;
    for (int q = threadIdx.x; q < 3 * Px; q += blockDim.x) {
        const int c = q >> dm.lx, kx = q & (Px - 1);
        if (kx < Pxh) {
            x[q] = in[wx_at(dm, s, c, k, j, kx, Pxh)];
        } else {  // X(Px - k) = conj X(k)
            const Cx<T> v = in[wx_at(dm, s, c, k, j, Px - kx, Pxh)];
            x[q] = Cx<T>{v.re, -v.im};
        }
    }
    __syncthreads();
    const Cx<T> *r = fft_lines<T, true>(x, y, 3, dm.lx, Px, (const Cx<T> *)dm.tw[0]);
    if (dm.stray) {
        // window cells i0 .. i0 + ncx_win - 1 of the track mesh
        const int org = origin[s];
        const int i0 = (org + dm.cx - 1) / dm.cx;
        T *out = (T *)dm.bstray;
        const int64_t cell0 = (int64_t)dm.ncx_win * (j + (int64_t)dm.ncy * k);
        for (int q = threadIdx.x; q < 3 * dm.ncx_win; q += blockDim.x) {
            const int c = q / dm.ncx_win, i = q - c * dm.ncx_win;
            out[((int64_t)s * 3 + c) * dm.ncell_win + cell0 + i] = r[c * Px + i0 + i].re;
        }
        return;
    }
    T *bd = (T *)dm.bd[stage];
    const T *add = (const T *)dm.bstray;
    const int64_t cell0 = (int64_t)dm.ncx * (j + (int64_t)dm.ncy * k);
    for (int q = threadIdx.x; q < 3 * dm.ncx; q += blockDim.x) {
        const int c = q / dm.ncx, i = q - c * dm.ncx;
        const int64_t o = ((int64_t)s * 3 + c) * dm.ncell + cell0 + i;
        bd[o] = add ? r[c * Px + i].re + add[o] : r[c * Px + i].re;
    }
}

template <typename T, typename U = double>
int run_demag(const DemagDev &dm, const T *S, int64_t ncs, const SysDev *sys,
                 const int32_t *origin, int stage, void *stream, const U *cells = nullptr)
{
    hipStream_t st = (hipStream_t)stream;
    const int Px = 1 << dm.lx, Py = 1 << dm.ly, Pz = 1 << dm.lz;
    const size_t cb = sizeof(Cx<T>);
    const dim3 blk(kDmThreads);
    const dim3 grows(dm.ncy * dm.ncz, dm.n_sys);
    if (cells)
        hipLaunchKernelGGL((k_dm_cells_x<T, U>), grows, blk, 2 * 3 * Px * cb, st, dm, cells);
    else
        hipLaunchKernelGGL(k_dm_gather_x<T>, grows, blk, 2 * 3 * Px * cb, st, dm, S, ncs, sys,
                           origin);
    const int Pxh = (Px >> 1) + 1;
    if (dm.yzf) {
        const dim3 g((Pxh * dm.n_sys + 7) / 8 * 8), b(kDmYzThreads);
        const size_t lds = demag_yz_lds_bytes(dm, (int)sizeof(T));
#define ASD_YZ(N)                                                                                  \
    case N: hipLaunchKernelGGL((k_dm_yz<T, N>), g, b, lds, st, dm); break;
        switch (dm.ncz) {
            ASD_YZ(1) ASD_YZ(2) ASD_YZ(3) ASD_YZ(4) ASD_YZ(5) ASD_YZ(6) ASD_YZ(7) ASD_YZ(8)
            ASD_YZ(9) ASD_YZ(10) ASD_YZ(11) ASD_YZ(12) ASD_YZ(13) ASD_YZ(14) ASD_YZ(15) ASD_YZ(16)
        default: return -1;
        }
#undef ASD_YZ
    } else {
        const dim3 gy((Pxh + dm.xb_y - 1) / dm.xb_y, 3 * dm.ncz, dm.n_sys);
        hipLaunchKernelGGL((k_dm_y<T, false>), gy, blk, 2 * dm.xb_y * (Py + 1) * cb, st, dm);
        const dim3 gz((Pxh + dm.xb_z - 1) / dm.xb_z, Py, dm.n_sys);
        hipLaunchKernelGGL(k_dm_z<T>, gz, blk, 2 * 3 * dm.xb_z * (Pz + 1) * cb, st, dm);
        hipLaunchKernelGGL((k_dm_y<T, true>), gy, blk, 2 * dm.xb_y * (Py + 1) * cb, st, dm);
    }
    hipLaunchKernelGGL(k_dm_x_out<T>, grows, blk, 2 * 3 * Px * cb, st, dm, stage, origin);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

size_t demag_yz_lds_bytes(const DemagDev &dm, int elem)
{
    // the unrolled sums keep their operands in registers: up to 16 planes
    // (12 in FP64)
    if (dm.ncz > (elem == 8 ? 12 : 16)) return 0;
    // two line buffers and the y twiddles
    return ((size_t)2 * 3 * dm.ncz * ((size_t)(1 << dm.ly) + 1) + std::max((1 << dm.ly) / 2, 1)) *
           2 * elem;
}

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

int launch_demag_cells(const DemagDev &dm, const double *cells, void *stream)
{
    return run_demag<double>(dm, nullptr, 0, nullptr, nullptr, 0, stream, cells);
}

int launch_demag_sums_f64(const DemagDev &dm, const double *sums, int stage, void *stream)
{
    return run_demag<double, double>(dm, nullptr, 0, nullptr, nullptr, stage, stream, sums);
}

int launch_demag_sums_f32(const DemagDev &dm, const float *sums, int stage, void *stream)
{
    return run_demag<float, float>(dm, nullptr, 0, nullptr, nullptr, stage, stream, sums);
}

}  // namespace asd
