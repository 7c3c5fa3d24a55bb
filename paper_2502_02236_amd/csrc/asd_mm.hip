// asd_mm.hip -- micromagnetic region (Sec. II): LLG without the thermal field
// (Eq. 1 in Landau-Lifshitz form) on a finite-difference mesh, classic RK4
// (the integrator the paper names for these regions, Sec. III), the
// magnetisation renormalised after each step.
//
// Field per cell (tesla), from the configuration u of the stage:
//   exchange   (2 A(T) / M_S(T)) lap u                 (Eq. 4, 6-point stencil,
//              neighbours in the order -x, +x, -y, +y, -z, +z; a missing
//              neighbour at an open face contributes nothing)
//   anisotropy (2 K(T) / M_S(T)) u_z z                 (Eq. 5)
//   write field p(n) B
// with M_S = M_S0 m_e, A = A_0 m_e^2, K = K_0 m_e^3, damping
// alpha = lambda (1 - min(T, T_C) / 3 T_C), and m_e(T) the largest root of
// m = L(3 T_C m / T + mu_s |B| / kB T) (Sec. II), found by 64 halvings of
// [0, 1] in FP64 for both precisions.  T per cell from the laser spot at
// the stage time t_n, t_n + dt/2, t_n + dt/2, t_n + dt.
//
// One launch per RK4 stage; stage inputs ping-pong between two buffers so
// that no launch overwrites what its neighbours read; the last stage writes
// the new magnetisation in place (each cell reads only its own old value).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "asd.h"
#include "asd_device.h"
#include "asd_pair.h"

namespace asd {
namespace {

constexpr int kMMTile = 256;
constexpr int kMMMaxBits = 1 << 16;
constexpr size_t kMMAlign = 256;

struct MMArgs {
    int32_t nx, ny, nz, n;
    int32_t per[3];
    double ih2[3];            // 1 / h^2 per axis
    double h[3];
    double Ms0, A0, K0, lambda, gamma, Tc, dt, b;  // b = mu_s |B| / kB (K)
    double B[3];
    int32_t n_bits, spot_mode;
    int64_t spb;
    double T_amb, T_peak, inv2s2, x0, y0, v;
    const uint8_t *bits;
    const int64_t *step;      // device step counter
    int32_t step_off;
    void *m, *ua, *ub, *acc;  // [3][n] in the handle precision
    double *me, *alpha;       // per cell, filled by the parameter pass
    const double *ghost[2];   // x-face neighbours [ny*nz][3] (zero: none), or null
    // a held field (T) per cell, added at every stage: cell (i, j, k) reads
    // bd[d][(bd_off + i) + bd_nx (j + ny k)] of a mesh bd_nx cells long; or null
    const double *bd;
    int32_t bd_nx, bd_off;
};

// Langevin function coth x - 1/x for x >= 0: series through x^11 below 0.1,
// coth from the portable exp above
__device__ __forceinline__ double langevin(double x)
{
    if (x < 0.1) {
        const double x2 = x * x;
        double p = -1382.0 / 638512875.0;
        p = 2.0 / 93555.0 + x2 * p;
        p = -1.0 / 4725.0 + x2 * p;
        p = 2.0 / 945.0 + x2 * p;
        p = -1.0 / 45.0 + x2 * p;
        p = 1.0 / 3.0 + x2 * p;
        return x * p;
    }
    const double e = f64::expn(-2.0 * x);
    return (1.0 + e) / (1.0 - e) - 1.0 / x;
}

__device__ __forceinline__ double equilibrium_m(double T, double Tc, double b)
{
    if (T <= 0.0) return 1.0;
    double lo = 0.0, hi = 1.0;
    for (int k = 0; k < 64; ++k) {
        const double mid = 0.5 * (lo + hi);
        const double f = langevin((3.0 * Tc * mid + b) / T) - mid;
        if (f >= 0.0)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// m_e and alpha of every cell at time t = (step + frac) dt
__global__ __launch_bounds__(kMMTile) void k_mm_params(MMArgs a, double frac)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const int i = c % a.nx, j = (c / a.nx) % a.ny;
    double T = a.T_amb;
    if (a.spot_mode != ASD_SPOT_NONE) {
        const double t0 = (double)(*a.step + a.step_off) * a.dt;
        const double t = frac == 0.0 ? t0 : (frac == 1.0 ? t0 + a.dt : t0 + 0.5 * a.dt);
        const double xc = a.spot_mode == ASD_SPOT_MOVING ? a.x0 + a.v * t : a.x0;
        const double dx = ((double)i + 0.5) * a.h[0] - xc;
        const double dy = ((double)j + 0.5) * a.h[1] - a.y0;
        const double q = (dx * dx + dy * dy) * a.inv2s2;
        T = a.T_amb + (a.T_peak - a.T_amb) * f64::expn(-q);
    }
    a.me[c] = equilibrium_m(T, a.Tc, a.b);
    const double Tr = T < a.Tc ? T : a.Tc;
    a.alpha[c] = a.lambda * (1.0 - Tr / (3.0 * a.Tc));
}

template <typename T>
struct M3 {
    T x, y, z;
};

template <typename T>
__device__ __forceinline__ int64_t mm_nb(const MMArgs &a, int i, int j, int k, int ax, int d)
{
    int c[3] = {i, j, k};
    const int n[3] = {a.nx, a.ny, a.nz};
    c[ax] += d;
    if (c[ax] < 0 || c[ax] >= n[ax]) {
        if (!a.per[ax]) return -1;
        c[ax] = (c[ax] + n[ax]) % n[ax];
    }
    return c[0] + (int64_t)n[0] * (c[1] + (int64_t)n[1] * c[2]);
}

// stage s: k_s from the stage input (m for s = 0, else the buffer the
// previous stage wrote); s < 3 writes the next input, s = 3 the new m
template <typename T>
__device__ __forceinline__ void mm_stage_cell(const MMArgs &a, int s, int c)
{
    if (c >= a.n) return;
    const int64_t n = a.n;
    const int i = c % a.nx, j = (c / a.nx) % a.ny, k = c / (a.nx * a.ny);
    T *m = (T *)a.m, *acc = (T *)a.acc;
    const T *u = s == 0 ? m : (s == 2 ? (const T *)a.ub : (const T *)a.ua);
    T *nxt = s == 1 ? (T *)a.ub : (T *)a.ua;  // written by s = 0, 1, 2
    const M3<T> mc{u[c], u[n + c], u[2 * n + c]};
    T lap[3] = {T(0), T(0), T(0)};
    for (int ax = 0; ax < 3; ++ax)
        for (int d = -1; d <= 1; d += 2) {
            const int64_t q = mm_nb<T>(a, i, j, k, ax, d);
            const T w = (T)a.ih2[ax];
            if (q < 0) {
                // the region across an x face: its direction (zero: nothing there)
                const double *g = ax == 0 ? a.ghost[d < 0 ? 0 : 1] : nullptr;
                if (!g) continue;
                const double *gv = g + 3 * ((int64_t)j + (int64_t)a.ny * k);
                if (gv[0] == 0.0 && gv[1] == 0.0 && gv[2] == 0.0) continue;
                lap[0] = lap[0] + ((T)gv[0] - mc.x) * w;
                lap[1] = lap[1] + ((T)gv[1] - mc.y) * w;
                lap[2] = lap[2] + ((T)gv[2] - mc.z) * w;
                continue;
            }
            lap[0] = lap[0] + (u[q] - mc.x) * w;
            lap[1] = lap[1] + (u[n + q] - mc.y) * w;
            lap[2] = lap[2] + (u[2 * n + q] - mc.z) * w;
        }
    const int64_t step = *a.step + a.step_off;
    T pol = T(1);
    if (a.n_bits > 0 && a.spb > 0) pol = a.bits[(step / a.spb) % a.n_bits] ? T(1) : T(-1);
    const double me = a.me[c];
    const T cex = (T)((2.0 * a.A0 * me) / a.Ms0);
    const T can = (T)((2.0 * a.K0 * (me * me)) / a.Ms0);
    T B[3];
    B[0] = cex * lap[0] + pol * (T)a.B[0];
    B[1] = cex * lap[1] + pol * (T)a.B[1];
    B[2] = cex * lap[2] + pol * (T)a.B[2];
    B[2] = B[2] + can * mc.z;
    if (a.bd) {
        const int64_t nb = (int64_t)a.bd_nx * a.ny * a.nz;
        const int64_t q = (a.bd_off + i) + (int64_t)a.bd_nx * (j + (int64_t)a.ny * k);
        B[0] = B[0] + (T)a.bd[q];
        B[1] = B[1] + (T)a.bd[nb + q];
        B[2] = B[2] + (T)a.bd[2 * nb + q];
    }
    const double al = a.alpha[c];
    const T alpha = (T)al;
    const T gp = (T)(-a.gamma / (1.0 + al * al));
    // Landau-Lifshitz right-hand side gp (m x B + alpha m x (m x B))
    const T cx = mc.y * B[2] - mc.z * B[1];
    const T cy = mc.z * B[0] - mc.x * B[2];
    const T cz = mc.x * B[1] - mc.y * B[0];
    const T ddx = mc.y * cz - mc.z * cy;
    const T ddy = mc.z * cx - mc.x * cz;
    const T ddz = mc.x * cy - mc.y * cx;
    const T f[3] = {gp * (cx + alpha * ddx), gp * (cy + alpha * ddy), gp * (cz + alpha * ddz)};
    const T dt = (T)a.dt;
    const T m0[3] = {m[c], m[n + c], m[2 * n + c]};
    if (s == 0) {
        for (int d = 0; d < 3; ++d) {
            acc[d * n + c] = f[d];
            nxt[d * n + c] = m0[d] + (T(0.5) * dt) * f[d];
        }
    } else if (s < 3) {
        for (int d = 0; d < 3; ++d) {
            acc[d * n + c] = acc[d * n + c] + T(2) * f[d];
            nxt[d * n + c] = m0[d] + (s == 1 ? T(0.5) * dt : dt) * f[d];
        }
    } else {
        T v[3];
        for (int d = 0; d < 3; ++d) v[d] = m0[d] + (dt / T(6)) * (acc[d * n + c] + f[d]);
        const T r = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        m[c] = v[0] / r;
        m[n + c] = v[1] / r;
        m[2 * n + c] = v[2] / r;
    }
}

template <typename T>
__global__ __launch_bounds__(kMMTile) void k_mm_stage(MMArgs a, int s)
{
    mm_stage_cell<T>(a, s, blockIdx.x * blockDim.x + threadIdx.x);
}

// stage s of two regions in one launch: blocks [0, blocks0) take region a0,
// the rest region a1 (the regions share nothing, so the results equal those
// of one launch per region)
template <typename T>
__global__ __launch_bounds__(kMMTile) void k_mm_stage_pair(MMArgs a0, MMArgs a1, int s, int blocks0)
{
    const int b = blockIdx.x;
    if (b < blocks0)
        mm_stage_cell<T>(a0, s, b * kMMTile + threadIdx.x);
    else
        mm_stage_cell<T>(a1, s, (b - blocks0) * kMMTile + threadIdx.x);
}

// face neighbours from vectors (normalised; zero stays zero)
__global__ void k_mm_set_face(double *ghost, const double *vec, int stride, int nyz)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nyz) return;
    const double x = vec[(int64_t)c * stride], y = vec[(int64_t)c * stride + 1],
                 z = vec[(int64_t)c * stride + 2];
    const double r = sqrt((x * x + y * y) + z * z);
    ghost[3 * c] = r > 0.0 ? x / r : 0.0;
    ghost[3 * c + 1] = r > 0.0 ? y / r : 0.0;
    ghost[3 * c + 2] = r > 0.0 ? z / r : 0.0;
}

// both regions' faces in one launch: threads [0, nyz) take g0/v0, the next
// nyz take g1/v1
__global__ void k_mm_set_face_pair(double *g0, const double *v0, double *g1, const double *v1,
                                   int stride, int nyz)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * nyz) return;
    const bool second = t >= nyz;
    const int c = second ? t - nyz : t;
    const double *vec = second ? v1 : v0;
    double *ghost = second ? g1 : g0;
    const double x = vec[(int64_t)c * stride], y = vec[(int64_t)c * stride + 1],
                 z = vec[(int64_t)c * stride + 2];
    const double r = sqrt((x * x + y * y) + z * z);
    ghost[3 * c] = r > 0.0 ? x / r : 0.0;
    ghost[3 * c + 1] = r > 0.0 ? y / r : 0.0;
    ghost[3 * c + 2] = r > 0.0 ? z / r : 0.0;
}

// directions of the cells of x face `face`
template <typename T>
__device__ __forceinline__ void mm_face_cell(const MMArgs &a, int face, double *dirs, int c)
{
    if (c >= a.ny * a.nz) return;
    const int64_t cell = (face == 0 ? 0 : a.nx - 1) + (int64_t)a.nx * c;
    const T *m = (const T *)a.m;
    for (int d = 0; d < 3; ++d) dirs[3 * c + d] = (double)m[d * (int64_t)a.n + cell];
}

template <typename T>
__global__ void k_mm_get_face(MMArgs a, int face, double *dirs)
{
    mm_face_cell<T>(a, face, dirs, blockIdx.x * blockDim.x + threadIdx.x);
}

// two regions' faces in one launch: blocks [0, b0) take region a0
template <typename T>
__global__ void k_mm_get_face_pair(MMArgs a0, int f0, double *d0, MMArgs a1, int f1, double *d1,
                                   int b0)
{
    if ((int)blockIdx.x < b0)
        mm_face_cell<T>(a0, f0, d0, blockIdx.x * blockDim.x + threadIdx.x);
    else
        mm_face_cell<T>(a1, f1, d1, (blockIdx.x - b0) * blockDim.x + threadIdx.x);
}

// What a region hands to the atomistic window by thermalisation (Sec. II):
// the reduced magnetisation M / M_S^0 = m_e(T) m of each cell of x face
// `face` at time t (s), out[3 c ..] with c = j + ny k; T from the spot at the
// cell centre as in k_mm_params
template <typename T>
__global__ void k_mm_face_moment(MMArgs a, int face, double t, double *out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ny * a.nz) return;
    const int i = face == 0 ? 0 : a.nx - 1, j = c % a.ny;
    double Tk = a.T_amb;
    if (a.spot_mode != ASD_SPOT_NONE) {
        const double xc = a.spot_mode == ASD_SPOT_MOVING ? a.x0 + a.v * t : a.x0;
        const double dx = ((double)i + 0.5) * a.h[0] - xc;
        const double dy = ((double)j + 0.5) * a.h[1] - a.y0;
        const double q = (dx * dx + dy * dy) * a.inv2s2;
        Tk = a.T_amb + (a.T_peak - a.T_amb) * f64::expn(-q);
    }
    const double me = equilibrium_m(Tk, a.Tc, a.b);
    const int64_t cell = i + (int64_t)a.nx * c;
    const T *m = (const T *)a.m;
    for (int d = 0; d < 3; ++d) out[3 * c + d] = me * (double)m[d * (int64_t)a.n + cell];
}

// The mesh moves one cell along +x with the window (Sec. II, Fig. 1): in each
// row (j, k) cell i takes the direction of cell i + 1 (rows run in order, so
// a cell is read before it is overwritten); the first cell's direction is
// copied to leave[3 c ..] (if given), the last takes enter[stride c ..]
// normalised (+z for a zero vector: a coarse cell with no magnetic site)
template <typename T>
__global__ void k_mm_shift(MMArgs a, const double *enter, int stride, double *leave)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ny * a.nz) return;
    const int64_t n = a.n, row = (int64_t)a.nx * c;
    T *m = (T *)a.m;
    if (leave)
        for (int d = 0; d < 3; ++d) leave[3 * c + d] = (double)m[d * n + row];
    for (int i = 0; i + 1 < a.nx; ++i)
        for (int d = 0; d < 3; ++d) m[d * n + row + i] = m[d * n + row + i + 1];
    const double *v = enter + (int64_t)stride * c;
    const double r = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    double e[3] = {0.0, 0.0, 1.0};
    if (r > 0.0)
        for (int d = 0; d < 3; ++d) e[d] = v[d] / r;
    for (int d = 0; d < 3; ++d) m[d * n + row + a.nx - 1] = (T)e[d];
}

__global__ void k_mm_advance(int64_t *step, int64_t n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *step += n;
}

__global__ void k_mm_advance_pair(int64_t *step0, int64_t *step1, int64_t n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *step0 += n;
        *step1 += n;
    }
}

size_t align_up(size_t v) { return (v + kMMAlign - 1) / kMMAlign * kMMAlign; }

// One region's part of the multiscale window's demagnetising sources.
struct MsdRegion {
    MMArgs a;                 // the region (its m, drive, T_C, M_S0 and cell edges)
    int32_t elem;             // 8: FP64 m, 4: FP32
    int32_t off;              // first cell along x of the combined mesh
    int32_t me_ready;         // a.me holds m_e(T) of every cell (a spot that does not move)
    double scale;             // M_S0 V / mu_s: the spin sum of a cell with m_e = 1
};

// Sources of Eq. 7 on the window laid out as one mesh of NX cells along x
// (left region, atomistic coarse cells, right region), in spin-sum units:
// set 0 every cell, set 1 the regions' cells only.  Region cell: (M_S0 V /
// mu_s) m_e(T) m with T at the cell centre at time t; atomistic cell: the
// coarse-grain sums (Eq. 6), sums[c][4] over the nA window cells.
__global__ void k_msd_sources(double *src, int NX, int ny, int nz, const double *sums, int nA,
                              int offA, MsdRegion L, int hasL, MsdRegion R, int hasR, double t)
{
    const int64_t ncell = (int64_t)NX * ny * nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int I = (int)(c % NX);
    const int64_t jk = c / NX;
    const int j = (int)(jk % ny);
    double v[3] = {0.0, 0.0, 0.0};
    bool region = false;
    if (I >= offA && I < offA + nA) {
        const double *sc = sums + 4 * ((I - offA) + (int64_t)nA * jk);
        for (int d = 0; d < 3; ++d) v[d] = sc[d];
    } else {
        const bool left = hasL && I < offA;
        if (left || hasR) {
            const MsdRegion &g = left ? L : R;
            const int i = I - g.off;
            const int64_t cell = i + (int64_t)g.a.nx * jk;
            double me;
            if (g.me_ready) {  // the region's own m_e(T) of a spot that does not move
                me = g.a.me[cell];
            } else {
                double Tk = g.a.T_amb;
                if (g.a.spot_mode != ASD_SPOT_NONE) {
                    const double xc = g.a.spot_mode == ASD_SPOT_MOVING ? g.a.x0 + g.a.v * t : g.a.x0;
                    const double dx = ((double)i + 0.5) * g.a.h[0] - xc;
                    const double dy = ((double)j + 0.5) * g.a.h[1] - g.a.y0;
                    const double q = (dx * dx + dy * dy) * g.a.inv2s2;
                    Tk = g.a.T_amb + (g.a.T_peak - g.a.T_amb) * f64::expn(-q);
                }
                me = equilibrium_m(Tk, g.a.Tc, g.a.b);
            }
            const double s = g.scale * me;
            for (int d = 0; d < 3; ++d)
                v[d] = s * (g.elem == 8 ? ((const double *)g.a.m)[d * (int64_t)g.a.n + cell]
                                        : (double)((const float *)g.a.m)[d * (int64_t)g.a.n + cell]);
            region = true;
        }
    }
    for (int d = 0; d < 3; ++d) {
        src[d * ncell + c] = v[d];
        src[(3 + d) * ncell + c] = region ? v[d] : 0.0;
    }
}

}  // namespace
}  // namespace asd

using namespace asd;

struct asd_mm_t {
    asd_mm_params p{};
    asd_drive drive{};
    std::vector<uint8_t> bits;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    int elem = 8;
    int64_t n = 0, step = 0;
    size_t off_m = 0, off_ua = 0, off_ub = 0, off_acc = 0, off_me = 0, off_al = 0,
           off_step = 0, off_bits = 0, off_ghost[2] = {0, 0}, off_fsum = 0, off_fdir = 0, bytes = 0;
    bool ghost_on[2] = {false, false};
    const double *bd = nullptr;  // held field of the multiscale window's demagnetising field
    int32_t bd_nx = 0, bd_off = 0;
    bool params_valid = false;  // m_e, alpha current for a spot that does not move
    hipGraphExec_t graph = nullptr;
    std::string err;
};

static thread_local std::string g_mm_err;

static int mm_fail(asd_mm_t *h, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    (h ? h->err : g_mm_err) = buf;
    return code;
}

#define MM_HIP(h, call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return mm_fail((h), ASD_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static int mm_check(const asd_mm_params *p)
{
    if (!p) return mm_fail(nullptr, ASD_EINVAL, "params is NULL");
    if (p->precision != ASD_FP64 && p->precision != ASD_FP32)
        return mm_fail(nullptr, ASD_EINVAL, "precision must be ASD_FP64 or ASD_FP32");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || (int64_t)p->nx * p->ny * p->nz > (1 << 28))
        return mm_fail(nullptr, ASD_EINVAL, "mesh must have 1 .. 2^28 cells");
    const int32_t bc[3] = {p->bc_x, p->bc_y, p->bc_z};
    for (int k = 0; k < 3; ++k)
        if (bc[k] != ASD_BC_OPEN && bc[k] != ASD_BC_PERIODIC)
            return mm_fail(nullptr, ASD_EINVAL, "micromagnetic faces are open or periodic");
    for (int k = 0; k < 3; ++k)
        if (!(p->h[k] > 0)) return mm_fail(nullptr, ASD_EINVAL, "cell edges must be positive");
    if (!(p->Ms0 > 0) || !(p->A0 >= 0) || !std::isfinite(p->K0) || !(p->lambda >= 0) ||
        !(p->gamma > 0) || !(p->Tc > 0) || !(p->mu_s >= 0) || !(p->dt > 0))
        return mm_fail(nullptr, ASD_EINVAL, "material constants out of range");
    if (p->graph_steps < 0) return mm_fail(nullptr, ASD_EINVAL, "graph_steps must be >= 0");
    return ASD_OK;
}

static void mm_layout(const asd_mm_params *p, asd_mm_t *h)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const size_t e = p->precision == ASD_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = align_up(off + b);
        return o;
    };
    h->off_m = take(3 * n * e);
    h->off_ua = take(3 * n * e);
    h->off_ub = take(3 * n * e);
    h->off_acc = take(3 * n * e);
    h->off_me = take(n * sizeof(double));
    h->off_al = take(n * sizeof(double));
    h->off_step = take(sizeof(int64_t));
    h->off_bits = take(kMMMaxBits);
    const size_t nyz = (size_t)p->ny * p->nz;
    h->off_ghost[0] = take(3 * nyz * sizeof(double));
    h->off_ghost[1] = take(3 * nyz * sizeof(double));
    h->off_fsum = take(4 * nyz * sizeof(double));  // coupling scratch
    h->off_fdir = take(3 * nyz * sizeof(double));
    h->bytes = off;
}

static MMArgs mm_args(const asd_mm_t *h, int step_off)
{
    const asd_mm_params &p = h->p;
    const asd_drive &d = h->drive;
    MMArgs a;
    std::memset(&a, 0, sizeof a);
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.n = (int32_t)h->n;
    a.per[0] = p.bc_x == ASD_BC_PERIODIC;
    a.per[1] = p.bc_y == ASD_BC_PERIODIC;
    a.per[2] = p.bc_z == ASD_BC_PERIODIC;
    for (int k = 0; k < 3; ++k) {
        a.h[k] = p.h[k];
        a.ih2[k] = 1.0 / (p.h[k] * p.h[k]);
        a.B[k] = d.B[k];
    }
    a.Ms0 = p.Ms0;
    a.A0 = p.A0;
    a.K0 = p.K0;
    a.lambda = p.lambda;
    a.gamma = p.gamma;
    a.Tc = p.Tc;
    a.dt = p.dt;
    const double bmag = std::sqrt((d.B[0] * d.B[0] + d.B[1] * d.B[1]) + d.B[2] * d.B[2]);
    a.b = p.mu_s * bmag / 1.380649e-23;
    a.n_bits = d.n_bits;
    a.spb = d.steps_per_bit;
    a.spot_mode = d.spot_mode;
    a.T_amb = d.T_amb;
    a.T_peak = d.T_peak;
    if (d.spot_mode != ASD_SPOT_NONE) {
        const double sd = d.fwhm / 2.3548200450309493;
        a.inv2s2 = 1.0 / ((2.0 * sd) * sd);
    }
    a.x0 = d.x0;
    a.y0 = d.y0;
    a.v = d.v;
    char *w = h->ws;
    a.bits = (const uint8_t *)(w + h->off_bits);
    a.step = (const int64_t *)(w + h->off_step);
    a.step_off = step_off;
    a.m = w + h->off_m;
    a.ua = w + h->off_ua;
    a.ub = w + h->off_ub;
    a.acc = w + h->off_acc;
    a.me = (double *)(w + h->off_me);
    a.alpha = (double *)(w + h->off_al);
    for (int f = 0; f < 2; ++f)
        a.ghost[f] = h->ghost_on[f] ? (const double *)(w + h->off_ghost[f]) : nullptr;
    a.bd = h->bd;
    a.bd_nx = h->bd_nx;
    a.bd_off = h->bd_off;
    return a;
}

// launches of one step (step_off after the device counter); the parameter
// pass runs per stage for a moving spot, else once when the drive changed
static int mm_launch_step(asd_mm_t *h, int step_off, bool params_now)
{
    const MMArgs a = mm_args(h, step_off);
    const dim3 grid((unsigned)((h->n + kMMTile - 1) / kMMTile)), blk(kMMTile);
    const bool moving = h->drive.spot_mode == ASD_SPOT_MOVING;
    const double frac[4] = {0.0, 0.5, 0.5, 1.0};
    for (int s = 0; s < 4; ++s) {
        if (moving ? (s != 2) : (s == 0 && params_now))
            hipLaunchKernelGGL(k_mm_params, grid, blk, 0, h->stream, a, frac[s]);
        if (h->elem == 8)
            hipLaunchKernelGGL(k_mm_stage<double>, grid, blk, 0, h->stream, a, s);
        else
            hipLaunchKernelGGL(k_mm_stage<float>, grid, blk, 0, h->stream, a, s);
    }
    return hipGetLastError() == hipSuccess ? ASD_OK
                                            : mm_fail(h, ASD_EHIP, "micromagnetic launch failed: %s",
                                                      hipGetErrorString(hipGetLastError()));
}

static void mm_drop_graph(asd_mm_t *h)
{
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
}

extern "C" {

int asd_mm_workspace_bytes(const asd_mm_params *p, size_t *bytes)
{
    int rc = mm_check(p);
    if (rc) return rc;
    if (!bytes) return mm_fail(nullptr, ASD_EINVAL, "bytes is NULL");
    asd_mm_t tmp;
    mm_layout(p, &tmp);
    *bytes = tmp.bytes;
    return ASD_OK;
}

int asd_mm_create(const asd_mm_params *p, void *workspace, size_t workspace_bytes, void *stream,
                  asd_mm_t **out)
{
    if (!out) return mm_fail(nullptr, ASD_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = mm_check(p);
    if (rc) return rc;
    asd_mm_t *h = new (std::nothrow) asd_mm_t();
    if (!h) return mm_fail(nullptr, ASD_ENOMEM, "host allocation failed");
    h->p = *p;
    mm_layout(p, h);
    if (!workspace || ((uintptr_t)workspace % kMMAlign) != 0 || workspace_bytes < h->bytes) {
        delete h;
        return mm_fail(nullptr, workspace_bytes < h->bytes ? ASD_ENOMEM : ASD_EINVAL,
                       "workspace must be 256-byte aligned and hold asd_mm_workspace_bytes");
    }
    h->ws = (char *)workspace;
    h->stream = (hipStream_t)stream;
    h->elem = p->precision == ASD_FP64 ? 8 : 4;
    h->n = (int64_t)p->nx * p->ny * p->nz;
    // zero everything, then m = +z
    hipError_t e = hipMemsetAsync(h->ws, 0, h->bytes, h->stream);
    std::vector<char> m0((size_t)3 * h->n * h->elem, 0);
    for (int64_t c = 0; c < h->n; ++c) {
        if (h->elem == 8) ((double *)m0.data())[2 * h->n + c] = 1.0;
        else ((float *)m0.data())[2 * h->n + c] = 1.0f;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->ws + h->off_m, m0.data(), m0.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete h;
        return mm_fail(nullptr, ASD_EHIP, "set-up copy failed: %s", hipGetErrorString(e));
    }
    *out = h;
    return ASD_OK;
}

int asd_mm_destroy(asd_mm_t *h)
{
    if (!h) return ASD_OK;
    mm_drop_graph(h);
    delete h;
    return ASD_OK;
}

int asd_mm_set_field_temperature(asd_mm_t *h, const asd_drive *d)
{
    if (!h || !d) return mm_fail(h, ASD_EINVAL, "NULL argument");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(d->B[k])) return mm_fail(h, ASD_EINVAL, "B must be finite");
    if (d->n_bits < 0 || d->n_bits > kMMMaxBits ||
        (d->n_bits > 0 && (!d->bits || d->steps_per_bit <= 0)))
        return mm_fail(h, ASD_EINVAL, "bits: 0..65536 entries with steps_per_bit > 0");
    if (d->spot_mode < ASD_SPOT_NONE || d->spot_mode > ASD_SPOT_LOCKED)
        return mm_fail(h, ASD_EINVAL, "unknown spot mode");
    if (!(d->T_amb >= 0) || (d->spot_mode != ASD_SPOT_NONE && !(d->T_peak >= 0 && d->fwhm > 0)))
        return mm_fail(h, ASD_EINVAL, "temperatures must be >= 0 and fwhm > 0 with a spot");
    h->drive = *d;
    h->drive.bits = nullptr;
    h->bits.assign(d->bits, d->bits + d->n_bits);
    if (d->n_bits > 0)
        MM_HIP(h, hipMemcpyAsync(h->ws + h->off_bits, h->bits.data(), h->bits.size(),
                                 hipMemcpyHostToDevice, h->stream));
    MM_HIP(h, hipStreamSynchronize(h->stream));
    h->params_valid = false;
    mm_drop_graph(h);
    return ASD_OK;
}

int asd_mm_set_m(asd_mm_t *h, const void *src, int32_t on_device)
{
    if (!h || !src) return mm_fail(h, ASD_EINVAL, "NULL argument");
    MM_HIP(h, hipMemcpyAsync(h->ws + h->off_m, src, (size_t)3 * h->n * h->elem,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             h->stream));
    MM_HIP(h, hipStreamSynchronize(h->stream));
    return ASD_OK;
}

int asd_mm_get_m(asd_mm_t *h, void *dst, int32_t on_device)
{
    if (!h || !dst) return mm_fail(h, ASD_EINVAL, "NULL argument");
    MM_HIP(h, hipMemcpyAsync(dst, h->ws + h->off_m, (size_t)3 * h->n * h->elem,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             h->stream));
    MM_HIP(h, hipStreamSynchronize(h->stream));
    return ASD_OK;
}

int asd_mm_step(asd_mm_t *h, int64_t n)
{
    if (!h) return mm_fail(nullptr, ASD_EINVAL, "NULL handle");
    if (n < 0) return mm_fail(h, ASD_EINVAL, "n must be >= 0");
    if (n == 0) return ASD_OK;
    int64_t *step = (int64_t *)(h->ws + h->off_step);
    int64_t done = 0;
    const int G = h->p.graph_steps;
    if (G > 0 && n >= G) {
        if (!h->params_valid) {  // graphs never hold the parameter pass of a static spot
            const MMArgs a = mm_args(h, 0);
            hipLaunchKernelGGL(k_mm_params, dim3((unsigned)((h->n + kMMTile - 1) / kMMTile)),
                               dim3(kMMTile), 0, h->stream, a, 0.0);
            h->params_valid = true;
        }
        if (!h->graph) {
            hipGraph_t g = nullptr;
            MM_HIP(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
            int rc = ASD_OK;
            for (int t = 0; t < G && rc == ASD_OK; ++t) rc = mm_launch_step(h, t, false);
            if (rc == ASD_OK) hipLaunchKernelGGL(k_mm_advance, dim3(1), dim3(1), 0, h->stream, step, (int64_t)G);
            hipError_t e = hipStreamEndCapture(h->stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return mm_fail(h, ASD_EHIP, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return mm_fail(h, ASD_EHIP, "graph instantiate failed: %s", hipGetErrorString(e));
        }
        while (n - done >= G) {
            MM_HIP(h, hipGraphLaunch(h->graph, h->stream));
            done += G;
        }
    }
    for (int64_t t = 0; t < n - done; ++t) {
        int rc = mm_launch_step(h, (int)t, !h->params_valid);
        if (rc) return rc;
        if (h->drive.spot_mode != ASD_SPOT_MOVING) h->params_valid = true;
    }
    if (n - done > 0)
        hipLaunchKernelGGL(k_mm_advance, dim3(1), dim3(1), 0, h->stream, step, n - done);
    MM_HIP(h, hipGetLastError());
    h->step += n;
    return ASD_OK;
}

int asd_mm_get_step(asd_mm_t *h, int64_t *step)
{
    if (!h || !step) return mm_fail(h, ASD_EINVAL, "NULL argument");
    *step = h->step;
    return ASD_OK;
}

int asd_mm_set_face(asd_mm_t *h, int32_t face, const double *vec, int32_t stride)
{
    if (!h) return mm_fail(nullptr, ASD_EINVAL, "NULL handle");
    if (face != 0 && face != 1) return mm_fail(h, ASD_EINVAL, "face is 0 (-x) or 1 (+x)");
    const bool per = h->p.bc_x == ASD_BC_PERIODIC;
    if (vec && per) return mm_fail(h, ASD_EINVAL, "a periodic x axis has no faces to couple");
    const bool was = h->ghost_on[face];
    if (!vec) {
        h->ghost_on[face] = false;
    } else {
        if (stride < 3) return mm_fail(h, ASD_EINVAL, "stride must be >= 3");
        const int nyz = h->p.ny * h->p.nz;
        hipLaunchKernelGGL(k_mm_set_face, dim3((nyz + 255) / 256), dim3(256), 0, h->stream,
                           (double *)(h->ws + h->off_ghost[face]), vec, (int)stride, nyz);
        MM_HIP(h, hipGetLastError());
        h->ghost_on[face] = true;
    }
    if (was != h->ghost_on[face]) mm_drop_graph(h);  // graphs bake the face pointers in
    return ASD_OK;
}

int asd_mm_get_face(asd_mm_t *h, int32_t face, double *dirs)
{
    if (!h || !dirs) return mm_fail(h, ASD_EINVAL, "NULL argument");
    if (face != 0 && face != 1) return mm_fail(h, ASD_EINVAL, "face is 0 (-x) or 1 (+x)");
    const MMArgs a = mm_args(h, 0);
    const int nyz = h->p.ny * h->p.nz;
    if (h->elem == 8)
        hipLaunchKernelGGL(k_mm_get_face<double>, dim3((nyz + 255) / 256), dim3(256), 0, h->stream,
                           a, (int)face, dirs);
    else
        hipLaunchKernelGGL(k_mm_get_face<float>, dim3((nyz + 255) / 256), dim3(256), 0, h->stream,
                           a, (int)face, dirs);
    MM_HIP(h, hipGetLastError());
    return ASD_OK;
}

// one RK4 step of two regions on one stream (same precision, spots that do
// not move): the launches of asd_mm_step(h, 1) for both, with the stages of
// the two merged into one launch each
static int mm_step_pair(asd_mm_t *L, asd_mm_t *R)
{
    asd_mm_t *r[2] = {L, R};
    for (asd_mm_t *h : r)
        if (!h->params_valid) {
            const MMArgs a = mm_args(h, 0);
            hipLaunchKernelGGL(k_mm_params, dim3((unsigned)((h->n + kMMTile - 1) / kMMTile)),
                               dim3(kMMTile), 0, h->stream, a, 0.0);
            h->params_valid = true;
        }
    const MMArgs a0 = mm_args(L, 0), a1 = mm_args(R, 0);
    const int b0 = (int)((L->n + kMMTile - 1) / kMMTile), b1 = (int)((R->n + kMMTile - 1) / kMMTile);
    const dim3 grid((unsigned)(b0 + b1)), blk(kMMTile);
    for (int s = 0; s < 4; ++s) {
        if (L->elem == 8)
            hipLaunchKernelGGL(k_mm_stage_pair<double>, grid, blk, 0, L->stream, a0, a1, s, b0);
        else
            hipLaunchKernelGGL(k_mm_stage_pair<float>, grid, blk, 0, L->stream, a0, a1, s, b0);
    }
    hipLaunchKernelGGL(k_mm_advance_pair, dim3(1), dim3(1), 0, L->stream,
                       (int64_t *)(L->ws + L->off_step), (int64_t *)(R->ws + R->off_step), (int64_t)1);
    MM_HIP(L, hipGetLastError());
    L->step += 1;
    R->step += 1;
    return ASD_OK;
}

// the checks asd_multiscale_step makes of a region beside the window
static int region_fits(asd_mm_t *m, double dt, const double edge[3], const int32_t cell[3], int ny,
                       int nz, void *st)
{
    if (std::fabs(m->p.dt - dt) > 1e-9 * dt)
        return mm_fail(m, ASD_EINVAL, "region dt %g s differs from the atomistic dt %g s", m->p.dt, dt);
    for (int k = 0; k < 3; ++k)
        if (std::fabs(m->p.h[k] - cell[k] * edge[k]) > 1e-9 * cell[k] * edge[k])
            return mm_fail(m, ASD_EINVAL, "region cell edge %d is %g m, not %d lattice cells (%g m)",
                           k, m->p.h[k], cell[k], cell[k] * edge[k]);
    if (m->stream != (hipStream_t)st)
        return mm_fail(m, ASD_EINVAL, "the region must run on the atomistic handle's stream");
    if (m->p.ny != (ny + cell[1] - 1) / cell[1] || m->p.nz != (nz + cell[2] - 1) / cell[2])
        return mm_fail(m, ASD_EINVAL, "region ny, nz must equal the window's coarse cells");
    if (m->p.bc_x == ASD_BC_PERIODIC) return mm_fail(m, ASD_EINVAL, "region x axis is periodic");
    return ASD_OK;
}

// The demagnetising field of the whole multiscale window: the combined mesh
// (left region, atomistic coarse cells, right region along x), its FFT
// pipeline in FP64 with two source sets (every cell; the regions' cells
// only), and the buffers in the caller's workspace.
struct asd_msd_t {
    asd_t *atoms = nullptr;
    int32_t sys = 0;
    asd_mm_t *left = nullptr, *right = nullptr;
    int32_t cell[3] = {1, 1, 1};
    int32_t nL = 0, nA = 0, nR = 0, NX = 0, ny = 0, nz = 0;
    double V = 0.0, mu_s = 0.0;
    DemagDev dm{};
    char *ws = nullptr;
    size_t off_src = 0, off_sums = 0, off_wx = 0, off_wy = 0, off_out = 0, off_K = 0,
           off_tw[3] = {0, 0, 0}, bytes = 0;
};

static int ilog2_up(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// geometry and workspace layout of the combined mesh; nonzero: invalid
static int msd_layout(asd_t *atoms, int32_t sys, const asd_mm_t *left, const asd_mm_t *right,
                      int32_t cx, int32_t cy, int32_t cz, asd_msd_t *m)
{
    if (!atoms || (!left && !right)) return mm_fail(nullptr, ASD_EINVAL, "need atoms and a region");
    if (cx < 1 || cy < 1 || cz < 1) return mm_fail(nullptr, ASD_EINVAL, "bad cell");
    int32_t nx, ny, nz;
    int rc = asd_window_size(atoms, sys, &nx, &ny, &nz);
    if (rc) return rc;
    void *st = nullptr;
    if ((rc = asd_get_stream(atoms, &st))) return rc;
    double dt, edge[3];
    lattice_cell(atoms, &dt, edge);
    const int32_t cell[3] = {cx, cy, cz};
    for (const asd_mm_t *r : {left, right})
        if (r && (rc = region_fits(const_cast<asd_mm_t *>(r), dt, edge, cell, ny, nz, st))) return rc;
    int32_t dcell[3], dmesh[3];
    if (demag_mesh(atoms, dcell, dmesh) != ASD_OK || dcell[0] != cx || dcell[1] != cy || dcell[2] != cz)
        return mm_fail(nullptr, ASD_EINVAL, "the atomistic handle needs demag_cell = (%d, %d, %d)", cx, cy, cz);
    if (nx % cx) return mm_fail(nullptr, ASD_EINVAL, "the window's columns must fill whole coarse cells");
    if (track_columns(atoms, sys) == 0) return mm_fail(nullptr, ASD_EINVAL, "system %d has no track", sys);
    m->atoms = atoms;
    m->sys = sys;
    m->left = const_cast<asd_mm_t *>(left);
    m->right = const_cast<asd_mm_t *>(right);
    m->cell[0] = cx;
    m->cell[1] = cy;
    m->cell[2] = cz;
    m->nL = left ? left->p.nx : 0;
    m->nR = right ? right->p.nx : 0;
    m->nA = nx / cx;
    m->NX = m->nL + m->nA + m->nR;
    m->ny = dmesh[1];
    m->nz = dmesh[2];
    if (m->NX > 512 || m->ny > 256 || m->nz > 256)
        return mm_fail(nullptr, ASD_EUNSUPPORTED, "the window's mesh is limited to 512 x 256 x 256 cells");
    m->V = ((cx * edge[0]) * (cy * edge[1])) * (cz * edge[2]);
    DemagDev &g = m->dm;
    std::memset(&g, 0, sizeof g);
    g.on = 1;
    g.cx = cx;
    g.cy = cy;
    g.cz = cz;
    g.ncx = m->NX;
    g.ncy = m->ny;
    g.ncz = m->nz;
    g.ncell = g.ncx * g.ncy * g.ncz;
    g.lx = ilog2_up(2 * g.ncx - 1);
    g.ly = ilog2_up(2 * g.ncy - 1);
    g.lz = ilog2_up(2 * g.ncz - 1);
    g.n_sys = 2;
    const int Px = 1 << g.lx, Py = 1 << g.ly, Pz = 1 << g.lz, Pxh = Px / 2 + 1;
    // x lines per workgroup of the y and z passes: two LDS buffers of at most
    // 1024 complex doubles, and no fewer than 512 workgroups while lines split
    int xb = 1;
    while (xb * 2 <= Pxh && xb * 2 * (Py + 1) <= 1024 &&
           (int64_t)((Pxh + 2 * xb - 1) / (xb * 2)) * 3 * g.ncz * 2 >= 512)
        xb *= 2;
    g.xb_y = xb;
    xb = 1;
    while (xb * 2 <= Pxh && xb * 2 * 3 * (Pz + 1) <= 1024 &&
           (int64_t)((Pxh + 2 * xb - 1) / (xb * 2)) * Py * 2 >= 512)
        xb *= 2;
    g.xb_z = xb;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = align_up(off + b);
        return o;
    };
    const size_t cplx = 16;
    m->off_src = take((size_t)2 * 3 * g.ncell * sizeof(double));
    m->off_sums = take((size_t)m->nA * m->ny * m->nz * 4 * sizeof(double));
    m->off_wx = take((size_t)2 * 3 * g.ncz * g.ncy * Pxh * cplx);
    m->off_wy = take((size_t)2 * 3 * g.ncz * Py * Pxh * cplx);
    m->off_out = take((size_t)2 * 3 * g.ncell * sizeof(double));
    m->off_K = take((size_t)6 * (Px / 2 + 1) * (Py / 2 + 1) * (Pz / 2 + 1) * sizeof(double));
    m->off_tw[0] = take((size_t)std::max(Px / 2, 1) * cplx);
    m->off_tw[1] = take((size_t)std::max(Py / 2, 1) * cplx);
    m->off_tw[2] = take((size_t)std::max(Pz / 2, 1) * cplx);
    m->bytes = off;
    return ASD_OK;
}

// n coupled steps; msd (may be null): the demagnetising field of the whole
// window, evaluated before each step from the state at its start
static int msd_prepare(asd_msd_t *m);

static int multiscale_run(asd_t *atoms, int32_t sys, asd_mm_t *left, asd_mm_t *right, int32_t cx,
                          int32_t cy, int32_t cz, int64_t n, asd_msd_t *msd)
{
    if (!atoms || (!left && !right)) return mm_fail(nullptr, ASD_EINVAL, "need atoms and a region");
    if (n < 0 || cx < 1 || cy < 1 || cz < 1) return mm_fail(nullptr, ASD_EINVAL, "bad sizes");
    int32_t nx, ny, nz;
    int rc = asd_window_size(atoms, sys, &nx, &ny, &nz);
    if (rc) return rc;
    int64_t step;
    int32_t org;
    if ((rc = asd_get_state(atoms, sys, &step, &org))) return rc;
    void *st = nullptr;
    if ((rc = asd_get_stream(atoms, &st))) return rc;
    double dt, edge[3];
    lattice_cell(atoms, &dt, edge);
    const int32_t cell[3] = {cx, cy, cz};
    // one RK4 step of a region per Heun step of the atoms, on cells that line
    // up with the window's coarse cells
    for (asd_mm_t *m : {left, right})
        if (m && (rc = region_fits(m, dt, edge, cell, ny, nz, st))) return rc;
    if (nx < cx || org < cx) return mm_fail(nullptr, ASD_EINVAL, "window too narrow or too close to the track start");
    // both regions in the same precision under a spot that does not move: one
    // launch per RK4 stage for the two
    const bool pair = left && right && left->elem == right->elem &&
                      left->drive.spot_mode != ASD_SPOT_MOVING &&
                      right->drive.spot_mode != ASD_SPOT_MOVING;
    if (pair && n > 0) {
        // the window's two boundary strips, the regions' facing faces and the
        // frozen columns beside the window: one launch for both sides each
        const int nyz = left->p.ny * left->p.nz;
        double *sumL = (double *)(left->ws + left->off_fsum), *sumR = (double *)(right->ws + right->off_fsum);
        double *dirL = (double *)(left->ws + left->off_fdir), *dirR = (double *)(right->ws + right->off_fdir);
        for (int f = 0; f < 2; ++f) {
            asd_mm_t *m = f == 0 ? left : right;
            const int face = f == 0 ? 1 : 0;
            if (!m->ghost_on[face]) {
                m->ghost_on[face] = true;
                mm_drop_graph(m);  // graphs bake the face pointers in
            }
        }
        const MMArgs aL = mm_args(left, 0), aR = mm_args(right, 0);
        const int bf = (nyz + 255) / 256;
        for (int64_t t = 0; t < n; ++t) {
            if (msd && (rc = msd_prepare(msd))) return rc;
            if ((rc = coarse_grain_pair(atoms, sys, org, org + nx - cx, cx, cx, cy, cz, sumL, sumR)))
                return rc;
            hipLaunchKernelGGL(k_mm_set_face_pair, dim3((unsigned)(2 * bf)), dim3(256), 0, left->stream,
                               (double *)(left->ws + left->off_ghost[1]), sumL,
                               (double *)(right->ws + right->off_ghost[0]), sumR, 4, nyz);
            if (left->elem == 8)
                hipLaunchKernelGGL(k_mm_get_face_pair<double>, dim3((unsigned)(2 * bf)), dim3(256), 0,
                                   left->stream, aL, 1, dirL, aR, 0, dirR, bf);
            else
                hipLaunchKernelGGL(k_mm_get_face_pair<float>, dim3((unsigned)(2 * bf)), dim3(256), 0,
                                   left->stream, aL, 1, dirL, aR, 0, dirR, bf);
            MM_HIP(left, hipGetLastError());
            if ((rc = set_columns_pair(atoms, sys, org - cx, org + nx, cx, cx, cy, cz, dirL, dirR)))
                return rc;
            if ((rc = asd_step(atoms, 1))) return rc;
            if ((rc = mm_step_pair(left, right))) return rc;
        }
        return ASD_OK;
    }
    for (int64_t t = 0; t < n; ++t) {
        if (msd && (rc = msd_prepare(msd))) return rc;
        // window -> regions: averaged boundary coarse columns
        if (left) {
            double *sum = (double *)(left->ws + left->off_fsum);
            if ((rc = asd_coarse_grain(atoms, sys, org, cx, cx, cy, cz, sum))) return rc;
            if ((rc = asd_mm_set_face(left, 1, sum, 4))) return rc;
        }
        if (right) {
            double *sum = (double *)(right->ws + right->off_fsum);
            if ((rc = asd_coarse_grain(atoms, sys, org + nx - cx, cx, cx, cy, cz, sum))) return rc;
            if ((rc = asd_mm_set_face(right, 0, sum, 4))) return rc;
        }
        // regions -> window: their boundary cells into the frozen columns
        if (left) {
            double *dir = (double *)(left->ws + left->off_fdir);
            if ((rc = asd_mm_get_face(left, 1, dir))) return rc;
            if ((rc = asd_set_columns(atoms, sys, org - cx, cx, cx, cy, cz, dir))) return rc;
        }
        if (right) {
            double *dir = (double *)(right->ws + right->off_fdir);
            if ((rc = asd_mm_get_face(right, 0, dir))) return rc;
            if ((rc = asd_set_columns(atoms, sys, org + nx, cx, cx, cy, cz, dir))) return rc;
        }
        if ((rc = asd_step(atoms, 1))) return rc;
        if (left && (rc = asd_mm_step(left, 1))) return rc;
        if (right && (rc = asd_mm_step(right, 1))) return rc;
    }
    return ASD_OK;
}

// the fields of the combined mesh from the state at the start of the step:
// sources, convolution, then the regions' held fields and the atoms' field
// of the regions
static int msd_prepare(asd_msd_t *m)
{
    int64_t step;
    int32_t org;
    int rc;
    if ((rc = asd_get_state(m->atoms, m->sys, &step, &org))) return rc;
    void *st = nullptr;
    if ((rc = asd_get_stream(m->atoms, &st))) return rc;
    double *sums = (double *)(m->ws + m->off_sums);
    if (m->nA > 0 && (rc = asd_coarse_grain(m->atoms, m->sys, org, m->nA * m->cell[0], m->cell[0],
                                            m->cell[1], m->cell[2], sums)))
        return rc;
    double dt, edge[3];
    lattice_cell(m->atoms, &dt, edge);
    MsdRegion L{}, R{};
    MsdRegion *rg[2] = {&L, &R};
    asd_mm_t *reg2[2] = {m->left, m->right};
    for (int k = 0; k < 2; ++k) {
        asd_mm_t *r = reg2[k];
        if (!r) continue;
        // a spot that does not move: the region's m_e(T) per cell, computed
        // once by its parameter pass, is the one at every time
        const bool still = r->drive.spot_mode != ASD_SPOT_MOVING;
        if (still && !r->params_valid) {
            const MMArgs a0 = mm_args(r, 0);
            hipLaunchKernelGGL(k_mm_params, dim3((unsigned)((r->n + kMMTile - 1) / kMMTile)),
                               dim3(kMMTile), 0, r->stream, a0, 0.0);
            r->params_valid = true;
        }
        rg[k]->a = mm_args(r, 0);
        rg[k]->elem = r->elem;
        rg[k]->off = k == 0 ? 0 : m->nL + m->nA;
        rg[k]->me_ready = still ? 1 : 0;
        rg[k]->scale = r->p.Ms0 * m->V / m->mu_s;
    }
    const double t = (double)step * dt;
    double *src = (double *)(m->ws + m->off_src);
    const int64_t ncell = m->dm.ncell;
    hipLaunchKernelGGL(k_msd_sources, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0,
                       (hipStream_t)st, src, m->NX, m->ny, m->nz, (const double *)sums, m->nA, m->nL,
                       L, m->left ? 1 : 0, R, m->right ? 1 : 0, t);
    if (hipGetLastError() != hipSuccess) return mm_fail(nullptr, ASD_EHIP, "demagnetising sources launch failed");
    if (launch_demag_cells(m->dm, src, st)) return mm_fail(nullptr, ASD_EHIP, "demagnetising field launch failed");
    const double *out = (const double *)(m->ws + m->off_out);
    // the atoms: the field of the regions' cells (source set 1)
    if ((rc = set_cell_field(m->atoms, m->sys, out + 3 * ncell, m->NX, m->nL))) return rc;
    // the regions: the field of every cell (set 0), held through the step
    asd_mm_t *reg[2] = {m->left, m->right};
    const int32_t off[2] = {0, m->nL + m->nA};
    for (int k = 0; k < 2; ++k) {
        asd_mm_t *r = reg[k];
        if (!r) continue;
        if (r->bd != out || r->bd_nx != m->NX || r->bd_off != off[k]) {
            r->bd = out;
            r->bd_nx = m->NX;
            r->bd_off = off[k];
            mm_drop_graph(r);
        }
    }
    return ASD_OK;
}

static void msd_release(asd_msd_t *m)
{
    for (asd_mm_t *r : {m->left, m->right})
        if (r && r->bd) {
            r->bd = nullptr;
            r->bd_nx = r->bd_off = 0;
            mm_drop_graph(r);
        }
    (void)clear_cell_field(m->atoms);
}

int asd_msd_workspace_bytes(asd_t *atoms, int32_t sys, const asd_mm_t *left,
                            const asd_mm_t *right, int32_t cx, int32_t cy, int32_t cz,
                            size_t *bytes)
{
    if (!bytes) return mm_fail(nullptr, ASD_EINVAL, "bytes is NULL");
    asd_msd_t m;
    int rc = msd_layout(atoms, sys, left, right, cx, cy, cz, &m);
    if (rc) return rc;
    *bytes = m.bytes;
    return ASD_OK;
}

int asd_msd_create(asd_t *atoms, int32_t sys, asd_mm_t *left, asd_mm_t *right, int32_t cx,
                   int32_t cy, int32_t cz, void *workspace, size_t workspace_bytes,
                   asd_msd_t **out)
{
    if (!out) return mm_fail(nullptr, ASD_EINVAL, "out is NULL");
    *out = nullptr;
    asd_msd_t *m = new (std::nothrow) asd_msd_t();
    if (!m) return mm_fail(nullptr, ASD_ENOMEM, "host allocation failed");
    int rc = msd_layout(atoms, sys, left, right, cx, cy, cz, m);
    if (rc) {
        delete m;
        return rc;
    }
    if (!workspace || ((uintptr_t)workspace % kMMAlign) != 0 || workspace_bytes < m->bytes) {
        const int code = workspace_bytes < m->bytes ? ASD_ENOMEM : ASD_EINVAL;
        delete m;
        return mm_fail(nullptr, code, "workspace must be 256-byte aligned and hold asd_msd_workspace_bytes");
    }
    m->ws = (char *)workspace;
    // mu_s from the spectrum's units: the atoms' moment
    double dt, edge[3];
    lattice_cell(atoms, &dt, edge);
    m->mu_s = atom_moment(atoms);
    void *stv = nullptr;
    (void)asd_get_stream(atoms, &stv);
    hipStream_t st = (hipStream_t)stv;
    DemagDev &g = m->dm;
    const int Px = 1 << g.lx, Py = 1 << g.ly, Pz = 1 << g.lz;
    const double dx = cx * edge[0], dy = cy * edge[1], dz = cz * edge[2];
    // the one-workgroup y-z pass (direct sums along z) where its LDS fits
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds_max = 0;
    const size_t need = demag_yz_lds_bytes(g, (int)sizeof(double));
    g.yzf = need > 0 && need <= (size_t)lds_max ? 1 : 0;
    std::vector<double> oct;
    if (g.yzf)
        demag_mixed(g.ncx, g.ncy, g.ncz, dx, dy, dz, g.lx, g.ly,
                    -1.25663706212e-6 * m->mu_s / (((dx * dy) * dz) * ((double)Px * Py)), oct);
    else
        demag_spectrum(g.ncx, g.ncy, g.ncz, dx, dy, dz, g.lx, g.ly, g.lz,
                       -1.25663706212e-6 * m->mu_s / (((dx * dy) * dz) * ((double)Px * Py * Pz)),
                       oct);
    hipError_t e = hipMemcpyAsync(m->ws + m->off_K, oct.data(), oct.size() * sizeof(double),
                                  hipMemcpyHostToDevice, st);
    std::vector<std::vector<double>> tw(3);
    const int lp[3] = {g.lx, g.ly, g.lz};
    for (int ax = 0; ax < 3 && e == hipSuccess; ++ax) {
        const int P = 1 << lp[ax], half = std::max(P / 2, 1);
        tw[ax].resize((size_t)2 * half);
        for (int q = 0; q < half; ++q) {
            const double ang = -2.0 * M_PI * (double)q / (double)P;
            tw[ax][2 * q] = std::cos(ang);
            tw[ax][2 * q + 1] = std::sin(ang);
        }
        e = hipMemcpyAsync(m->ws + m->off_tw[ax], tw[ax].data(), tw[ax].size() * sizeof(double),
                           hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete m;
        return mm_fail(nullptr, ASD_EHIP, "demagnetising set-up copy failed: %s", hipGetErrorString(e));
    }
    g.wx = m->ws + m->off_wx;
    g.wy = m->ws + m->off_wy;
    g.bd[0] = m->ws + m->off_out;
    g.bd[1] = nullptr;
    g.K = m->ws + m->off_K;
    for (int ax = 0; ax < 3; ++ax) g.tw[ax] = m->ws + m->off_tw[ax];
    g.bstray = nullptr;
    *out = m;
    return ASD_OK;
}

int asd_msd_destroy(asd_msd_t *m)
{
    if (!m) return ASD_OK;
    msd_release(m);
    delete m;
    return ASD_OK;
}

int asd_multiscale_step_demag(asd_msd_t *m, int64_t n)
{
    if (!m) return mm_fail(nullptr, ASD_EINVAL, "NULL multiscale demagnetising field");
    const int rc = multiscale_run(m->atoms, m->sys, m->left, m->right, m->cell[0], m->cell[1],
                                  m->cell[2], n, m);
    msd_release(m);
    return rc;
}

int asd_msd_fields(asd_msd_t *m, double *all, double *regions, int32_t *mesh)
{
    if (!m) return mm_fail(nullptr, ASD_EINVAL, "NULL multiscale demagnetising field");
    void *st = nullptr;
    int rc = asd_get_stream(m->atoms, &st);
    if (rc) return rc;
    const size_t n = (size_t)3 * m->dm.ncell;
    const double *out = (const double *)(m->ws + m->off_out);
    hipError_t e = hipSuccess;
    if (all) e = hipMemcpyAsync(all, out, n * sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)st);
    if (regions && e == hipSuccess)
        e = hipMemcpyAsync(regions, out + n, n * sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)st);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)st);
    if (e != hipSuccess) return mm_fail(nullptr, ASD_EHIP, "field copy failed: %s", hipGetErrorString(e));
    if (mesh) {
        mesh[0] = m->NX;
        mesh[1] = m->ny;
        mesh[2] = m->nz;
    }
    return ASD_OK;
}

int asd_multiscale_step(asd_t *atoms, int32_t sys, asd_mm_t *left, asd_mm_t *right, int32_t cx,
                        int32_t cy, int32_t cz, int64_t n)
{
    return multiscale_run(atoms, sys, left, right, cx, cy, cz, n, nullptr);
}

int asd_multiscale_shift(asd_t *atoms, int32_t sys, asd_mm_t *left, asd_mm_t *right, int32_t cx,
                         int32_t cy, int32_t cz, const double *enter, double *leave)
{
    if (!atoms || (!left && !right)) return mm_fail(nullptr, ASD_EINVAL, "need atoms and a region");
    if (cx < 1 || cy < 1 || cz < 1) return mm_fail(nullptr, ASD_EINVAL, "bad cell");
    if (right && !enter) return mm_fail(right, ASD_EINVAL, "the right region needs the track ahead");
    int32_t nx, ny, nz;
    int rc = asd_window_size(atoms, sys, &nx, &ny, &nz);
    if (rc) return rc;
    int64_t step;
    int32_t org;
    if ((rc = asd_get_state(atoms, sys, &step, &org))) return rc;
    void *st = nullptr;
    if ((rc = asd_get_stream(atoms, &st))) return rc;
    double dt, edge[3];
    lattice_cell(atoms, &dt, edge);
    const int32_t cell[3] = {cx, cy, cz};
    for (asd_mm_t *m : {left, right})
        if (m && (rc = region_fits(m, dt, edge, cell, ny, nz, st))) return rc;
    if (nx < cx) return mm_fail(nullptr, ASD_EINVAL, "window narrower than a coarse cell");
    // the entering columns and the moved window must lie on the track
    const int32_t sx = track_columns(atoms, sys);
    if (sx == 0) return mm_fail(nullptr, ASD_EINVAL, "system %d has no track", sys);
    if ((int64_t)org + nx + cx > sx)
        return mm_fail(nullptr, ASD_ESTATE, "the window would leave its track of %d columns", sx);
    const int nyz = (left ? left : right)->p.ny * (left ? left : right)->p.nz;
    const int blocks = (nyz + 255) / 256;
    // 1. trailing end: the leaving atomistic columns, averaged, become the left
    // region's new last cells
    if (left) {
        double *sum = (double *)(left->ws + left->off_fsum);
        if ((rc = asd_coarse_grain(atoms, sys, org, cx, cx, cy, cz, sum))) return rc;
        const MMArgs a = mm_args(left, 0);
        if (left->elem == 8)
            hipLaunchKernelGGL(k_mm_shift<double>, dim3(blocks), dim3(256), 0, left->stream, a, sum, 4, leave);
        else
            hipLaunchKernelGGL(k_mm_shift<float>, dim3(blocks), dim3(256), 0, left->stream, a, sum, 4, leave);
        MM_HIP(left, hipGetLastError());
    }
    // 2. leading end: the right region's first cells enter the atoms by
    // thermalisation around m_e(T) m, then the region moves down one cell
    if (right) {
        double *mface = (double *)(right->ws + right->off_fdir);
        const MMArgs a = mm_args(right, 0);
        const double t = (double)step * right->p.dt;
        if (right->elem == 8) {
            hipLaunchKernelGGL(k_mm_face_moment<double>, dim3(blocks), dim3(256), 0, right->stream, a, 0, t, mface);
        } else {
            hipLaunchKernelGGL(k_mm_face_moment<float>, dim3(blocks), dim3(256), 0, right->stream, a, 0, t, mface);
        }
        MM_HIP(right, hipGetLastError());
        if ((rc = asd_thermalise_columns(atoms, sys, org + nx, cx, cx, cy, cz, mface, (uint32_t)step)))
            return rc;
        if (right->elem == 8)
            hipLaunchKernelGGL(k_mm_shift<double>, dim3(blocks), dim3(256), 0, right->stream, a, enter, 3, nullptr);
        else
            hipLaunchKernelGGL(k_mm_shift<float>, dim3(blocks), dim3(256), 0, right->stream, a, enter, 3, nullptr);
        MM_HIP(right, hipGetLastError());
    }
    // 3. the atomistic window moves
    return asd_shift_window(atoms, cx);
}

const char *asd_mm_last_error(const asd_mm_t *h) { return h ? h->err.c_str() : g_mm_err.c_str(); }

}  // extern "C"
