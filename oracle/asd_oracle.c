/*
 * asd_oracle.c -- plain, slow, FP64 CPU oracle for the stochastic
 * Landau-Lifshitz-Gilbert (sLLG) Heun step of atomistic spin dynamics.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  It shares no code,
 * header, table or constant generator with the GPU library; the two agree
 * only because both follow the same written definitions.
 *
 * What it follows (Gija et al., "Multiscale micromagnetic / atomistic
 * modeling of heat assisted magnetic recording", arXiv 2502.02236):
 *   - Eq. 1   sLLG equation (Gilbert form), integrated here in the
 *             algebraically equivalent explicit Landau-Lifshitz form with
 *             prefactor gamma/(1+alpha^2), by Heun's predictor-corrector
 *             with renormalisation of every stage (the paper names no
 *             atomistic integrator; Heun is this project's reading).
 *   - Sec. II thermal field: Gaussian, zero mean, standard deviation
 *             sqrt(2 alpha kB T / (gamma mu_s dt)) (tesla form of the
 *             paper's A/m expression), drawn fresh every time step and
 *             shared by the predictor and the corrector.
 *   - Eq. 2   exchange field (1/mu_s) sum_j J_ij S_j over neighbour shells
 *             (SC: 6 nearest neighbours; L1_0 Fe sublattice: shells).
 *   - Eq. 3   uniaxial anisotropy field (2 k_u/mu_s)(S.z) z.
 *   - Sec. II/III Zeeman write field with bit-timed polarity and a
 *             Gaussian laser-spot temperature profile (Fig. 2).
 *   - Sec. II Voronoi construction of exchange-decoupled grains.
 *   - Eq. 6   moment sums (per-grain magnetisation sums, coarse cells of
 *             the window-end transfer and of the demagnetising field).
 *   - Eq. 7   demagnetising field on coarse cells, H = -sum N M, with
 *             Newell's cell-averaged tensor, summed directly.
 *
 * Floating point: FP64, compiled with -ffp-contract=off.  The
 * transcendentals the noise and the temperature need (ln, sin/cos of
 * 2*pi*u, exp) are this file's own fixed-order series built from + - * /
 * only, so that the result is a function of the definitions alone and not
 * of a vendor math library.  Random numbers: Philox4x32 with R rounds as
 * defined by Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "asd_oracle.h"

/* ------------------------------------------------------------------ */
/* Philox4x32-R (Salmon et al. 2011, Sec. 4.3 / Table 2).             */
/* One round: the two 32x32->64 products of the S-box, xor with the  */
/* key and the other two words, then the key is bumped by the Weyl   */
/* constants.  The first round uses the key as given.                */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32(int rounds, uint32_t k0, uint32_t k1, const uint32_t ctr[4],
                    uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int r = 0; r < rounds; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox_batch(int rounds, uint64_t seed, const uint32_t *ctr, uint32_t *out,
                      int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        orc_philox4x32(rounds, (uint32_t)seed, (uint32_t)(seed >> 32), ctr + 4 * i,
                       out + 4 * i);
}

/* ------------------------------------------------------------------ */
/* Portable FP64 transcendentals (own definitions, fixed order).      */
/* ------------------------------------------------------------------ */
static const double LN2_HI = 6.93147180369123816490e-01; /* 22 trailing zero bits */
static const double LN2_LO = 1.90821492927058770002e-10;
static const double SQRT_HALF = 0.70710678118654752440;
static const double PIO2 = 1.57079632679489661923;
static const double INV_LN2 = 1.44269504088896340736;

/* ln(u) for u > 0 finite: u = m 2^e with m in [sqrt(1/2), sqrt(2)),
 * ln m = 2 atanh(z), z = (m-1)/(m+1), atanh series through z^21. */
double orc_ln(double u)
{
    int e;
    double m = frexp(u, &e); /* exact: m in [0.5, 1) */
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
    double lnm = (2.0 * z) * p;
    double de = (double)e;
    return de * LN2_HI + (de * LN2_LO + lnm);
}

/* sin(2 pi u), cos(2 pi u) for u in [0, 1): exact quadrant split of 4u,
 * then Taylor polynomials on th = (4u - q) pi/2 in [-pi/4, pi/4]:
 * sin th = th - th^3 P(th^2), P through the th^21 term;
 * cos th = 1 - th^2 C(th^2), C through the th^20 term. */
void orc_sincos2pi(double u, double *s_out, double *c_out)
{
    double t = 4.0 * u;
    double q = floor(t + 0.5);
    double x = t - q;
    double th = x * PIO2;
    double th2 = th * th;
    double ps = -1.0 / 51090942171709440000.0;
    ps = 1.0 / 121645100408832000.0 + th2 * ps;
    ps = -1.0 / 355687428096000.0 + th2 * ps;
    ps = 1.0 / 1307674368000.0 + th2 * ps;
    ps = -1.0 / 6227020800.0 + th2 * ps;
    ps = 1.0 / 39916800.0 + th2 * ps;
    ps = -1.0 / 362880.0 + th2 * ps;
    ps = 1.0 / 5040.0 + th2 * ps;
    ps = -1.0 / 120.0 + th2 * ps;
    ps = 1.0 / 6.0 + th2 * ps;
    double s = th - (th * th2) * ps;
    double pc = -1.0 / 2432902008176640000.0;
    pc = 1.0 / 6402373705728000.0 + th2 * pc;
    pc = -1.0 / 20922789888000.0 + th2 * pc;
    pc = 1.0 / 87178291200.0 + th2 * pc;
    pc = -1.0 / 479001600.0 + th2 * pc;
    pc = 1.0 / 3628800.0 + th2 * pc;
    pc = -1.0 / 40320.0 + th2 * pc;
    pc = 1.0 / 720.0 + th2 * pc;
    pc = -1.0 / 24.0 + th2 * pc;
    pc = 0.5 + th2 * pc;
    double c = 1.0 - th2 * pc;
    int quad = ((int)q) & 3;
    switch (quad) {
    case 0: *s_out = s; *c_out = c; break;
    case 1: *s_out = c; *c_out = -s; break;
    case 2: *s_out = -s; *c_out = -c; break;
    default: *s_out = -c; *c_out = s; break;
    }
}

/* exp(x) for finite x <= 0: x = k ln2 + r with k = floor(x/ln2 + 1/2),
 * r reduced with the split ln2, Taylor polynomial through r^13, then an
 * exact scaling by 2^k.  Below -700 the result is 0. */
double orc_exp(double x)
{
    if (x < -700.0)
        return 0.0;
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

/* ------------------------------------------------------------------ */
/* Gaussian triple for one site and step (Box-Muller on Philox words) */
/* counter = (site, step, system, stage), key = (lo32 seed, hi32 seed) */
/* u_r = (w + 1/2) 2^-32 in (0,1), u_t = w 2^-32 in [0,1)             */
/* (gx, gy) = r (cos, sin)(2 pi u_t) from (w0, w1); gz = r cos(...) of */
/* (w2, w3); the fourth Gaussian is not used.                          */
/* ------------------------------------------------------------------ */
static const double TWO_M32 = 2.3283064365386962890625e-10; /* 2^-32 */

static void box_muller(uint32_t wr, uint32_t wt, double *g_cos, double *g_sin)
{
    double ur = ((double)wr + 0.5) * TWO_M32;
    double ut = (double)wt * TWO_M32;
    double r = sqrt(-2.0 * orc_ln(ur));
    double s, c;
    orc_sincos2pi(ut, &s, &c);
    *g_cos = r * c;
    *g_sin = r * s;
}

void orc_gauss3(int rounds, uint64_t seed, uint32_t site, uint32_t step, uint32_t sys,
                uint32_t stage, double g[3])
{
    uint32_t ctr[4] = {site, step, sys, stage};
    uint32_t w[4];
    orc_philox4x32(rounds, (uint32_t)seed, (uint32_t)(seed >> 32), ctr, w);
    double gx, gy, gz, unused;
    box_muller(w[0], w[1], &gx, &gy);
    box_muller(w[2], w[3], &gz, &unused);
    g[0] = gx; g[1] = gy; g[2] = gz;
}

void orc_ln_batch(const double *u, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_ln(u[i]);
}
void orc_exp_batch(const double *x, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_exp(x[i]);
}
void orc_sincos2pi_batch(const double *u, double *s, double *c, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) orc_sincos2pi(u[i], s + i, c + i);
}
void orc_gauss3_batch(int rounds, uint64_t seed, const uint32_t *site, const uint32_t *step,
                      uint32_t sys, uint32_t stage, double *g, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) orc_gauss3(rounds, seed, site[i], step[i], sys, stage, g + 3 * i);
}

/* ------------------------------------------------------------------ */
/* Lattices by brute-force geometry.                                  */
/* Sites carry integer coordinates (X, Y, Z) in units (hx, hy, hz).   */
/* SC: X = x, Y = y, Z = z, units (a, a, a).                          */
/* L1_0 Fe sublattice (Appendix A, Fig. 5): Fe at the corners and the */
/* centre of the a x a face of every a x a x c cell: X = 2x + s,      */
/* Y = 2y + s, Z = z with units (a/2, a/2, c), s = 0, 1.              */
/* Site index: SC x + nx (y + ny z); L1_0 2 (x + nx (y + ny z)) + s.  */
/* Neighbours: every site within the cutoff, found by scanning a box  */
/* of integer offsets, with minimum-image wrap on periodic axes; each */
/* is assigned to the shell whose radius it matches.  Row order:      */
/* shell ascending, then the offset (dZ, dY, dX) lexicographically.   */
/* ------------------------------------------------------------------ */
static void site_coords(int kind, int nx, int ny, int64_t i, int64_t *X, int64_t *Y, int64_t *Z)
{
    if (kind == ORC_SC) {
        *X = i % nx;
        *Y = (i / nx) % ny;
        *Z = i / ((int64_t)nx * ny);
    } else {
        int64_t cell = i / 2, s = i % 2;
        int64_t cx = cell % nx, cy = (cell / nx) % ny, cz = cell / ((int64_t)nx * ny);
        *X = 2 * cx + s;
        *Y = 2 * cy + s;
        *Z = cz;
    }
}

/* returns site index or -1 if no site sits at (X, Y, Z) */
static int64_t site_at(int kind, int nx, int ny, int nz, int64_t X, int64_t Y, int64_t Z)
{
    if (kind == ORC_SC) {
        if (X < 0 || X >= nx || Y < 0 || Y >= ny || Z < 0 || Z >= nz) return -1;
        return X + (int64_t)nx * (Y + (int64_t)ny * Z);
    }
    if (X < 0 || X >= 2 * (int64_t)nx || Y < 0 || Y >= 2 * (int64_t)ny || Z < 0 || Z >= nz)
        return -1;
    if (((X - Y) % 2) != 0) return -1;
    int64_t s = X % 2;
    int64_t cx = (X - s) / 2, cy = (Y - s) / 2;
    return 2 * (cx + (int64_t)nx * (cy + (int64_t)ny * Z)) + s;
}

static int64_t wrap(int64_t v, int64_t L) { return ((v % L) + L) % L; }

typedef struct {
    int shell;
    int64_t dz, dy, dx;
    int64_t j;
} nb_entry;

static int nb_cmp(const void *a, const void *b)
{
    const nb_entry *p = (const nb_entry *)a, *q = (const nb_entry *)b;
    if (p->shell != q->shell) return p->shell < q->shell ? -1 : 1;
    if (p->dz != q->dz) return p->dz < q->dz ? -1 : 1;
    if (p->dy != q->dy) return p->dy < q->dy ? -1 : 1;
    if (p->dx != q->dx) return p->dx < q->dx ? -1 : 1;
    return 0;
}

int64_t orc_lattice_sites(int kind, int nx, int ny, int nz)
{
    return (kind == ORC_SC ? 1 : 2) * (int64_t)nx * ny * nz;
}

/* Pass row_ptr/col/shell = NULL to get the number of neighbour entries. */
int64_t orc_build_neighbours(int kind, int nx, int ny, int nz, const int periodic[3], double a,
                             double c, int n_shells, const double *radius, int64_t *row_ptr,
                             int32_t *col, int8_t *shell)
{
    double hx = kind == ORC_SC ? a : 0.5 * a;
    double hy = hx;
    double hz = kind == ORC_SC ? a : c;
    double rmax = 0.0;
    for (int s = 0; s < n_shells; ++s) rmax = radius[s] > rmax ? radius[s] : rmax;
    int64_t mx = (int64_t)ceil(rmax / hx) + 1, my = (int64_t)ceil(rmax / hy) + 1,
            mz = (int64_t)ceil(rmax / hz) + 1;
    int64_t LX = kind == ORC_SC ? nx : 2 * (int64_t)nx;
    int64_t LY = kind == ORC_SC ? ny : 2 * (int64_t)ny;
    int64_t LZ = nz;
    int64_t n = orc_lattice_sites(kind, nx, ny, nz);
    nb_entry *buf = (nb_entry *)malloc(sizeof(nb_entry) * (size_t)((2 * mx + 1) * (2 * my + 1) * (2 * mz + 1)));
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t X, Y, Z;
        site_coords(kind, nx, ny, i, &X, &Y, &Z);
        int cnt = 0;
        for (int64_t dz = -mz; dz <= mz; ++dz)
            for (int64_t dy = -my; dy <= my; ++dy)
                for (int64_t dx = -mx; dx <= mx; ++dx) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    int64_t Xj = X + dx, Yj = Y + dy, Zj = Z + dz;
                    if (periodic[0]) Xj = wrap(Xj, LX);
                    if (periodic[1]) Yj = wrap(Yj, LY);
                    if (periodic[2]) Zj = wrap(Zj, LZ);
                    int64_t j = site_at(kind, nx, ny, nz, Xj, Yj, Zj);
                    if (j < 0 || j == i) continue;
                    double ddx = (double)dx * hx, ddy = (double)dy * hy, ddz = (double)dz * hz;
                    double d = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
                    for (int s = 0; s < n_shells; ++s) {
                        if (fabs(d - radius[s]) <= 1e-6 * radius[s]) {
                            buf[cnt].shell = s;
                            buf[cnt].dz = dz; buf[cnt].dy = dy; buf[cnt].dx = dx;
                            buf[cnt].j = j;
                            ++cnt;
                            break;
                        }
                    }
                }
        qsort(buf, (size_t)cnt, sizeof(nb_entry), nb_cmp);
        if (row_ptr) row_ptr[i] = total;
        for (int k = 0; k < cnt; ++k) {
            if (col) col[total + k] = (int32_t)buf[k].j;
            if (shell) shell[total + k] = (int8_t)buf[k].shell;
        }
        total += cnt;
    }
    if (row_ptr) row_ptr[n] = total;
    free(buf);
    return total;
}

/* in-plane site positions in metres, in the frame of the stored lattice */
void orc_site_positions(int kind, int nx, int ny, int nz, double a, double *px, double *py)
{
    double h = kind == ORC_SC ? a : 0.5 * a;
    int64_t n = orc_lattice_sites(kind, nx, ny, nz);
    for (int64_t i = 0; i < n; ++i) {
        int64_t X, Y, Z;
        site_coords(kind, nx, ny, i, &X, &Y, &Z);
        px[i] = (double)X * h;
        py[i] = (double)Y * h;
    }
}

/* ------------------------------------------------------------------ */
/* Columnar Voronoi grains (Sec. II "Voronoi construction", Sec. III). */
/* Integer geometry in units of a/Q (SC) or a/(2Q) half-cells (L1_0). */
/* Site p = (X Q, Y Q).  Label = index of the nearest seed (squared   */
/* distance, minimum image on periodic axes; ties to the lower index). */
/* A site is non-magnetic (label -1) when some other seed j has        */
/* (d_j^2 - d_g^2)^2 < w^2 |s_j - s_g|^2, i.e. it lies closer than w/2 */
/* to the bisector of its own seed g and seed j.  Brute force over all */
/* seeds.                                                              */
/* ------------------------------------------------------------------ */
static int64_t min_image(int64_t d, int64_t L, int periodic)
{
    if (!periodic) return d;
    d = ((d % L) + L) % L;
    if (2 * d > L) d -= L;
    return d;
}

void orc_voronoi_labels(int kind, int nx, int ny, int nz, const int periodic[2], int Q,
                        const int32_t *seeds_xy, int n_seeds, int64_t w_units, int32_t *labels)
{
    int64_t LX = (kind == ORC_SC ? nx : 2 * (int64_t)nx) * (int64_t)Q;
    int64_t LY = (kind == ORC_SC ? ny : 2 * (int64_t)ny) * (int64_t)Q;
    int64_t n = orc_lattice_sites(kind, nx, ny, nz);
    int64_t *dxs = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_seeds);
    int64_t *dys = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_seeds);
    for (int64_t i = 0; i < n; ++i) {
        int64_t X, Y, Z;
        site_coords(kind, nx, ny, i, &X, &Y, &Z);
        int64_t px = X * Q, py = Y * Q;
        int g = -1;
        int64_t best = 0;
        for (int k = 0; k < n_seeds; ++k) {
            dxs[k] = min_image(px - seeds_xy[2 * k], LX, periodic[0]);
            dys[k] = min_image(py - seeds_xy[2 * k + 1], LY, periodic[1]);
            int64_t d2 = dxs[k] * dxs[k] + dys[k] * dys[k];
            if (g < 0 || d2 < best) {
                g = k;
                best = d2;
            }
        }
        int magnetic = 1;
        for (int k = 0; k < n_seeds && magnetic; ++k) {
            if (k == g) continue;
            int64_t d2 = dxs[k] * dxs[k] + dys[k] * dys[k];
            int64_t diff = d2 - best;
            int64_t sx = dxs[g] - dxs[k], sy = dys[g] - dys[k];
            int64_t sep2 = sx * sx + sy * sy;
            if (diff * diff < w_units * w_units * sep2) magnetic = 0;
        }
        labels[i] = magnetic ? g : -1;
    }
    free(dxs);
    free(dys);
}

/* ------------------------------------------------------------------ */
/* sLLG right-hand side in Landau-Lifshitz form (Eq. 1 rewritten):    */
/*   dS/dt = gp (S x B + alpha S x (S x B)),  gp = -gamma/(1+alpha^2) */
/* ------------------------------------------------------------------ */
static void ll_rhs(double gp, double alpha, const double S[3], const double B[3], double f[3])
{
    double cx = S[1] * B[2] - S[2] * B[1];
    double cy = S[2] * B[0] - S[0] * B[2];
    double cz = S[0] * B[1] - S[1] * B[0];
    double dx = S[1] * cz - S[2] * cy;
    double dy = S[2] * cx - S[0] * cz;
    double dz = S[0] * cy - S[1] * cx;
    f[0] = gp * (cx + alpha * dx);
    f[1] = gp * (cy + alpha * dy);
    f[2] = gp * (cz + alpha * dz);
}

static void normalise(double v[3])
{
    double n = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    v[0] = v[0] / n;
    v[1] = v[1] / n;
    v[2] = v[2] / n;
}

/* write-field polarity at step n (bit sequence by field polarity): bit
 * (n / steps_per_bit) mod n_bits, +1 when set; +1 without a pattern */
static double bit_polarity(int n_bits, const uint8_t *bits, int64_t steps_per_bit, int64_t n)
{
    if (n_bits <= 0 || steps_per_bit <= 0) return 1.0;
    int64_t k = (n / steps_per_bit) % n_bits;
    return bits[k] ? 1.0 : -1.0;
}

static double polarity(const orc_system *s, int64_t n)
{
    return bit_polarity(s->n_bits, s->bits, s->steps_per_bit, n);
}

/* Gaussian laser spot (Sec. III, Fig. 2): T = Tamb + (Tpk-Tamb) exp(-r^2/2s^2),
 * s = FWHM / (2 sqrt(2 ln 2)), r the in-plane distance to the spot centre. */
static double site_temperature(const orc_system *s, int64_t i, int64_t n)
{
    if (s->spot_mode == ORC_SPOT_NONE) return s->T_amb;
    double xc;
    if (s->spot_mode == ORC_SPOT_MOVING)
        xc = s->x0 + s->v * ((double)n * s->dt);
    else
        xc = (double)s->origin * s->hx + s->x0;
    double sd = s->fwhm / 2.3548200450309493;
    double inv2s2 = 1.0 / ((2.0 * sd) * sd);
    double dx = s->px[i] - xc;
    double dy = s->py[i] - s->y0;
    double q = (dx * dx + dy * dy) * inv2s2;
    return s->T_amb + (s->T_peak - s->T_amb) * orc_exp(-q);
}

static int magnetic(const orc_system *s, int64_t i) { return s->label[i] >= 0; }
static int evolves(const orc_system *s, int64_t i)
{
    return magnetic(s, i) && (s->active == NULL || s->active[i]);
}

/* B at site i for spin configuration (Sx,Sy,Sz): Eq. 2 grouped by shell,
 * + Eq. 3 + write field + thermal field, in this order. */
static void field(const orc_system *s, const double *Sx, const double *Sy, const double *Sz,
                  int64_t i, double pol, const double bth[3], const double *bd, double B[3])
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int sh = 0; sh < s->n_shells; ++sh) {
        double part[3] = {0.0, 0.0, 0.0};
        for (int64_t k = s->row_ptr[i]; k < s->row_ptr[i + 1]; ++k) {
            if (s->shell[k] != sh) continue;
            int64_t j = s->col[k];
            if (s->label[j] != s->label[i]) continue; /* exchange-decoupled grains */
            part[0] = part[0] + Sx[j];
            part[1] = part[1] + Sy[j];
            part[2] = part[2] + Sz[j];
        }
        double cex = s->J[sh] / s->mu_s;
        acc[0] = acc[0] + cex * part[0];
        acc[1] = acc[1] + cex * part[1];
        acc[2] = acc[2] + cex * part[2];
    }
    double ku = s->ku_grain ? s->ku_grain[s->label[i]] : s->ku;
    double can = (2.0 * ku) / s->mu_s;
    double ban[3] = {0.0, 0.0, can * Sz[i]};
    for (int k = 0; k < 3; ++k)
        B[k] = ((acc[k] + ban[k]) + pol * s->B[k]) + bth[k];
    /* demagnetising field of the site's coarse cell, evaluated from the same
     * configuration as the exchange and anisotropy terms */
    if (bd && s->dcell[i] >= 0) {
        int64_t nc = (int64_t)s->dn[0] * s->dn[1] * s->dn[2];
        for (int k = 0; k < 3; ++k) B[k] = B[k] + bd[k * nc + s->dcell[i]];
    }
}

static int demag_cells(const orc_system *s, const double *Sx, const double *Sy, const double *Sz,
                       double *out);

int orc_heun_steps(const orc_system *s, double *Sx, double *Sy, double *Sz, int64_t step0,
                   int64_t nsteps)
{
    int64_t n = s->n_sites;
    double *Px = (double *)malloc(sizeof(double) * (size_t)n);
    double *Py = (double *)malloc(sizeof(double) * (size_t)n);
    double *Pz = (double *)malloc(sizeof(double) * (size_t)n);
    double *f0 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *bth = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int64_t nc = s->dn[0] > 0 ? (int64_t)s->dn[0] * s->dn[1] * s->dn[2] : 0;
    double *bd = nc ? (double *)malloc(sizeof(double) * 3 * (size_t)nc) : NULL;
    if (!Px || !Py || !Pz || !f0 || !bth || (nc && !bd)) {
        free(Px); free(Py); free(Pz); free(f0); free(bth); free(bd);
        return -1;
    }
    double gp = -s->gamma / (1.0 + s->alpha * s->alpha);
    double h = 0.5 * s->dt;
    double cth = ((2.0 * s->alpha) * ORC_KB) / ((s->gamma * s->mu_s) * s->dt);

    for (int64_t t = 0; t < nsteps; ++t) {
        int64_t step = step0 + t;
        double pol = polarity(s, step);
        if (bd && demag_cells(s, Sx, Sy, Sz, bd) != 0) {
            free(Px); free(Py); free(Pz); free(f0); free(bth); free(bd);
            return -1;
        }
        /* thermal field: one Gaussian triple per site and step */
        for (int64_t i = 0; i < n; ++i) {
            if (!evolves(s, i)) continue;
            double T = site_temperature(s, i, step);
            double sigma = sqrt(cth * T);
            double g[3];
            orc_gauss3(s->rounds, s->seed, s->ctr0[i], (uint32_t)step, s->sys_id, 0u, g);
            bth[3 * i + 0] = sigma * g[0];
            bth[3 * i + 1] = sigma * g[1];
            bth[3 * i + 2] = sigma * g[2];
        }
        /* predictor at every site before any corrector */
        for (int64_t i = 0; i < n; ++i) {
            if (!evolves(s, i)) {
                Px[i] = Sx[i]; Py[i] = Sy[i]; Pz[i] = Sz[i];
                continue;
            }
            double B[3], f[3], S[3] = {Sx[i], Sy[i], Sz[i]};
            field(s, Sx, Sy, Sz, i, pol, bth + 3 * i, bd, B);
            ll_rhs(gp, s->alpha, S, B, f);
            double P[3] = {S[0] + s->dt * f[0], S[1] + s->dt * f[1], S[2] + s->dt * f[2]};
            normalise(P);
            Px[i] = P[0]; Py[i] = P[1]; Pz[i] = P[2];
            f0[3 * i + 0] = f[0]; f0[3 * i + 1] = f[1]; f0[3 * i + 2] = f[2];
        }
        /* corrector with the predicted configuration and the same noise (the
         * demagnetising field of S' too, unless it is held through the step) */
        if (bd && !s->demag_once && demag_cells(s, Px, Py, Pz, bd) != 0) {
            free(Px); free(Py); free(Pz); free(f0); free(bth); free(bd);
            return -1;
        }
        for (int64_t i = 0; i < n; ++i) {
            if (!evolves(s, i)) continue;
            double B[3], f[3], Sp[3] = {Px[i], Py[i], Pz[i]};
            field(s, Px, Py, Pz, i, pol, bth + 3 * i, bd, B);
            ll_rhs(gp, s->alpha, Sp, B, f);
            double Q[3] = {Sx[i] + h * (f0[3 * i + 0] + f[0]), Sy[i] + h * (f0[3 * i + 1] + f[1]),
                           Sz[i] + h * (f0[3 * i + 2] + f[2])};
            normalise(Q);
            Sx[i] = Q[0]; Sy[i] = Q[1]; Sz[i] = Q[2];
        }
    }
    free(Px); free(Py); free(Pz); free(f0); free(bth); free(bd);
    return 0;
}

/* The per-site drive and the deterministic field, exported so that tests
 * can check them against closed forms: the spot temperature of site i at
 * step n, the write-field polarity of step n, and B_i without the thermal
 * and demagnetising terms (exchange, anisotropy and the polarised write
 * field, exactly as the Heun stages assemble it). */
double orc_site_temperature(const orc_system *s, int64_t i, int64_t n)
{
    return site_temperature(s, i, n);
}

double orc_polarity(const orc_system *s, int64_t n) { return polarity(s, n); }

void orc_field(const orc_system *s, const double *Sx, const double *Sy, const double *Sz,
               int64_t i, int64_t n, double B[3])
{
    const double none[3] = {0.0, 0.0, 0.0};
    field(s, Sx, Sy, Sz, i, polarity(s, n), none, NULL, B);
}

/* ------------------------------------------------------------------ */
/* Reductions: Neumaier-compensated sums.                             */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

/* per grain g (label g >= 0): (sum Sx, sum Sy, sum Sz, count) into out[4 g..];
 * total over all magnetic sites into tot[4] (Eq. 6 moment sums / mu_s).
 * Only sites inside the window (active, when a mask is set) are summed. */
void orc_magnetisation(const orc_system *s, const double *Sx, const double *Sy, const double *Sz,
                       int n_grains, double *per_grain, double tot[4])
{
    nsum *acc = (nsum *)calloc((size_t)(4 * (n_grains + 1)), sizeof(nsum));
    for (int64_t i = 0; i < s->n_sites; ++i) {
        int g = s->label[i];
        if (g < 0 || (s->active && !s->active[i])) continue;
        double v[4] = {Sx[i], Sy[i], Sz[i], 1.0};
        for (int k = 0; k < 4; ++k) {
            if (g < n_grains) nadd(&acc[4 * g + k], v[k]);
            nadd(&acc[4 * n_grains + k], v[k]);
        }
    }
    for (int g = 0; g < n_grains; ++g)
        for (int k = 0; k < 4; ++k) per_grain[4 * g + k] = nval(&acc[4 * g + k]);
    for (int k = 0; k < 4; ++k) tot[k] = nval(&acc[4 * n_grains + k]);
    free(acc);
}

/* energy (J) of the Hamiltonian whose field is Eqs. 2-3 + write field:
 * E = -1/2 sum_i sum_j J_ij S_i.S_j - sum_i k_u S_iz^2 - sum_i mu_s B.S_i,
 * with i over the magnetic sites of the window (active sites when a mask
 * is set; j over all their neighbours); out = (exchange, anisotropy,
 * Zeeman, total). */
void orc_energy(const orc_system *s, const double *Sx, const double *Sy, const double *Sz,
                int64_t step, double out[4])
{
    nsum ex = {0, 0}, an = {0, 0}, ze = {0, 0};
    double pol = polarity(s, step);
    for (int64_t i = 0; i < s->n_sites; ++i) {
        if (!magnetic(s, i) || (s->active && !s->active[i])) continue;
        for (int64_t k = s->row_ptr[i]; k < s->row_ptr[i + 1]; ++k) {
            int64_t j = s->col[k];
            if (s->label[j] != s->label[i]) continue;
            double d = Sx[i] * Sx[j] + Sy[i] * Sy[j] + Sz[i] * Sz[j];
            nadd(&ex, -0.5 * s->J[s->shell[k]] * d);
        }
        double ku = s->ku_grain ? s->ku_grain[s->label[i]] : s->ku;
        nadd(&an, -ku * Sz[i] * Sz[i]);
        nadd(&ze, -s->mu_s * pol * (s->B[0] * Sx[i] + s->B[1] * Sy[i] + s->B[2] * Sz[i]));
    }
    out[0] = nval(&ex);
    out[1] = nval(&an);
    out[2] = nval(&ze);
    out[3] = (out[0] + out[1]) + out[2];
}

/* ------------------------------------------------------------------ */
/* Window-end transfer between the atomistic lattice and a coarse     */
/* (micromagnetic) grid (Sec. II, Eq. 6).  Cells are boxes of         */
/* cx x cy x cz lattice cells over the stored columns [x0, x0+ncols)  */
/* of a lattice of sx x ny x nz cells, numbered i + ncx (j + ncy k)   */
/* with ncx = ceil(ncols/cx), ncy = ceil(ny/cy); both L1_0 sites of a */
/* lattice cell belong to its coarse cell.                            */
/* ------------------------------------------------------------------ */
static int64_t coarse_cell(int kind, int sx, int ny, int64_t site, int x0, int ncols, int cx,
                           int cy, int cz)
{
    int64_t cell = kind == ORC_SC ? site : site / 2;
    int64_t x = cell % sx, y = (cell / sx) % ny, z = cell / ((int64_t)sx * ny);
    if (x < x0 || x >= x0 + ncols) return -1;
    int64_t ncx = (ncols + cx - 1) / cx, ncy = (ny + cy - 1) / cy;
    return (x - x0) / cx + ncx * (y / cy + ncy * (z / cz));
}

/* Eq. 6 read forwards: per coarse cell the sum of the unit spins of its
 * magnetic sites and their number, out[ncell][4] = (sum mx, sum my, sum mz,
 * N).  M = mu_s / V * sum m, and M / M_S^0 = |sum m| / N (all N aligned). */
void orc_coarse_grain(int kind, int sx, int ny, int nz, const int32_t *label, const double *Sx,
                      const double *Sy, const double *Sz, int x0, int ncols, int cx, int cy,
                      int cz, double *out)
{
    int64_t ncell = (int64_t)((ncols + cx - 1) / cx) * ((ny + cy - 1) / cy) * ((nz + cz - 1) / cz);
    int64_t n = (kind == ORC_SC ? 1 : 2) * (int64_t)sx * ny * nz;
    for (int64_t k = 0; k < 4 * ncell; ++k) out[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (label[i] < 0) continue;
        int64_t c = coarse_cell(kind, sx, ny, i, x0, ncols, cx, cy, cz);
        if (c < 0) continue;
        out[4 * c + 0] += Sx[i];
        out[4 * c + 1] += Sy[i];
        out[4 * c + 2] += Sz[i];
        out[4 * c + 3] += 1.0;
    }
}

/* Maximum polar angle of the cone that rebuilds a reduced magnetisation m
 * (Sec. II, inverse transfer), as printed:
 * (5 pi / 9) sqrt(1 - sqrt(1 + 6 (m - 1) / 5)).  The expression is real on
 * [1/6, 1]; m is clamped to that range (reading: below 1/6 the widest cone,
 * 100 degrees). */
double orc_cone_theta_max(double m)
{
    if (m > 1.0) m = 1.0;
    if (m < 1.0 / 6.0) m = 1.0 / 6.0;
    double t = 1.0 + (6.0 * (m - 1.0)) / 5.0;
    if (t < 0.0) t = 0.0;
    return 1.7453292519943295 * sqrt(1.0 - sqrt(t));
}

/* One spin drawn in the cone around the unit direction n (n = z when the
 * coarse magnetisation vanishes), from Philox words (w0, w1) of counter
 * (site, step, system, 1) with u1 = (w0 + 1/2) 2^-32, u2 = w1 2^-32; the
 * azimuth 2 pi u2 is measured in the orthonormal basis of Duff, Burgess,
 * Christensen, Hery, Kensler, Liani and Villemin, "Building an orthonormal
 * basis, revisited" (JCGT 2017): s = sign(n_z) (+1 at 0),
 * a = -1 / (s + n_z), b = n_x n_y a, b1 = (1 + s n_x^2 a, s b, -s n_x),
 * b2 = (b, s + n_y^2 a, -n_y).  The polar angle, by the cone reading:
 *   ORC_CONE_PRINTED: uniform on [0, theta_max(m)] with the printed
 *     theta_max (the paper's formula; the mean spin is not m n);
 *   ORC_CONE_CAP: uniform over the spherical cap cos theta >= 2 m - 1
 *     (m clamped to [0, 1]), cos theta = 1 - u1 (2 - 2 m): the mean of
 *     cos theta over the cap is m, so the cell average of many such spins
 *     returns the magnetisation the spins were drawn from. */
void orc_cone_spin_mode(int mode, const double mvec[3], int rounds, uint64_t seed, uint32_t site,
                        uint32_t step, uint32_t sys, double out[3])
{
    double m = sqrt((mvec[0] * mvec[0] + mvec[1] * mvec[1]) + mvec[2] * mvec[2]);
    double nx = 0.0, ny = 0.0, nz = 1.0;
    if (m > 0.0) {
        nx = mvec[0] / m;
        ny = mvec[1] / m;
        nz = mvec[2] / m;
    }
    uint32_t ctr[4] = {site, step, sys, 1u};
    uint32_t w[4];
    orc_philox4x32(rounds, (uint32_t)seed, (uint32_t)(seed >> 32), ctr, w);
    double u1 = ((double)w[0] + 0.5) * TWO_M32;
    double u2 = (double)w[1] * TWO_M32;
    double st, ct, sp, cp;
    if (mode == ORC_CONE_CAP) {
        double mc = m > 1.0 ? 1.0 : m;
        ct = 1.0 - u1 * (2.0 - 2.0 * mc);
        st = sqrt((1.0 - ct) * (1.0 + ct));
    } else {
        double th = u1 * orc_cone_theta_max(m);
        orc_sincos2pi(th / 6.283185307179586, &st, &ct);
    }
    orc_sincos2pi(u2, &sp, &cp);
    double s = nz >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (s + nz);
    double b = (nx * ny) * a;
    double b1[3] = {1.0 + ((s * nx) * nx) * a, s * b, -s * nx};
    double b2[3] = {b, s + (ny * ny) * a, -ny};
    double ex = st * cp, ey = st * sp;
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = (ex * b1[k] + ey * b2[k]) + ct * (k == 0 ? nx : (k == 1 ? ny : nz));
    normalise(v);
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
}

void orc_cone_spin(const double mvec[3], int rounds, uint64_t seed, uint32_t site, uint32_t step,
                   uint32_t sys, double out[3])
{
    orc_cone_spin_mode(ORC_CONE_PRINTED, mvec, rounds, seed, site, step, sys, out);
}

/* Eq. 6 read backwards: the magnetic sites of columns [x0, x0+ncols) take
 * cone spins around the reduced magnetisation mcell[3 c .. 3 c + 2] of
 * their coarse cell c (|m| <= 1); other sites are left as they are.
 * Counter word 0 is the stored site index. */
void orc_cone_columns(int kind, int sx, int ny, int nz, const int32_t *label, double *Sx,
                      double *Sy, double *Sz, int x0, int ncols, int cx, int cy, int cz,
                      const double *mcell, int rounds, uint64_t seed, uint32_t step, uint32_t sys)
{
    orc_cone_columns_mode(ORC_CONE_PRINTED, kind, sx, ny, nz, label, Sx, Sy, Sz, x0, ncols, cx, cy,
                          cz, mcell, rounds, seed, step, sys);
}

void orc_cone_columns_mode(int mode, int kind, int sx, int ny, int nz, const int32_t *label,
                           double *Sx, double *Sy, double *Sz, int x0, int ncols, int cx, int cy,
                           int cz, const double *mcell, int rounds, uint64_t seed, uint32_t step,
                           uint32_t sys)
{
    int64_t n = (kind == ORC_SC ? 1 : 2) * (int64_t)sx * ny * nz;
    for (int64_t i = 0; i < n; ++i) {
        if (label[i] < 0) continue;
        int64_t c = coarse_cell(kind, sx, ny, i, x0, ncols, cx, cy, cz);
        if (c < 0) continue;
        double v[3];
        orc_cone_spin_mode(mode, mcell + 3 * c, rounds, seed, (uint32_t)i, step, sys, v);
        Sx[i] = v[0];
        Sy[i] = v[1];
        Sz[i] = v[2];
    }
}

/* ------------------------------------------------------------------ */
/* Demagnetising field, Eq. 7: H_i = -sum_j N(r_j - r_i) M_j with the  */
/* cell-averaged tensor of Newell, Williams and Dunlop, "A generalization */
/* of the demagnetizing tensor for nonuniform magnetization", J.      */
/* Geophys. Res. 98, 9551 (1993).  Each component is a 27-point       */
/* second difference (per axis: -1, 2, -1 at -d, 0, +d) of an         */
/* auxiliary function, divided by 4 pi times the cell volume:         */
/* f for the diagonal, g for the off-diagonal terms.                  */
/* ------------------------------------------------------------------ */
#define ORC_MU0 1.25663706212e-6 /* vacuum permeability, N/A^2 (CODATA 2018) */
#define ORC_PI 3.14159265358979323846

/* Newell's f.  A term whose coefficient vanishes is left out, which also
 * keeps its inverse hyperbolic sine or arctangent away from 0/0. */
static double newell_f(double x, double y, double z)
{
    double x2 = x * x, y2 = y * y, z2 = z * z;
    double R = sqrt(x2 + y2 + z2);
    if (R == 0.0) return 0.0;
    double t = ((2.0 * x2 - y2) - z2) * R / 6.0;
    if (y != 0.0 && z2 != x2) t += 0.5 * y * (z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (z != 0.0 && y2 != x2) t += 0.5 * z * (y2 - x2) * asinh(z / sqrt(x2 + y2));
    if (x != 0.0 && y != 0.0 && z != 0.0) t -= x * y * z * atan(y * z / (x * R));
    return t;
}

/* Newell's g (off-diagonal xy term). */
static double newell_g(double x, double y, double z)
{
    double x2 = x * x, y2 = y * y, z2 = z * z;
    double R = sqrt(x2 + y2 + z2);
    if (R == 0.0) return 0.0;
    double t = -(x * y * R) / 3.0;
    if (x != 0.0 && y != 0.0 && z != 0.0) t += x * y * z * asinh(z / sqrt(x2 + y2));
    if (y != 0.0 && 3.0 * z2 != y2) t += y / 6.0 * (3.0 * z2 - y2) * asinh(x / sqrt(y2 + z2));
    if (x != 0.0 && 3.0 * z2 != x2) t += x / 6.0 * (3.0 * z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (z != 0.0) {
        t -= z * z2 / 6.0 * atan(x * y / (z * R));
        if (y != 0.0) t -= z * y2 / 2.0 * atan(x * z / (y * R));
        if (x != 0.0) t -= z * x2 / 2.0 * atan(y * z / (x * R));
    }
    return t;
}

/* sum over e in {-1,0,1}^3 of w(e) F(X + ex dx, Y + ey dy, Z + ez dz),
 * w = product over the axes of (2 if e = 0, else -1), over 4 pi dx dy dz */
static double newell_stencil(double (*F)(double, double, double), double X, double Y, double Z,
                             double dx, double dy, double dz)
{
    double acc = 0.0;
    for (int ex = -1; ex <= 1; ++ex)
        for (int ey = -1; ey <= 1; ++ey)
            for (int ez = -1; ez <= 1; ++ez) {
                double w = (ex ? -1.0 : 2.0) * (ey ? -1.0 : 2.0) * (ez ? -1.0 : 2.0);
                acc += w * F(X + ex * dx, Y + ey * dy, Z + ez * dz);
            }
    return acc / (4.0 * ORC_PI * dx * dy * dz);
}

/* N_yy, N_zz follow from N_xx and N_xz, N_yz from N_xy by relabelling the
 * axes (coordinates and cell edges together). */
void orc_newell_tensor(double X, double Y, double Z, double dx, double dy, double dz, double N[6])
{
    N[0] = newell_stencil(newell_f, X, Y, Z, dx, dy, dz); /* xx */
    N[1] = newell_stencil(newell_f, Y, X, Z, dy, dx, dz); /* yy */
    N[2] = newell_stencil(newell_f, Z, Y, X, dz, dy, dx); /* zz */
    N[3] = newell_stencil(newell_g, X, Y, Z, dx, dy, dz); /* xy */
    N[4] = newell_stencil(newell_g, X, Z, Y, dx, dz, dy); /* xz */
    N[5] = newell_stencil(newell_g, Y, Z, X, dy, dz, dx); /* yz */
}

/* Eq. 7 summed directly.  The tensor depends only on the displacement, so
 * it is evaluated once per displacement (index (ix, iy, iz) + (n - 1)). */
void orc_demag_direct(int nx, int ny, int nz, double dx, double dy, double dz, const double *M,
                      double *H)
{
    int64_t n = (int64_t)nx * ny * nz;
    int64_t tx = 2 * nx - 1, ty = 2 * ny - 1, tz = 2 * nz - 1;
    double *T = (double *)malloc(sizeof(double) * 6 * (size_t)(tx * ty * tz));
    if (!T) return;
    for (int64_t kz = 0; kz < tz; ++kz)
        for (int64_t ky = 0; ky < ty; ++ky)
            for (int64_t kx = 0; kx < tx; ++kx)
                orc_newell_tensor((double)(kx - (nx - 1)) * dx, (double)(ky - (ny - 1)) * dy,
                                  (double)(kz - (nz - 1)) * dz, dx, dy, dz,
                                  T + 6 * (kx + tx * (ky + ty * kz)));
    for (int64_t i = 0; i < n; ++i) {
        int64_t ix = i % nx, iy = (i / nx) % ny, iz = i / ((int64_t)nx * ny);
        double h[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            int64_t jx = j % nx, jy = (j / nx) % ny, jz = j / ((int64_t)nx * ny);
            const double *N = T + 6 * ((jx - ix + nx - 1) + tx * ((jy - iy + ny - 1) +
                                                                   ty * (jz - iz + nz - 1)));
            double mx = M[j], my = M[n + j], mz = M[2 * n + j];
            h[0] -= (N[0] * mx + N[3] * my) + N[4] * mz;
            h[1] -= (N[3] * mx + N[1] * my) + N[5] * mz;
            h[2] -= (N[4] * mx + N[5] * my) + N[2] * mz;
        }
        H[i] = h[0];
        H[n + i] = h[1];
        H[2 * n + i] = h[2];
    }
    free(T);
}

/* The demagnetising flux density mu0 H_d (T) per coarse cell of the evolving
 * magnetic sites: Eq. 6 (M = mu_s sum m / V) then Eq. 7.  out [3][ncell]. */
static int demag_cells(const orc_system *s, const double *Sx, const double *Sy, const double *Sz,
                       double *out)
{
    int64_t nc = (int64_t)s->dn[0] * s->dn[1] * s->dn[2];
    double *M = (double *)calloc(3 * (size_t)nc, sizeof(double));
    double *H = (double *)malloc(sizeof(double) * 3 * (size_t)nc);
    if (!M || !H) {
        free(M); free(H);
        return -1;
    }
    for (int64_t i = 0; i < s->n_sites; ++i) {
        if (!evolves(s, i) || s->dcell[i] < 0) continue;
        int64_t c = s->dcell[i];
        M[c] += Sx[i];
        M[nc + c] += Sy[i];
        M[2 * nc + c] += Sz[i];
    }
    double k = s->mu_s / ((s->dd[0] * s->dd[1]) * s->dd[2]);
    for (int64_t c = 0; c < 3 * nc; ++c) M[c] = k * M[c];
    orc_demag_direct(s->dn[0], s->dn[1], s->dn[2], s->dd[0], s->dd[1], s->dd[2], M, H);
    for (int64_t c = 0; c < 3 * nc; ++c) out[c] = ORC_MU0 * H[c];
    if (s->bstray)
        for (int64_t c = 0; c < 3 * nc; ++c) out[c] = out[c] + s->bstray[c];
    free(M);
    free(H);
    return 0;
}


/* ------------------------------------------------------------------ */
/* Metropolis Monte Carlo of the same Hamiltonian (the calibration of */
/* the exchange constant, Sec. III with Eq. 8).  Site energy          */
/*   E_i(S) = -mu_s S . (B_ex + p B) - k_u S_z^2,                      */
/* B_ex = Eq. 2 summed by shell as in the field above.  A sweep visits */
/* the sites of colour 0 in index order, then those of colour 1; no    */
/* two neighbours share a colour, so the order within a colour does    */
/* not matter.  A visit takes Philox words (site, sweep, system, 2):   */
/* trial direction uniform on the sphere, S_z = 2 u0 - 1 with          */
/* u0 = (w0 + 1/2) 2^-32 and azimuth 2 pi w1 2^-32; the trial is       */
/* accepted when dE <= 0 or (w2 + 1/2) 2^-32 < exp(-dE / kB T), with   */
/* T the system's ambient temperature.                                 */
/* ------------------------------------------------------------------ */
static void mc_visit(const orc_system *s, double *Sx, double *Sy, double *Sz, int64_t i,
                     int64_t sweep, double pol)
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int sh = 0; sh < s->n_shells; ++sh) {
        double part[3] = {0.0, 0.0, 0.0};
        for (int64_t k = s->row_ptr[i]; k < s->row_ptr[i + 1]; ++k) {
            if (s->shell[k] != sh) continue;
            int64_t j = s->col[k];
            if (s->label[j] != s->label[i]) continue;
            part[0] = part[0] + Sx[j];
            part[1] = part[1] + Sy[j];
            part[2] = part[2] + Sz[j];
        }
        double cex = s->J[sh] / s->mu_s;
        acc[0] = acc[0] + cex * part[0];
        acc[1] = acc[1] + cex * part[1];
        acc[2] = acc[2] + cex * part[2];
    }
    double h[3] = {acc[0] + pol * s->B[0], acc[1] + pol * s->B[1], acc[2] + pol * s->B[2]};
    uint32_t ctr[4] = {s->ctr0[i], (uint32_t)sweep, s->sys_id, 2u};
    uint32_t w[4];
    orc_philox4x32(s->rounds, (uint32_t)s->seed, (uint32_t)(s->seed >> 32), ctr, w);
    double z = 2.0 * (((double)w[0] + 0.5) * TWO_M32) - 1.0;
    double r = sqrt(1.0 - z * z);
    double sp, cp;
    orc_sincos2pi((double)w[1] * TWO_M32, &sp, &cp);
    double t[3] = {r * cp, r * sp, z};
    double d[3] = {t[0] - Sx[i], t[1] - Sy[i], t[2] - Sz[i]};
    double ku = s->ku_grain ? s->ku_grain[s->label[i]] : s->ku;
    double dE = -s->mu_s * ((d[0] * h[0] + d[1] * h[1]) + d[2] * h[2]) -
                ku * (t[2] * t[2] - Sz[i] * Sz[i]);
    int accept = dE <= 0.0;
    if (!accept && s->T_amb > 0.0) {
        double u = ((double)w[2] + 0.5) * TWO_M32;
        accept = u < orc_exp(-(dE / (ORC_KB * s->T_amb)));
    }
    if (accept) {
        Sx[i] = t[0];
        Sy[i] = t[1];
        Sz[i] = t[2];
    }
}

int orc_mc_sweeps(const orc_system *s, const int8_t *colour, int n_colours, double *Sx,
                  double *Sy, double *Sz, int64_t sweep0, int64_t nsweeps)
{
    for (int64_t t = 0; t < nsweeps; ++t) {
        int64_t sweep = sweep0 + t;
        double pol = polarity(s, sweep);
        for (int c = 0; c < n_colours; ++c)
            for (int64_t i = 0; i < s->n_sites; ++i)
                if (evolves(s, i) && colour[i] == c) mc_visit(s, Sx, Sy, Sz, i, sweep, pol);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Micromagnetic region (Sec. II): LLG without the thermal field (Eq. 1 */
/* in Landau-Lifshitz form) on a finite-difference mesh, integrated by  */
/* classic RK4 (the paper's integrator for these regions, Sec. III) with */
/* the magnetisation renormalised after each step.  Field (tesla):       */
/*   exchange   (2 A(T) / M_S(T)) lap m           (Eq. 4, 6-point stencil) */
/*   anisotropy (2 K(T) / M_S(T)) (m . z) z       (Eq. 5)                 */
/*   write field p(n) B                                                    */
/* with M_S = M_S0 m_e, A = A_0 m_e^2, K = K_0 m_e^3 and the damping      */
/* alpha = lambda (1 - T / 3 T_C) (Sec. II); m_e(T) is the root of        */
/* m = L(3 T_C m / T + mu_s |B| / kB T), L the Langevin function.  T per  */
/* cell from the laser spot at the stage time.                            */
/* ------------------------------------------------------------------ */

/* Langevin function coth x - 1/x for x >= 0; below 0.1 its Taylor series
 * through x^11 (coefficients 2^2n B_2n / (2n)!, the closed form cancels
 * there); coth from this file's exp. */
double orc_langevin(double x)
{
    if (x < 0.1) {
        double x2 = x * x;
        double p = -1382.0 / 638512875.0;
        p = 2.0 / 93555.0 + x2 * p;
        p = -1.0 / 4725.0 + x2 * p;
        p = 2.0 / 945.0 + x2 * p;
        p = -1.0 / 45.0 + x2 * p;
        p = 1.0 / 3.0 + x2 * p;
        return x * p;
    }
    double e = orc_exp(-2.0 * x);
    return (1.0 + e) / (1.0 - e) - 1.0 / x;
}

/* m_e(T): 64 halvings of [0, 1] keeping f(lo) >= 0 > f(hi), f(m) =
 * L((3 T_C m + b) / T) - m, b = mu_s |B| / kB (kelvin).  This brackets the
 * largest root: the ordered one below T_C, 0 above it when b = 0. */
double orc_mm_me(double T, double Tc, double b)
{
    if (T <= 0.0) return 1.0;
    double lo = 0.0, hi = 1.0;
    for (int k = 0; k < 64; ++k) {
        double mid = 0.5 * (lo + hi);
        double f = orc_langevin((3.0 * Tc * mid + b) / T) - mid;
        if (f >= 0.0)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

static double mm_temperature(const orc_mm *p, int i, int j, double t)
{
    if (p->spot_mode == ORC_SPOT_NONE) return p->T_amb;
    double xc = p->spot_mode == ORC_SPOT_MOVING ? p->x0 + p->v * t : p->x0;
    double sd = p->fwhm / 2.3548200450309493;
    double inv2s2 = 1.0 / ((2.0 * sd) * sd);
    double dx = ((double)i + 0.5) * p->h[0] - xc;
    double dy = ((double)j + 0.5) * p->h[1] - p->y0;
    double q = (dx * dx + dy * dy) * inv2s2;
    return p->T_amb + (p->T_peak - p->T_amb) * orc_exp(-q);
}

double orc_mm_temperature(const orc_mm *p, int i, int j, double t)
{
    return mm_temperature(p, i, j, t);
}

double orc_mm_polarity(const orc_mm *p, int64_t n)
{
    return bit_polarity(p->n_bits, p->bits, p->steps_per_bit, n);
}

/* neighbour of cell (i, j, k) along axis ax, direction d (+-1), or -1 */
static int64_t mm_nb(const orc_mm *p, int i, int j, int k, int ax, int d)
{
    int c[3] = {i, j, k};
    int n[3] = {p->nx, p->ny, p->nz};
    c[ax] += d;
    if (c[ax] < 0 || c[ax] >= n[ax]) {
        if (!p->periodic[ax]) return -1;
        c[ax] = (c[ax] + n[ax]) % n[ax];
    }
    return c[0] + (int64_t)n[0] * (c[1] + (int64_t)n[1] * c[2]);
}

/* k = dm/dt at configuration u (all cells) and time t */
static void mm_rhs(const orc_mm *p, const double *u, double t, double pol, double *k)
{
    int64_t n = (int64_t)p->nx * p->ny * p->nz;
    double bmag = sqrt((p->B[0] * p->B[0] + p->B[1] * p->B[1]) + p->B[2] * p->B[2]);
    double b = p->mu_s * bmag / ORC_KB;
    double ih2[3] = {1.0 / (p->h[0] * p->h[0]), 1.0 / (p->h[1] * p->h[1]),
                     1.0 / (p->h[2] * p->h[2])};
    for (int64_t c = 0; c < n; ++c) {
        int i = (int)(c % p->nx), j = (int)((c / p->nx) % p->ny), kk = (int)(c / ((int64_t)p->nx * p->ny));
        double T = mm_temperature(p, i, j, t);
        double me = orc_mm_me(T, p->Tc, b);
        double Tr = T < p->Tc ? T : p->Tc;
        double alpha = p->lambda * (1.0 - Tr / (3.0 * p->Tc));
        double gp = -p->gamma / (1.0 + alpha * alpha);
        double m[3] = {u[c], u[n + c], u[2 * n + c]};
        double lap[3] = {0.0, 0.0, 0.0};
        for (int ax = 0; ax < 3; ++ax)
            for (int d = -1; d <= 1; d += 2) {
                int64_t q = mm_nb(p, i, j, kk, ax, d);
                if (q < 0) {
                    /* the other region across an x face: its direction */
                    const double *g = ax == 0 ? p->ghost[d < 0 ? 0 : 1] : NULL;
                    if (!g) continue;
                    const double *gv = g + 3 * ((int64_t)j + (int64_t)p->ny * kk);
                    if (gv[0] == 0.0 && gv[1] == 0.0 && gv[2] == 0.0) continue; /* nothing there */
                    for (int s = 0; s < 3; ++s) lap[s] = lap[s] + (gv[s] - m[s]) * ih2[ax];
                    continue;
                }
                for (int s = 0; s < 3; ++s) lap[s] = lap[s] + (u[s * n + q] - m[s]) * ih2[ax];
            }
        double cex = (2.0 * p->A0 * me) / p->Ms0;
        double can = (2.0 * p->K0 * (me * me)) / p->Ms0;
        double B[3];
        for (int s = 0; s < 3; ++s) B[s] = cex * lap[s] + pol * p->B[s];
        B[2] = B[2] + can * m[2];
        if (p->bd)
            for (int s = 0; s < 3; ++s) B[s] = B[s] + p->bd[s * n + c];
        double f[3];
        ll_rhs(gp, alpha, m, B, f);
        k[c] = f[0];
        k[n + c] = f[1];
        k[2 * n + c] = f[2];
    }
}

int orc_mm_rk4(const orc_mm *p, double *m, int64_t step0, int64_t nsteps)
{
    int64_t n = (int64_t)p->nx * p->ny * p->nz;
    double *k1 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *k2 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *k3 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *k4 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *u = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!k1 || !k2 || !k3 || !k4 || !u) {
        free(k1); free(k2); free(k3); free(k4); free(u);
        return -1;
    }
    const double dt = p->dt;
    for (int64_t s = 0; s < nsteps; ++s) {
        int64_t step = step0 + s;
        double pol = bit_polarity(p->n_bits, p->bits, p->steps_per_bit, step);
        double t = (double)step * dt;
        mm_rhs(p, m, t, pol, k1);
        for (int64_t q = 0; q < 3 * n; ++q) u[q] = m[q] + (0.5 * dt) * k1[q];
        mm_rhs(p, u, t + 0.5 * dt, pol, k2);
        for (int64_t q = 0; q < 3 * n; ++q) u[q] = m[q] + (0.5 * dt) * k2[q];
        mm_rhs(p, u, t + 0.5 * dt, pol, k3);
        for (int64_t q = 0; q < 3 * n; ++q) u[q] = m[q] + dt * k3[q];
        mm_rhs(p, u, t + dt, pol, k4);
        for (int64_t c = 0; c < n; ++c) {
            double v[3];
            for (int d = 0; d < 3; ++d) {
                int64_t q = d * n + c;
                v[d] = m[q] + (dt / 6.0) * (((k1[q] + 2.0 * k2[q]) + 2.0 * k3[q]) + k4[q]);
            }
            normalise(v);
            m[c] = v[0];
            m[n + c] = v[1];
            m[2 * n + c] = v[2];
        }
    }
    free(k1); free(k2); free(k3); free(k4); free(u);
    return 0;
}


/* The region's mesh moved one cell along +x together with the simulation
 * window (Sec. II, Fig. 1): cell (i, j, k) takes the direction of cell
 * (i + 1, j, k); the column i = 0, which leaves the region, is copied to
 * leave[3 (j + ny k) ..] (when leave is not NULL); the column i = nx - 1
 * takes the direction of enter[stride (j + ny k) ..] (+z for a zero
 * vector: a cell with no magnetic site). */
void orc_mm_shift(const orc_mm *p, double *m, const double *enter, int stride, double *leave)
{
    int64_t n = (int64_t)p->nx * p->ny * p->nz;
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j) {
            int64_t row = (int64_t)p->nx * (j + (int64_t)p->ny * k);
            int64_t f = (int64_t)j + (int64_t)p->ny * k;
            if (leave)
                for (int s = 0; s < 3; ++s) leave[3 * f + s] = m[s * n + row];
            for (int i = 0; i + 1 < p->nx; ++i)
                for (int s = 0; s < 3; ++s) m[s * n + row + i] = m[s * n + row + i + 1];
            const double *v = enter + (int64_t)stride * f;
            double r = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
            double d[3] = {0.0, 0.0, 1.0};
            if (r > 0.0)
                for (int s = 0; s < 3; ++s) d[s] = v[s] / r;
            for (int s = 0; s < 3; ++s) m[s * n + row + p->nx - 1] = d[s];
        }
}

/* Reduced magnetisation M / M_S^0 = m_e(T) m of the cells on x face `face`
 * (0: i = 0, 1: i = nx - 1) at time t, out[3 (j + ny k) ..]: what the
 * region hands to the atomistic window by thermalisation (Sec. II). */
void orc_mm_face_moment(const orc_mm *p, const double *m, int face, double t, double *out)
{
    int64_t n = (int64_t)p->nx * p->ny * p->nz;
    double bmag = sqrt((p->B[0] * p->B[0] + p->B[1] * p->B[1]) + p->B[2] * p->B[2]);
    double b = p->mu_s * bmag / ORC_KB;
    int i = face == 0 ? 0 : p->nx - 1;
    for (int k = 0; k < p->nz; ++k)
        for (int j = 0; j < p->ny; ++j) {
            int64_t c = i + (int64_t)p->nx * (j + (int64_t)p->ny * k);
            double me = orc_mm_me(mm_temperature(p, i, j, t), p->Tc, b);
            int64_t f = (int64_t)j + (int64_t)p->ny * k;
            for (int s = 0; s < 3; ++s) out[3 * f + s] = me * m[s * n + c];
        }
}

/* The magnetic sites of stored columns [x0, x0 + ncols) take the direction
 * of their coarse cell, mcell[c] / |mcell[c]| (+z for a zero cell): the
 * micromagnetic neighbours just outside the atomistic window (Sec. II). */
void orc_set_columns(int kind, int sx, int ny, int nz, const int32_t *label, double *Sx,
                     double *Sy, double *Sz, int x0, int ncols, int cx, int cy, int cz,
                     const double *mcell)
{
    int64_t n = (kind == ORC_SC ? 1 : 2) * (int64_t)sx * ny * nz;
    for (int64_t i = 0; i < n; ++i) {
        if (label[i] < 0) continue;
        int64_t c = coarse_cell(kind, sx, ny, i, x0, ncols, cx, cy, cz);
        if (c < 0) continue;
        const double *v = mcell + 3 * c;
        double m = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        if (m > 0.0) {
            Sx[i] = v[0] / m;
            Sy[i] = v[1] / m;
            Sz[i] = v[2] / m;
        } else {
            Sx[i] = 0.0;
            Sy[i] = 0.0;
            Sz[i] = 1.0;
        }
    }
}
