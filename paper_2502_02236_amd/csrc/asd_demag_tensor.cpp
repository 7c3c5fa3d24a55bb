// asd_demag_tensor.cpp -- host set-up of the demagnetising field (Eq. 7):
// Newell's cell-averaged tensor on the coarse mesh and its spectrum.
//
// Newell, Williams and Dunlop, J. Geophys. Res. 98, 9551 (1993): the mutual
// demagnetising tensor of two equal cells displaced by (X, Y, Z) is, per
// component, a second difference along each axis (weights -1, 2, -1 at
// -d, 0, +d) of an auxiliary function over 4 pi V; f gives the diagonal and
// g the off-diagonal components.  f is even in each argument and g is odd
// in its first two, so both are tabulated once on the non-negative lattice
// of cell offsets and every stencil point is a table read.
#include <cmath>
#include <complex>
#include <vector>

#include "asd_internal.h"

namespace asd {

namespace {

double aux_f(double x, double y, double z)
{
    const double xx = x * x, yy = y * y, zz = z * z, r = std::sqrt(xx + yy + zz);
    if (r == 0.0) return 0.0;
    double v = ((2.0 * xx - yy) - zz) * r / 6.0;
    if (y != 0.0 && zz != xx) v += 0.5 * y * (zz - xx) * std::asinh(y / std::sqrt(xx + zz));
    if (z != 0.0 && yy != xx) v += 0.5 * z * (yy - xx) * std::asinh(z / std::sqrt(xx + yy));
    if (x != 0.0 && y != 0.0 && z != 0.0) v -= x * y * z * std::atan((y * z) / (x * r));
    return v;
}

double aux_g(double x, double y, double z)
{
    const double xx = x * x, yy = y * y, zz = z * z, r = std::sqrt(xx + yy + zz);
    if (r == 0.0) return 0.0;
    double v = -(x * y * r) / 3.0;
    if (x != 0.0 && y != 0.0 && z != 0.0) v += x * y * z * std::asinh(z / std::sqrt(xx + yy));
    if (y != 0.0 && 3.0 * zz != yy) v += y / 6.0 * (3.0 * zz - yy) * std::asinh(x / std::sqrt(yy + zz));
    if (x != 0.0 && 3.0 * zz != xx) v += x / 6.0 * (3.0 * zz - xx) * std::asinh(y / std::sqrt(xx + zz));
    if (z != 0.0) {
        v -= z * zz / 6.0 * std::atan((x * y) / (z * r));
        if (y != 0.0) v -= z * yy / 2.0 * std::atan((x * z) / (y * r));
        if (x != 0.0) v -= z * xx / 2.0 * std::atan((y * z) / (x * r));
    }
    return v;
}

// table of an auxiliary function over offsets (i, j, k) >= 0, i <= mx, ...
struct Table {
    int mx, my, mz;
    std::vector<double> v;
    double at(int i, int j, int k) const { return v[((size_t)k * (my + 1) + j) * (mx + 1) + i]; }
};

// in-place radix-2 FFT of n = 2^l points at stride st
void fft1(std::complex<double> *a, int l, size_t st)
{
    const size_t n = (size_t)1 << l;
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i * st], a[j * st]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = -2.0 * M_PI / (double)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> w(std::cos(ang * (double)k), std::sin(ang * (double)k));
                const std::complex<double> u = a[(i + k) * st], t = w * a[(i + k + len / 2) * st];
                a[(i + k) * st] = u + t;
                a[(i + k + len / 2) * st] = u - t;
            }
    }
}

}  // namespace

namespace {

// the auxiliary-function table of tensor component comp (xx yy zz xy xz yz)
// over cell offsets 0..nc (a stencil reaches one beyond nc - 1)
Table component_table(int comp, int ncx, int ncy, int ncz, double dx, double dy, double dz)
{
    Table t{ncx, ncy, ncz, std::vector<double>((size_t)(ncx + 1) * (ncy + 1) * (ncz + 1))};
    for (int k = 0; k <= ncz; ++k)
        for (int j = 0; j <= ncy; ++j)
            for (int i = 0; i <= ncx; ++i) {
                const double X = i * dx, Y = j * dy, Z = k * dz;
                double v = 0.0;
                switch (comp) {
                case 0: v = aux_f(X, Y, Z); break;  // xx: f(x, y, z)
                case 1: v = aux_f(Y, X, Z); break;  // yy: f(y, x, z)
                case 2: v = aux_f(Z, Y, X); break;  // zz: f(z, y, x)
                case 3: v = aux_g(X, Y, Z); break;  // xy: g(x, y, z)
                case 4: v = aux_g(X, Z, Y); break;  // xz: g(x, z, y)
                default: v = aux_g(Y, Z, X); break; // yz: g(y, z, x)
                }
                t.v[((size_t)k * (ncy + 1) + j) * (ncx + 1) + i] = v;
            }
    return t;
}

// axes in which each component is odd: xy -> (x, y), xz -> (x, z), yz -> (y, z)
const bool kOdd[6][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};

// component comp of the tensor between cells displaced by (I, J, K) cells,
// times 4 pi V: the second difference along each axis of the table
double tensor_element(const Table &t, int comp, int I, int J, int K)
{
    double acc = 0.0;
    for (int ez = -1; ez <= 1; ++ez)
        for (int ey = -1; ey <= 1; ++ey)
            for (int ex = -1; ex <= 1; ++ex) {
                const int ii = I + ex, jj = J + ey, kk = K + ez;
                double sg = 1.0;
                if (kOdd[comp][0] && ii < 0) sg = -sg;
                if (kOdd[comp][1] && jj < 0) sg = -sg;
                if (kOdd[comp][2] && kk < 0) sg = -sg;
                const double w = (ex ? -1.0 : 2.0) * (ey ? -1.0 : 2.0) * (ez ? -1.0 : 2.0);
                acc += w * sg * t.at(std::abs(ii), std::abs(jj), std::abs(kk));
            }
    return acc;
}

}  // namespace

// Spectrum of the six tensor components on the zero-padded mesh (padded
// sizes 2^lx x 2^ly x 2^lz), times `scale`, kept on the octant kx <= Px/2,
// ky <= Py/2, kz <= Pz/2: [6][Py/2+1][Px/2+1][Pz/2+1] (xx yy zz xy xz yz;
// kz fastest, the order in which the z pass reads it).
// The components are real and even or odd in each wavenumber by the
// symmetry of the tensor, so the octant determines the whole spectrum.
void demag_spectrum(int ncx, int ncy, int ncz, double dx, double dy, double dz, int lx, int ly,
                    int lz, double scale, std::vector<double> &octant)
{
    const int Px = 1 << lx, Py = 1 << ly, Pz = 1 << lz;
    const int ox = Px / 2 + 1, oy = Py / 2 + 1, oz = Pz / 2 + 1;
    octant.assign((size_t)6 * ox * oy * oz, 0.0);
    const double inv4piV = 1.0 / (4.0 * M_PI * dx * dy * dz);
    std::vector<std::complex<double>> a((size_t)Px * Py * Pz);
    for (int comp = 0; comp < 6; ++comp) {
        const Table t = component_table(comp, ncx, ncy, ncz, dx, dy, dz);
        std::fill(a.begin(), a.end(), std::complex<double>(0.0, 0.0));
        for (int K = -(ncz - 1); K <= ncz - 1; ++K)
            for (int J = -(ncy - 1); J <= ncy - 1; ++J)
                for (int I = -(ncx - 1); I <= ncx - 1; ++I) {
                    const size_t ix = (size_t)((I + Px) % Px), iy = (size_t)((J + Py) % Py),
                                 iz = (size_t)((K + Pz) % Pz);
                    a[(iz * Py + iy) * Px + ix] = tensor_element(t, comp, I, J, K) * inv4piV * scale;
                }
        for (size_t r = 0; r < (size_t)Py * Pz; ++r) fft1(a.data() + r * Px, lx, 1);
        for (size_t z = 0; z < (size_t)Pz; ++z)
            for (size_t x = 0; x < (size_t)Px; ++x) fft1(a.data() + z * Py * Px + x, ly, Px);
        for (size_t r = 0; r < (size_t)Py * Px; ++r) fft1(a.data() + r, lz, (size_t)Py * Px);
        for (int kz = 0; kz < oz; ++kz)
            for (int ky = 0; ky < oy; ++ky)
                for (int kx = 0; kx < ox; ++kx)
                    octant[(((size_t)comp * oy + ky) * ox + kx) * oz + kz] =
                        a[((size_t)(kz % Pz) * Py + (ky % Py)) * Px + (kx % Px)].real();
    }
}

// The same tensor transformed along x and y only, at the plane offsets
// dz = 0 .. ncz-1: [Px/2+1][6][ncz][Py/2+1] (ky fastest, the order in which
// neighbouring lanes of the y-z pass read it), times `scale`.
// Along x and y the components are real and even or odd in each wavenumber
// as above; xx, yy, zz and xy are real, xz and yz (odd along one in-plane
// axis) imaginary, stored as their imaginary part.  Along z, xz and yz are
// odd in dz, the others even.
void demag_mixed(int ncx, int ncy, int ncz, double dx, double dy, double dz, int lx, int ly,
                 double scale, std::vector<double> &table)
{
    const int Px = 1 << lx, Py = 1 << ly;
    const int ox = Px / 2 + 1, oy = Py / 2 + 1;
    table.assign((size_t)6 * ox * oy * ncz, 0.0);
    const double inv4piV = 1.0 / (4.0 * M_PI * dx * dy * dz);
    std::vector<std::complex<double>> a((size_t)Px * Py);
    for (int comp = 0; comp < 6; ++comp) {
        const Table t = component_table(comp, ncx, ncy, ncz, dx, dy, dz);
        for (int K = 0; K < ncz; ++K) {
            std::fill(a.begin(), a.end(), std::complex<double>(0.0, 0.0));
            for (int J = -(ncy - 1); J <= ncy - 1; ++J)
                for (int I = -(ncx - 1); I <= ncx - 1; ++I) {
                    const size_t ix = (size_t)((I + Px) % Px), iy = (size_t)((J + Py) % Py);
                    a[iy * Px + ix] = tensor_element(t, comp, I, J, K) * inv4piV * scale;
                }
            for (size_t r = 0; r < (size_t)Py; ++r) fft1(a.data() + r * Px, lx, 1);
            for (size_t x = 0; x < (size_t)Px; ++x) fft1(a.data() + x, ly, Px);
            const bool imag = comp >= 4;
            for (int ky = 0; ky < oy; ++ky)
                for (int kx = 0; kx < ox; ++kx) {
                    const std::complex<double> v = a[(size_t)(ky % Py) * Px + (kx % Px)];
                    table[(((size_t)kx * 6 + comp) * ncz + K) * oy + ky] = imag ? v.imag() : v.real();
                }
        }
    }
}

}  // namespace asd
