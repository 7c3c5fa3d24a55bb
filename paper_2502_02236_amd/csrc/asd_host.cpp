// asd_host.cpp -- the C ABI of libasd (include/asd.h): descriptor checks,
// workspace layout, host construction of lattices, grain labels and
// neighbour tables, uploads, and the enqueueing of Heun steps, window
// shifts and FP64 reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "asd.h"
#include "asd_internal.h"
#include "asd_pair.h"
#include "asd_variants.h"

using namespace asd;

namespace {

constexpr double kBoltzmann = 1.380649e-23;  // J/K (exact SI)
constexpr double kMu0 = 1.25663706212e-6;     // vacuum permeability, N/A^2 (CODATA 2018)
constexpr size_t kAlign = 256;
constexpr int kMaxBits = 1 << 16;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// in-plane L1_0 half-cell offsets (dx, dy, dz) by shell, each shell ordered
// by (dz, dy, dx): shells a/sqrt2 (4), c (2), a (4), sqrt(a^2/2 + c^2) (8)
const int kL10Off[kL10Degree][3] = {
    {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 1, 0},                 // shell 0
    {0, 0, -1},  {0, 0, 1},                                          // shell 1
    {0, -2, 0},  {-2, 0, 0}, {2, 0, 0},  {0, 2, 0},                  // shell 2
    {-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1},              // shell 3, dz = -1
    {-1, -1, 1},  {1, -1, 1},  {-1, 1, 1},  {1, 1, 1}};              // shell 3, dz = +1
const int kL10ShellEnd[4] = {4, 6, 10, 18};
// SC offsets (dx, dy, dz) ordered by (dz, dy, dx)
const int kScOffH[6][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

struct HostSys {
    asd_system_desc desc;
    std::vector<int32_t> labels;  // per stored site, -1 non-magnetic
    std::vector<double> ku_grain;
    int32_t n_grains = 1;
    int64_t n_stored = 0, n_window = 0;
    int32_t sx = 0;
};

struct Layout {
    int64_t n_total = 0;   // stored sites over all systems (+ zero slot)
    int64_t ncs = 0;       // component stride
    int64_t zero_site = 0;
    int32_t n_grains = 0;  // over all systems
    int32_t n_tiles = 0;   // plain tiles
    int32_t n_ftiles = 0;  // fused tiles
    size_t off_S[3] = {0, 0, 0};
    size_t off_F0 = 0, off_Bt = 0;  // stash buffers of the two-pass variant 1
    size_t off_can32 = 0;
    size_t off_label = 0, off_ell = 0, off_sys = 0, off_tile = 0, off_ftile = 0, off_can = 0,
           off_ku = 0, off_gsys = 0, off_gptr = 0, off_gsites = 0, off_step = 0, off_origin = 0,
           off_bits = 0, off_gout = 0, off_sout = 0, off_mom = 0, off_epart = 0, off_eout = 0;
    // demagnetising field (when asd_params.demag_cell is set)
    DemagDev dm{};            // geometry; pointers filled at create
    size_t off_dwx = 0, off_dwy = 0, off_dbd[2] = {0, 0}, off_dK = 0, off_dtw[3] = {0, 0, 0};
    size_t off_dcs[2] = {0, 0};  // cell sums of the cell-row and fused stage kernels
    size_t dcs_bytes = 0;
    DemagDev dmT{};           // stray field of the frozen track (track systems only)
    size_t off_twx = 0, off_twy = 0, off_tK = 0, off_ttw = 0, off_tstray = 0;
    size_t bytes = 0;
};

}  // namespace

struct asd_t {
    asd_params p{};
    std::vector<HostSys> sys;
    std::vector<SysDev> dev;
    Layout L;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    int cur = 0;              // buffer holding the current spins
    int64_t step = 0;         // host copy of the step counter
    std::vector<int32_t> origin;
    asd_drive drive{};
    std::vector<uint8_t> bits;
    int kernel = ASD_KERNEL_PLAIN;
    int tile_cfg = 0;
    std::string err;
    int elem = 8;
    int device = 0;           // HIP device current at asd_create (holds the workspace)
    int cone = ASD_CONE_PRINTED;  // reading of the inverse transfer's cone
    // graphs: one per starting buffer parity
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_steps = 0;
    int graph_kernel = -1, graph_tile = -1;
    int n_ftiles = 0;         // fused tiles of the current variant
    DemagDev dm{};            // demagnetising field (dm.on = 0: none)
    DemagDev dmT{};           // stray field of the frozen track (dmT.on = 0: none)
    bool stray_dirty = true;  // the frozen track changed since the stray field was computed
    bool external_field = false;  // the stray-field buffer holds a field set from outside
};

static thread_local std::string g_err;

static int fail(asd_t *h, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    g_err = buf;
    return code;
}

#define HIP_OK(h, call)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((h), ASD_EHIP, "%s: %s", #call, hipGetErrorString(e_));             \
    } while (0)

// ------------------------------------------------------------------ validation
static int check_params(const asd_params *p)
{
    if (!p) return fail(nullptr, ASD_EINVAL, "params is NULL");
    if (p->lattice != ASD_SC && p->lattice != ASD_L10)
        return fail(nullptr, ASD_EINVAL, "lattice must be ASD_SC or ASD_L10");
    if (p->precision != ASD_FP64 && p->precision != ASD_FP32)
        return fail(nullptr, ASD_EINVAL, "precision must be ASD_FP64 or ASD_FP32");
    if (p->lattice == ASD_SC && p->n_shells != 1)
        return fail(nullptr, ASD_EINVAL, "SC lattice has exactly one shell");
    if (p->lattice == ASD_L10 && (p->n_shells < 1 || p->n_shells > 4))
        return fail(nullptr, ASD_EINVAL, "L1_0 n_shells must be 1..4");
    if (!(p->a > 0) || (p->lattice == ASD_L10 && !(p->c > 0)))
        return fail(nullptr, ASD_EINVAL, "lattice constants must be positive");
    if (!(p->mu_s > 0) || !(p->gamma > 0) || !(p->dt > 0) || !(p->alpha >= 0))
        return fail(nullptr, ASD_EINVAL, "mu_s, gamma, dt must be positive and alpha >= 0");
    if (!std::isfinite(p->k_u)) return fail(nullptr, ASD_EINVAL, "k_u must be finite");
    for (int s = 0; s < p->n_shells; ++s)
        if (!std::isfinite(p->J[s])) return fail(nullptr, ASD_EINVAL, "J must be finite");
    if (p->philox_rounds != 10 && p->philox_rounds != 7)
        return fail(nullptr, ASD_EINVAL, "philox_rounds must be 10 or 7");
    if (p->kernel < ASD_KERNEL_AUTO || p->kernel > ASD_KERNEL_FUSED)
        return fail(nullptr, ASD_EINVAL, "unknown kernel selector");
    if (p->graph_steps < 0 || (p->graph_steps % 2) != 0)
        return fail(nullptr, ASD_EINVAL, "graph_steps must be a non-negative even number");
    return ASD_OK;
}

static int check_system(const asd_params *p, const asd_system_desc *d, int idx)
{
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return fail(nullptr, ASD_EINVAL, "system %d: sizes must be >= 1", idx);
    const int bc[3] = {d->bc_x, d->bc_y, d->bc_z};
    const int n[3] = {d->nx, d->ny, d->nz};
    for (int k = 0; k < 3; ++k) {
        if (bc[k] != ASD_BC_OPEN && bc[k] != ASD_BC_PERIODIC && !(k == 0 && bc[k] == ASD_BC_TRACK))
            return fail(nullptr, ASD_EINVAL, "system %d: bad boundary condition on axis %d", idx, k);
        if (bc[k] == ASD_BC_PERIODIC && n[k] < 3)
            return fail(nullptr, ASD_EINVAL, "system %d: periodic axis %d needs >= 3 cells", idx, k);
    }
    if (d->bc_x == ASD_BC_TRACK && d->track_nx < d->nx)
        return fail(nullptr, ASD_EINVAL, "system %d: track_nx must be >= nx", idx);
    int64_t sxv = d->bc_x == ASD_BC_TRACK ? d->track_nx : d->nx;
    int64_t stored = (p->lattice == ASD_SC ? 1 : 2) * sxv * d->ny * d->nz;
    if (stored >= (int64_t)1 << 31)
        return fail(nullptr, ASD_EINVAL, "system %d: more than 2^31 stored sites", idx);
    if (d->n_seeds < 0) return fail(nullptr, ASD_EINVAL, "system %d: n_seeds < 0", idx);
    if (d->n_seeds > 0 && (!d->seeds_xy || d->voronoi_q < 1 || d->boundary_w_units < 0))
        return fail(nullptr, ASD_EINVAL, "system %d: Voronoi needs seeds, q >= 1, w >= 0", idx);
    if (d->n_seeds > 0 && d->labels)
        return fail(nullptr, ASD_EINVAL, "system %d: give either Voronoi seeds or labels", idx);
    if (d->n_seeds > (int)kNoGrain)
        return fail(nullptr, ASD_EINVAL, "system %d: at most 65535 grains", idx);
    if (d->n_k_u_grain < 0 || (d->n_k_u_grain > 0 && !d->k_u_grain))
        return fail(nullptr, ASD_EINVAL, "system %d: bad per-grain k_u table", idx);
    return ASD_OK;
}

// ------------------------------------------------------------------ lattice setup
static int64_t min_image(int64_t d, int64_t L, bool periodic)
{
    if (!periodic) return d;
    d %= L;
    if (d < 0) d += L;
    if (2 * d > L) d -= L;
    return d;
}

// Columnar Voronoi labels: computed for each in-plane site of the stored
// lattice and extruded along z.
static void voronoi_plane(const asd_params *p, const asd_system_desc *d, int32_t sx,
                          std::vector<int32_t> &plane)
{
    const bool l10 = p->lattice == ASD_L10;
    const int per_cell = l10 ? 2 : 1;
    const int64_t Q = d->voronoi_q;
    const int64_t LX = (l10 ? 2 * (int64_t)sx : sx) * Q;
    const int64_t LY = (l10 ? 2 * (int64_t)d->ny : d->ny) * Q;
    const bool px = d->bc_x == ASD_BC_PERIODIC, py = d->bc_y == ASD_BC_PERIODIC;
    const int ns = d->n_seeds;
    const int64_t w2 = d->boundary_w_units * d->boundary_w_units;
    plane.assign((size_t)sx * d->ny * per_cell, -1);
    std::vector<int64_t> vx(ns), vy(ns);
    for (int32_t y = 0; y < d->ny; ++y)
        for (int32_t x = 0; x < sx; ++x)
            for (int s = 0; s < per_cell; ++s) {
                const int64_t X = l10 ? 2 * (int64_t)x + s : x;
                const int64_t Y = l10 ? 2 * (int64_t)y + s : y;
                int best = 0;
                int64_t bd = INT64_MAX;
                for (int k = 0; k < ns; ++k) {
                    vx[k] = min_image(X * Q - d->seeds_xy[2 * k], LX, px);
                    vy[k] = min_image(Y * Q - d->seeds_xy[2 * k + 1], LY, py);
                    const int64_t d2 = vx[k] * vx[k] + vy[k] * vy[k];
                    if (d2 < bd) {
                        bd = d2;
                        best = k;
                    }
                }
                bool mag = true;
                for (int k = 0; k < ns && mag; ++k) {
                    if (k == best) continue;
                    const int64_t gap = vx[k] * vx[k] + vy[k] * vy[k] - bd;
                    const int64_t ex = vx[best] - vx[k], ey = vy[best] - vy[k];
                    if (gap * gap < w2 * (ex * ex + ey * ey)) mag = false;
                }
                plane[((size_t)y * sx + x) * per_cell + s] = mag ? best : -1;
            }
}

// global-frame neighbour of stored site (SC cell or L1_0 half-cell coords);
// returns local stored index or -1
static int64_t neighbour_local(const asd_params *p, const asd_system_desc *d, int32_t sx, int64_t X,
                               int64_t Y, int64_t Z, int dx, int dy, int dz)
{
    const bool l10 = p->lattice == ASD_L10;
    const int64_t LX = l10 ? 2 * (int64_t)(d->bc_x == ASD_BC_TRACK ? sx : d->nx) : (d->bc_x == ASD_BC_TRACK ? sx : d->nx);
    const int64_t LY = l10 ? 2 * (int64_t)d->ny : d->ny;
    const int64_t LZ = d->nz;
    X += dx;
    Y += dy;
    Z += dz;
    if (X < 0 || X >= LX) {
        if (d->bc_x != ASD_BC_PERIODIC) return -1;
        X = (X % LX + LX) % LX;
    }
    if (Y < 0 || Y >= LY) {
        if (d->bc_y != ASD_BC_PERIODIC) return -1;
        Y = (Y % LY + LY) % LY;
    }
    if (Z < 0 || Z >= LZ) {
        if (d->bc_z != ASD_BC_PERIODIC) return -1;
        Z = (Z % LZ + LZ) % LZ;
    }
    if (!l10) return X + (int64_t)sx * (Y + (int64_t)d->ny * Z);
    const int64_t s = X & 1;
    return 2 * ((X >> 1) + (int64_t)sx * ((Y >> 1) + (int64_t)d->ny * Z)) + s;
}

static void site_coords(const asd_params *p, const HostSys &hs, int64_t i, int64_t &X, int64_t &Y,
                        int64_t &Z)
{
    const asd_system_desc *d = &hs.desc;
    if (p->lattice == ASD_SC) {
        X = i % hs.sx;
        Y = (i / hs.sx) % d->ny;
        Z = i / ((int64_t)hs.sx * d->ny);
    } else {
        const int64_t s = i & 1, cell = i >> 1;
        X = 2 * (cell % hs.sx) + s;
        Y = 2 * ((cell / hs.sx) % d->ny) + s;
        Z = cell / ((int64_t)hs.sx * d->ny);
    }
}

static int n_neighbour_slots(const asd_params *p)
{
    return p->lattice == ASD_SC ? 6 : kL10ShellEnd[p->n_shells - 1];
}

static int64_t slot_neighbour(const asd_params *p, const HostSys &hs, int64_t i, int k)
{
    int64_t X, Y, Z;
    site_coords(p, hs, i, X, Y, Z);
    const int *o = p->lattice == ASD_SC ? kScOffH[k] : kL10Off[k];
    return neighbour_local(p, &hs.desc, hs.sx, X, Y, Z, o[0], o[1], o[2]);
}

static int slot_shell(const asd_params *p, int k)
{
    if (p->lattice == ASD_SC) return 0;
    return k < 4 ? 0 : (k < 6 ? 1 : (k < 10 ? 2 : 3));
}

static int build_system(const asd_params *p, const asd_system_desc *d, int idx, HostSys &hs)
{
    hs.desc = *d;
    hs.desc.seeds_xy = nullptr;
    hs.desc.labels = nullptr;
    hs.desc.k_u_grain = nullptr;
    hs.sx = d->bc_x == ASD_BC_TRACK ? d->track_nx : d->nx;
    const int per_cell = p->lattice == ASD_SC ? 1 : 2;
    hs.n_stored = (int64_t)per_cell * hs.sx * d->ny * d->nz;
    hs.n_window = (int64_t)per_cell * d->nx * d->ny * d->nz;
    hs.labels.assign((size_t)hs.n_stored, 0);
    if (d->n_seeds > 0) {
        std::vector<int32_t> plane;
        voronoi_plane(p, d, hs.sx, plane);
        const size_t pn = plane.size();
        for (int64_t z = 0; z < d->nz; ++z)
            std::memcpy(&hs.labels[(size_t)z * pn], plane.data(), pn * sizeof(int32_t));
        hs.n_grains = d->n_seeds;
    } else if (d->labels) {
        int32_t mx = -1;
        for (int64_t i = 0; i < hs.n_stored; ++i) {
            int32_t l = d->labels[i];
            if (l < -1 || l >= (int32_t)kNoGrain)
                return fail(nullptr, ASD_EINVAL, "system %d: label out of range at %lld", idx,
                            (long long)i);
            hs.labels[i] = l;
            mx = std::max(mx, l);
        }
        hs.n_grains = std::max(mx + 1, 1);
    } else {
        hs.n_grains = 1;
    }
    if (d->n_k_u_grain > 0) {
        if (d->n_k_u_grain < hs.n_grains)
            return fail(nullptr, ASD_EINVAL, "system %d: k_u table shorter than the grain count", idx);
        hs.ku_grain.assign(d->k_u_grain, d->k_u_grain + hs.n_grains);
    }
    // no two magnetic neighbours may belong to different grains: the kernels
    // rely on non-magnetic boundaries to decouple grains
    const int slots = n_neighbour_slots(p);
    for (int64_t i = 0; i < hs.n_stored; ++i) {
        const int32_t li = hs.labels[i];
        if (li < 0) continue;
        for (int k = 0; k < slots; ++k) {
            const int64_t j = slot_neighbour(p, hs, i, k);
            if (j >= 0 && hs.labels[j] >= 0 && hs.labels[j] != li)
                return fail(nullptr, ASD_EUNSUPPORTED,
                            "system %d: magnetic neighbours %lld and %lld belong to different grains "
                            "(boundaries thinner than the neighbour range)",
                            idx, (long long)i, (long long)j);
        }
    }
    return ASD_OK;
}

static int grain_count_of(const asd_params *p, const asd_system_desc *d)
{
    (void)p;
    if (d->n_seeds > 0) return d->n_seeds;
    if (d->labels) {
        int64_t sxv = d->bc_x == ASD_BC_TRACK ? d->track_nx : d->nx;
        int64_t n = (p->lattice == ASD_SC ? 1 : 2) * sxv * d->ny * d->nz;
        int32_t mx = -1;
        for (int64_t i = 0; i < n; ++i) mx = std::max(mx, d->labels[i]);
        return std::max(mx + 1, 1);
    }
    return 1;
}

// tiles of fused variant tile_cfg along x, y, z (and the z chunk length);
// stage: the stage kernels of the step with the demagnetising field, whose
// whole extended tile is interior
static void fused_tiles_of(const asd_params *p, const asd_system_desc *d, int tile_cfg, int *tx,
                           int *ty, int *tz = nullptr, int *lz = nullptr, bool stage = false)
{
    int bx, by;
    const bool l10 = p->lattice == ASD_L10;
    fused_tile_interior(p->precision == ASD_FP64, tile_cfg, &bx, &by, l10);
    if (stage) {
        bx += 2;
        by += 2;
    }
    *tx = (d->nx + bx - 1) / bx;
    *ty = (d->ny + by - 1) / by;
    const FusedVariant f = fused_pick(l10, p->precision == ASD_FP64, tile_cfg);
    const int len = f.lz > 0 ? std::min(f.lz, d->nz) : d->nz;
    if (lz) *lz = len;
    if (tz) *tz = (d->nz + len - 1) / len;
}

// partial-sum slots of the fused kernels with the demagnetising field, SC
// variant v (stage: the halo-free stage kernels, else the one-launch step):
// how many tiles one coarse cell can meet along x, y and z
static void stage_slots(const asd_params *p, const asd_system_desc *d, const int32_t *cell, int v,
                        int *nsx, int *nsy, int *ns, bool stage = true)
{
    int bx, by, fx, fy, fz, len;
    fused_tile_interior(p->precision == ASD_FP64, v, &bx, &by, false);
    if (stage) {  // the stage kernels' tiles have no halo
        bx += 2;
        by += 2;
    }
    fused_tiles_of(p, d, v, &fx, &fy, &fz, &len, stage);
    *nsx = (cell[0] - 1) / bx + 2;
    *nsy = (cell[1] - 1) / by + 2;
    const int nsz = fz > 1 ? (cell[2] - 1) / len + 2 : 1;
    *ns = *nsx * *nsy * nsz;
}

static FastDivH host_fastdiv(uint32_t d)
{
    FastDivH f;
    f.d = d;
    uint32_t l = 0;
    while (l < 32 && ((uint64_t)1 << l) < d) ++l;
    f.l = l;
    f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
    return f;
}

static int ilog2_ceil(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// coarse mesh and padded FFT sizes of the demagnetising field; nullptr when
// the descriptors allow it, else the reason
static const char *demag_geometry(const asd_params *p, const asd_system_desc *sys, int n_sys,
                                  DemagDev *g)
{
    std::memset(g, 0, sizeof *g);
    const int32_t *c = p->demag_cell;
    if (c[0] == 0 && c[1] == 0 && c[2] == 0) return nullptr;
    if (c[0] < 1 || c[1] < 1 || c[2] < 1) return "demag_cell must be all positive or all zero";
    for (int s = 1; s < n_sys; ++s)
        if (sys[s].nx != sys[0].nx || sys[s].ny != sys[0].ny || sys[s].nz != sys[0].nz)
            return "the demagnetising field needs every system to have the same window size";
    g->on = 1;
    g->cx = c[0];
    g->cy = c[1];
    g->cz = c[2];
    g->ncx = (sys[0].nx + c[0] - 1) / c[0];
    g->ncy = (sys[0].ny + c[1] - 1) / c[1];
    g->ncz = (sys[0].nz + c[2] - 1) / c[2];
    if (g->ncx > 256 || g->ncy > 256 || g->ncz > 256)
        return "the demagnetising mesh is limited to 256 coarse cells per axis";
    for (int s = 0; s < n_sys; ++s)
        if (sys[s].bc_x == ASD_BC_TRACK && (sys[s].track_nx + c[0] - 1) / c[0] + 2 > 256)
            return "the stray field of a track needs at most 254 coarse cells along the track";
    g->ncell = g->ncx * g->ncy * g->ncz;
    // zero padding to a power of two >= 2 n - 1 (none for a single cell)
    g->lx = ilog2_ceil(2 * g->ncx - 1);
    g->ly = ilog2_ceil(2 * g->ncy - 1);
    g->lz = ilog2_ceil(2 * g->ncz - 1);
    // x lines per workgroup of the y and z passes: two LDS buffers of at
    // most 1024 (FP64) / 2048 (FP32) complex values (lines padded by one),
    // and no fewer than 1024 workgroups while the lines can be split
    const int budget = p->precision == ASD_FP64 ? 1024 : 2048;
    const int Px = 1 << g->lx, Py = 1 << g->ly, Pz = 1 << g->lz;
    const int Pxh = Px / 2 + 1;  // kept columns of the Hermitian x transform
    int xb = 1;
    while (xb * 2 <= Pxh && xb * 2 * (Py + 1) <= budget &&
           (int64_t)((Pxh + 2 * xb - 1) / (xb * 2)) * 3 * g->ncz * n_sys >= 1024)
        xb *= 2;
    g->xb_y = xb;
    xb = 1;
    while (xb * 2 <= Pxh && xb * 2 * 3 * (Pz + 1) <= budget &&
           (int64_t)((Pxh + 2 * xb - 1) / (xb * 2)) * Py * n_sys >= 1024)
        xb *= 2;
    g->xb_z = xb;
    g->n_sys = n_sys;
    g->fd_cx = host_fastdiv((uint32_t)c[0]);
    g->fd_cy = host_fastdiv((uint32_t)c[1]);
    g->fd_cz = host_fastdiv((uint32_t)c[2]);
    // cell-row kernels: whole cells across the 64 lanes of a wavefront
    g->cr_cells = c[0] <= 64 ? 64 / c[0] : 0;
    g->cr_segs = g->cr_cells ? (g->ncx + g->cr_cells - 1) / g->cr_cells : 0;
    return nullptr;
}

static Layout make_layout(const asd_params *p, const asd_system_desc *sys, int n_sys)
{
    Layout L;
    int64_t n = 0;
    int32_t g = 0, tiles = 0, ftiles = 0;
    for (int s = 0; s < n_sys; ++s) {
        const asd_system_desc *d = &sys[s];
        int64_t sxv = d->bc_x == ASD_BC_TRACK ? d->track_nx : d->nx;
        int per = p->lattice == ASD_SC ? 1 : 2;
        n += per * sxv * d->ny * d->nz;
        g += grain_count_of(p, d);
        int64_t nw = (int64_t)per * d->nx * d->ny * d->nz;
        tiles += (int32_t)((nw + kPlainTile - 1) / kPlainTile);
        int fx = 0, fy = 0, fz = 0;
        int maxf = 0;
        for (int v = 0; v < fused_count(p->lattice == ASD_L10, p->precision == ASD_FP64); ++v) {
            fused_tiles_of(p, d, v, &fx, &fy, &fz);
            maxf = std::max(maxf, fx * fy * fz);
        }
        ftiles += maxf;
    }
    L.n_total = n + 1;  // + zero slot
    L.zero_site = n;
    L.ncs = (int64_t)align_up((size_t)L.n_total, 64);
    L.n_grains = g;
    L.n_tiles = tiles;
    L.n_ftiles = ftiles;
    const size_t elem = p->precision == ASD_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    for (int b = 0; b < 3; ++b) L.off_S[b] = take(3 * (size_t)L.ncs * elem);
    L.off_F0 = take(3 * (size_t)L.ncs * elem);
    L.off_Bt = take(3 * (size_t)L.ncs * elem);
    L.off_label = take((size_t)L.ncs * sizeof(uint16_t));
    L.off_ell = p->lattice == ASD_L10 ? take((size_t)kL10Degree * L.ncs * sizeof(int32_t)) : 0;
    L.off_sys = take((size_t)n_sys * sizeof(SysDev));
    L.off_tile = take((size_t)std::max(tiles, 1) * sizeof(int32_t));
    L.off_ftile = take((size_t)std::max(ftiles, 1) * sizeof(int32_t));
    L.off_can = take((size_t)std::max(g, 1) * sizeof(double));
    L.off_can32 = take((size_t)std::max(g, 1) * sizeof(float));
    L.off_ku = take((size_t)std::max(g, 1) * sizeof(double));
    L.off_gsys = take((size_t)std::max(g, 1) * sizeof(int32_t));
    L.off_gptr = take((size_t)(g + 1) * sizeof(int64_t));
    L.off_gsites = take((size_t)std::max<int64_t>(n, 1) * sizeof(int32_t));
    L.off_step = take(sizeof(int64_t));
    L.off_origin = take((size_t)n_sys * sizeof(int32_t));
    L.off_bits = take(kMaxBits);
    L.off_gout = take((size_t)std::max(g, 1) * 4 * sizeof(double));
    L.off_sout = take((size_t)n_sys * 4 * sizeof(double));
    L.off_mom = take((size_t)n_sys * 5 * sizeof(double));
    L.off_epart = take((size_t)std::max(tiles, 1) * 3 * sizeof(double));
    L.off_eout = take((size_t)n_sys * 4 * sizeof(double));
    (void)demag_geometry(p, sys, n_sys, &L.dm);
    if (L.dm.on) {
        const DemagDev &g = L.dm;
        const size_t Px = (size_t)1 << g.lx, Py = (size_t)1 << g.ly, Pz = (size_t)1 << g.lz;
        const size_t cplx = 2 * elem;
        const size_t Pxh = Px / 2 + 1;  // kept columns of the Hermitian x transform
        L.off_dwx = take((size_t)n_sys * 3 * g.ncz * g.ncy * Pxh * cplx);
        L.off_dwy = take((size_t)n_sys * 3 * g.ncz * Py * Pxh * cplx);
        for (int b = 0; b < 2; ++b) L.off_dbd[b] = take((size_t)n_sys * 3 * g.ncell * elem);
        // cell sums: one slot (cell-row kernels) or the fused stage kernels' partial slots
        int ns_max = 1;
        if (p->lattice == ASD_SC)
            for (int v = 0; v < fused_count(false, p->precision == ASD_FP64); ++v)
                for (bool stage : {true, false}) {
                    int nsx, nsy, ns;
                    stage_slots(p, &sys[0], p->demag_cell, v, &nsx, &nsy, &ns, stage);
                    ns_max = std::max(ns_max, ns);
                }
        for (int b = 0; b < 2; ++b)
            L.off_dcs[b] = take((size_t)n_sys * 3 * ns_max * g.ncell * elem);
        L.dcs_bytes = (size_t)n_sys * 3 * ns_max * g.ncell * elem;
        L.off_dK = take(6 * (Px / 2 + 1) * (Py / 2 + 1) * (Pz / 2 + 1) * elem);
        L.off_dtw[0] = take(std::max<size_t>(Px / 2, 1) * cplx);
        L.off_dtw[1] = take(std::max<size_t>(Py / 2, 1) * cplx);
        L.off_dtw[2] = take(std::max<size_t>(Pz / 2, 1) * cplx);
        bool track = false;
        int32_t sxmax = 0;
        for (int s = 0; s < n_sys; ++s) {
            if (sys[s].bc_x == ASD_BC_TRACK) track = true;
            sxmax = std::max(sxmax, sys[s].bc_x == ASD_BC_TRACK ? sys[s].track_nx : sys[s].nx);
        }
        if (track) {
            // the window's cells continued over the whole track: at most
            // ceil(track / cx) + 1 of them hold sites
            DemagDev &t = L.dmT;
            t = g;
            t.stray = 1;
            t.ncx_win = g.ncx;
            t.ncell_win = g.ncell;
            t.ncx = (sxmax + g.cx - 1) / g.cx + 2;
            t.ncell = t.ncx * g.ncy * g.ncz;
            t.lx = ilog2_ceil(2 * t.ncx - 1);
            const size_t PxT = (size_t)1 << t.lx;
            const int budget = p->precision == ASD_FP64 ? 1024 : 2048;
            const int PxTh = (int)PxT / 2 + 1;
            int xb = 1;
            while (xb * 2 <= PxTh && xb * 2 * ((int)Py + 1) <= budget &&
                   (int64_t)((PxTh + 2 * xb - 1) / (xb * 2)) * 3 * g.ncz * n_sys >= 1024)
                xb *= 2;
            t.xb_y = xb;
            xb = 1;
            while (xb * 2 <= PxTh && xb * 2 * 3 * ((int)Pz + 1) <= budget &&
                   (int64_t)((PxTh + 2 * xb - 1) / (xb * 2)) * Py * n_sys >= 1024)
                xb *= 2;
            t.xb_z = xb;
            L.off_twx = take((size_t)n_sys * 3 * g.ncz * g.ncy * (PxT / 2 + 1) * cplx);
            L.off_twy = take((size_t)n_sys * 3 * g.ncz * Py * (PxT / 2 + 1) * cplx);
            L.off_tK = take(6 * (PxT / 2 + 1) * (Py / 2 + 1) * (Pz / 2 + 1) * elem);
            L.off_ttw = take(std::max<size_t>(PxT / 2, 1) * cplx);
            L.off_tstray = take((size_t)n_sys * 3 * g.ncell * elem);
        }
    }
    L.bytes = off;
    return L;
}

// ------------------------------------------------------------------ C ABI
// (definitions take C linkage from their declarations in asd.h)

const char *asd_strerror(int code)
{
    switch (code) {
    case ASD_OK: return "ok";
    case ASD_EINVAL: return "invalid argument";
    case ASD_ENOMEM: return "workspace too small";
    case ASD_EHIP: return "HIP runtime error";
    case ASD_ESTATE: return "invalid state";
    case ASD_ENONFINITE: return "non-finite value in a reduction";
    case ASD_EUNSUPPORTED: return "unsupported";
    default: return "unknown error";
    }
}

const char *asd_last_error(const asd_t *h) { return h ? h->err.c_str() : g_err.c_str(); }

int asd_workspace_bytes(const asd_params *p, const asd_system_desc *sys, int32_t n_sys,
                        size_t *bytes)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (!sys || n_sys < 1 || !bytes) return fail(nullptr, ASD_EINVAL, "need >= 1 system and bytes");
    for (int s = 0; s < n_sys; ++s)
        if ((rc = check_system(p, &sys[s], s))) return rc;
    DemagDev g;
    if (const char *why = demag_geometry(p, sys, n_sys, &g)) {
        const bool bad_arg = std::strstr(why, "must") != nullptr;
        return fail(nullptr, bad_arg ? ASD_EINVAL : ASD_EUNSUPPORTED, "%s", why);
    }
    *bytes = make_layout(p, sys, n_sys).bytes;
    return ASD_OK;
}

static double T_of(const asd_t *h, int s)
{
    return h->sys[s].desc.T_system >= 0 ? h->sys[s].desc.T_system : h->drive.T_amb;
}

static int upload_sysdev(asd_t *h)
{
    for (size_t s = 0; s < h->sys.size(); ++s) h->dev[s].T_amb = T_of(h, (int)s);
    HIP_OK(h, hipMemcpyAsync(h->ws + h->L.off_sys, h->dev.data(), h->dev.size() * sizeof(SysDev),
                             hipMemcpyHostToDevice, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    return ASD_OK;
}

static void drop_graphs(asd_t *h)
{
    for (int k = 0; k < 2; ++k)
        if (h->graph[k]) {
            (void)hipGraphExecDestroy(h->graph[k]);
            h->graph[k] = nullptr;
        }
}

static const char *fused_unsupported(const asd_t *h);
static const char *cell_rows_unsupported(const asd_t *h);
static int setup_fused_tiles(asd_t *h, int v);

int asd_create(const asd_params *p, const asd_system_desc *sys, int32_t n_sys, void *workspace,
               size_t workspace_bytes, void *stream, asd_t **out)
{
    if (!out) return fail(nullptr, ASD_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    int rc = asd_workspace_bytes(p, sys, n_sys, &need);
    if (rc) return rc;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0)
        return fail(nullptr, ASD_EINVAL, "workspace must be a 256-byte aligned device pointer");
    if (workspace_bytes < need)
        return fail(nullptr, ASD_ENOMEM, "workspace of %zu bytes < %zu needed", workspace_bytes, need);
    asd_t *h = new (std::nothrow) asd_t();
    if (!h) return fail(nullptr, ASD_ENOMEM, "host allocation failed");
    h->p = *p;
    h->ws = (char *)workspace;
    h->stream = (hipStream_t)stream;
    h->elem = p->precision == ASD_FP64 ? 8 : 4;
    h->kernel = ASD_KERNEL_PLAIN;
    h->graph_steps = p->graph_steps;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(nullptr, ASD_EHIP, "hipGetDevice failed");
    }
    h->sys.resize(n_sys);
    h->L = make_layout(p, sys, n_sys);
    for (int s = 0; s < n_sys; ++s)
        if ((rc = build_system(p, &sys[s], s, h->sys[s]))) {
            delete h;
            return rc;
        }
    const Layout &L = h->L;
    // device descriptors, tile maps, grain tables
    h->dev.resize(n_sys);
    std::vector<int32_t> tile_sys, gsys;
    std::vector<double> can, ku;
    std::vector<float> can32;
    std::vector<int64_t> gptr(1, 0);
    std::vector<int32_t> gsites;
    std::vector<uint16_t> lab((size_t)L.ncs, kNoGrain);
    int64_t base = 0;
    int32_t gbase = 0;
    for (int s = 0; s < n_sys; ++s) {
        HostSys &hs = h->sys[s];
        SysDev &d = h->dev[s];
        std::memset(&d, 0, sizeof d);
        d.kind = p->lattice;
        d.nx = hs.desc.nx;
        d.ny = hs.desc.ny;
        d.nz = hs.desc.nz;
        d.sx = hs.sx;
        d.bcx = hs.desc.bc_x;
        d.bcy = hs.desc.bc_y;
        d.bcz = hs.desc.bc_z;
        d.track = hs.desc.bc_x == ASD_BC_TRACK;
        d.grain_base = gbase;
        d.n_grains = hs.n_grains;
        d.tile_base = (int32_t)tile_sys.size();
        d.n_tiles = (int32_t)((hs.n_window + kPlainTile - 1) / kPlainTile);
        for (int t = 0; t < d.n_tiles; ++t) tile_sys.push_back(s);
        d.sys_id = (uint32_t)s;
        d.fd_nx = host_fastdiv((uint32_t)d.nx);
        d.fd_ny = host_fastdiv((uint32_t)d.ny);
        d.base = base;
        d.n_stored = hs.n_stored;
        d.n_window = hs.n_window;
        for (int64_t i = 0; i < hs.n_stored; ++i)
            lab[(size_t)(base + i)] = hs.labels[i] < 0 ? kNoGrain : (uint16_t)hs.labels[i];
        d.columnar = 1;
        {
            const int64_t pn = (p->lattice == ASD_SC ? 1 : 2) * (int64_t)hs.sx * hs.desc.ny;
            for (int64_t i = pn; i < hs.n_stored && d.columnar; ++i)
                if (hs.labels[i] != hs.labels[i % pn]) d.columnar = 0;
        }
        // grain site lists, ascending site index within each grain
        std::vector<int64_t> cnt(hs.n_grains + 1, 0);
        for (int64_t i = 0; i < hs.n_stored; ++i)
            if (hs.labels[i] >= 0) ++cnt[hs.labels[i] + 1];
        for (int g = 0; g < hs.n_grains; ++g) cnt[g + 1] += cnt[g];
        std::vector<int32_t> sites(cnt[hs.n_grains]);
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (int64_t i = 0; i < hs.n_stored; ++i)
            if (hs.labels[i] >= 0) sites[fill[hs.labels[i]]++] = (int32_t)i;
        const int64_t off0 = (int64_t)gsites.size();
        gsites.insert(gsites.end(), sites.begin(), sites.end());
        for (int g = 0; g < hs.n_grains; ++g) {
            gptr.push_back(off0 + cnt[g + 1]);
            gsys.push_back(s);
            double kug = hs.ku_grain.empty() ? p->k_u : hs.ku_grain[g];
            ku.push_back(kug);
            can.push_back((2.0 * kug) / p->mu_s);
        }
        base += hs.n_stored;
        gbase += hs.n_grains;
    }
    // fused tile map is filled per variant at step time; start with variant 0
    h->origin.assign(n_sys, 0);
    char *w = h->ws;
    hipStream_t st = h->stream;
    // zero everything: spin buffers (incl. the zero slot), counters, outputs
    HIP_OK(h, hipMemsetAsync(w, 0, L.bytes, st));
    HIP_OK(h, hipMemcpyAsync(w + L.off_label, lab.data(), lab.size() * sizeof(uint16_t),
                             hipMemcpyHostToDevice, st));
    HIP_OK(h, hipMemcpyAsync(w + L.off_tile, tile_sys.data(), tile_sys.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, st));
    if (!can.empty()) {
        HIP_OK(h, hipMemcpyAsync(w + L.off_can, can.data(), can.size() * sizeof(double),
                                 hipMemcpyHostToDevice, st));
        can32.assign(can.begin(), can.end());
        HIP_OK(h, hipMemcpyAsync(w + L.off_can32, can32.data(), can32.size() * sizeof(float),
                                 hipMemcpyHostToDevice, st));
        HIP_OK(h, hipMemcpyAsync(w + L.off_ku, ku.data(), ku.size() * sizeof(double),
                                 hipMemcpyHostToDevice, st));
        HIP_OK(h, hipMemcpyAsync(w + L.off_gsys, gsys.data(), gsys.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
    }
    HIP_OK(h, hipMemcpyAsync(w + L.off_gptr, gptr.data(), gptr.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, st));
    if (!gsites.empty())
        HIP_OK(h, hipMemcpyAsync(w + L.off_gsites, gsites.data(), gsites.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
    std::vector<int32_t> ell;
    if (p->lattice == ASD_L10) {
        // ELL neighbour table [slot][site]; absent neighbours and unused
        // slots point at the zero slot
        ell.assign((size_t)kL10Degree * L.ncs, (int32_t)L.zero_site);
        const int slots = n_neighbour_slots(p);
        for (int s = 0; s < n_sys; ++s) {
            const HostSys &hs = h->sys[s];
            const int64_t b = h->dev[s].base;
            for (int64_t i = 0; i < hs.n_stored; ++i)
                for (int k = 0; k < slots; ++k) {
                    int64_t j = slot_neighbour(p, hs, i, k);
                    if (j >= 0) ell[(size_t)k * L.ncs + b + i] = (int32_t)(b + j);
                }
        }
        HIP_OK(h, hipMemcpyAsync(w + L.off_ell, ell.data(), ell.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
    }
    // initial spins: +z on magnetic sites, both ping-pong buffers
    {
        std::vector<char> S((size_t)3 * L.ncs * h->elem, 0);
        for (int64_t i = 0; i < L.ncs; ++i)
            if (lab[(size_t)i] != kNoGrain && i < L.zero_site) {
                if (h->elem == 8) ((double *)S.data())[2 * L.ncs + i] = 1.0;
                else ((float *)S.data())[2 * L.ncs + i] = 1.0f;
            }
        for (int b = 0; b < 2; ++b)
            HIP_OK(h, hipMemcpyAsync(w + L.off_S[b], S.data(), S.size(), hipMemcpyHostToDevice, st));
        HIP_OK(h, hipStreamSynchronize(st));
    }
    if (L.dm.on) {
        // demagnetising field: tensor spectrum and twiddles (host FP64)
        DemagDev g = L.dm;
        const double ex = p->a, ey = p->a, ez = p->lattice == ASD_SC ? p->a : p->c;
        const double dx = g.cx * ex, dy = g.cy * ey, dz = g.cz * ez;
        const int Px = 1 << g.lx, Py = 1 << g.ly, Pz = 1 << g.lz;
        // the one-workgroup y-z pass (direct sums along z) where its LDS fits
        int lds_max = 0;
        if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) !=
            hipSuccess)
            lds_max = 0;
        auto yz_fits = [&](const DemagDev &d) {
            const size_t need = demag_yz_lds_bytes(d, h->elem);
            return need > 0 && need <= (size_t)lds_max ? 1 : 0;
        };
        g.yzf = yz_fits(g);
        std::vector<double> oct;
        if (g.yzf)
            demag_mixed(g.ncx, g.ncy, g.ncz, dx, dy, dz, g.lx, g.ly,
                        -kMu0 * p->mu_s / (((dx * dy) * dz) * ((double)Px * Py)), oct);
        else
            demag_spectrum(g.ncx, g.ncy, g.ncz, dx, dy, dz, g.lx, g.ly, g.lz,
                           -kMu0 * p->mu_s / (((dx * dy) * dz) * ((double)Px * Py * Pz)), oct);
        std::vector<char> buf(oct.size() * h->elem);
        for (size_t i = 0; i < oct.size(); ++i) {
            if (h->elem == 8) ((double *)buf.data())[i] = oct[i];
            else ((float *)buf.data())[i] = (float)oct[i];
        }
        HIP_OK(h, hipMemcpyAsync(w + L.off_dK, buf.data(), buf.size(), hipMemcpyHostToDevice, st));
        std::vector<std::vector<char>> tw(3);
        const int lp[3] = {g.lx, g.ly, g.lz};
        for (int ax = 0; ax < 3; ++ax) {
            const int P = 1 << lp[ax], half = std::max(P / 2, 1);
            tw[ax].resize((size_t)half * 2 * h->elem);
            for (int t = 0; t < half; ++t) {
                const double ang = -2.0 * M_PI * (double)t / (double)P;
                if (h->elem == 8) {
                    ((double *)tw[ax].data())[2 * t] = std::cos(ang);
                    ((double *)tw[ax].data())[2 * t + 1] = std::sin(ang);
                } else {
                    ((float *)tw[ax].data())[2 * t] = (float)std::cos(ang);
                    ((float *)tw[ax].data())[2 * t + 1] = (float)std::sin(ang);
                }
            }
            HIP_OK(h, hipMemcpyAsync(w + L.off_dtw[ax], tw[ax].data(), tw[ax].size(),
                                     hipMemcpyHostToDevice, st));
        }
        g.wx = w + L.off_dwx;
        g.wy = w + L.off_dwy;
        g.bd[0] = w + L.off_dbd[0];
        g.bd[1] = w + L.off_dbd[1];
        g.cs[0] = w + L.off_dcs[0];
        g.cs[1] = w + L.off_dcs[1];
        g.K = w + L.off_dK;
        for (int ax = 0; ax < 3; ++ax) g.tw[ax] = w + L.off_dtw[ax];
        if (L.dmT.on) {
            DemagDev t = L.dmT;
            const int PxT = 1 << t.lx;
            t.yzf = yz_fits(t);
            if (t.yzf)
                demag_mixed(t.ncx, t.ncy, t.ncz, dx, dy, dz, t.lx, t.ly,
                            -kMu0 * p->mu_s / (((dx * dy) * dz) * ((double)PxT * Py)), oct);
            else
                demag_spectrum(t.ncx, t.ncy, t.ncz, dx, dy, dz, t.lx, t.ly, t.lz,
                               -kMu0 * p->mu_s / (((dx * dy) * dz) * ((double)PxT * Py * Pz)), oct);
            buf.assign(oct.size() * h->elem, 0);
            for (size_t i = 0; i < oct.size(); ++i) {
                if (h->elem == 8) ((double *)buf.data())[i] = oct[i];
                else ((float *)buf.data())[i] = (float)oct[i];
            }
            HIP_OK(h, hipMemcpyAsync(w + L.off_tK, buf.data(), buf.size(), hipMemcpyHostToDevice, st));
            std::vector<char> twT((size_t)std::max(PxT / 2, 1) * 2 * h->elem);
            for (int q = 0; q < std::max(PxT / 2, 1); ++q) {
                const double ang = -2.0 * M_PI * (double)q / (double)PxT;
                if (h->elem == 8) {
                    ((double *)twT.data())[2 * q] = std::cos(ang);
                    ((double *)twT.data())[2 * q + 1] = std::sin(ang);
                } else {
                    ((float *)twT.data())[2 * q] = (float)std::cos(ang);
                    ((float *)twT.data())[2 * q + 1] = (float)std::sin(ang);
                }
            }
            HIP_OK(h, hipMemcpyAsync(w + L.off_ttw, twT.data(), twT.size(), hipMemcpyHostToDevice, st));
            t.wx = w + L.off_twx;
            t.wy = w + L.off_twy;
            t.K = w + L.off_tK;
            t.tw[0] = w + L.off_ttw;
            t.tw[1] = g.tw[1];
            t.tw[2] = g.tw[2];
            t.bstray = w + L.off_tstray;
            t.bd[0] = t.bd[1] = nullptr;
            t.cs[0] = t.cs[1] = nullptr;
            h->dmT = t;
            g.bstray = t.bstray;  // the window's field includes the track's
            HIP_OK(h, hipStreamSynchronize(st));
        }
        h->dm = g;
        HIP_OK(h, hipStreamSynchronize(st));
    }
    h->drive = asd_drive{};
    int r2 = upload_sysdev(h);
    if (r2) {
        delete h;
        return r2;
    }
    HIP_OK(h, hipStreamSynchronize(st));
    // AUTO: fused where it applies; FUSED: required
    if (p->kernel != ASD_KERNEL_PLAIN) {
        const char *why = fused_unsupported(h);
        if (!why) {
            int r3 = asd_set_variant(h, ASD_KERNEL_FUSED, 0);
            if (r3) {
                delete h;
                return r3;
            }
        } else if (p->kernel == ASD_KERNEL_FUSED) {
            fail(nullptr, ASD_EUNSUPPORTED, "%s", why);
            delete h;
            return ASD_EUNSUPPORTED;
        }
    }
    // with the demagnetising field the two-pass kernels default to the
    // cell-row variant, which forms the cell sums as it writes the spins
    if (h->kernel == ASD_KERNEL_PLAIN && !cell_rows_unsupported(h)) h->tile_cfg = kCellRowVariant;
    *out = h;
    return ASD_OK;
}

int asd_destroy(asd_t *h)
{
    if (!h) return ASD_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    delete h;
    return ASD_OK;
}

int asd_set_field_temperature(asd_t *h, const asd_drive *d)
{
    if (!h || !d) return fail(h, ASD_EINVAL, "NULL argument");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(d->B[k])) return fail(h, ASD_EINVAL, "B must be finite");
    if (d->n_bits < 0 || d->n_bits > kMaxBits || (d->n_bits > 0 && (!d->bits || d->steps_per_bit <= 0)))
        return fail(h, ASD_EINVAL, "bits: 0..65536 entries with steps_per_bit > 0");
    if (d->spot_mode < ASD_SPOT_NONE || d->spot_mode > ASD_SPOT_LOCKED)
        return fail(h, ASD_EINVAL, "unknown spot mode");
    if (!(d->T_amb >= 0) || (d->spot_mode != ASD_SPOT_NONE && !(d->T_peak >= 0 && d->fwhm > 0)))
        return fail(h, ASD_EINVAL, "temperatures must be >= 0 and fwhm > 0 with a spot");
    h->drive = *d;
    h->drive.bits = nullptr;
    h->bits.assign(d->bits, d->bits + d->n_bits);
    if (d->n_bits > 0)
        HIP_OK(h, hipMemcpyAsync(h->ws + h->L.off_bits, h->bits.data(), h->bits.size(),
                                 hipMemcpyHostToDevice, h->stream));
    drop_graphs(h);  // constants are baked into captured launches
    return upload_sysdev(h);
}

static size_t spin_bytes(const asd_t *h, int s) { return (size_t)h->sys[s].n_stored * h->elem; }

int asd_set_spins(asd_t *h, int32_t s, const void *src, int32_t on_device)
{
    if (!h || !src) return fail(h, ASD_EINVAL, "NULL argument");
    if (s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad system index");
    const SysDev &d = h->dev[s];
    const size_t nb = spin_bytes(h, s);
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int b = 0; b < 2; ++b) {
        char *dst = h->ws + h->L.off_S[b];
        for (int k = 0; k < 3; ++k)
            HIP_OK(h, hipMemcpyAsync(dst + ((size_t)k * h->L.ncs + d.base) * h->elem,
                                     (const char *)src + k * nb, nb, kind, h->stream));
        if (launch_mask_spins(h->p.precision, dst, h->L.ncs,
                              (const uint16_t *)(h->ws + h->L.off_label), d, h->stream))
            return fail(h, ASD_EHIP, "mask kernel launch failed");
    }
    h->stray_dirty = true;
    HIP_OK(h, hipStreamSynchronize(h->stream));
    return ASD_OK;
}

int asd_get_spins(asd_t *h, int32_t s, void *dst, int32_t on_device)
{
    if (!h || !dst) return fail(h, ASD_EINVAL, "NULL argument");
    if (s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad system index");
    const SysDev &d = h->dev[s];
    const size_t nb = spin_bytes(h, s);
    const char *src = h->ws + h->L.off_S[h->cur];
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int k = 0; k < 3; ++k)
        HIP_OK(h, hipMemcpyAsync((char *)dst + k * nb, src + ((size_t)k * h->L.ncs + d.base) * h->elem,
                                 nb, kind, h->stream));
    if (!on_device) HIP_OK(h, hipStreamSynchronize(h->stream));
    return ASD_OK;
}

static StepConsts make_consts(const asd_t *h)
{
    const asd_params &p = h->p;
    const asd_drive &dr = h->drive;
    StepConsts c;
    std::memset(&c, 0, sizeof c);
    for (int s = 0; s < p.n_shells; ++s) c.cex[s] = p.J[s] / p.mu_s;
    c.can = (2.0 * p.k_u) / p.mu_s;
    c.gp = -p.gamma / (1.0 + p.alpha * p.alpha);
    c.alpha = p.alpha;
    c.dt = p.dt;
    c.h = 0.5 * p.dt;
    c.cth = ((2.0 * p.alpha) * kBoltzmann) / ((p.gamma * p.mu_s) * p.dt);
    for (int k = 0; k < 3; ++k) c.B[k] = dr.B[k];
    c.T_peak = dr.T_peak;
    if (dr.spot_mode != ASD_SPOT_NONE) {
        double sd = dr.fwhm / 2.3548200450309493;
        c.inv2s2 = 1.0 / ((2.0 * sd) * sd);
    }
    c.x0 = dr.x0;
    c.y0 = dr.y0;
    c.v = dr.v;
    c.hx = p.lattice == ASD_SC ? p.a : 0.5 * p.a;
    c.spb = dr.steps_per_bit;
    c.n_bits = dr.n_bits;
    c.spot_mode = dr.spot_mode;
    c.n_shells = p.n_shells;
    c.rounds = p.philox_rounds;
    c.k0 = (uint32_t)p.seed;
    c.k1 = (uint32_t)(p.seed >> 32);
    bool per_grain = false;
    for (const HostSys &hs : h->sys)
        if (!hs.ku_grain.empty()) per_grain = true;
    c.has_can_grain = per_grain ? 1 : 0;
    return c;
}

template <typename T>
static StepArgs<T> make_args(const asd_t *h, int cur, int step_off)
{
    const Layout &L = h->L;
    char *w = h->ws;
    StepArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.S = (const T *)(w + L.off_S[cur]);
    a.So = (T *)(w + L.off_S[1 - cur]);
    a.Sp = (T *)(w + L.off_S[2]);
    a.F0 = (T *)(w + L.off_F0);
    a.Bt = (T *)(w + L.off_Bt);
    a.ncs = L.ncs;
    a.sys = (const SysDev *)(w + L.off_sys);
    a.tile_sys = (const int32_t *)(w + (h->kernel == ASD_KERNEL_FUSED ? L.off_ftile : L.off_tile));
    a.ell = h->p.lattice == ASD_L10 ? (const int32_t *)(w + L.off_ell) : nullptr;
    a.label = (const uint16_t *)(w + L.off_label);
    a.can_grain = (const double *)(w + L.off_can);
    a.can_grain32 = (const float *)(w + L.off_can32);
    a.step_base = (const int64_t *)(w + L.off_step);
    a.origin = (const int32_t *)(w + L.off_origin);
    a.bits = (const uint8_t *)(w + L.off_bits);
    a.zero_site = L.zero_site;
    a.step_off = step_off;
    a.tile_cfg = h->tile_cfg;
    a.lattice = h->p.lattice;
    for (const HostSys &hs : h->sys)
        if (hs.desc.bc_z == ASD_BC_PERIODIC) a.any_zper = 1;
    a.c = make_consts(h);
    a.dm = h->dm;
    return a;
}

static int launch_one(asd_t *h, int cur, int step_off)
{
    int rc;
    const bool fused = h->kernel == ASD_KERNEL_FUSED;
    const int blocks = fused ? h->n_ftiles : h->L.n_tiles;
    if (h->p.precision == ASD_FP64) {
        StepArgs<double> a = make_args<double>(h, cur, step_off);
        rc = fused ? launch_fused_step_f64(a, blocks, h->stream) : launch_plain_step_f64(a, blocks, h->stream);
    } else {
        StepArgs<float> a = make_args<float>(h, cur, step_off);
        rc = fused ? launch_fused_step_f32(a, blocks, h->stream) : launch_plain_step_f32(a, blocks, h->stream);
    }
    if (rc == -2) return fail(h, ASD_EUNSUPPORTED, "fused kernel not available for this lattice");
    if (rc) return fail(h, ASD_EHIP, "step kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    return ASD_OK;
}

// stray field of the frozen track, recomputed when the track changed
// (spins set, window shifted, columns thermalised)
static int refresh_stray(asd_t *h)
{
    if (!h->dmT.on || !h->stray_dirty || h->external_field) return ASD_OK;
    const char *w = h->ws;
    const SysDev *sys = (const SysDev *)(w + h->L.off_sys);
    const int32_t *org = (const int32_t *)(w + h->L.off_origin);
    int rc;
    if (h->elem == 8)
        rc = launch_demag(h->dmT, (const double *)(w + h->L.off_S[h->cur]), h->L.ncs, sys, org, 0,
                          h->stream);
    else
        rc = launch_demag(h->dmT, (const float *)(w + h->L.off_S[h->cur]), h->L.ncs, sys, org, 0,
                          h->stream);
    if (rc) return fail(h, ASD_EHIP, "stray field launch failed: %s", hipGetErrorString(hipGetLastError()));
    h->stray_dirty = false;
    return ASD_OK;
}

static int capture_graph(asd_t *h, int cur)
{
    hipGraph_t g = nullptr;
    HIP_OK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int rc = ASD_OK;
    int c = cur;
    for (int t = 0; t < h->graph_steps && rc == ASD_OK; ++t) {
        rc = launch_one(h, c, t);
        c = 1 - c;
    }
    if (rc == ASD_OK && launch_advance_step((int64_t *)(h->ws + h->L.off_step), h->graph_steps, h->stream))
        rc = fail(h, ASD_EHIP, "advance launch failed");
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(h, ASD_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&h->graph[cur], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(h, ASD_EHIP, "graph instantiate failed: %s", hipGetErrorString(e));
    // move the graph to the device now, so its first launch does not pay for it
    HIP_OK(h, hipGraphUpload(h->graph[cur], h->stream));
    h->graph_kernel = h->kernel;
    h->graph_tile = h->tile_cfg;
    return ASD_OK;
}

int asd_step(asd_t *h, int64_t n)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (n < 0) return fail(h, ASD_EINVAL, "n must be >= 0");
    if (h->step + n >= ((int64_t)1 << 32))
        return fail(h, ASD_ESTATE, "step counter would exceed 2^32 (Philox counter word)");
    if (n == 0) return ASD_OK;
    if (int rc = refresh_stray(h)) return rc;
    int64_t done = 0;
    if (h->graph_steps > 0 && n >= h->graph_steps) {
        if (h->graph_kernel != h->kernel || h->graph_tile != h->tile_cfg) drop_graphs(h);
        while (n - done >= h->graph_steps) {
            if (!h->graph[h->cur]) {
                int rc = capture_graph(h, h->cur);
                if (rc) return rc;
            }
            HIP_OK(h, hipGraphLaunch(h->graph[h->cur], h->stream));
            done += h->graph_steps;
            h->step += h->graph_steps;  // graph_steps is even: the parity is unchanged
        }
    }
    const int64_t rest = n - done;
    for (int64_t t = 0; t < rest; ++t) {
        int rc = launch_one(h, h->cur, (int)t);
        if (rc) return rc;
        h->cur = 1 - h->cur;
    }
    if (rest > 0) {
        if (launch_advance_step((int64_t *)(h->ws + h->L.off_step), rest, h->stream))
            return fail(h, ASD_EHIP, "advance launch failed");
        h->step += rest;
    }
    return ASD_OK;
}

int asd_prepare(asd_t *h)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (h->graph_steps <= 0) return ASD_OK;
    if (h->graph_kernel != h->kernel || h->graph_tile != h->tile_cfg) drop_graphs(h);
    for (int c = 0; c < 2; ++c)
        if (!h->graph[c]) {
            int rc = capture_graph(h, c);
            if (rc) return rc;
        }
    return ASD_OK;
}

int asd_shift_window(asd_t *h, int32_t columns)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (columns < 0) return fail(h, ASD_EINVAL, "columns must be >= 0");
    bool any = false;
    for (size_t s = 0; s < h->sys.size(); ++s) {
        const SysDev &d = h->dev[s];
        if (!d.track) continue;
        any = true;
        if ((int64_t)h->origin[s] + d.nx + columns > d.sx)
            return fail(h, ASD_ESTATE, "system %zu: window would leave its track", s);
    }
    if (!any) return fail(h, ASD_EINVAL, "no system has a track");
    if (columns == 0) return ASD_OK;
    char *cur = h->ws + h->L.off_S[h->cur];
    char *oth = h->ws + h->L.off_S[1 - h->cur];
    for (size_t s = 0; s < h->sys.size(); ++s) {
        const SysDev &d = h->dev[s];
        if (!d.track) continue;
        // leaving columns freeze with their current spins in both buffers
        if (launch_copy_columns(h->p.precision, oth, cur, h->L.ncs, d, h->origin[s], columns, h->stream))
            return fail(h, ASD_EHIP, "column copy failed");
        h->origin[s] += columns;
    }
    h->stray_dirty = true;
    if (launch_set_i32((int32_t *)(h->ws + h->L.off_origin), h->origin.data(), (int)h->origin.size(),
                       h->stream))
        return fail(h, ASD_EHIP, "origin update failed");
    return ASD_OK;
}

static RedArgs red_args(const asd_t *h)
{
    const Layout &L = h->L;
    char *w = h->ws;
    RedArgs a;
    std::memset(&a, 0, sizeof a);
    a.S = w + L.off_S[h->cur];
    a.prec = h->p.precision;
    a.ncs = L.ncs;
    a.sys = (const SysDev *)(w + L.off_sys);
    a.grain_sys = (const int32_t *)(w + L.off_gsys);
    a.grain_ptr = (const int64_t *)(w + L.off_gptr);
    a.grain_sites = (const int32_t *)(w + L.off_gsites);
    a.origin = (const int32_t *)(w + L.off_origin);
    a.grain_out = (double *)(w + L.off_gout);
    a.sys_out = (double *)(w + L.off_sout);
    a.moments = (double *)(w + L.off_mom);
    a.n_grains = L.n_grains;
    a.n_sys = (int)h->sys.size();
    return a;
}

int asd_reduce_magnetization(asd_t *h, double *per_grain, double *per_system)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    RedArgs a = red_args(h);
    if (launch_reduce_grains(a, h->stream) || launch_reduce_systems(a, 0, 0, h->stream))
        return fail(h, ASD_EHIP, "reduction launch failed");
    std::vector<double> g((size_t)4 * std::max(a.n_grains, 1)), s((size_t)4 * a.n_sys);
    HIP_OK(h, hipMemcpyAsync(g.data(), a.grain_out, (size_t)4 * a.n_grains * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipMemcpyAsync(s.data(), a.sys_out, s.size() * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    if (per_grain) std::memcpy(per_grain, g.data(), (size_t)4 * a.n_grains * sizeof(double));
    if (per_system) std::memcpy(per_system, s.data(), s.size() * sizeof(double));
    for (double v : s)
        if (!std::isfinite(v)) return fail(h, ASD_ENONFINITE, "non-finite magnetisation");
    return ASD_OK;
}

// ------------------------------------------------------ static scratch sums
// asd_reduce_magnetization_static keeps the per-grain and per-system sums in
// this file-scope device array instead of the handle's workspace.  Host code
// never passes the array's name to a kernel or copy: it takes the array's
// address on each device from hipGetSymbolAddress, once per device, with that
// device current, and uses only that address.
constexpr int64_t kScratchDoubles = int64_t(1) << 17;  // 1 MiB per device
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

static int scratch_on_device(asd_t *h, double **out)
{
    if (h->device < 0 || h->device >= kMaxDevices)
        return fail(h, ASD_EUNSUPPORTED, "device %d beyond the %d the static scratch serves",
                    h->device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[h->device]) {
        int cur = 0;
        HIP_OK(h, hipGetDevice(&cur));
        if (cur != h->device) HIP_OK(h, hipSetDevice(h->device));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != h->device) HIP_OK(h, hipSetDevice(cur));
        if (e != hipSuccess)
            return fail(h, ASD_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[h->device] = (double *)ptr;
    }
    *out = g_scratch_ptr[h->device];
    return ASD_OK;
}

int asd_reduce_magnetization_static(asd_t *h, double *per_grain, double *per_system)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    RedArgs a = red_args(h);
    const int64_t need = 4 * ((int64_t)a.n_grains + a.n_sys);
    if (need > kScratchDoubles)
        return fail(h, ASD_EINVAL,
                    "%d grains + %d systems need %lld scratch doubles; the static scratch holds "
                    "%lld (at most %lld grains and systems together)",
                    a.n_grains, a.n_sys, (long long)need, (long long)kScratchDoubles,
                    (long long)(kScratchDoubles / 4));
    if (!per_grain && !per_system) return ASD_OK;
    double *sc = nullptr;
    int rc = scratch_on_device(h, &sc);
    if (rc) return rc;
    // every slot the kernels read is written first in the same call: nothing
    // of an earlier call's contents is used
    a.grain_out = sc;
    a.sys_out = sc + 4 * (int64_t)a.n_grains;
    if (launch_reduce_grains(a, h->stream) || launch_reduce_systems(a, 0, 0, h->stream))
        return fail(h, ASD_EHIP, "reduction launch failed");
    if (per_grain && a.n_grains > 0)
        HIP_OK(h, hipMemcpyAsync(per_grain, a.grain_out, (size_t)4 * a.n_grains * sizeof(double),
                                 hipMemcpyDeviceToHost, h->stream));
    if (per_system)
        HIP_OK(h, hipMemcpyAsync(per_system, a.sys_out, (size_t)4 * a.n_sys * sizeof(double),
                                 hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    const double *chk = per_system ? per_system : per_grain;
    const int64_t n_chk = per_system ? 4 * (int64_t)a.n_sys : 4 * (int64_t)a.n_grains;
    for (int64_t k = 0; k < n_chk; ++k)
        if (!std::isfinite(chk[k])) return fail(h, ASD_ENONFINITE, "non-finite magnetisation");
    return ASD_OK;
}

int asd_accumulate_moments(asd_t *h, int32_t reset)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    RedArgs a = red_args(h);
    if (launch_reduce_grains(a, h->stream) || launch_reduce_systems(a, 1, reset ? 1 : 0, h->stream))
        return fail(h, ASD_EHIP, "reduction launch failed");
    return ASD_OK;
}

int asd_get_moment_stats(asd_t *h, double *per_system)
{
    if (!h || !per_system) return fail(h, ASD_EINVAL, "NULL argument");
    HIP_OK(h, hipMemcpyAsync(per_system, h->ws + h->L.off_mom, h->sys.size() * 5 * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    for (size_t k = 0; k < h->sys.size() * 5; ++k)
        if (!std::isfinite(per_system[k])) return fail(h, ASD_ENONFINITE, "non-finite moment");
    return ASD_OK;
}

int asd_reduce_energy(asd_t *h, double *per_system)
{
    if (!h || !per_system) return fail(h, ASD_EINVAL, "NULL argument");
    const Layout &L = h->L;
    char *w = h->ws;
    int rc;
    const int saved = h->kernel;
    h->kernel = ASD_KERNEL_PLAIN;  // energy uses the plain tile map
    if (h->p.precision == ASD_FP64) {
        EnergyArgs<double> e;
        std::memset(&e, 0, sizeof e);
        e.st = make_args<double>(h, h->cur, 0);
        e.partial = (double *)(w + L.off_epart);
        for (int s = 0; s < 4; ++s) e.J[s] = h->p.J[s];
        e.mu_s = h->p.mu_s;
        e.ku = h->p.k_u;
        e.ku_grain = (const double *)(w + L.off_ku);
        rc = launch_energy_f64(e, L.n_tiles, h->stream);
    } else {
        EnergyArgs<float> e;
        std::memset(&e, 0, sizeof e);
        e.st = make_args<float>(h, h->cur, 0);
        e.partial = (double *)(w + L.off_epart);
        for (int s = 0; s < 4; ++s) e.J[s] = h->p.J[s];
        e.mu_s = h->p.mu_s;
        e.ku = h->p.k_u;
        e.ku_grain = (const double *)(w + L.off_ku);
        rc = launch_energy_f32(e, L.n_tiles, h->stream);
    }
    h->kernel = saved;
    if (rc || launch_energy_finish((const double *)(w + L.off_epart), (const SysDev *)(w + L.off_sys),
                                   (int)h->sys.size(), (double *)(w + L.off_eout), h->stream))
        return fail(h, ASD_EHIP, "energy launch failed");
    HIP_OK(h, hipMemcpyAsync(per_system, w + L.off_eout, h->sys.size() * 4 * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    for (size_t k = 0; k < h->sys.size() * 4; ++k)
        if (!std::isfinite(per_system[k])) return fail(h, ASD_ENONFINITE, "non-finite energy");
    return ASD_OK;
}

int asd_grain_count(asd_t *h, int32_t s, int32_t *n)
{
    if (!h || !n || s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad argument");
    *n = h->sys[s].n_grains;
    return ASD_OK;
}

int asd_stored_sites(asd_t *h, int32_t s, int64_t *n)
{
    if (!h || !n || s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad argument");
    *n = h->sys[s].n_stored;
    return ASD_OK;
}

int asd_get_grain_labels(asd_t *h, int32_t s, int32_t *labels)
{
    if (!h || !labels || s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad argument");
    std::memcpy(labels, h->sys[s].labels.data(), h->sys[s].labels.size() * sizeof(int32_t));
    return ASD_OK;
}

int asd_neighbour_count(asd_t *h, int32_t s, int64_t *n_entries)
{
    if (!h || !n_entries || s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad argument");
    const HostSys &hs = h->sys[s];
    const int slots = n_neighbour_slots(&h->p);
    int64_t c = 0;
    for (int64_t i = 0; i < hs.n_stored; ++i)
        for (int k = 0; k < slots; ++k)
            if (slot_neighbour(&h->p, hs, i, k) >= 0) ++c;
    *n_entries = c;
    return ASD_OK;
}

int asd_get_neighbours(asd_t *h, int32_t s, int64_t *row_ptr, int32_t *col, int8_t *shell)
{
    if (!h || !row_ptr || !col || !shell || s < 0 || s >= (int)h->sys.size())
        return fail(h, ASD_EINVAL, "bad argument");
    const HostSys &hs = h->sys[s];
    const int slots = n_neighbour_slots(&h->p);
    int64_t c = 0;
    for (int64_t i = 0; i < hs.n_stored; ++i) {
        row_ptr[i] = c;
        for (int k = 0; k < slots; ++k) {
            int64_t j = slot_neighbour(&h->p, hs, i, k);
            if (j < 0) continue;
            col[c] = (int32_t)j;
            shell[c] = (int8_t)slot_shell(&h->p, k);
            ++c;
        }
    }
    row_ptr[hs.n_stored] = c;
    return ASD_OK;
}

int asd_host_grain_labels(const asd_params *p, const asd_system_desc *sys, int32_t *labels)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (!sys || !labels) return fail(nullptr, ASD_EINVAL, "NULL argument");
    if ((rc = check_system(p, sys, 0))) return rc;
    HostSys hs;
    rc = build_system(p, sys, 0, hs);
    if (rc && rc != ASD_EUNSUPPORTED) return rc;
    std::memcpy(labels, hs.labels.data(), hs.labels.size() * sizeof(int32_t));
    return rc;
}

int asd_host_neighbours(const asd_params *p, const asd_system_desc *sys, int64_t *n_entries,
                        int64_t *row_ptr, int32_t *col, int8_t *shell)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (!sys || !n_entries) return fail(nullptr, ASD_EINVAL, "NULL argument");
    if ((rc = check_system(p, sys, 0))) return rc;
    HostSys hs;
    hs.desc = *sys;
    hs.desc.seeds_xy = nullptr;
    hs.desc.labels = nullptr;
    hs.sx = sys->bc_x == ASD_BC_TRACK ? sys->track_nx : sys->nx;
    hs.n_stored = (p->lattice == ASD_SC ? 1 : 2) * (int64_t)hs.sx * sys->ny * sys->nz;
    const int slots = n_neighbour_slots(p);
    int64_t c = 0;
    for (int64_t i = 0; i < hs.n_stored; ++i) {
        if (row_ptr) row_ptr[i] = c;
        for (int k = 0; k < slots; ++k) {
            int64_t j = slot_neighbour(p, hs, i, k);
            if (j < 0) continue;
            if (col) col[c] = (int32_t)j;
            if (shell) shell[c] = (int8_t)slot_shell(p, k);
            ++c;
        }
    }
    if (row_ptr) row_ptr[hs.n_stored] = c;
    *n_entries = c;
    return ASD_OK;
}

// coarse cells over stored columns [x0, x0 + ncols) of system s
static int transfer_args(asd_t *h, int32_t s, int32_t x0, int32_t ncols, int32_t cx, int32_t cy,
                         int32_t cz, TransferArgs *a)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad system index");
    const SysDev &d = h->dev[s];
    if (x0 < 0 || ncols < 1 || (int64_t)x0 + ncols > d.sx)
        return fail(h, ASD_EINVAL, "columns [%d, %d) outside the %d stored columns", x0, x0 + ncols, d.sx);
    if (cx < 1 || cy < 1 || cz < 1) return fail(h, ASD_EINVAL, "coarse cells need cx, cy, cz >= 1");
    std::memset(a, 0, sizeof *a);
    a->prec = h->p.precision;
    a->S[0] = h->ws + h->L.off_S[h->cur];
    a->S[1] = h->ws + h->L.off_S[1 - h->cur];
    a->ncs = h->L.ncs;
    a->d = d;
    a->label = (const uint16_t *)(h->ws + h->L.off_label);
    a->x0 = x0;
    a->ncols = ncols;
    a->cx = cx;
    a->cy = cy;
    a->cz = cz;
    a->ncx = (ncols + cx - 1) / cx;
    a->ncy = (d.ny + cy - 1) / cy;
    const int64_t ncell = (int64_t)a->ncx * a->ncy * ((d.nz + cz - 1) / cz);
    if (ncell > INT32_MAX) return fail(h, ASD_EINVAL, "too many coarse cells");
    a->ncell = (int32_t)ncell;
    a->per = h->p.lattice == ASD_SC ? 1 : 2;
    return ASD_OK;
}

int asd_coarse_grain(asd_t *h, int32_t s, int32_t x0, int32_t ncols, int32_t cx, int32_t cy,
                     int32_t cz, double *out)
{
    TransferArgs a;
    int rc = transfer_args(h, s, x0, ncols, cx, cy, cz, &a);
    if (rc) return rc;
    if (!out) return fail(h, ASD_EINVAL, "NULL output");
    a.out = out;
    if (launch_coarse_grain(a, h->stream)) return fail(h, ASD_EHIP, "coarse-grain launch failed");
    return ASD_OK;
}

int asd_thermalise_columns(asd_t *h, int32_t s, int32_t x0, int32_t ncols, int32_t cx,
                           int32_t cy, int32_t cz, const double *mcell, uint32_t step)
{
    TransferArgs a;
    int rc = transfer_args(h, s, x0, ncols, cx, cy, cz, &a);
    if (rc) return rc;
    if (!mcell) return fail(h, ASD_EINVAL, "NULL cell magnetisation");
    a.mcell = mcell;
    a.k0 = (uint32_t)h->p.seed;
    a.k1 = (uint32_t)(h->p.seed >> 32);
    a.step = step;
    a.rounds = h->p.philox_rounds;
    a.cap = h->cone == ASD_CONE_CAP;
    if (launch_cone_columns(a, h->stream)) return fail(h, ASD_EHIP, "cone launch failed");
    h->stray_dirty = true;
    return ASD_OK;
}

int asd_set_demag_reading(asd_t *h, int32_t reading)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (reading != ASD_DEMAG_EACH_STAGE && reading != ASD_DEMAG_ONCE)
        return fail(h, ASD_EINVAL, "reading must be ASD_DEMAG_EACH_STAGE or ASD_DEMAG_ONCE");
    if (!h->dm.on) return fail(h, ASD_ESTATE, "the handle has no demagnetising field");
    h->dm.once = reading == ASD_DEMAG_ONCE ? 1 : 0;
    drop_graphs(h);
    // the fused kernels' tiles and partial-sum slots depend on the reading
    if (h->kernel == ASD_KERNEL_FUSED) return setup_fused_tiles(h, h->tile_cfg);
    return ASD_OK;
}

int asd_set_cone_reading(asd_t *h, int32_t reading)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (reading != ASD_CONE_PRINTED && reading != ASD_CONE_CAP)
        return fail(h, ASD_EINVAL, "cone reading must be ASD_CONE_PRINTED or ASD_CONE_CAP");
    h->cone = reading;
    return ASD_OK;
}

int asd_mc_sweep(asd_t *h, int64_t n)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (n < 0) return fail(h, ASD_EINVAL, "n must be >= 0");
    if (h->dm.on)
        return fail(h, ASD_EUNSUPPORTED, "Metropolis sweeps do not include the demagnetising field");
    for (const HostSys &hs : h->sys) {
        const asd_system_desc &d = hs.desc;
        if ((d.bc_x == ASD_BC_PERIODIC && d.nx % 2) || (d.bc_y == ASD_BC_PERIODIC && d.ny % 2) ||
            (d.bc_z == ASD_BC_PERIODIC && d.nz % 2))
            return fail(h, ASD_EUNSUPPORTED,
                        "the Monte Carlo colours need an even length along every periodic axis");
    }
    if (h->step + n >= ((int64_t)1 << 32))
        return fail(h, ASD_ESTATE, "step counter would exceed 2^32 (Philox counter word)");
    if (n == 0) return ASD_OK;
    // in place on the current buffer (a Heun step only reads the window of the
    // current buffer; the other one's window is overwritten)
    for (int64_t t = 0; t < n; ++t) {
        int rc;
        if (h->p.precision == ASD_FP64) {
            MCArgs<double> m;
            m.st = make_args<double>(h, h->cur, (int)t);
            m.st.tile_sys = (const int32_t *)(h->ws + h->L.off_tile);
            m.st.So = (double *)(h->ws + h->L.off_S[h->cur]);
            m.mu_s = h->p.mu_s;
            m.ku = h->p.k_u;
            m.ku_grain = (const double *)(h->ws + h->L.off_ku);
            rc = launch_mc_sweep_f64(m, h->L.n_tiles, h->stream);
        } else {
            MCArgs<float> m;
            m.st = make_args<float>(h, h->cur, (int)t);
            m.st.tile_sys = (const int32_t *)(h->ws + h->L.off_tile);
            m.st.So = (float *)(h->ws + h->L.off_S[h->cur]);
            m.mu_s = h->p.mu_s;
            m.ku = h->p.k_u;
            m.ku_grain = (const double *)(h->ws + h->L.off_ku);
            rc = launch_mc_sweep_f32(m, h->L.n_tiles, h->stream);
        }
        if (rc) return fail(h, ASD_EHIP, "Metropolis launch failed: %s", hipGetErrorString(hipGetLastError()));
    }
    if (launch_advance_step((int64_t *)(h->ws + h->L.off_step), n, h->stream))
        return fail(h, ASD_EHIP, "advance launch failed");
    h->step += n;
    return ASD_OK;
}

int asd_set_columns(asd_t *h, int32_t s, int32_t x0, int32_t ncols, int32_t cx, int32_t cy,
                    int32_t cz, const double *mcell)
{
    TransferArgs a;
    int rc = transfer_args(h, s, x0, ncols, cx, cy, cz, &a);
    if (rc) return rc;
    if (!mcell) return fail(h, ASD_EINVAL, "NULL cell direction");
    a.mcell = mcell;
    a.exact = 1;
    if (launch_cone_columns(a, h->stream)) return fail(h, ASD_EHIP, "column launch failed");
    h->stray_dirty = true;
    return ASD_OK;
}

namespace asd {

double atom_moment(const asd_t *h) { return h->p.mu_s; }

void lattice_cell(const asd_t *h, double *dt, double edge[3])
{
    *dt = h->p.dt;
    edge[0] = edge[1] = h->p.a;
    edge[2] = h->p.lattice == ASD_L10 ? h->p.c : h->p.a;
}

int coarse_grain_pair(asd_t *h, int32_t s, int32_t xa, int32_t xb, int32_t ncols, int32_t cx,
                      int32_t cy, int32_t cz, double *outa, double *outb)
{
    TransferArgs a, b;
    int rc = transfer_args(h, s, xa, ncols, cx, cy, cz, &a);
    if (rc || (rc = transfer_args(h, s, xb, ncols, cx, cy, cz, &b))) return rc;
    if (!outa || !outb) return fail(h, ASD_EINVAL, "NULL output");
    a.out = outa;
    b.out = outb;
    if (launch_coarse_grain_pair(a, b, h->stream)) return fail(h, ASD_EHIP, "coarse-grain launch failed");
    return ASD_OK;
}

int demag_mesh(const asd_t *h, int32_t cell[3], int32_t mesh[3])
{
    if (!h || !h->dm.on) return ASD_ESTATE;
    cell[0] = h->dm.cx;
    cell[1] = h->dm.cy;
    cell[2] = h->dm.cz;
    mesh[0] = h->dm.ncx;
    mesh[1] = h->dm.ncy;
    mesh[2] = h->dm.ncz;
    return ASD_OK;
}

int set_cell_field(asd_t *h, int32_t s, const double *src, int32_t src_nx, int32_t src_off)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad system index");
    if (!h->dm.on || !h->dmT.on || !h->dm.bstray)
        return fail(h, ASD_ESTATE, "a field per coarse cell needs a track system with demag_cell");
    const DemagDev &g = h->dm;
    if (!src || src_off < 0 || src_off + g.ncx > src_nx) return fail(h, ASD_EINVAL, "bad source mesh");
    char *dst = (char *)g.bstray + (size_t)s * 3 * g.ncell * h->elem;
    if (launch_cells_from_mesh(h->p.precision, dst, src, src_nx, src_off, g.ncx, g.ncy, g.ncz,
                               h->stream))
        return fail(h, ASD_EHIP, "cell field launch failed");
    h->external_field = true;
    return ASD_OK;
}

int clear_cell_field(asd_t *h)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (h->external_field) {
        h->external_field = false;
        h->stray_dirty = true;
    }
    return ASD_OK;
}

int32_t track_columns(const asd_t *h, int32_t s)
{
    if (!h || s < 0 || s >= (int)h->sys.size() || !h->dev[s].track) return 0;
    return h->dev[s].sx;
}

int set_columns_pair(asd_t *h, int32_t s, int32_t xa, int32_t xb, int32_t ncols, int32_t cx,
                     int32_t cy, int32_t cz, const double *ma, const double *mb)
{
    TransferArgs a, b;
    int rc = transfer_args(h, s, xa, ncols, cx, cy, cz, &a);
    if (rc || (rc = transfer_args(h, s, xb, ncols, cx, cy, cz, &b))) return rc;
    if (!ma || !mb) return fail(h, ASD_EINVAL, "NULL cell direction");
    a.mcell = ma;
    b.mcell = mb;
    a.exact = b.exact = 1;
    if (launch_cone_columns_pair(a, b, h->stream)) return fail(h, ASD_EHIP, "column launch failed");
    h->stray_dirty = true;
    return ASD_OK;
}

}  // namespace asd

int asd_window_size(asd_t *h, int32_t s, int32_t *nx, int32_t *ny, int32_t *nz)
{
    if (!h || !nx || !ny || !nz) return fail(h, ASD_EINVAL, "NULL argument");
    if (s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad system index");
    *nx = h->sys[s].desc.nx;
    *ny = h->sys[s].desc.ny;
    *nz = h->sys[s].desc.nz;
    return ASD_OK;
}

int asd_get_stream(asd_t *h, void **stream)
{
    if (!h || !stream) return fail(h, ASD_EINVAL, "NULL argument");
    *stream = (void *)h->stream;
    return ASD_OK;
}

int asd_demag_field(asd_t *h, double *per_cell, int32_t *mesh)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (!h->dm.on) return fail(h, ASD_ESTATE, "the handle has no demagnetising field");
    if (!per_cell) return fail(h, ASD_EINVAL, "per_cell is NULL");
    const DemagDev &g = h->dm;
    const char *w = h->ws;
    const size_t n = (size_t)g.n_sys * 3 * g.ncell;
    int rc = refresh_stray(h);
    if (rc) return rc;
    if (h->elem == 8)
        rc = launch_demag(g, (const double *)(w + h->L.off_S[h->cur]), h->L.ncs,
                          (const SysDev *)(w + h->L.off_sys), (const int32_t *)(w + h->L.off_origin),
                          0, h->stream);
    else
        rc = launch_demag(g, (const float *)(w + h->L.off_S[h->cur]), h->L.ncs,
                          (const SysDev *)(w + h->L.off_sys), (const int32_t *)(w + h->L.off_origin),
                          0, h->stream);
    if (rc) return fail(h, ASD_EHIP, "demag launch failed: %s", hipGetErrorString(hipGetLastError()));
    std::vector<char> buf(n * h->elem);
    HIP_OK(h, hipMemcpyAsync(buf.data(), g.bd[0], buf.size(), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    for (size_t i = 0; i < n; ++i)
        per_cell[i] = h->elem == 8 ? ((const double *)buf.data())[i] : (double)((const float *)buf.data())[i];
    if (mesh) {
        mesh[0] = g.ncx;
        mesh[1] = g.ncy;
        mesh[2] = g.ncz;
    }
    return ASD_OK;
}

int asd_get_state(asd_t *h, int32_t s, int64_t *step, int32_t *origin)
{
    if (!h || s < 0 || s >= (int)h->sys.size()) return fail(h, ASD_EINVAL, "bad argument");
    if (step) *step = h->step;
    if (origin) *origin = h->origin[s];
    return ASD_OK;
}

int asd_set_step(asd_t *h, int64_t step)
{
    if (!h || step < 0 || step >= ((int64_t)1 << 32)) return fail(h, ASD_EINVAL, "bad step");
    HIP_OK(h, hipMemcpyAsync(h->ws + h->L.off_step, &step, sizeof step, hipMemcpyHostToDevice,
                             h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    h->step = step;
    return ASD_OK;
}

int asd_philox(uint64_t seed, int32_t rounds, const uint32_t *ctr, uint32_t *out, int64_t n,
               void *stream)
{
    if (n < 0 || (n > 0 && (!ctr || !out))) return fail(nullptr, ASD_EINVAL, "bad arguments");
    if (rounds < 1 || rounds > 10) return fail(nullptr, ASD_EINVAL, "rounds must be 1..10");
    if (launch_philox_export(seed, rounds, ctr, out, n, stream))
        return fail(nullptr, ASD_EHIP, "philox launch failed");
    return ASD_OK;
}

// reason the fused kernel cannot serve this handle, or NULL
static const char *fused_unsupported(const asd_t *h)
{
    if (h->dm.on) {
        // the step runs as the predictor and corrector stages of the SC kernel
        if (h->p.lattice != ASD_SC)
            return "the demagnetising field needs the convolution between the two Heun stages; "
                   "the fused L1_0 kernel runs both stages in one launch";
        for (const HostSys &hs : h->sys)
            if (hs.desc.bc_z != ASD_BC_OPEN)
                return "the fused stage kernels for the demagnetising field march open z only";
    }
    const int64_t elem = h->p.precision == ASD_FP64 ? 8 : 4;
    for (const HostSys &hs : h->sys) {
        if (hs.desc.bc_z != ASD_BC_OPEN && hs.desc.bc_z != ASD_BC_PERIODIC)
            return "the fused kernels march z with open or periodic ends";
        if (hs.n_stored * elem > 0x7FFFFFFF)
            return "the fused kernel addresses a system with 32-bit byte offsets (2 GiB per component)";
    }
    bool per_grain = false;
    for (const HostSys &hs : h->sys)
        if (!hs.ku_grain.empty()) per_grain = true;
    if (per_grain)
        for (const SysDev &d : h->dev)
            if (!d.columnar) return "per-grain anisotropy in the fused kernel needs grains that span whole z columns";
    return nullptr;
}

// reason the cell-row kernels (two-pass variant 2) cannot serve this handle, or NULL
static const char *cell_rows_unsupported(const asd_t *h)
{
    if (!h->dm.on) return "the cell-row kernels serve handles with the demagnetising field";
    if (h->dm.cr_cells < 1) return "the cell-row kernels need coarse cells of at most 64 lattice cells along x";
    return nullptr;
}

// fill the fused tile map for variant v and upload it with the descriptors
static int setup_fused_tiles(asd_t *h, int v)
{
    std::vector<int32_t> map;
    for (size_t s = 0; s < h->sys.size(); ++s) {
        int fx, fy, fz, lz;
        fused_tiles_of(&h->p, &h->sys[s].desc, v, &fx, &fy, &fz, &lz, h->dm.on && !h->dm.once);
        SysDev &d = h->dev[s];
        d.ftile_base = (int32_t)map.size();
        d.ftiles_x = fx;
        d.ftiles_y = fy;
        d.ftiles_z = fz;
        d.fz_len = lz;
        d.fd_ftx = host_fastdiv((uint32_t)fx);
        d.fd_fty = host_fastdiv((uint32_t)fy);
        for (int t = 0; t < fx * fy * fz; ++t) map.push_back((int32_t)s);
    }
    h->n_ftiles = (int)map.size();
    HIP_OK(h, hipMemcpyAsync(h->ws + h->L.off_ftile, map.data(), map.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, h->stream));
    if (h->dm.on) {
        // partial-sum slots of the stage kernels; slots no tile writes stay zero
        int nsx, nsy, ns;
        stage_slots(&h->p, &h->sys[0].desc, h->p.demag_cell, v, &nsx, &nsy, &ns, !h->dm.once);
        h->dm.nsx = nsx;
        h->dm.nsy = nsy;
        h->dm.ns = ns;
        for (int b = 0; b < 2; ++b)
            HIP_OK(h, hipMemsetAsync(h->ws + h->L.off_dcs[b], 0, h->L.dcs_bytes, h->stream));
    }
    return upload_sysdev(h);
}

int asd_set_variant(asd_t *h, int32_t kernel, int32_t tile)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (kernel != ASD_KERNEL_PLAIN && kernel != ASD_KERNEL_FUSED)
        return fail(h, ASD_EINVAL, "kernel must be PLAIN or FUSED");
    const int nvar = kernel == ASD_KERNEL_PLAIN
                         ? kPlainVariants
                         : fused_count(h->p.lattice == ASD_L10, h->p.precision == ASD_FP64);
    if (tile < 0 || tile >= nvar) return fail(h, ASD_EINVAL, "variant out of range");
    if (kernel == ASD_KERNEL_PLAIN && tile == kCellRowVariant) {
        const char *why = cell_rows_unsupported(h);
        if (why) return fail(h, ASD_EUNSUPPORTED, "%s", why);
    }
    if (kernel == ASD_KERNEL_FUSED) {
        const char *why = fused_unsupported(h);
        if (why) return fail(h, ASD_EUNSUPPORTED, "%s", why);
        int rc = setup_fused_tiles(h, tile);
        if (rc) return rc;
    } else if (h->dm.on) {
        h->dm.ns = h->dm.nsx = h->dm.nsy = 1;  // the cell-row kernels write whole sums
    }
    h->kernel = kernel;
    h->tile_cfg = tile;
    drop_graphs(h);
    return ASD_OK;
}

int asd_variant_count(asd_t *h, int32_t kernel, int32_t *count)
{
    if (!h || !count) return fail(h, ASD_EINVAL, "NULL argument");
    if (kernel == ASD_KERNEL_PLAIN)
        *count = kPlainVariants;
    else if (kernel == ASD_KERNEL_FUSED)
        *count = fused_count(h->p.lattice == ASD_L10, h->p.precision == ASD_FP64);
    else
        return fail(h, ASD_EINVAL, "kernel must be PLAIN or FUSED");
    return ASD_OK;
}

int asd_get_variant(asd_t *h, int32_t *kernel, int32_t *tile)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    if (kernel) *kernel = h->kernel;
    if (tile) *tile = h->tile_cfg;
    return ASD_OK;
}

int asd_variant_name(asd_t *h, char *buf, size_t len)
{
    if (!h || !buf || len == 0) return fail(h, ASD_EINVAL, "bad argument");
    const bool fp64 = h->p.precision == ASD_FP64;
    const char *T = fp64 ? "double" : "float";
    char tmp[256];
    if (h->kernel == ASD_KERNEL_FUSED) {
        const bool l10 = h->p.lattice == ASD_L10;
        const FusedVariant f = fused_pick(l10, fp64, h->tile_cfg);
        bool zper = false;
        for (const HostSys &hs : h->sys)
            if (hs.desc.bc_z == ASD_BC_PERIODIC) zper = true;
        if (l10)
            snprintf(tmp, sizeof tmp, "k_fused_l10<%s, %d, %d, %d>", T, f.txe, f.waves, f.rows);
        else if (h->dm.on && h->dm.once)  // one launch, the field of S held (open z only)
            snprintf(tmp, sizeof tmp, "k_fused_sc<%s, %d, %d, %d, false, 3>", T, f.txe, f.waves,
                     f.rows);
        else if (h->dm.on)  // the predictor and corrector stages (open z only)
            snprintf(tmp, sizeof tmp, "k_fused_sc<%s, %d, %d, %d, false, 1>+k_fused_sc<%s, %d, %d, %d, false, 2>",
                     T, f.txe, f.waves, f.rows, T, f.txe, f.waves, f.rows);
        else
            snprintf(tmp, sizeof tmp, "k_fused_sc<%s, %d, %d, %d, %s, 0>", T, f.txe, f.waves, f.rows,
                     zper ? "true" : "false");
    } else if (h->tile_cfg == 1) {
        snprintf(tmp, sizeof tmp, "k_plain_predictor<%s, true>+k_stash_corrector<%s>", T, T);
    } else if (h->tile_cfg == kCellRowVariant) {
        snprintf(tmp, sizeof tmp, "k_cell_step<%s, false>+k_cell_step<%s, true>", T, T);
    } else {
        snprintf(tmp, sizeof tmp, "k_plain_predictor<%s, false>+k_plain_corrector<%s>", T, T);
    }
    if (strlen(tmp) + 1 > len) return fail(h, ASD_EINVAL, "buffer too small");
    memcpy(buf, tmp, strlen(tmp) + 1);
    return ASD_OK;
}

// ------------------------------------------------------------------ autotuning
static std::string tune_key(const asd_t *h)
{
    char buf[256];
    int64_t sites = 0;
    for (const HostSys &hs : h->sys) sites += hs.n_window;
    const asd_system_desc &d = h->sys[0].desc;
    // the variant table is part of the key: an entry names a variant by index
    const bool l10 = h->p.lattice == ASD_L10, fp64 = h->p.precision == ASD_FP64;
    uint32_t tab = 2166136261u;  // FNV-1a over (txe, waves, rows, lz) of every variant
    for (int v = 0; v < fused_count(l10, fp64); ++v) {
        const FusedVariant f = fused_pick(l10, fp64, v);
        for (int x : {f.txe, f.waves, f.rows, f.lz}) tab = (tab ^ (uint32_t)x) * 16777619u;
    }
    int len = snprintf(buf, sizeof buf, "lat%d_prec%d_%dx%dx%d_n%zu_w%lld_t%08x", h->p.lattice,
                       h->p.precision, d.nx, d.ny, d.nz, h->sys.size(), (long long)sites, tab);
    // the demagnetising field changes the candidates and their cost
    if (h->dm.on && len > 0 && len < (int)sizeof buf)
        snprintf(buf + len, sizeof buf - len, "_dm%dx%dx%d%s", h->dm.cx, h->dm.cy, h->dm.cz,
                 h->dm.once ? "_once" : "");
    return buf;
}

static bool tune_cache_lookup(const char *path, const std::string &key, int *kernel, int *tile)
{
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    fclose(f);
    const std::string pat = "\"" + key + "\": {\"kernel\": ";
    size_t p = text.find(pat);
    if (p == std::string::npos) return false;
    return sscanf(text.c_str() + p + pat.size(), "%d, \"tile\": %d", kernel, tile) == 2;
}

static void tune_cache_store(const char *path, const std::string &key, int kernel, int tile,
                             double ms)
{
    if (!path) return;
    std::string text;
    if (FILE *f = fopen(path, "r")) {
        char buf[4096];
        size_t n;
        while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
        fclose(f);
    }
    // one entry per line between braces: {"key": {...},\n ...}
    std::vector<std::string> lines;
    size_t a = 0;
    while (a < text.size()) {
        size_t b = text.find('\n', a);
        if (b == std::string::npos) b = text.size();
        std::string ln = text.substr(a, b - a);
        if (ln.find("\"kernel\"") != std::string::npos && ln.find("\"" + key + "\"") == std::string::npos) {
            while (!ln.empty() && (ln.back() == ',' || ln.back() == ' ')) ln.pop_back();
            size_t q = ln.find('"');
            lines.push_back(ln.substr(q));
        }
        a = b + 1;
    }
    char e[512];
    snprintf(e, sizeof e, "\"%s\": {\"kernel\": %d, \"tile\": %d, \"ms_per_step\": %.6f}", key.c_str(),
             kernel, tile, ms);
    lines.push_back(e);
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fputs("{\n", f);
    for (size_t i = 0; i < lines.size(); ++i) fprintf(f, "  %s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
    fputs("}\n", f);
    fclose(f);
    rename(tmp.c_str(), path);
}

// time `steps` eager steps of the current variant (ms per step)
static int time_variant(asd_t *h, int steps, double *ms)
{
    hipEvent_t e0, e1;
    HIP_OK(h, hipEventCreate(&e0));
    HIP_OK(h, hipEventCreate(&e1));
    int rc = asd_step(h, 2);  // warm-up
    if (!rc) {
        (void)hipEventRecord(e0, h->stream);
        rc = asd_step(h, steps);
        (void)hipEventRecord(e1, h->stream);
    }
    float t = 0.f;
    if (!rc) {
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&t, e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / steps;
    return rc;
}

int asd_autotune(asd_t *h, const char *cache_path)
{
    if (!h) return fail(nullptr, ASD_EINVAL, "NULL handle");
    const std::string key = tune_key(h);
    int kern = 0, tile = 0;
    if (tune_cache_lookup(cache_path, key, &kern, &tile) &&
        (kern == ASD_KERNEL_PLAIN || kern == ASD_KERNEL_FUSED))
        return asd_set_variant(h, kern, tile);
    // save spins and counters; every trial runs from the same state
    const size_t nb = (size_t)3 * h->L.ncs * h->elem;
    std::vector<char> saved(nb);
    HIP_OK(h, hipMemcpyAsync(saved.data(), h->ws + h->L.off_S[h->cur], nb, hipMemcpyDeviceToHost,
                             h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    const int64_t step0 = h->step;
    const int cur0 = h->cur;
    const int gsteps = h->graph_steps;
    h->graph_steps = 0;
    struct Cand {
        int kernel, tile;
    };
    std::vector<Cand> cands;
    for (int v = 0; v < kPlainVariants; ++v)
        if (v != kCellRowVariant || !cell_rows_unsupported(h)) cands.push_back({ASD_KERNEL_PLAIN, v});
    if (!fused_unsupported(h))
        for (int v = 0; v < fused_count(h->p.lattice == ASD_L10, h->p.precision == ASD_FP64); ++v)
            cands.push_back({ASD_KERNEL_FUSED, v});
    // pass 1: every candidate for 20 steps; pass 2: the three fastest, three
    // interleaved rounds of 60 steps each, ranked by their median
    double best = 1e30;
    Cand pick = cands[0];
    int rc = ASD_OK;
    std::vector<std::pair<double, size_t>> first;
    for (size_t i = 0; i < cands.size() && !rc; ++i) {
        double ms = 0;
        if ((rc = asd_set_variant(h, cands[i].kernel, cands[i].tile))) break;
        if ((rc = time_variant(h, 20, &ms))) break;
        first.push_back({ms, i});
    }
    std::sort(first.begin(), first.end());
    const size_t nf = std::min<size_t>(3, first.size());
    std::vector<std::vector<double>> rounds(nf);
    for (int rd = 0; rd < 3 && !rc; ++rd)
        for (size_t j = 0; j < nf && !rc; ++j) {
            double ms = 0;
            const Cand &c = cands[first[j].second];
            if ((rc = asd_set_variant(h, c.kernel, c.tile))) break;
            if ((rc = time_variant(h, 60, &ms))) break;
            rounds[j].push_back(ms);
        }
    for (size_t j = 0; j < nf && !rc; ++j) {
        std::vector<double> v = rounds[j];
        std::sort(v.begin(), v.end());
        const double med = v[v.size() / 2];
        if (med < best) {
            best = med;
            pick = cands[first[j].second];
        }
    }
    h->graph_steps = gsteps;
    // restore the state into both ping-pong buffers and the step counter
    h->cur = cur0;
    for (int b = 0; b < 2; ++b)
        HIP_OK(h, hipMemcpyAsync(h->ws + h->L.off_S[b], saved.data(), nb, hipMemcpyHostToDevice,
                                 h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    int r2 = asd_set_step(h, step0);
    if (rc) return rc;
    if (r2) return r2;
    if ((rc = asd_set_variant(h, pick.kernel, pick.tile))) return rc;
    tune_cache_store(cache_path, key, pick.kernel, pick.tile, best);
    return ASD_OK;
}
