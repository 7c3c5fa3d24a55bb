// asd_internal.h -- layout shared by the host code and the kernels of libasd.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace asd {

struct FastDivH {            // mirror of the device FastDiv (d, multiplier, shift)
    uint32_t d, m, l;
};

constexpr int kPlainTile = 256;      // window sites per block in the two-pass kernels
constexpr uint16_t kNoGrain = 0xFFFF; // label of a non-magnetic site
constexpr int kL10Degree = 18;        // ELL slots of the 4-shell L1_0 table

// Per-system descriptor, resident in device memory.
struct SysDev {
    int32_t kind;             // ASD_SC / ASD_L10
    int32_t nx, ny, nz;       // window cells
    int32_t sx;               // stored x cells (track_nx or nx)
    int32_t bcx, bcy, bcz;    // ASD_BC_*
    int32_t track;            // 1 when x is a track
    int32_t grain_base;       // first global grain index
    int32_t n_grains;
    int32_t tile_base;        // first tile of this system (plain kernels)
    int32_t n_tiles;
    int32_t ftile_base;       // first tile of this system (fused kernel)
    int32_t ftiles_x, ftiles_y, ftiles_z;
    int32_t fz_len;           // z planes per fused tile
    int32_t columnar;         // 1 when every stored column lies in one grain
    uint32_t sys_id;          // Philox counter word 2
    FastDivH fd_nx, fd_ny;    // division by nx, ny (window)
    FastDivH fd_ftx, fd_fty;  // division by ftiles_x, ftiles_y
    int64_t base;             // first stored site in the global arrays
    int64_t n_stored;
    int64_t n_window;         // sites in the window
    double T_amb;             // ambient temperature of this system (K)
};

// Per-step constants (kernel argument, by value).
struct StepConsts {
    double cex[4];            // J_s / mu_s per shell
    double can;               // 2 k_u / mu_s (uniform)
    double gp;                // -gamma / (1 + alpha^2)
    double alpha, dt, h;      // h = dt / 2
    double cth;               // 2 alpha kB / (gamma mu_s dt)
    double B[3];              // write field (T), before polarity
    double T_peak, inv2s2, x0, y0, v;
    double hx;                // x, y site unit (m): a (SC) or a/2 (L1_0)
    int64_t spb;              // steps per bit
    int32_t n_bits, spot_mode, n_shells, rounds;
    uint32_t k0, k1;          // Philox key
    int32_t has_can_grain;
    int32_t pad;
};

// Demagnetising field (Eq. 7) of every system's window on a coarse mesh of
// cx x cy x cz lattice cells (Eq. 6), by zero-padded FFT convolution.  All
// systems share the window size, so they share the mesh and the tensor.
struct DemagDev {
    int32_t on;               // 0: no demagnetising field
    int32_t cx, cy, cz;       // lattice cells per coarse cell
    int32_t ncx, ncy, ncz;    // coarse cells per axis (last ones ragged)
    int32_t ncell;            // ncx * ncy * ncz
    int32_t lx, ly, lz;       // log2 of the padded sizes Px, Py, Pz
    int32_t xb_y, xb_z;       // x lines per workgroup in the y and z passes
    int32_t yzf;              // 1: the y and z passes as one workgroup per (kx,
                              // system) with direct sums along z (ncz <= 16), K
                              // the tensor transformed along x and y only
                              // (demag_mixed)
    int32_t n_sys;
    FastDivH fd_cx, fd_cy, fd_cz;
    // stray field of a frozen track: the same pipeline on a mesh that
    // extends the window's cells along x over the whole stored track
    // (window cell i is cell i + ceil(origin / cx) of this mesh); its
    // sources are the stored sites outside the window and its output is
    // kept at the window cells only
    int32_t stray;            // 1 for the track mesh
    int32_t ncx_win;          // track mesh: window cells along x
    int32_t ncell_win;        // track mesh: cells of the window mesh
    void *bstray;             // window mesh: added to the result when not null;
                              // track mesh: the output [S][3][ncell_win]
    void *wx;                 // complex [S][3][ncz][ncy][Px/2+1] (Hermitian half in x)
    void *wy;                 // complex [S][3][ncz][Py][Px/2+1]
    void *bd[2];              // field (T) per coarse cell, [S][3][ncell], one per Heun stage
    // cell-row step kernels (two-pass variant 2): the spin sums of every
    // coarse cell (T, [S][3][ncell]) as the kernels write the spins, [0] of
    // S' (predictor), [1] of the next spins (corrector); a workgroup takes
    // cr_cells cells along x of one layer (j, k), cr_segs workgroups per layer
    // The fused stage kernels write partial sums per tile instead: slot
    // (sz nsy + sy) nsx + sx of [S][3][ns][ncell] holds the part of a cell in
    // the tile that is (sx, sy, sz) tiles past the first tile the cell meets
    // (ns = nsx nsy nsz); the field pass adds the ns slots in order.  The
    // cell-row kernels use one slot.
    void *cs[2];
    int32_t cr_cells, cr_segs;
    int32_t ns, nsx, nsy;
    int32_t once;             // 1: the field of S only, held through both stages
    const void *K;            // tensor spectrum, octant [6][Py/2+1][Px/2+1][Pz/2+1]
                              // (yzf: [Px/2+1][6][ncz][Py/2+1], see demag_mixed)
    const void *tw[3];        // twiddles exp(-2 pi i t / P), t < P / 2, per axis
};

template <typename T>
struct StepArgs {
    const T *S;               // current spins [3][ncs]
    T *Sp;                    // predicted spins (two-pass) [3][ncs]
    T *So;                    // next spins [3][ncs]
    T *F0;                    // stash: f at the start of the step [3][ncs]
    T *Bt;                    // stash: thermal field [3][ncs]
    int64_t ncs;              // component stride
    const SysDev *sys;
    const int32_t *tile_sys;  // block -> system
    const int32_t *ell;       // L1_0 neighbours [kL10Degree][ncs] (absent: zero_site)
    const uint16_t *label;    // local grain label per stored site
    const double *can_grain;  // 2 k_u,g / mu_s per global grain
    const float *can_grain32; // the same rounded to FP32 (FP32 kernels)
    const int64_t *step_base; // device step counter
    const int32_t *origin;    // window origin per system
    const uint8_t *bits;      // polarity bits
    int64_t zero_site;        // an always-zero slot
    int32_t step_off;         // step = *step_base + step_off
    int32_t tile_cfg;         // tile variant
    int32_t n_blocks;         // blocks of the launch (XCD-contiguous tile order)
    int32_t lattice;          // ASD_SC / ASD_L10
    int32_t any_zper;         // some system is periodic along z
    StepConsts c;
    DemagDev dm;
};

// the same pipeline in FP64 from given cell sums cells [n_sys][3][ncell]
// (spin-sum units) into dm.bd[0]
int launch_demag_cells(const DemagDev &dm, const double *cells, void *stream);
// the same in the handle's precision from cell sums in that precision into
// dm.bd[stage]
int launch_demag_sums_f64(const DemagDev &dm, const double *sums, int stage, void *stream);
int launch_demag_sums_f32(const DemagDev &dm, const float *sums, int stage, void *stream);
inline int launch_demag_sums(const DemagDev &dm, const double *sums, int stage, void *stream)
{
    return launch_demag_sums_f64(dm, sums, stage, stream);
}
inline int launch_demag_sums(const DemagDev &dm, const float *sums, int stage, void *stream)
{
    return launch_demag_sums_f32(dm, sums, stage, stream);
}
// demagnetising field of spins S (both [3][ncs]) into dm.bd[stage]
int launch_demag_f64(const DemagDev &dm, const double *S, int64_t ncs, const SysDev *sys,
                     const int32_t *origin, int stage, void *stream);
int launch_demag_f32(const DemagDev &dm, const float *S, int64_t ncs, const SysDev *sys,
                     const int32_t *origin, int stage, void *stream);
inline int launch_demag(const DemagDev &dm, const double *S, int64_t ncs, const SysDev *sys,
                        const int32_t *origin, int stage, void *stream)
{
    return launch_demag_f64(dm, S, ncs, sys, origin, stage, stream);
}
inline int launch_demag(const DemagDev &dm, const float *S, int64_t ncs, const SysDev *sys,
                        const int32_t *origin, int stage, void *stream)
{
    return launch_demag_f32(dm, S, ncs, sys, origin, stage, stream);
}
// host set-up (asd_demag_tensor.cpp): tensor spectrum octant, times scale
void demag_spectrum(int ncx, int ncy, int ncz, double dx, double dy, double dz, int lx, int ly,
                    int lz, double scale, std::vector<double> &octant);
// the tensor transformed along x and y only, at plane offsets 0 .. ncz-1
void demag_mixed(int ncx, int ncy, int ncz, double dx, double dy, double dz, int lx, int ly,
                 double scale, std::vector<double> &table);
// dynamic LDS bytes of the one-workgroup y-z pass (0: ncz above 16); the
// pass runs where this fits the device
size_t demag_yz_lds_bytes(const DemagDev &dm, int elem);

// launchers (asd_step_f64.hip / asd_step_f32.hip)
int launch_plain_step_f64(const StepArgs<double> &a, int n_blocks, void *stream);
int launch_plain_step_f32(const StepArgs<float> &a, int n_blocks, void *stream);
int launch_fused_step_f64(const StepArgs<double> &a, int n_blocks, void *stream);
int launch_fused_step_f32(const StepArgs<float> &a, int n_blocks, void *stream);

// misc kernels (asd_misc.hip)
int launch_philox_export(uint64_t seed, int rounds, const uint32_t *ctr, uint32_t *out, int64_t n,
                         void *stream);
int launch_advance_step(int64_t *step_base, int64_t n, void *stream);
int launch_set_i32(int32_t *dst, const int32_t *vals, int n, void *stream);
// dst [3][ncx ncy ncz] (handle precision) from cells [off, off + ncx) of a
// mesh of src_nx cells along x, src [3][src_nx ncy ncz] (FP64)
int launch_cells_from_mesh(int prec, void *dst, const double *src, int src_nx, int src_off, int ncx,
                           int ncy, int ncz, void *stream);
// copy stored columns [x0, x0 + ncols) of system d from src to dst (both [3][ncs])
int launch_copy_columns(int prec, void *dst, const void *src, int64_t ncs, const SysDev &d, int x0,
                        int ncols, void *stream);
// zero the spins of non-magnetic sites of system d in buf ([3][ncs])
int launch_mask_spins(int prec, void *buf, int64_t ncs, const uint16_t *label, const SysDev &d,
                      void *stream);
struct RedArgs {
    const void *S;            // spins [3][ncs]
    int prec;                 // 0 FP64, 1 FP32
    int64_t ncs;
    const SysDev *sys;
    const int32_t *grain_sys;   // global grain -> system
    const int64_t *grain_ptr;   // global grain -> [begin, end) in grain_sites
    const int32_t *grain_sites; // local stored site indices, grain-major
    const int32_t *origin;
    double *grain_out;          // [G][4]
    double *sys_out;            // [S][4]
    double *moments;            // [S][5]
    int n_grains, n_sys;
};
int launch_reduce_grains(const RedArgs &a, void *stream);
int launch_reduce_systems(const RedArgs &a, int accumulate_moments, int reset, void *stream);
template <typename T>
struct EnergyArgs {
    StepArgs<T> st;           // spins, tables, constants (S = current)
    double *partial;          // [n_tiles][3]: exchange, anisotropy, Zeeman
    double J[4];              // exchange per shell (J)
    double mu_s, ku;          // J/T, J
    const double *ku_grain;   // per global grain (J) when has_can_grain
};
// window-end transfer to and from a coarse grid (Eq. 6): cells of cx x cy
// x cz lattice cells over stored columns [x0, x0 + ncols) of system d
struct TransferArgs {
    int prec;                 // ASD_FP64 / ASD_FP32
    void *S[2];               // both spin buffers [3][ncs] (coarse-grain reads S[0])
    int64_t ncs;
    SysDev d;
    const uint16_t *label;    // global label array
    int32_t x0, ncols, cx, cy, cz, ncx, ncy, ncell;
    int32_t per;              // sites per lattice cell (1 SC, 2 L1_0)
    double *out;              // coarse-grain: [ncell][4]
    const double *mcell;      // cone: [ncell][3]
    uint32_t k0, k1, step;    // cone: Philox key and counter word 1
    int32_t rounds;
    int32_t exact;            // 1: each magnetic site takes its cell's direction, no cone
    int32_t cap;              // cone reading: 0 the printed theta_max, 1 the cap of mean m
};
int launch_coarse_grain(const TransferArgs &a, void *stream);
int launch_cone_columns(const TransferArgs &a, void *stream);
// sum the energy partials of each system's tiles in order -> [S][4]
int launch_energy_finish(const double *partial, const SysDev *sys, int n_sys, double *sys_out,
                         void *stream);
int launch_energy_f64(const EnergyArgs<double> &a, int n_tiles, void *stream);
int launch_energy_f32(const EnergyArgs<float> &a, int n_tiles, void *stream);
// Metropolis sweeps in place on st.S (checkerboard colour 0, then 1); the
// sweep index is the step counter + st.step_off
template <typename T>
struct MCArgs {
    StepArgs<T> st;           // S = So = the current buffer
    double mu_s, ku;          // J/T, J (uniform anisotropy)
    const double *ku_grain;   // per global grain (J) when st.c.has_can_grain
};
int launch_mc_sweep_f64(const MCArgs<double> &a, int n_tiles, void *stream);
int launch_mc_sweep_f32(const MCArgs<float> &a, int n_tiles, void *stream);

}  // namespace asd
