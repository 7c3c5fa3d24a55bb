/*
 * asd_oracle.h -- declarations of the FP64 CPU oracle (test infrastructure
 * only; see asd_oracle.c).  Nothing in the GPU library includes this file.
 */
#ifndef ASD_ORACLE_H
#define ASD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_SC 0
#define ORC_L10 1

#define ORC_SPOT_NONE 0   /* uniform T_amb */
#define ORC_SPOT_MOVING 1 /* centre x0 + v n dt (absolute frame) */
#define ORC_SPOT_LOCKED 2 /* centre origin*hx + x0 (moves with the window) */

/* Boltzmann constant, J/K (exact SI value) */
#define ORC_KB 1.380649e-23

typedef struct orc_system {
    /* lattice and neighbour shells (CSR) */
    int64_t n_sites;
    const int64_t *row_ptr; /* [n_sites + 1] */
    const int32_t *col;     /* neighbour site */
    const int8_t *shell;    /* shell of each neighbour entry */
    const int32_t *label;   /* grain label per site, -1 = non-magnetic */
    const uint8_t *active;  /* 1 = evolves this step, 0 = frozen; NULL = all */
    const double *px, *py;  /* in-plane positions (m) */
    const uint32_t *ctr0;   /* Philox counter word 0 per site (absolute index) */
    uint32_t sys_id;        /* Philox counter word 2 */
    double hx;              /* x unit of the window origin (m) */
    int64_t origin;         /* window origin in x units (locked spot) */
    /* material */
    int n_shells;
    double J[4];            /* exchange per shell (J) */
    double mu_s, alpha, gamma, dt;
    double ku;              /* uniaxial anisotropy (J/atom) */
    const double *ku_grain; /* per-grain k_u or NULL */
    /* drive */
    double B[3];            /* write field (T) */
    int n_bits;             /* polarity bits (0 = constant +1) */
    const uint8_t *bits;
    int64_t steps_per_bit;
    int spot_mode;
    double T_amb, T_peak, fwhm, x0, y0, v;
    /* noise */
    uint64_t seed;
    int rounds;
    /* demagnetising field of the evolving sites (Eq. 7 on the coarse cells
     * of Eq. 6), evaluated at both Heun stages from that stage's spins (or
     * once per step, demag_once); dcell[i] = coarse cell of site i or -1;
     * dn[0] = 0 switches it off */
    int dn[3];              /* coarse mesh, cells along x, y, z */
    double dd[3];           /* coarse cell edges (m) */
    const int32_t *dcell;
    const double *bstray;   /* [3][ncell] field (T) of sources outside the
                               evolving sites, added per coarse cell; or NULL */
    int demag_once;         /* 0: the field is evaluated at both Heun stages
                               from that stage's spins; 1: once per step, from
                               the step's starting spins, and held through
                               both stages */
} orc_system;

void orc_philox4x32(int rounds, uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]);
void orc_philox_batch(int rounds, uint64_t seed, const uint32_t *ctr, uint32_t *out, int64_t n);
double orc_ln(double u);
void orc_sincos2pi(double u, double *s, double *c);
double orc_exp(double x);
void orc_gauss3(int rounds, uint64_t seed, uint32_t site, uint32_t step, uint32_t sys,
                uint32_t stage, double g[3]);
void orc_ln_batch(const double *u, double *out, int64_t n);
void orc_exp_batch(const double *x, double *out, int64_t n);
void orc_sincos2pi_batch(const double *u, double *s, double *c, int64_t n);
void orc_gauss3_batch(int rounds, uint64_t seed, const uint32_t *site, const uint32_t *step,
                      uint32_t sys, uint32_t stage, double *g, int64_t n);

int64_t orc_lattice_sites(int kind, int nx, int ny, int nz);
int64_t orc_build_neighbours(int kind, int nx, int ny, int nz, const int periodic[3], double a,
                             double c, int n_shells, const double *radius, int64_t *row_ptr,
                             int32_t *col, int8_t *shell);
void orc_site_positions(int kind, int nx, int ny, int nz, double a, double *px, double *py);
void orc_voronoi_labels(int kind, int nx, int ny, int nz, const int periodic[2], int Q,
                        const int32_t *seeds_xy, int n_seeds, int64_t w_units, int32_t *labels);

int orc_heun_steps(const orc_system *s, double *Sx, double *Sy, double *Sz, int64_t step0,
                   int64_t nsteps);
/* spot temperature (K) of site i at step n; write-field polarity (+-1) of
 * step n; deterministic field (T) at site i: exchange + anisotropy +
 * polarised write field (no thermal or demagnetising term) */
double orc_site_temperature(const orc_system *s, int64_t i, int64_t n);
double orc_polarity(const orc_system *s, int64_t n);
void orc_field(const orc_system *s, const double *Sx, const double *Sy, const double *Sz,
               int64_t i, int64_t n, double B[3]);
void orc_magnetisation(const orc_system *s, const double *Sx, const double *Sy, const double *Sz,
                       int n_grains, double *per_grain, double tot[4]);
/* window-end transfer (Sec. II, Eq. 6): coarse cells of cx x cy x cz
 * lattice cells over stored columns [x0, x0 + ncols) */
void orc_coarse_grain(int kind, int sx, int ny, int nz, const int32_t *label, const double *Sx,
                      const double *Sy, const double *Sz, int x0, int ncols, int cx, int cy,
                      int cz, double *out);
void orc_set_columns(int kind, int sx, int ny, int nz, const int32_t *label, double *Sx,
                     double *Sy, double *Sz, int x0, int ncols, int cx, int cy, int cz,
                     const double *mcell);
double orc_cone_theta_max(double m);
#define ORC_CONE_PRINTED 0 /* polar angle uniform on [0, printed theta_max] */
#define ORC_CONE_CAP 1     /* uniform over the cap cos theta >= 2 m - 1 (mean m) */
void orc_cone_spin_mode(int mode, const double mvec[3], int rounds, uint64_t seed, uint32_t site,
                        uint32_t step, uint32_t sys, double out[3]);
void orc_cone_columns_mode(int mode, int kind, int sx, int ny, int nz, const int32_t *label,
                           double *Sx, double *Sy, double *Sz, int x0, int ncols, int cx, int cy,
                           int cz, const double *mcell, int rounds, uint64_t seed, uint32_t step,
                           uint32_t sys);
void orc_cone_spin(const double mvec[3], int rounds, uint64_t seed, uint32_t site, uint32_t step,
                   uint32_t sys, double out[3]);
void orc_cone_columns(int kind, int sx, int ny, int nz, const int32_t *label, double *Sx,
                      double *Sy, double *Sz, int x0, int ncols, int cx, int cy, int cz,
                      const double *mcell, int rounds, uint64_t seed, uint32_t step, uint32_t sys);
/* demagnetising tensor (Newell, Williams, Dunlop 1993) between two cells
 * of edges (dx, dy, dz) displaced by (X, Y, Z); N = (xx, yy, zz, xy, xz, yz) */
void orc_newell_tensor(double X, double Y, double Z, double dx, double dy, double dz,
                       double N[6]);
/* Eq. 7 by direct summation on a mesh of nx*ny*nz cells (x fastest):
 * H_i = -sum_j N(r_j - r_i) M_j, M and H [3][n] in A/m */
void orc_demag_direct(int nx, int ny, int nz, double dx, double dy, double dz, const double *M,
                      double *H);
/* Metropolis sweeps (colours 0 .. n_colours-1 in turn per sweep, no two
 * neighbours sharing one; colour -1: never visited) at the system's ambient
 * temperature; see asd_oracle.c */
int orc_mc_sweeps(const orc_system *s, const int8_t *colour, int n_colours, double *Sx,
                  double *Sy, double *Sz, int64_t sweep0, int64_t nsweeps);
/* micromagnetic region: LLG (no thermal field) by RK4 on a finite-difference
 * mesh with temperature-dependent parameters; see asd_oracle.c */
typedef struct orc_mm {
    int nx, ny, nz;
    int periodic[3];
    double h[3];            /* cell edges (m) */
    double Ms0, A0, K0;     /* A/m, J/m, J/m^3 at 0 K */
    double lambda, gamma, Tc, mu_s, dt;
    double B[3];
    int n_bits;
    const uint8_t *bits;
    int64_t steps_per_bit;
    int spot_mode;
    double T_amb, T_peak, fwhm, x0, y0, v;
    /* exchange coupling across the x faces (Sec. II): direction [ny*nz][3]
     * taken as the -x (ghost[0]) or +x (ghost[1]) neighbour of the boundary
     * cells of an open face; NULL: no neighbour */
    const double *ghost[2];
    /* a field (T) per cell [3][n] added to the effective field at every
     * stage, held through the step (the demagnetising field of the
     * multiscale window, Sec. II, Eq. 7); NULL: none */
    const double *bd;
} orc_mm;
double orc_langevin(double x);
double orc_mm_me(double T, double Tc, double b);
int orc_mm_rk4(const orc_mm *p, double *m, int64_t step0, int64_t nsteps);
/* temperature (K) of cell (i, j) at time t (s); polarity of step n */
double orc_mm_temperature(const orc_mm *p, int i, int j, double t);
double orc_mm_polarity(const orc_mm *p, int64_t n);
void orc_mm_shift(const orc_mm *p, double *m, const double *enter, int stride, double *leave);
void orc_mm_face_moment(const orc_mm *p, const double *m, int face, double t, double *out);
void orc_energy(const orc_system *s, const double *Sx, const double *Sy, const double *Sz,
                int64_t step, double out[4]);

#ifdef __cplusplus
}
#endif
#endif
