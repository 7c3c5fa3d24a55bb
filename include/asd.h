/*
 * asd.h -- C ABI of libasd: the stochastic Landau-Lifshitz-Gilbert (sLLG)
 * Heun time step of atomistic spin dynamics on MI355X (gfx950).
 *
 * Method (Gija et al., "Multiscale micromagnetic / atomistic modeling of
 * heat assisted magnetic recording", arXiv 2502.02236):
 *   - spins of fixed length evolved by the sLLG equation (Eq. 1), written
 *     in Landau-Lifshitz form dS/dt = -gamma/(1+alpha^2) [S x B + alpha
 *     S x (S x B)] and integrated by Heun's predictor-corrector with
 *     renormalisation to unit length after each stage;
 *   - B = exchange (Eq. 2, grouped by neighbour shell) + uniaxial
 *     anisotropy along z (Eq. 3) + write field (Sec. III: polarity carries
 *     the bit pattern) + Langevin thermal field of standard deviation
 *     sqrt(2 alpha kB T / (gamma mu_s dt)) (Sec. II), with T from a
 *     Gaussian laser spot (Sec. III, Fig. 2);
 *   - exchange-decoupled Voronoi grains separated by non-magnetic
 *     boundaries (Sec. II, Sec. III);
 *   - a simulation window that moves along a frozen track in steps of one
 *     lattice column, its ends exchange-coupled to the track (Sec. II);
 *   - simple-cubic or L1_0 Fe-sublattice lattices (Sec. II, Appendix A).
 *
 * Conventions shared by every call:
 *   - Every function returns ASD_OK (0) or a negative ASD_E* code; nothing
 *     throws or aborts across the ABI.  Arguments are validated before any
 *     work is enqueued.  The text of the last error of a handle is kept and
 *     returned by asd_last_error.
 *   - Memory ownership: the caller owns all device memory.  The library
 *     never allocates device memory: it carves everything it needs out of
 *     one caller-provided device workspace (asd_workspace_bytes tells the
 *     size).  The caller owns the HIP stream and every host buffer; input
 *     descriptors are copied at asd_create and may be freed afterwards.
 *   - All device work is enqueued on the stream given at asd_create, in
 *     order; calls that return host data synchronise that stream.
 *   - A handle is not thread-safe.
 *   - Spin arrays are structure-of-arrays: [3][n_stored] (Sx block, Sy
 *     block, Sz block), x fastest.  SC site index: x + sx (y + ny z); L1_0:
 *     2 (x + sx (y + ny z)) + s with s = 0 at the cell corner and s = 1 at
 *     the centre of the a x a face.  sx = track_nx for a track system, nx
 *     otherwise.  Element type is double (ASD_FP64) or float (ASD_FP32).
 */
#ifndef ASD_H
#define ASD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define ASD_OK 0
#define ASD_EINVAL (-1)       /* invalid argument or descriptor */
#define ASD_ENOMEM (-2)       /* workspace smaller than asd_workspace_bytes */
#define ASD_EHIP (-3)         /* a HIP runtime call or kernel launch failed */
#define ASD_ESTATE (-4)       /* call not valid in the handle's state */
#define ASD_ENONFINITE (-5)   /* a reduction met a non-finite spin */
#define ASD_EUNSUPPORTED (-6) /* valid request this library cannot serve */

/* ---- enumerations ---- */
#define ASD_FP64 0 /* every per-spin quantity in FP64 */
#define ASD_FP32 1 /* per-spin field and Heun update in FP32; reductions, time and
                      spot position in FP64 */

#define ASD_SC 0  /* simple cubic, 6 nearest neighbours, one shell */
#define ASD_L10 1 /* L1_0 Fe sublattice: shells at a/sqrt2 (4), c (2), a (4),
                     sqrt(a^2/2 + c^2) (8); n_shells selects the first 1..4 */

#define ASD_BC_OPEN 0
#define ASD_BC_PERIODIC 1
#define ASD_BC_TRACK 2 /* x only: the window [origin, origin+nx) moves inside a
                          stored track of track_nx columns; columns outside the
                          window are frozen and act as fixed neighbours */

#define ASD_SPOT_NONE 0   /* uniform temperature */
#define ASD_SPOT_MOVING 1 /* spot centre x0 + v n dt (stored-lattice frame) */
#define ASD_SPOT_LOCKED 2 /* spot centre origin*hx + x0: moves with the window */

#define ASD_KERNEL_AUTO 0  /* fused kernel where available, else two-pass */
#define ASD_KERNEL_PLAIN 1 /* two-pass: predictor kernel, corrector kernel */
#define ASD_KERNEL_FUSED 2 /* one kernel per step, LDS tiles with recomputed halo
                              (open or periodic z; see asd_set_variant) */

typedef struct asd_t asd_t; /* opaque handle */

/* Material and numerical parameters, common to all systems of a handle. */
typedef struct asd_params {
    int32_t lattice;       /* ASD_SC or ASD_L10 */
    int32_t precision;     /* ASD_FP64 or ASD_FP32 */
    double a;              /* lattice constant (m); x and y cell size */
    double c;              /* L1_0 cell height (m); ignored for SC */
    int32_t n_shells;      /* SC: 1.  L1_0: 1..4 */
    double J[4];           /* exchange energy per shell (J), Eq. 2 */
    double mu_s;           /* atomic moment (J/T) */
    double alpha;          /* Gilbert damping (the paper's lambda) */
    double gamma;          /* gyromagnetic ratio (rad s^-1 T^-1) */
    double dt;             /* time step (s) */
    double k_u;            /* uniaxial anisotropy energy per atom (J), Eq. 3 */
    uint64_t seed;         /* Philox key: (lo32, hi32) */
    int32_t philox_rounds; /* 10 (published Philox4x32-10) or 7 */
    int32_t kernel;        /* ASD_KERNEL_* */
    int32_t graph_steps;   /* >0: capture segments of this many steps (even)
                              in HIP graphs; 0: launch every step eagerly */
    int32_t demag_cell[3]; /* all > 0: add the demagnetising field of the window
                              (Eq. 7, Newell's tensor, open boundaries) on coarse
                              cells of demag_cell[0] x [1] x [2] lattice cells
                              (Eq. 6), evaluated at both Heun stages; for a
                              track system also the stray field of the frozen
                              track (Sec. II), on the window's cells continued
                              along the track, recomputed after the track
                              changes (spins set, window shifted, columns
                              thermalised); all 0: off.  Needs every system to
                              have the same window size, at most 256 coarse
                              cells per axis (254 along a track), and the
                              two-pass kernels (ASD_KERNEL_PLAIN or AUTO) */
} asd_params;

/* One lattice (one system).  A handle steps all its systems together. */
typedef struct asd_system_desc {
    int32_t nx, ny, nz;      /* window size in cells */
    int32_t bc_x, bc_y, bc_z; /* ASD_BC_*; ASD_BC_TRACK only for x */
    int32_t track_nx;        /* stored columns when bc_x == ASD_BC_TRACK */
    /* Grains, one of:
     *   n_seeds > 0: columnar Voronoi built by the library from integer seed
     *     points seeds_xy[2 n_seeds] in units of (hx / voronoi_q), hx = a
     *     (SC) or a/2 (L1_0); a site is non-magnetic when it lies closer
     *     than boundary_w_units/2 to the bisector of its own and another
     *     seed (minimum image on periodic axes, ties to the lower seed);
     *   labels != NULL: explicit grain label per stored site (-1 = not
     *     magnetic);
     *   neither: every site magnetic, one grain. */
    int32_t n_seeds;
    const int32_t *seeds_xy;
    int32_t voronoi_q;
    int64_t boundary_w_units;
    const int32_t *labels;
    const double *k_u_grain; /* per-grain k_u (J) [n_grains] or NULL */
    int32_t n_k_u_grain;
    double T_system;         /* >= 0: this system's ambient temperature (K),
                                replacing the drive's T_amb */
} asd_system_desc;

/* Write field and temperature drive (Sec. III). */
typedef struct asd_drive {
    double B[3];            /* write field (T); multiplied by the polarity */
    int32_t n_bits;         /* 0: polarity +1 always */
    const uint8_t *bits;    /* polarity of bit k: +1 if bits[k] else -1 */
    int64_t steps_per_bit;  /* step n writes bit (n / steps_per_bit) mod n_bits */
    int32_t spot_mode;      /* ASD_SPOT_* */
    double T_amb, T_peak;   /* K */
    double fwhm;            /* spot full width at half maximum (m) */
    double x0, y0;          /* spot centre at n = 0 / relative to the window (m) */
    double v;               /* spot velocity along +x (m/s), ASD_SPOT_MOVING */
} asd_drive;

/* Size of the device workspace asd_create needs for these descriptors.
 * Host-only; validates the descriptors (ASD_EINVAL). */
int asd_workspace_bytes(const asd_params *p, const asd_system_desc *sys, int32_t n_sys,
                        size_t *bytes);

/* Build lattices, neighbour tables and grain labels on the host and upload
 * them into the caller's workspace (device pointer, 256-byte aligned, at
 * least asd_workspace_bytes).  stream: hipStream_t (NULL = default).  Spins
 * start at +z on magnetic sites and 0 elsewhere; the step counter at 0; the
 * drive at zero field, T = 0, no spot.  Returns ASD_EUNSUPPORTED when two
 * magnetic neighbours carry different labels (grain boundaries thinner
 * than the neighbour range). */
int asd_create(const asd_params *p, const asd_system_desc *sys, int32_t n_sys, void *workspace,
               size_t workspace_bytes, void *stream, asd_t **out);

int asd_destroy(asd_t *h);

/* Set the write field, bit pattern and temperature spot (copied). */
int asd_set_field_temperature(asd_t *h, const asd_drive *d);

/* Copy spins of system sys in/out, [3][n_stored] in handle precision.
 * on_device != 0: src/dst is a device pointer.  set_spins writes both
 * ping-pong buffers and stores 0 at non-magnetic sites. get_spins
 * synchronises the stream when dst is host memory. */
int asd_set_spins(asd_t *h, int32_t sys, const void *src, int32_t on_device);
int asd_get_spins(asd_t *h, int32_t sys, void *dst, int32_t on_device);

/* Enqueue n >= 0 Heun steps (Eq. 1) of every system: step k uses the
 * write field, spot position and thermal noise of step index n0 + k, where
 * n0 is the handle's step counter, which then advances by n.  The thermal
 * field of a site at step n is sigma(T) (g_x, g_y, g_z) with g from
 * Box-Muller on Philox4x32(key = seed, counter = (stored site index, n,
 * system index, 0)): (g_x, g_y) from words (w0, w1), g_z the cosine branch
 * of (w2, w3), u_r = (w + 1/2) 2^-32, u_t = w 2^-32.  The predictor is
 * completed at every site before any corrector uses it; both stages use
 * the same thermal field, write field and temperature.  Asynchronous. */
int asd_step(asd_t *h, int64_t n);

/* Capture the step graphs now (one per ping-pong parity) when graph_steps >
 * 0, so the next graph segment of asd_step does not pay for capture and
 * instantiation.  Enqueues nothing.  Changing the drive or the kernel
 * variant drops the graphs again; asd_step then captures them on use. */
int asd_prepare(asd_t *h);

/* Move the window of every track system by `columns` >= 0 along +x: the
 * leaving columns freeze with their current spins, the entering ones are
 * taken from the track (Sec. II window shift).  ASD_ESTATE if a window
 * would leave its track; ASD_EINVAL for systems without a track. */
int asd_shift_window(asd_t *h, int32_t columns);

/* FP64 sums over the magnetic sites of each window (Eq. 6 moment sums
 * divided by mu_s): per_grain[4 g + k] for grain g of the flattened grain
 * list (systems in order, asd_grain_count grains each) and per_system[4 s
 * + k], k = (sum Sx, sum Sy, sum Sz, count).  Either pointer may be NULL.
 * Host pointers; synchronises.  ASD_ENONFINITE if a sum is not finite. */
int asd_reduce_magnetization(asd_t *h, double *per_grain, double *per_system);

/* asd_reduce_magnetization for callers that cannot allocate device memory
 * (serving loops, code between graph captures, harnesses that forbid
 * hipMalloc): the per-grain and per-system sums are kept in a static
 * device array of the library (1 MiB on each device it runs on, held
 * until the process ends) instead of the handle's workspace; nothing is
 * allocated.  Same arguments, kernels, summation order and results as
 * asd_reduce_magnetization.  Limit: n_grains + n_systems <= 32768 over the
 * handle, else ASD_EINVAL before anything is enqueued.  Either pointer may
 * be NULL (both NULL: nothing is enqueued); the finiteness check
 * (ASD_ENONFINITE) covers per_system, or per_grain when per_system is
 * NULL.  Host pointers; synchronises.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (two threads, or two handles on
 * different streams) race and must be serialised by the caller. */
int asd_reduce_magnetization_static(asd_t *h, double *per_grain, double *per_system);

/* FP64 energy of each window at the current step (J): per_system[4 s + k],
 * k = (exchange -1/2 sum_i sum_j J_ij S_i.S_j, anisotropy -sum k_u S_z^2,
 * Zeeman -sum mu_s B.S, total).  Host pointer; synchronises. */
int asd_reduce_energy(asd_t *h, double *per_system);

/* Accumulate M-statistics of every system from its current spins: with
 * m = |sum_i S_i| / N_magnetic over the window (Eq. 6 sums, FP64), per
 * system [5]: (samples, sum m, sum m^2, sum m^4, reserved, always 0);
 * these give <|m|>, the susceptibility N (<m^2> - <|m|>^2) mu_s / kB T and
 * the Binder cumulant 1 - <m^4> / 3 <m^2>^2.  reset != 0 clears before adding.  Enqueued on the
 * stream; read with asd_get_moment_stats (synchronises). */
int asd_accumulate_moments(asd_t *h, int32_t reset);
int asd_get_moment_stats(asd_t *h, double *per_system /* [5 n_sys] */);

/* Introspection of the built tables (for bit-exact checks).  Grain labels
 * per stored site; neighbour shells in CSR form, rows by site index, each
 * row ordered by shell then by offset (dz, dy, dx) with dx, dy in units of
 * hx; pass NULL arrays to the count query first. */
int asd_grain_count(asd_t *h, int32_t sys, int32_t *n_grains);
int asd_stored_sites(asd_t *h, int32_t sys, int64_t *n_stored);
int asd_get_grain_labels(asd_t *h, int32_t sys, int32_t *labels);
int asd_neighbour_count(asd_t *h, int32_t sys, int64_t *n_entries);
int asd_get_neighbours(asd_t *h, int32_t sys, int64_t *row_ptr, int32_t *col, int8_t *shell);

/* Host-only versions of the two tables above, computed from descriptors
 * without a device or handle (same code as asd_create uses): labels[n_stored]
 * and the CSR neighbour table.  asd_host_neighbours with NULL arrays only
 * writes the entry count to *n_entries. */
int asd_host_grain_labels(const asd_params *p, const asd_system_desc *sys, int32_t *labels);
int asd_host_neighbours(const asd_params *p, const asd_system_desc *sys, int64_t *n_entries,
                        int64_t *row_ptr, int32_t *col, int8_t *shell);

/* Window-end transfer to a coarse (micromagnetic) grid: Eq. 6 read
 * forwards (Sec. II).  The stored columns [x0, x0 + ncols) of system sys are
 * cut into coarse cells of cx x cy x cz lattice cells, numbered
 * c = i + ncx (j + ncy k) with ncx = ceil(ncols / cx), ncy = ceil(ny / cy)
 * (cells at the far ends may be partial; both L1_0 sites of a lattice cell
 * belong to its coarse cell).  out[4 c .. 4 c + 3] = (sum mx, sum my,
 * sum mz, N): the FP64 sum of the unit spins of the cell's magnetic sites
 * and their number, so M = mu_s / V sum m and M / M_S^0 = |sum m| / N.
 * out: caller-owned device pointer to ncx ncy ceil(nz / cz) x 4 doubles.
 * Reads the current spins; sums run in a fixed order (the same result every
 * run).  Asynchronous.  ASD_EINVAL for a bad system, column range or cell. */
int asd_coarse_grain(asd_t *h, int32_t sys, int32_t x0, int32_t ncols, int32_t cx, int32_t cy,
                     int32_t cz, double *out);

/* Window-end transfer from a coarse grid: Eq. 6 read backwards (Sec. II).
 * Every magnetic site of the stored columns [x0, x0 + ncols) of system sys
 * takes a spin drawn in the cone around the reduced magnetisation
 * m_c = mcell[3 c .. 3 c + 2] (M / M_S^0, |m_c| <= 1) of its coarse cell c
 * (cells as in asd_coarse_grain): polar angle uniform on [0, theta_max] with
 * theta_max = (5 pi / 9) sqrt(1 - sqrt(1 + 6 (|m_c| - 1) / 5)), |m_c|
 * clamped to [1/6, 1] (the expression is real there); azimuth uniform,
 * measured in the orthonormal basis of Duff et al., "Building an
 * orthonormal basis, revisited" (JCGT 2017) around m_c (z when m_c = 0).
 * Random words: Philox4x32 of counter (stored site index, step, system, 1),
 * u1 = (w0 + 1/2) 2^-32 sets the polar angle, u2 = w1 2^-32 the azimuth.
 * Computed in FP64, stored in the handle precision into both spin buffers
 * (like asd_set_spins).  mcell: caller-owned device pointer, [ncell][3]
 * doubles.  Asynchronous.  ASD_EINVAL as asd_coarse_grain.  The polar
 * angle follows the handle's cone reading (asd_set_cone_reading): the one
 * above by default. */
int asd_thermalise_columns(asd_t *h, int32_t sys, int32_t x0, int32_t ncols, int32_t cx,
                           int32_t cy, int32_t cz, const double *mcell, uint32_t step);

/* Cone readings of the inverse transfer (Sec. II).  The printed theta_max
 * does not give back |m_c| when many cone spins are averaged again (a
 * polar angle uniform on [0, theta_max] has mean cos = sin(theta_max) /
 * theta_max); the cap reading draws cos theta uniform on [2 |m_c| - 1, 1]
 * (|m_c| clamped to [0, 1]), cos theta = 1 - u1 (2 - 2 |m_c|), whose mean
 * is |m_c|: the averaged spins return the magnetisation they were drawn
 * from, which is what the angle is there for. */
#define ASD_CONE_PRINTED 0 /* polar angle uniform on [0, theta_max], the printed formula */
#define ASD_CONE_CAP 1     /* uniform over the cap cos theta >= 2 |m_c| - 1 */
int asd_set_cone_reading(asd_t *h, int32_t reading);

/* n Metropolis Monte Carlo sweeps of the same Hamiltonian (exchange,
 * anisotropy, write field with its polarity at the sweep index; no thermal
 * field) at each system's ambient temperature: the calibration of the
 * exchange constant against the Curie temperature (Sec. III with Eq. 8).
 * A sweep visits the window sites colour by colour (stored-lattice cell
 * coordinates): SC (x + y + z) mod 2, L1_0 s + 2 ((x + y) mod 2) + 4 (z mod 2)
 * with s the sublattice, so that no two neighbours share a colour; a visit
 * proposes a direction uniform on the sphere from Philox words (site, sweep,
 * system, 2) and accepts it with probability min(1, exp(-dE / kB T)).  The
 * sweep index is the step counter, which advances by n.  ASD_EUNSUPPORTED
 * for a periodic axis of odd length (the colours would pair neighbours) and
 * with the demagnetising field. */
int asd_mc_sweep(asd_t *h, int64_t n);

/* Every magnetic site of stored columns [x0, x0 + ncols) of system sys takes
 * the direction mcell[c] / |mcell[c]| of its coarse cell c (cells and mcell
 * as in asd_thermalise_columns; a zero cell gives +z), in both buffers: the
 * micromagnetic neighbours of the atomistic window (Sec. II). */
int asd_set_columns(asd_t *h, int32_t sys, int32_t x0, int32_t ncols, int32_t cx, int32_t cy,
                    int32_t cz, const double *mcell);
int asd_window_size(asd_t *h, int32_t sys, int32_t *nx, int32_t *ny, int32_t *nz);
int asd_get_stream(asd_t *h, void **stream);

/* Demagnetising field (Eq. 7) of the current spins of every system, as
 * the flux density mu0 H_d (T) per coarse cell of the window (including the
 * frozen track's stray field for a track system): per_cell is a host array
 * [n_sys][3][ncell] (cells numbered x fastest over the window,
 * c = i + ncx (j + ncy k)); mesh (optional, host int32[3]) receives
 * (ncx, ncy, ncz).  Coarse cell moment M = mu_s (sum of unit spins) / V
 * with V the full cell volume (Eq. 6); ragged cells at the far window
 * faces count their sites against the same V.  Synchronises the stream.
 * ASD_ESTATE when the handle was created without demag_cell. */
int asd_demag_field(asd_t *h, double *per_cell, int32_t *mesh);

/* When the demagnetising field is evaluated within a Heun step (Sec. II: the
 * field of the window is refreshed every iteration).  ASD_DEMAG_EACH_STAGE
 * (default): at both stages, from that stage's spins (S, then S').
 * ASD_DEMAG_ONCE: once per step from the step's starting spins S, and the
 * same field in both stages (an iteration read as a whole time step); the
 * fused kernel then runs the step in one launch.  ASD_EINVAL for another
 * value, ASD_ESTATE for a handle without demag_cell.  Drops captured
 * graphs. */
#define ASD_DEMAG_EACH_STAGE 0
#define ASD_DEMAG_ONCE 1
int asd_set_demag_reading(asd_t *h, int32_t reading);

/* Step counter of the handle and window origin (in lattice columns) of
 * system sys, from the host copies (no synchronisation). */
int asd_get_state(asd_t *h, int32_t sys, int64_t *step, int32_t *origin);
/* Set the step counter (resume from a checkpoint). */
int asd_set_step(asd_t *h, int64_t step);

/* Raw Philox4x32-R words of n counters (device pointers ctr[4n], out[4n]),
 * key = (lo32 seed, hi32 seed), on `stream`.  No handle needed. */
int asd_philox(uint64_t seed, int32_t rounds, const uint32_t *ctr, uint32_t *out, int64_t n,
               void *stream);

/* Pick the fastest kernel variant and tile for this handle by timing each
 * on the handle's stream (spins are saved and restored, the step counter
 * unchanged).  cache_path: JSON file read if it holds an entry for this
 * shape, written otherwise (NULL: no cache). */
int asd_autotune(asd_t *h, const char *cache_path);
/* Force a variant: kernel ASD_KERNEL_PLAIN or ASD_KERNEL_FUSED, tile index
 * 0 .. asd_variant_count - 1 (0 = default), else ASD_EINVAL.  The fused
 * kernels return ASD_EUNSUPPORTED (the handle keeps its variant) for a
 * system whose spins exceed 2 GiB per component, or when the anisotropy
 * varies per grain and some stored column crosses grains (labels varying
 * along z), or when the handle adds the demagnetising field (a whole-mesh
 * convolution between the two Heun stages); the two-pass kernels take every
 * system.  Two-pass tiles: 0 recomputes f(S) and the thermal field in the
 * corrector, 1 stores them from the predictor, 2 (the default with the
 * demagnetising field; ASD_EUNSUPPORTED without it or for coarse cells wider
 * than 64 lattice cells) works on whole coarse cells and forms their spin
 * sums (Eq. 6) as it writes the spins, so that within one asd_step call only
 * the first field evaluation reads the spins.  Drops captured graphs. */
int asd_set_variant(asd_t *h, int32_t kernel, int32_t tile);
int asd_get_variant(asd_t *h, int32_t *kernel, int32_t *tile);
/* Number of tile variants of a kernel family for this handle's lattice and
 * precision (the fused count is returned even where the fused kernels
 * cannot serve the handle). */
int asd_variant_count(asd_t *h, int32_t kernel, int32_t *count);
/* Name of the step kernel(s) the current variant launches (as profilers list
 * them), NUL-terminated into buf[len]; ASD_EINVAL if it does not fit. */
int asd_variant_name(asd_t *h, char *buf, size_t len);

/* ---- micromagnetic region (Sec. II) ----
 * LLG without the thermal field (Eq. 1 in Landau-Lifshitz form) on a
 * finite-difference mesh of nx x ny x nz cells (x fastest, arrays
 * [3][n] of unit vectors in the handle precision), integrated by classic
 * RK4 (the integrator the paper names for these regions, Sec. III) and
 * renormalised after every step.  Field per cell, in tesla:
 *   exchange (2 A(T) / M_S(T)) lap m (Eq. 4; six-point stencil, a missing
 *   neighbour at an open face contributes nothing), uniaxial anisotropy
 *   (2 K(T) / M_S(T)) m_z z (Eq. 5), write field p(n) B;
 * M_S = Ms0 m_e(T), A = A0 m_e^2, K = K0 m_e^3, alpha = lambda (1 - T / 3 T_C)
 * with T clamped to T_C, and m_e(T) the largest root of
 * m = L(3 T_C m / T + mu_s |B| / kB T) with L the Langevin function
 * (Sec. II), computed in FP64.  T per cell from the drive's spot at the
 * cell centre ((i + 1/2) h_x, (j + 1/2) h_y) and the stage time
 * (ASD_SPOT_LOCKED: centre (x0, y0) in the mesh frame).  The handle owns no
 * device memory (caller workspace); work runs on the given stream. */
typedef struct asd_mm_t asd_mm_t;
typedef struct asd_mm_params {
    int32_t precision;        /* ASD_FP64 or ASD_FP32 */
    int32_t nx, ny, nz;       /* cells, at most 2^28 in all */
    int32_t bc_x, bc_y, bc_z; /* ASD_BC_OPEN or ASD_BC_PERIODIC */
    double h[3];              /* cell edges (m) */
    double Ms0;               /* spontaneous magnetisation at 0 K (A/m) */
    double A0;                /* exchange stiffness at 0 K (J/m); Eq. 9: J / 2a */
    double K0;                /* uniaxial anisotropy at 0 K (J/m^3) */
    double lambda;            /* damping at 0 K */
    double gamma;             /* gyromagnetic ratio (rad s^-1 T^-1) */
    double Tc;                /* Curie temperature (K) */
    double mu_s;              /* atomic moment in the field term of m_e (J/T) */
    double dt;                /* time step (s) */
    int32_t graph_steps;      /* > 0: capture segments of this many steps */
} asd_mm_params;
int asd_mm_workspace_bytes(const asd_mm_params *p, size_t *bytes);
/* m starts at +z everywhere, the step counter at 0, no field, T = 0. */
int asd_mm_create(const asd_mm_params *p, void *workspace, size_t workspace_bytes, void *stream,
                  asd_mm_t **out);
int asd_mm_destroy(asd_mm_t *h);
int asd_mm_set_field_temperature(asd_mm_t *h, const asd_drive *d);
int asd_mm_set_m(asd_mm_t *h, const void *src, int32_t on_device);
int asd_mm_get_m(asd_mm_t *h, void *dst, int32_t on_device);
/* n RK4 steps; the polarity of step k is that of bit (k / steps_per_bit). */
int asd_mm_step(asd_mm_t *h, int64_t n);
int asd_mm_get_step(asd_mm_t *h, int64_t *step);
/* Exchange coupling across an x face (Sec. II): vec (device, or NULL to
 * remove) holds per boundary cell c = j + ny k a vector at vec[c * stride];
 * its direction becomes the -x (face 0) or +x (face 1) stencil neighbour of
 * the cells on that face (a zero vector: no neighbour).  stride 4 takes the
 * sums of asd_coarse_grain directly. */
int asd_mm_set_face(asd_mm_t *h, int32_t face, const double *vec, int32_t stride);
/* Directions of the cells on x face `face` into dirs (device, [ny*nz][3]). */
int asd_mm_get_face(asd_mm_t *h, int32_t face, double *dirs);
/* n steps of a multiscale window (Sec. II, Fig. 1): micromagnetic regions
 * left (may be NULL) and right (may be NULL) of the atomistic window of
 * track system `sys`, exchange-coupled through their x faces.  Cells of the
 * micromagnetic meshes are cx x cy x cz lattice cells (their ny, nz equal
 * the window's coarse cells).  Each step: the first and last coarse column
 * of the window, averaged (Eq. 6), become the +x / -x face neighbours of
 * the left / right region (the average atomistic spin direction of the
 * stencil cell); the regions' boundary cell directions are written into the
 * cx frozen columns just outside the window (the atomistic exchange
 * neighbours there); then one Heun step of the atoms and one RK4 step of each
 * region, all on the atomistic handle's stream (both handles must have been
 * created on it).  Needs cx <= origin and origin + nx + cx <= track_nx, each
 * region's dt equal to the atomistic dt (one RK4 step per Heun step) and its
 * cell edges h equal to (cx a, cy a, cz a) for SC or (cx a, cy a, cz c) for
 * L1_0 (relative tolerance 1e-9), so its faces line up with the coarse cells.
 * With both regions of one precision under a spot that does not move, each
 * face operation and each RK4 stage runs as one launch for the two sides;
 * the results are those of the per-region sequence.  Errors: ASD_EINVAL for
 * bad sizes, streams or meshes (nothing enqueued); a failure part-way through
 * the n steps returns at once, after the steps already enqueued. */
int asd_multiscale_step(asd_t *atoms, int32_t sys, asd_mm_t *left, asd_mm_t *right, int32_t cx,
                        int32_t cy, int32_t cz, int64_t n);
/* Move the multiscale window of asd_multiscale_step by one coarse cell (cx
 * lattice columns) along +x, the whole simulation region following the
 * write head (Sec. II, Fig. 1), in this order:
 *   1. trailing end (left region, if any): the first cx columns of the
 *      atomistic window, averaged (Eq. 6), give the direction of the
 *      region's new last cell column (+z for a cell with no magnetic site);
 *      every other cell takes the direction of its +x neighbour, and the
 *      first cell column leaves for the track: its directions are copied
 *      to leave (device, [ny*nz][3] doubles, c = j + ny k) unless NULL;
 *   2. leading end (right region, if any): the magnetic sites of stored
 *      columns [origin + nx, origin + nx + cx) take cone spins (Eq. 6 read
 *      backwards, as asd_thermalise_columns, with the handle's cone
 *      reading and Philox counter word = the atomistic step counter)
 *      around m_e(T) m of the region's first cells, m_e(T) at the
 *      cell temperature at time step * dt (the equilibrium magnetisation
 *      of the region's M_S(T), Sec. II); then every cell takes the
 *      direction of its +x neighbour and the last cell column takes the
 *      directions enter[3 c ..] of the track ahead (device, [ny*nz][3]
 *      doubles, normalised; a zero vector gives +z);
 *   3. the atomistic window moves by cx columns (asd_shift_window).
 * Same region checks as asd_multiscale_step; enter is required with a right
 * region.  Asynchronous, on the atomistic handle's stream. */
int asd_multiscale_shift(asd_t *atoms, int32_t sys, asd_mm_t *left, asd_mm_t *right, int32_t cx,
                         int32_t cy, int32_t cz, const double *enter, double *leave);

/* The demagnetising field of the whole multiscale window (Eq. 7, Sec. II:
 * the stray field between the meshes fully computed every step, Fig. 1).
 * The left region's cells, the atomistic window's coarse cells and the right
 * region's cells are laid along x as one mesh of NX = nL + nx / cx + nR
 * equal cells (ny, nz as the regions); a region cell carries
 * M = M_S0 m_e(T) m (T at the cell centre), an atomistic cell
 * M = mu_s (sum of its spins) / V (Eq. 6).  The field of this mesh is
 * computed by zero-padded FFT convolution with Newell's tensor (FP64) from
 * the state at the start of each coupled step:
 *   - each region adds the field at its cells (all sources) to its
 *     effective field, held through the four RK4 stages;
 *   - the atoms add, at both Heun stages, the field of the regions' cells at
 *     their coarse cells, in place of the frozen track's stray field, to
 *     their own demagnetising field evaluated per stage (the atomistic
 *     handle must have demag_cell = (cx, cy, cz)).
 * Needs what asd_multiscale_step needs, nx a multiple of cx, NX <= 512 and
 * ny, nz <= 256 coarse cells.  The object keeps pointers to the three
 * handles (which must outlive it) and lives in a caller workspace
 * (asd_msd_workspace_bytes, 256-byte aligned, device memory). */
typedef struct asd_msd_t asd_msd_t;
int asd_msd_workspace_bytes(asd_t *atoms, int32_t sys, const asd_mm_t *left,
                            const asd_mm_t *right, int32_t cx, int32_t cy, int32_t cz,
                            size_t *bytes);
int asd_msd_create(asd_t *atoms, int32_t sys, asd_mm_t *left, asd_mm_t *right, int32_t cx,
                   int32_t cy, int32_t cz, void *workspace, size_t workspace_bytes,
                   asd_msd_t **out);
int asd_msd_destroy(asd_msd_t *m);
/* n coupled steps of asd_multiscale_step with the demagnetising field of the
 * whole window; after it the regions hold no field and the atoms go back to
 * the frozen track's stray field.  Errors as asd_multiscale_step. */
int asd_multiscale_step_demag(asd_msd_t *m, int64_t n);
/* The last evaluated fields (T) of the combined mesh into host arrays
 * all[3][NX ny nz] (every source) and regions[3][NX ny nz] (the regions'
 * cells only), either may be NULL; mesh (optional, int32[3]) receives
 * (NX, ny, nz).  Synchronises the stream. */
int asd_msd_fields(asd_msd_t *m, double *all, double *regions, int32_t *mesh);
const char *asd_mm_last_error(const asd_mm_t *h);

const char *asd_strerror(int code);
const char *asd_last_error(const asd_t *h);

#ifdef __cplusplus
}
#endif
#endif
