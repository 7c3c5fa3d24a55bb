// asd_pair.h -- the two boundary strips of a window in one launch each (the
// coupled multiscale step moves data across both x faces every step; the
// launches, not the bytes, dominate there).  Library-internal: not part of
// the C ABI.
#pragma once

#include "asd.h"
#include "asd_internal.h"

namespace asd {

// both transfer kernels over two strips of the same shape; -1 on a shape or
// precision mismatch or a launch error
int launch_coarse_grain_pair(const TransferArgs &a0, const TransferArgs &a1, void *stream);
int launch_cone_columns_pair(const TransferArgs &a0, const TransferArgs &a1, void *stream);

// asd_coarse_grain of columns [xa, xa + ncols) into outa and of
// [xb, xb + ncols) into outb, in one launch; same checks and error codes
int coarse_grain_pair(asd_t *h, int32_t s, int32_t xa, int32_t xb, int32_t ncols, int32_t cx,
                      int32_t cy, int32_t cz, double *outa, double *outb);
// the handle's time step and lattice cell edges (x, y: a; z: a for SC, c for
// L1_0), for the checks of the multiscale window
void lattice_cell(const asd_t *h, double *dt, double edge[3]);
// the atomic moment mu_s (J/T) of the handle
double atom_moment(const asd_t *h);
// stored columns of track system s (0 for a system without a track or a bad index)
int32_t track_columns(const asd_t *h, int32_t s);
// the demagnetising mesh of a handle: coarse cell (lattice cells) and cells
// per axis; ASD_ESTATE when the handle has no demagnetising field
int demag_mesh(const asd_t *h, int32_t cell[3], int32_t mesh[3]);
// the field (T) that system s adds per coarse cell at both Heun stages in
// place of the frozen track's stray field: cells [off, off + ncx) of a wider
// mesh of src_nx cells along x (src [3][src_nx ncy ncz], device, FP64),
// copied now; clear_cell_field goes back to the track's stray field
int set_cell_field(asd_t *h, int32_t s, const double *src, int32_t src_nx, int32_t src_off);
int clear_cell_field(asd_t *h);
// asd_set_columns of two strips in one launch
int set_columns_pair(asd_t *h, int32_t s, int32_t xa, int32_t xb, int32_t ncols, int32_t cx,
                     int32_t cy, int32_t cz, const double *ma, const double *mb);

}  // namespace asd
