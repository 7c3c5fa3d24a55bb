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
// stored columns of track system s (0 for a system without a track or a bad index)
int32_t track_columns(const asd_t *h, int32_t s);
// asd_set_columns of two strips in one launch
int set_columns_pair(asd_t *h, int32_t s, int32_t xa, int32_t xb, int32_t ncols, int32_t cx,
                     int32_t cy, int32_t cz, const double *ma, const double *mb);

}  // namespace asd
