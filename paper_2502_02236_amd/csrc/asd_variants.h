// asd_variants.h -- kernel variants (host and device).
#pragma once

namespace asd {

// Two-pass kernel variants: 0 recomputes f(S) and the thermal field in the
// corrector; 1 stashes them from the predictor; 2 (handles with the
// demagnetising field only) recomputes them in kernels that take whole
// coarse cells and form the cells' spin sums for the next field evaluation.
constexpr int kPlainVariants = 3;
constexpr int kCellRowVariant = 2;

// Fused SC kernel variant: TXE lanes across x (64, 32 or 16), WAVES
// wavefronts, R column slots per lane, z planes per tile LZ (0: all).
// Extended tile TXE x TYE with TYE = WAVES R 64 / TXE; interior
// (TXE - 2) x (TYE - 2) x LZ.
struct FusedVariant {
    int txe, waves, rows, lz;
};

inline int fused_variant_count(bool fp64) { return fp64 ? 9 : 18; }

// Variant 0 is the default before any tuning (narrow tiles, z-chunks of 11:
// enough workgroups for ~1M-site lattices); the others cover wider tiles for
// large batches and the R = 2 and 16-lane shapes.  The twelve-wave tiles fill
// a CU with one workgroup at three waves per SIMD (the occupancy of the R = 1
// kernels' register count), on taller tiles: 32 x 24 extended columns
// recompute 1.16x the interior where 64 x 8 recompute 1.38x.
inline FusedVariant fused_variant(bool fp64, int v)
{
    static const FusedVariant f32v[18] = {
        {32, 4, 1, 11}, {64, 4, 2, 0},  {16, 4, 2, 11}, {32, 8, 1, 11}, {32, 4, 1, 17},
        {32, 8, 1, 17}, {32, 8, 1, 0},  {32, 4, 2, 11}, {64, 8, 2, 17}, {16, 4, 1, 11},
        {16, 8, 1, 11}, {16, 8, 1, 0},  {32, 8, 2, 8},  {32, 12, 1, 0}, {64, 12, 1, 0},
        {16, 12, 1, 0}, {32, 12, 1, 11}, {32, 6, 1, 0}};
    static const FusedVariant f64v[9] = {{32, 4, 1, 11}, {64, 4, 2, 0},  {32, 8, 1, 17},
                                         {32, 4, 1, 0},  {32, 8, 1, 11}, {16, 4, 1, 11},
                                         {32, 4, 2, 11}, {32, 12, 1, 0}, {32, 12, 1, 11}};
    const int n = fused_variant_count(fp64);
    if (v < 0 || v >= n) v = 0;
    return fp64 ? f64v[v] : f32v[v];
}

// Fused L1_0 kernel variants (cell tiles, both sublattices per column).
inline int fused_l10_variant_count(bool fp64) { return fp64 ? 3 : 5; }

inline FusedVariant fused_l10_variant(bool fp64, int v)
{
    static const FusedVariant f32v[5] = {{32, 4, 1, 9}, {32, 4, 1, 0}, {32, 8, 1, 9}, {16, 4, 1, 9},
                                         {32, 8, 1, 0}};
    static const FusedVariant f64v[3] = {{32, 4, 1, 9}, {32, 4, 1, 0}, {16, 4, 1, 9}};
    const int n = fused_l10_variant_count(fp64);
    if (v < 0 || v >= n) v = 0;
    return fp64 ? f64v[v] : f32v[v];
}

inline int fused_count(bool l10, bool fp64)
{
    return l10 ? fused_l10_variant_count(fp64) : fused_variant_count(fp64);
}

inline FusedVariant fused_pick(bool l10, bool fp64, int v)
{
    return l10 ? fused_l10_variant(fp64, v) : fused_variant(fp64, v);
}

inline void fused_tile_interior(bool fp64, int v, int *tx, int *ty, bool l10 = false)
{
    FusedVariant f = fused_pick(l10, fp64, v);
    *tx = f.txe - 2;
    *ty = f.waves * f.rows * 64 / f.txe - 2;
}

}  // namespace asd
