// asd_variants.h -- tile variants of the fused SC kernel (host and device).
#pragma once

namespace asd {

// fused kernel variant v: WAVES wavefronts of 64 lanes, R rows per wave;
// extended tile 64 x (WAVES R), interior 62 x (WAVES R - 2)
inline int fused_variant_count(bool fp64) { return fp64 ? 3 : 4; }

inline void fused_variant_geom(bool fp64, int v, int *waves, int *rows)
{
    static const int f32w[4] = {8, 4, 8, 4}, f32r[4] = {4, 4, 2, 2};
    static const int f64w[3] = {4, 8, 8}, f64r[3] = {2, 2, 1};
    const int n = fused_variant_count(fp64);
    if (v < 0 || v >= n) v = 0;
    *waves = fp64 ? f64w[v] : f32w[v];
    *rows = fp64 ? f64r[v] : f32r[v];
}

inline void fused_tile_interior(bool fp64, int v, int *tx, int *ty)
{
    int w, r;
    fused_variant_geom(fp64, v, &w, &r);
    *tx = 62;
    *ty = w * r - 2;
}

}  // namespace asd
