// Grid and tile index arithmetic of the NUFFT stage, shared by the plan-time
// sort, the interpolation / spreading kernels and a CPU build of the same
// functions (the tests compile this header with a host compiler to check that
// a point's stencil never leaves the tile it is sorted into).
//
// Grid: the oversampled Theta grid has spacing 2 pi / Ntheta along the
// stretched colatitude Theta = theta pi / theta_max (Sec. II, step 3) and
// spacing 2 pi / Nphi in longitude.  A point at grid coordinates
// (X, Y) = (theta sx, phi sy) touches rows a0 .. a0 + W - 1 with
// a0 = ceil(X - W/2), and columns b0 .. b0 + W - 1 (mod Nphi),
// b0 = ceil(Y - W/2).  Only the rows row_lo .. row_lo + rows_used - 1 are
// stored; tiles cover tile_x x tile_y stencil origins.
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define PSHT_HD __host__ __device__
#else
#define PSHT_HD
#endif

namespace psht {

struct TileGeom {
    double sx, sy;
    int W, row_lo, rows_used, Nphi, tile_x, tile_y, ntx, nty;
};

PSHT_HD inline int stencil_origin(double X, int W) { return (int)ceil(X - 0.5 * W); }

// Degree of the polynomial kernel table of the inner taps: FP64 plans
// max(W + 1, 12); FP32 plans, whose table is evaluated in float,
// max(W + 2, 10) (its float evaluation error is about 1e-7).
PSHT_HD constexpr int es_poly_degree(int W, bool fp32) {
    return fp32 ? (W + 2 > 10 ? W + 2 : 10) : (W + 1 > 12 ? W + 1 : 12);
}

// b0 reduced to [0, Nphi).  A point's b0 lies in [-W/2, Nphi): a compare or
// one add; the remainder only for other values.
PSHT_HD inline int wrap_col(int b0, int Nphi) {
    if (b0 >= 0 && b0 < Nphi) return b0;
    if (b0 < 0 && b0 >= -Nphi) return b0 + Nphi;
    int b = b0 % Nphi;
    return b < 0 ? b + Nphi : b;
}

// Grid coordinates of a point; phi is reduced to [0, 2 pi).
PSHT_HD inline void point_grid(const TileGeom &a, double theta, double phi, double &X, double &Y) {
    const double twopi = 2.0 * M_PI;
    double f = phi - twopi * floor(phi / twopi);
    if (f >= twopi) f -= twopi;
    if (f < 0.0) f = 0.0;
    X = theta * a.sx;
    Y = f * a.sy;
    if (Y >= (double)a.Nphi) Y -= (double)a.Nphi;
}

// Tile of a point (clamped to the tile grid).
PSHT_HD inline int point_tile(const TileGeom &a, double X, double Y) {
    const int a0 = stencil_origin(X, a.W);
    const int b0m = wrap_col(stencil_origin(Y, a.W), a.Nphi);
    int tx = (a0 - a.row_lo) / a.tile_x;
    int ty = b0m / a.tile_y;
    tx = tx < 0 ? 0 : (tx > a.ntx - 1 ? a.ntx - 1 : tx);
    ty = ty < 0 ? 0 : (ty > a.nty - 1 ? a.nty - 1 : ty);
    return tx * a.nty + ty;
}

// Stencil origin of a point relative to tile t, unclamped: (li, lj) lies in
// [0, tile_x) x [0, tile_y) exactly when the point's stencil stays inside the
// tile's subgrid.
PSHT_HD inline void tile_local(const TileGeom &a, double X, double Y, int t, int &li, int &lj) {
    const int tx = t / a.nty, ty = t - tx * a.nty;
    li = stencil_origin(X, a.W) - a.row_lo - tx * a.tile_x;
    lj = wrap_col(stencil_origin(Y, a.W), a.Nphi) - ty * a.tile_y;
}

PSHT_HD inline bool in_tile(const TileGeom &a, int li, int lj) {
    return li >= 0 && li < a.tile_x && lj >= 0 && lj < a.tile_y;
}

}  // namespace psht
