// CPU build of the NUFFT tile arithmetic (paper_2603_17166_amd/csrc/nufft_index.h):
// for a plan geometry given on the command line, sweeps colatitudes over
// [theta_min, theta_star] and longitudes over and around [0, 2 pi), with the
// values where a stencil origin jumps (X - W/2 or Y - W/2 an integer) and
// their neighbouring doubles, and counts points whose stencil origin falls
// outside the tile point_tile assigns them.  Prints "checked <n> outside <k>".
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "nufft_index.h"

int main(int argc, char **argv) {
    if (argc != 13) {
        std::fprintf(stderr, "usage: sx sy W row_lo rows_used Nphi tile_x tile_y ntx nty theta_min theta_star\n");
        return 2;
    }
    psht::TileGeom g;
    g.sx = std::atof(argv[1]);
    g.sy = std::atof(argv[2]);
    g.W = std::atoi(argv[3]);
    g.row_lo = std::atoi(argv[4]);
    g.rows_used = std::atoi(argv[5]);
    g.Nphi = std::atoi(argv[6]);
    g.tile_x = std::atoi(argv[7]);
    g.tile_y = std::atoi(argv[8]);
    g.ntx = std::atoi(argv[9]);
    g.nty = std::atoi(argv[10]);
    const double tmin = std::atof(argv[11]), tmax = std::atof(argv[12]);
    std::vector<double> th, ph;
    for (int i = 0; i <= 4000; ++i) th.push_back(tmin + (tmax - tmin) * i / 4000.0);
    // colatitudes where X - W/2 crosses an integer, and the doubles next to them
    for (int k = (int)std::floor(tmin * g.sx - 0.5 * g.W) - 1; k <= (int)std::ceil(tmax * g.sx - 0.5 * g.W) + 1; ++k) {
        const double t = (k + 0.5 * g.W) / g.sx;
        for (double v : {t, std::nextafter(t, 0.0), std::nextafter(t, 10.0)})
            if (v >= tmin && v <= tmax) th.push_back(v);
    }
    th.push_back(tmin);
    th.push_back(tmax);
    const double twopi = 2.0 * M_PI;
    for (int i = 0; i <= 2000; ++i) ph.push_back(-3.0 * twopi + 7.0 * twopi * i / 2000.0);
    for (int k = -1; k <= g.Nphi + 1; k += 1) {
        const double p = (k + 0.5 * g.W) / g.sy;
        for (double v : {p, std::nextafter(p, -100.0), std::nextafter(p, 100.0), p - twopi, p + twopi}) ph.push_back(v);
    }
    for (double v : {0.0, -0.0, -1e-300, 1e-300, twopi, std::nextafter(twopi, 0.0), std::nextafter(twopi, 10.0),
                     -twopi, 1e6, -1e6})
        ph.push_back(v);
    long long n = 0, bad = 0;
    for (double t : th)
        for (double p : ph) {
            double X, Y;
            psht::point_grid(g, t, p, X, Y);
            const int tile = psht::point_tile(g, X, Y);
            int li, lj;
            psht::tile_local(g, X, Y, tile, li, lj);
            ++n;
            if (!psht::in_tile(g, li, lj) || !(Y >= 0.0 && Y < g.Nphi)) ++bad;
        }
    std::printf("checked %lld outside %lld\n", n, bad);
    return 0;
}
