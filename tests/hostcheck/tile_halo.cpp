// Host-side check of the halo coverage of the LDS tiles (tiles.h), built by
// tests/test_tile_halo.py.  It stages one plane the way the tiled kernels do
// (thread t stages elements t + k NT) into an array prefilled with NaN --
// what the kernels' debug mode does to their LDS -- and then reads every
// value the kernels read: the in-plane 5-point stencil of every component at
// the own site and the halo-ring site of every thread.  A value never staged
// reads as NaN; a staged value from the wrong lattice site reads as a wrong
// value; a site of the halo-1 plane that no thread evaluates (or two do) is
// counted too.  argv[1] plants a mistake in the staging: 0 none, 1 the last
// halo column is never staged, 2 the first halo row is never staged.
// Prints "nan bad cover" summed over a set of tile positions and lattices.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_0901_3293_amd/csrc/tiles.h"

using hlb::wrapi;
using S = hlb::KernelTile;
using M = hlb::TileMap<S>;

static double tag(int c, int off) { return 1e7 * c + off; }

int main(int argc, char **argv)
{
    const int drop = argc > 1 ? std::atoi(argv[1]) : 0;
    const int NC = 5;
    const int cases[][4] = {{128, 128, 0, 0},   {128, 128, 96, 120}, {100, 37, 96, 32}, {4, 4, 0, 0},
                            {13, 7, 0, 0},      {70, 5, 64, 0},      {255, 129, 224, 128}, {33, 9, 32, 8}};
    long nan = 0, bad = 0, cover = 0;
    for (const auto &cs : cases) {
        const int nx = cs[0], ny = cs[1], x0 = cs[2], y0 = cs[3];
        std::vector<double> slot(NC * S::RN, std::nan(""));
        for (int t = 0; t < S::NT; ++t)
            for (int e = t; e < NC * S::RN; e += S::NT) {
                int comp, off;
                M::staged(e, x0, y0, nx, ny, comp, off);
                const int r = e - comp * S::RN, ri = r % S::RX, rj = r / S::RX;
                if ((drop == 1 && ri == S::RX - 1) || (drop == 2 && rj == 0)) continue;
                slot[e] = tag(comp, off);
            }
        std::vector<int> evaluated(S::PN, 0);
        for (int t = 0; t < S::NT; ++t) {
            int pc, rc, hp, hr;
            M::own(t, pc, rc);
            M::halo(t, hp, hr);
            ++evaluated[pc];
            if (hp >= 0) ++evaluated[hp];
            for (int r : {rc, hr}) {
                if (r < 0) continue;
                for (int c = 0; c < NC; ++c)
                    for (int d : {0, 1, -1, S::RX, -S::RX}) {
                        const int o = r + d;
                        const double v = slot[c * S::RN + o];
                        if (std::isnan(v)) {
                            ++nan;
                            continue;
                        }
                        const int gx = wrapi(x0 - 2 + o % S::RX, nx), gy = wrapi(y0 - 2 + o / S::RX, ny);
                        if (v != tag(c, gx + nx * gy)) ++bad;
                    }
            }
        }
        for (int v : evaluated) cover += v != 1;
    }
    std::printf("%ld %ld %ld\n", nan, bad, cover);
    return 0;
}
