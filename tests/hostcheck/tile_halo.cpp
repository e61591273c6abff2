// Host-side check of the halo coverage of the LDS tiles (tiles.h), built by
// tests/test_tile_halo.py.  It stages one plane the way the tiled kernels do
// (thread t of a block of NB stages elements t + k NB, in the component given
// by comp_base / comp_split) into an array prefilled with NaN -- what the
// kernels' debug mode does to their LDS -- and then reads every value the
// kernels read: the in-plane 5-point stencil of every component at the
// evaluation point of every thread (its z-neighbours are read at the same
// staged coordinate).  A value never staged reads as NaN; a staged value from
// the wrong lattice site or component reads as a wrong value; a point of the
// halo-1 plane that no thread evaluates (or two do), or a tile site that is
// not its thread's own, is counted too.  argv[1] plants a mistake in the
// staging: 0 none, 1 the last halo column is never staged, 2 the first halo
// row is never staged, 3 the component split of k = 1 is taken 8 elements late.
// Prints "nan bad cover" summed over a set of tile positions and lattices,
// one line for each tile shape (FP32, FP64).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_0901_3293_amd/csrc/tiles.h"

using hlb::wrapi;

static double tag(int c, int off) { return 1e7 * c + off; }

template <class S>
static void check(int drop)
{
    using M = hlb::TileMap<S>;
    const int NC = 5;
    // lattice (nx, ny) and tile origin (x0, y0): origins of both tile shapes,
    // last tiles that overhang the lattice, lattices smaller than a tile
    const int cases[][4] = {{128, 128, 0, 0},     {128, 128, 96, 120},  {100, 37, 96, 32}, {4, 4, 0, 0},
                            {13, 7, 0, 0},        {70, 5, 64, 0},       {255, 129, 224, 128}, {33, 9, 32, 8},
                            {128, 128, 112, 120}, {100, 37, 96, 36},    {255, 129, 240, 120}, {33, 9, 32, 0}};
    long nan = 0, bad = 0, cover = 0;
    for (const auto &cs : cases) {
        const int nx = cs[0], ny = cs[1], x0 = cs[2], y0 = cs[3];
        std::vector<double> slot(NC * S::RN, std::nan(""));
        const int nk = (NC * S::RN + S::NB - 1) / S::NB;
        for (int t = 0; t < S::NB; ++t)
            for (int k = 0; k < nk; ++k) {
                const int e = t + k * S::NB;
                if (e >= NC * S::RN) continue;
                int comp, off;
                M::staged(e, x0, y0, nx, ny, comp, off);
                const int r = e - comp * S::RN, ri = r % S::RX, rj = r / S::RX;
                if ((drop == 1 && ri == S::RX - 1) || (drop == 2 && rj == 0)) continue;
                // the component the kernels' loader takes for this element
                int lc = M::comp_base(k) + (t >= M::comp_split(k) ? 1 : 0);
                if (drop == 3 && k == 1) lc = M::comp_base(k) + (t >= M::comp_split(k) + 8 ? 1 : 0);
                slot[e] = tag(lc, off);
            }
        std::vector<int> evaluated(S::PN, 0);
        for (int t = 0; t < S::NB; ++t) {
            int pc, rc;
            if (!M::point(t, pc, rc)) continue;
            ++evaluated[pc];
            if (t < S::NT) {
                int opc, orc;
                M::own(t, opc, orc);
                if (opc != pc || orc != rc) ++cover;
            }
            for (int r : {rc}) {
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
}

int main(int argc, char **argv)
{
    const int drop = argc > 1 ? std::atoi(argv[1]) : 0;
    check<hlb::KernelTile<float>>(drop);   // one line per tile shape
    check<hlb::KernelTile<double>>(drop);
    return 0;
}
