// tiles.h -- geometry of the 2.5D z-marching tiles used by the fused
// Q-side kernels.  A block of TX*TY threads owns a TX x TY column of sites and
// marches along z through a chunk of planes.  Input planes are staged in LDS
// with a two-site halo (ring of three planes); intermediate quantities that
// are needed at stencil neighbours (the stress, the predictor stage) are
// evaluated on the tile plus a one-site halo ring.
#pragma once

#include <hip/hip_runtime.h>

namespace hlb {

template <int TX_, int TY_>
struct TileShape {
    static constexpr int TX = TX_, TY = TY_;
    static constexpr int NT = TX * TY;                  // threads
    static constexpr int RX = TX + 4, RY = TY + 4;      // staged input plane (halo 2)
    static constexpr int RN = RX * RY;
    static constexpr int PX = TX + 2, PY = TY + 2;      // evaluated plane (halo 1)
    static constexpr int PN = PX * PY;
    static constexpr int NH = PN - NT;                  // halo-ring points
    static_assert(NH <= NT, "halo ring must fit in one pass of the block");

    // Halo-ring point h in [0, NH) -> (i, j) in halo-1 plane coordinates:
    // bottom row, top row, then left/right columns.
    __host__ __device__ static __forceinline__ void halo_point(int h, int &i, int &j)
    {
        if (h < PX) {
            i = h;
            j = 0;
        } else if (h < 2 * PX) {
            i = h - PX;
            j = PY - 1;
        } else {
            const int k = h - 2 * PX;
            j = 1 + (k >> 1);
            i = (k & 1) ? PX - 1 : 0;
        }
    }
};

// The tile of the fused Q-side kernels: 32 x 8 sites per block.
using KernelTile = TileShape<32, 8>;

__host__ __device__ __forceinline__ int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Index maps of the tile kernels, shared by the kernels and the host-side
// check of their halo coverage.
template <class S>
struct TileMap {
    // Own site of thread t: its place on the halo-1 plane (pc) and on the
    // staged plane (rc).
    __host__ __device__ static __forceinline__ void own(int t, int &pc, int &rc)
    {
        const int tx = t % S::TX, ty = t / S::TX;
        pc = (ty + 1) * S::PX + (tx + 1);
        rc = (ty + 2) * S::RX + (tx + 2);
    }
    // Halo-ring point of thread t < NH on the halo-1 plane (hp) and on the
    // staged plane (hr); -1 for the other threads.
    __host__ __device__ static __forceinline__ void halo(int t, int &hp, int &hr)
    {
        hp = hr = -1;
        if (t < S::NH) {
            int i, j;
            S::halo_point(t, i, j);
            hp = j * S::PX + i;
            hr = (j + 1) * S::RX + (i + 1);
        }
    }
    // Element e of an NC-component staged plane (component-major, RN points
    // per component): its component and its in-plane offset in the lattice
    // for a tile at (x0, y0), periodic wrap.  The block stages element
    // e = t + k NT from thread t, k = 0, 1, ...
    __host__ __device__ static __forceinline__ void staged(int e, int x0, int y0, int nx, int ny, int &comp, int &off)
    {
        comp = e / S::RN;
        const int r = e - comp * S::RN;
        const int ri = r % S::RX, rj = r / S::RX;
        off = wrapi(x0 - 2 + ri, nx) + nx * wrapi(y0 - 2 + rj, ny);
    }
};

// Block decomposition shared by the fused kernels: tiles over x and y, chunks
// of `tz` planes over z.  Consecutive logical blocks share planes, so the
// hardware block id is remapped so that each of the 8 XCDs (which receive
// workgroups round-robin) walks a contiguous range of logical blocks and
// keeps the z-halo planes in its own L2.
struct TileGrid {
    int tiles_x, tiles_y, chunks_z, tz, total, launch;
};

inline TileGrid tile_grid(int nx, int ny, int nz, int TX, int TY, int tz)
{
    TileGrid g;
    g.tiles_x = (nx + TX - 1) / TX;
    g.tiles_y = (ny + TY - 1) / TY;
    g.tz = tz;
    g.chunks_z = (nz + tz - 1) / tz;
    g.total = g.tiles_x * g.tiles_y * g.chunks_z;
    g.launch = (g.total + 7) / 8 * 8;
    return g;
}

__device__ __forceinline__ int xcd_logical_block()
{
    const int per = gridDim.x >> 3;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

}  // namespace hlb
