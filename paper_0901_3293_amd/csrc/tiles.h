// tiles.h -- geometry of the 2.5D z-marching tiles used by the fused
// Q-side kernels.  A block owns a TX x TY column of sites and marches along z
// through a chunk of planes.  Quantities needed at stencil neighbours (the
// stress, the predictor stage) are evaluated on the tile plus a one-site halo
// ring, the "evaluation plane" of PX x PY points; every thread of the block
// owns one evaluation point for the whole march (threads [0, NT) the tile's
// own sites, [NT, PN) the ring, the last few none), so its z-neighbours can
// stay in registers.  Input planes are staged in LDS with a two-site halo.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace hlb {

template <int TX_, int TY_>
struct TileShape {
    static constexpr int TX = TX_, TY = TY_;
    static constexpr int NT = TX * TY;                  // tile sites
    static constexpr int RX = TX + 4, RY = TY + 4;      // staged input plane (halo 2)
    static constexpr int RN = RX * RY;
    static constexpr int PX = TX + 2, PY = TY + 2;      // evaluated plane (halo 1)
    static constexpr int PN = PX * PY;
    static constexpr int NH = PN - NT;                  // halo-ring points
    static constexpr int NB = (PN + 63) / 64 * 64;      // threads per block (whole waves)
    static_assert(NB <= 1024, "one evaluation point per thread");

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

// The tile of the fused Q-side kernels, per precision.  FP32: 32 x 8 sites
// (340 evaluation points, six waves; three blocks of the stress kernel or two
// of the Q update share a CU).  FP64: 16 x 12 sites (252 points, four waves):
// the FP64 kernels hold about 180 and 254 registers, two waves per SIMD, so
// two four-wave blocks share a CU where a six-wave block would run alone with
// a quarter of the CU's wave slots empty.
template <typename T>
using KernelTile = typename std::conditional<sizeof(T) == 8, TileShape<16, 12>, TileShape<32, 8>>::type;

__host__ __device__ __forceinline__ int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Index maps of the tile kernels, shared by the kernels and the host-side
// check of their halo coverage.
template <class S>
struct TileMap {
    // Tile site t in [0, NT): its place on the halo-1 plane (pc) and on the
    // staged plane (rc).
    __host__ __device__ static __forceinline__ void own(int t, int &pc, int &rc)
    {
        const int tx = t % S::TX, ty = t / S::TX;
        pc = (ty + 1) * S::PX + (tx + 1);
        rc = (ty + 2) * S::RX + (tx + 2);
    }
    // Halo-ring point t < NH on the halo-1 plane (hp) and on the staged plane
    // (hr); -1 otherwise.
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
    // Evaluation point of thread t of a block: tile site t for t < NT, ring
    // point t - NT for NT <= t < PN (pc, rc as above); returns false, with
    // pc = rc = -1, for the threads past PN.
    __host__ __device__ static __forceinline__ bool point(int t, int &pc, int &rc)
    {
        if (t < S::NT) {
            own(t, pc, rc);
            return true;
        }
        halo(t - S::NT, pc, rc);
        return pc >= 0;
    }
    // Thread t of a block stages the elements e = t + k NB (k = 0, 1, ...) of
    // a staged plane (component-major, RN points per component).  Since
    // NB <= RN, the elements of one k lie in component comp_base(k) for
    // t < comp_split(k) and in the next one above.
    static_assert(S::NB <= S::RN, "the elements of one k span at most two components");
    __host__ __device__ static constexpr int comp_base(int k) { return k * S::NB / S::RN; }
    __host__ __device__ static constexpr int comp_split(int k) { return (comp_base(k) + 1) * S::RN - k * S::NB; }
    // Element e of an NC-component staged plane: its component and its
    // in-plane offset in the lattice for a tile at (x0, y0), periodic wrap.
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
