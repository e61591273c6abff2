// kernels.hip -- HIP kernels of the hybrid step for gfx950 and their launchers.
//
// Data layout in HBM (structure-of-arrays, component-major, x fastest):
//   g[2]  19 x N  deviation populations g_i = f_i - w_i rho0 (ping-pong, pull)
//   Q[2]   5 x N  order parameter (xx, xy, xz, yy, yz); Q[qcur] is the state,
//                 the other copy holds the predictor stage or the next Q
//   u      3 x N  velocity of the last LB step
//   Pi    12 x N  chemical stress, 9 planes (its first 3 hold F in the tiled
//                 schedule), or the 12 planes of the split coupling (sigma^xi,
//                 tau, h; see sitekern.h)
// Scalars of one run are passed by value (Coef<T>).
//
// Five schedules of one step (Sec. 2.2), chosen per lattice and precision by
// the autotuner:
//  SITES (4 sweeps, one site per thread, neighbours through L2; 95 values
//  per site cross HBM):
//   k_stress  Q^n -> Pi;  k_lb  g, div Pi -> g', u^n;
//   k_qpred   Q^n, u^n -> Q*;  k_qcorr  Q*, u^n -> Q^{n+1} (in place)
//  TILED (3 sweeps; the stress and the predictor stage live in LDS of 2.5D
//  z-marching tiles and are recomputed on a one-site halo ring; 65 values):
//   k_qforce  Q^n -> F^n;  k_lbf  g, F^n -> g', u^n;  k_qupdate  Q^n, u^n -> Q^{n+1}
//  MIXED (3 sweeps: the per-site stress and LB, then the tiled Q update;
//  77 values):  k_stress, k_lb, k_qupdate
//  FUSED (3 sweeps: the stress of the tiles fused with the LB step, then the
//  per-site predictor and corrector; 77 values):
//   k_qlb  Q^n, g -> g', u^n;  k_qpred;  k_qcorr
//  FUSED_TILED (2 sweeps; 59 values):  k_qlb, k_qupdate
// The split coupling (Sec. 2.2) runs the SITES and MIXED schedules with
// k_stress / k_lb writing and reading the split terms (101 and 83 values),
// and the FUSED and FUSED_TILED schedules with k_qlb<T, true>, which
// evaluates them in its tiles (77 and 59 values).
// The population sweeps (k_lb, k_lbf, k_qlb, the second D3Q15 pass k_pc2)
// load and store the populations nontemporally, and the first D3Q15 pass
// k_pc1 stores its predicted populations so (pop_load / pop_store in
// sitekern.h).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "site.h"
#include "sitekern.h"
#include "tiles.h"

namespace hlb {

namespace {

constexpr int BLK = 256;  // per-site kernels

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int logical_block() { return xcd_logical_block(); }

// Fixed-order block reduction of NV doubles per thread into out[NV] (each
// round folds the upper part of the live range onto the lower one; for a
// power-of-two block this is the usual halving tree).
template <int NV, int NTH>
__device__ __forceinline__ void block_sum(double v[NV], double *out)
{
    __shared__ double buf[NV][NTH];
#pragma unroll
    for (int k = 0; k < NV; ++k) buf[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int n = NTH; n > 1;) {
        const int h = (n + 1) / 2;
        if (int(threadIdx.x) < n - h)
#pragma unroll
            for (int k = 0; k < NV; ++k) buf[k][threadIdx.x] += buf[k][threadIdx.x + h];
        __syncthreads();
        n = h;
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = buf[k][0];
}

// Debug mode of the tiled kernels: every LDS plane is overwritten with NaN
// (by all threads, independently of the loaders' element mapping) before the
// plane is staged or evaluated into it; the caller puts a workgroup barrier
// between the fill and the writes that follow.
template <typename T>
__device__ __forceinline__ void nan_fill(T *slot, int n)
{
    const T q = __builtin_nan("");
    for (int i = int(threadIdx.x); i < n; i += int(blockDim.x)) slot[i] = q;
}

// Staging of one z-plane of an NC-component field into an LDS slot with a
// two-site halo in x and y (periodic wrap of the global coordinates) by the
// NB threads of a block.  The element -> (component, in-plane offset)
// assignment is computed once per block.
template <class Shape, int NC>
struct PlaneLoader {
    static constexpr int NE = NC * Shape::RN;
    static constexpr int NL = (NE + Shape::NB - 1) / Shape::NB;
    // only the last k has elements past the end (t >= LAST)
    static constexpr int LAST = NE - (NL - 1) * Shape::NB;
    int off[NL];  // in-plane lattice offset of the element

    __device__ __forceinline__ void init(const Geom &G, int x0, int y0)
    {
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = int(threadIdx.x) + k * Shape::NB;
            int comp = 0;
            off[k] = 0;
            if (e < NE) TileMap<Shape>::staged(e, x0, y0, G.nx, G.ny, comp, off[k]);
        }
    }

    __device__ __forceinline__ static bool valid(int k) { return k < NL - 1 || int(threadIdx.x) < LAST; }

    template <typename T>
    __device__ __forceinline__ const T *elem(const T *__restrict__ src, size_t N, int plane_off, int k) const
    {
        const int cb = TileMap<Shape>::comp_base(k);
        const T *base = int(threadIdx.x) < TileMap<Shape>::comp_split(k) ? src + size_t(cb) * N : src + size_t(cb + 1) * N;
        return base + (plane_off + off[k]);
    }

    template <typename T>
    __device__ __forceinline__ void load(const T *__restrict__ src, size_t N, int plane_off,
                                         T *__restrict__ slot) const
    {
#pragma unroll
        for (int k = 0; k < NL; ++k)
            if (valid(k)) slot[int(threadIdx.x) + k * Shape::NB] = *elem(src, N, plane_off, k);
    }

    // Software pipelining: issue the global loads of a plane into registers
    // now, park them in LDS after the compute of the current plane.
    template <typename T>
    __device__ __forceinline__ void fetch(const T *__restrict__ src, size_t N, int plane_off, T reg[NL]) const
    {
#pragma unroll
        for (int k = 0; k < NL; ++k) reg[k] = valid(k) ? *elem(src, N, plane_off, k) : T(0);
    }

    template <typename T>
    __device__ __forceinline__ void store(const T reg[NL], T *__restrict__ slot) const
    {
#pragma unroll
        for (int k = 0; k < NL; ++k)
            if (valid(k)) slot[int(threadIdx.x) + k * Shape::NB] = reg[k];
    }
};

// Derivatives of the 5-component Q at staged coordinate r of plane p: the
// value and its in-plane neighbours from the staged slot `mid` (two-site
// halo, RN points per component), the z-neighbours from `lo` (plane p-1,
// registers of the thread owning the point) and the staged slot `hi`
// (plane p+1).
template <class Shape, typename T>
__device__ __forceinline__ void stencil_staged(const T lo[5], const T *mid, const T *hi, int r, T q[5],
                                               T d[3][5], T lap[5])
{
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int o = k * Shape::RN + r;
        const T v = mid[o];
        const T xp = mid[o + 1], xm = mid[o - 1];
        const T yp = mid[o + Shape::RX], ym = mid[o - Shape::RX];
        const T zp = hi[o], zm = lo[k];
        q[k] = v;
        d[0][k] = T(0.5) * (xp - xm);
        d[1][k] = T(0.5) * (yp - ym);
        d[2][k] = T(0.5) * (zp - zm);
        lap[k] = ((xp + xm) + (yp + ym)) + (zp + zm) - T(6) * v;
    }
}

// Same for the three-slot form (all of planes p-1, p, p+1 staged).
template <class Shape, typename T>
__device__ __forceinline__ void stencil_ring(const T *lo, const T *mid, const T *hi, int r, T q[5],
                                             T d[3][5], T lap[5])
{
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int o = k * Shape::RN + r;
        const T v = mid[o];
        const T xp = mid[o + 1], xm = mid[o - 1];
        const T yp = mid[o + Shape::RX], ym = mid[o - Shape::RX];
        const T zp = hi[o], zm = lo[o];
        q[k] = v;
        d[0][k] = T(0.5) * (xp - xm);
        d[1][k] = T(0.5) * (yp - ym);
        d[2][k] = T(0.5) * (zp - zm);
        lap[k] = ((xp + xm) + (yp + ym)) + (zp + zm) - T(6) * v;
    }
}

// Derivatives of a 5-component field held on the evaluation plane (PX x PY,
// PN points per component) at point r: value and in-plane neighbours from
// `mid`, z-neighbours from registers.
template <class Shape, typename T>
__device__ __forceinline__ void stencil_eval(const T lo[5], const T *mid, const T hi[5], int r, T q[5],
                                             T d[3][5], T lap[5])
{
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int o = k * Shape::PN + r;
        const T v = mid[o];
        const T xp = mid[o + 1], xm = mid[o - 1];
        const T yp = mid[o + Shape::PX], ym = mid[o - Shape::PX];
        const T zp = hi[k], zm = lo[k];
        q[k] = v;
        d[0][k] = T(0.5) * (xp - xm);
        d[1][k] = T(0.5) * (yp - ym);
        d[2][k] = T(0.5) * (zp - zm);
        lap[k] = ((xp + xm) + (yp + ym)) + (zp + zm) - T(6) * v;
    }
}

// u and its centred gradient W_ab = d_b u_a at staged coordinate r of plane
// p: in-plane from `mid`, z from `lo` (registers, plane p-1) and `hi`.
template <class Shape, typename T>
__device__ __forceinline__ void velocity_staged(const T lo[3], const T *mid, const T *hi, int r, T uc[3],
                                                T W[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int o = a * Shape::RN + r;
        uc[a] = mid[o];
        W[a][0] = T(0.5) * (mid[o + 1] - mid[o - 1]);
        W[a][1] = T(0.5) * (mid[o + Shape::RX] - mid[o - Shape::RX]);
        W[a][2] = T(0.5) * (hi[o] - lo[a]);
    }
}

struct Block {
    int x0, y0, z0, z1;
    bool ok;
};

template <class Shape>
__device__ __forceinline__ Block block_of(const Geom &G, const TileGrid &tg)
{
    Block b;
    const int lb = logical_block();
    b.ok = lb < tg.total;
    const int bx = lb % tg.tiles_x;
    const int by = (lb / tg.tiles_x) % tg.tiles_y;
    const int bz = lb / (tg.tiles_x * tg.tiles_y);
    b.x0 = bx * Shape::TX;
    b.y0 = by * Shape::TY;
    b.z0 = bz * tg.tz;
    b.z1 = min(b.z0 + tg.tz, G.nz);
    return b;
}

// ---------------------------------------------------------------- k_qforce
// F = div Pi(Q) (Eqs. (6)-(8), (19)).  Every thread owns one point of the
// evaluation plane (a tile site or a ring point).  Per plane p: evaluate the
// stress at the own point from the staged planes p-1, p, p+1 (ring points
// only where a tile site needs them), keep its z column in registers and put
// its x and y columns into one of two LDS buffers; the tile threads finish
// F(p-1) from the other buffer (the stress of plane p-1) and the z columns of
// planes p and p-2, and the plane p+2, fetched into registers at the start,
// goes into the fourth staging slot.  One barrier per plane: no slot or
// buffer is written in the plane in which it is read.  With WITH_F the block
// also sums the free-energy density of its sites.
// FP32: at most 96 registers, five waves per SIMD (three blocks per CU).  In
// FP64 (about 180 registers, two four-wave blocks per CU) a bound that would
// let a third block in spills (36 bytes per lane); with six-wave blocks such
// a bound spilled and ran slower.
template <typename T, bool WITH_F>
__global__ __launch_bounds__(KernelTile<T>::NB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 1 : 5))) void k_qforce(Geom G, Coef<T> c, TileGrid tg,
                                                      const T *__restrict__ Q, T *__restrict__ F,
                                                      double *__restrict__ fpart, bool dbg_nan)
{
    using Shape = KernelTile<T>;
    __shared__ T sQ[4][5 * Shape::RN];
    __shared__ T sP[2][6 * Shape::PN];
    const Block B = block_of<Shape>(G, tg);
    if (!B.ok) return;
    if (dbg_nan) {
        nan_fill(&sQ[0][0], 4 * 5 * Shape::RN);
        nan_fill(&sP[0][0], 2 * 6 * Shape::PN);
        __syncthreads();
    }
    const size_t N = G.N;
    const int sxy = G.nx * G.ny;
    const int t = int(threadIdx.x);
    int pc, rc;
    const bool eval = TileMap<Shape>::point(t, pc, rc);
    const bool tile = t < Shape::NT;
    const int gx = B.x0 + t % Shape::TX, gy = B.y0 + t / Shape::TX;
    const bool mine = tile && gx < G.nx && gy < G.ny;

    PlaneLoader<Shape, 5> L;
    L.init(G, B.x0, B.y0);
    int s0 = 0, s1 = 1, s2 = 2, s3 = 3;  // s1, s2, s3: planes p-1, p, p+1; s0 free
    L.load(Q, N, wrapi(B.z0 - 2, G.nz) * sxy, sQ[s1]);
    L.load(Q, N, wrapi(B.z0 - 1, G.nz) * sxy, sQ[s2]);
    L.load(Q, N, wrapi(B.z0, G.nz) * sxy, sQ[s3]);
    __syncthreads();

    T Pz1[3] = {T(0), T(0), T(0)}, Pz2[3] = {T(0), T(0), T(0)};
    double facc = 0.0;
    constexpr int NL = PlaneLoader<Shape, 5>::NL;
    T pre[NL];
    for (int p = B.z0 - 1; p <= B.z1; ++p) {
        const bool more = p + 2 <= B.z1 + 1;
        if (more) L.fetch(Q, N, wrapi(p + 2, G.nz) * sxy, pre);
        T *Pc = sP[p & 1];        // stress of plane p (written now)
        const T *Pp = sP[~p & 1];  // stress of plane p-1 (written in the last plane)
        T Pz[3] = {T(0), T(0), T(0)};
        // ring points: only the planes whose in-plane divergence is output
        if (eval && (tile || (p >= B.z0 && p < B.z1))) {
            T q[5], d[3][5], lap[5], P[3][3], fd, H[5];
            stencil_ring<Shape>(sQ[s1], sQ[s2], sQ[s3], rc, q, d, lap);
            site_stress(c, q, d, lap, P, fd, H);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Pc[a * Shape::PN + pc] = P[a][0];
                Pc[(3 + a) * Shape::PN + pc] = P[a][1];
                Pz[a] = P[a][2];
            }
            if (WITH_F && mine && p >= B.z0 && p < B.z1) facc += double(fd);
        }
        if (tile) {
            if (mine && p - 1 >= B.z0) {
                const size_t o = size_t(p - 1) * sxy + size_t(gy) * G.nx + gx;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const T Fin = (Pp[a * Shape::PN + pc + 1] - Pp[a * Shape::PN + pc - 1])
                                + (Pp[(3 + a) * Shape::PN + pc + Shape::PX] - Pp[(3 + a) * Shape::PN + pc - Shape::PX]);
                    F[a * N + o] = T(0.5) * (Fin + (Pz[a] - Pz2[a]));
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Pz2[a] = Pz1[a];
                Pz1[a] = Pz[a];
            }
        }
        if (dbg_nan) {  // the free slot and the stress of plane p-1 are no longer read
            __syncthreads();
            nan_fill(sQ[s0], 5 * Shape::RN);
            nan_fill(const_cast<T *>(Pp), 6 * Shape::PN);
            __syncthreads();
        }
        if (more) L.store(pre, sQ[s0]);  // plane p+2 into the free slot
        __syncthreads();
        const int o = s0;
        s0 = s1;
        s1 = s2;
        s2 = s3;
        s3 = o;
    }
    if (WITH_F) {
        double v[1] = {facc};
        block_sum<1, Shape::NB>(v, fpart + logical_block());
    }
}

// ---------------------------------------------------------------- k_qlb
// The stress kernel fused with the LB step (Eqs. (6)-(8), (19) with the
// collision and streaming of Sec. 2.2): the plane march of k_qforce, but
// instead of writing F(p-1) each tile thread collides its site of plane p-1
// with it, pulling the populations from gin and writing gout and u^n, so F
// never goes to HBM.  The 19 pulled populations are loaded at the start of
// the plane and arrive while the stress is evaluated (loaded after it, the
// FP64 kernel ran 4% slower).
// SPLIT (Eqs. (17)-(21)): the evaluation gives sigma^xi, tau and h; the LDS
// buffers hold tau (xy, xz, yz) for the in-plane differences of the body
// force b_a = d_b tau_ab + h_a, and a tile thread keeps sigma^xi and h of its
// site of plane p-1 in registers for the collision with sigma^xi in the
// equilibrium.
// FP32: at most 128 registers (four waves per SIMD, two blocks per CU); FP64:
// about 230 (two waves per SIMD, two four-wave blocks per CU).
template <typename T, bool SPLIT>
__global__ __launch_bounds__(KernelTile<T>::NB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 1 : 4))) void k_qlb(Geom G, Coef<T> c, TileGrid tg,
                                                      const T *__restrict__ Q, const T *__restrict__ gin,
                                                      T *__restrict__ gout, T *__restrict__ u, bool dbg_nan)
{
    using Shape = KernelTile<T>;
    __shared__ T sQ[4][5 * Shape::RN];
    __shared__ T sP[2][6 * Shape::PN];
    const Block B = block_of<Shape>(G, tg);
    if (!B.ok) return;
    if (dbg_nan) {
        nan_fill(&sQ[0][0], 4 * 5 * Shape::RN);
        nan_fill(&sP[0][0], 2 * 6 * Shape::PN);
        __syncthreads();
    }
    const int N = G.N;
    const int sxy = G.nx * G.ny;
    const int t = int(threadIdx.x);
    int pc, rc;
    const bool eval = TileMap<Shape>::point(t, pc, rc);
    const bool tile = t < Shape::NT;
    const int gx = B.x0 + t % Shape::TX, gy = B.y0 + t / Shape::TX;
    const bool mine = tile && gx < G.nx && gy < G.ny;

    PlaneLoader<Shape, 5> L;
    L.init(G, B.x0, B.y0);
    int s0 = 0, s1 = 1, s2 = 2, s3 = 3;  // s1, s2, s3: planes p-1, p, p+1; s0 free
    L.load(Q, size_t(N), wrapi(B.z0 - 2, G.nz) * sxy, sQ[s1]);
    L.load(Q, size_t(N), wrapi(B.z0 - 1, G.nz) * sxy, sQ[s2]);
    L.load(Q, size_t(N), wrapi(B.z0, G.nz) * sxy, sQ[s3]);
    __syncthreads();

    // z columns of the own point at planes p-1 and p-2: Pi_az, or (SPLIT) tau xz, yz
    T Pz1[3] = {T(0), T(0), T(0)}, Pz2[3] = {T(0), T(0), T(0)};
    T sig1[6], h1[3];  // SPLIT: sigma^xi and h of the own site at plane p-1
    constexpr int NL = PlaneLoader<Shape, 5>::NL;
    T pre[NL];
    for (int p = B.z0 - 1; p <= B.z1; ++p) {
        const bool more = p + 2 <= B.z1 + 1;
        if (more) L.fetch(Q, size_t(N), wrapi(p + 2, G.nz) * sxy, pre);
        const bool lb = mine && p - 1 >= B.z0;  // this plane collides site (gx, gy, p-1)
        Off<T> O;
        T g[19];
        if (lb) {
            O = offsets<T>(nbr_at(G, (p - 1) * sxy + gy * G.nx + gx, gx, gy, p - 1));
#pragma unroll
            for (int i = 0; i < 19; ++i) g[i] = pop_load<true>(plane(gin, i, N), pull_off(O, CX[i], CY[i], CZ[i]));
        }
        T *Pc = sP[p & 1];         // stress (tau) of plane p (written now)
        const T *Pp = sP[~p & 1];  // stress (tau) of plane p-1 (written in the last plane)
        T Pz[3] = {T(0), T(0), T(0)};
        T sig0[6], h0[3];
        // ring points: only the planes whose in-plane divergence is used
        if (eval && (tile || (p >= B.z0 && p < B.z1))) {
            T q[5], d[3][5], lap[5], fd;
            stencil_ring<Shape>(sQ[s1], sQ[s2], sQ[s3], rc, q, d, lap);
            if constexpr (SPLIT) {
                T tau3[3];
                site_split(c, q, d, lap, sig0, tau3, h0, fd);
#pragma unroll
                for (int k = 0; k < 3; ++k) Pc[k * Shape::PN + pc] = tau3[k];
                Pz[0] = tau3[1];
                Pz[1] = tau3[2];
            } else {
                T P[3][3], H[5];
                site_stress(c, q, d, lap, P, fd, H);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    Pc[a * Shape::PN + pc] = P[a][0];
                    Pc[(3 + a) * Shape::PN + pc] = P[a][1];
                    Pz[a] = P[a][2];
                }
            }
        }
        if (tile) {
            if (lb) {
                T f[3], uu[3], rho;
                if constexpr (SPLIT) {
                    // b_a = d_b tau_ab + h_a at plane p-1: in-plane differences from LDS,
                    // z differences from the own point's tau at planes p and p-2
                    const T *txy = Pp, *txz = Pp + Shape::PN, *tyz = Pp + 2 * Shape::PN;
                    f[0] = T(0.5) * ((txy[pc + Shape::PX] - txy[pc - Shape::PX]) + (Pz[0] - Pz2[0])) + h1[0];
                    f[1] = T(0.5) * ((Pz[1] - Pz2[1]) - (txy[pc + 1] - txy[pc - 1])) + h1[1];
                    f[2] = T(0.5) * (-(txz[pc + 1] - txz[pc - 1]) - (tyz[pc + Shape::PX] - tyz[pc - Shape::PX])) +
                           h1[2];
                    lb_collide_split(c, g, f, sig1, uu, rho);
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const T Fin = (Pp[a * Shape::PN + pc + 1] - Pp[a * Shape::PN + pc - 1])
                                    + (Pp[(3 + a) * Shape::PN + pc + Shape::PX] - Pp[(3 + a) * Shape::PN + pc - Shape::PX]);
                        f[a] = T(0.5) * (Fin + (Pz[a] - Pz2[a]));
                    }
                    lb_collide(c, g, f, uu, rho);
                }
#pragma unroll
                for (int i = 0; i < 19; ++i) pop_store<true>(plane(gout, i, N), O.s, g[i]);
#pragma unroll
                for (int a = 0; a < 3; ++a) *at(plane(u, a, N), O.s) = uu[a];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Pz2[a] = Pz1[a];
                Pz1[a] = Pz[a];
            }
            if constexpr (SPLIT) {
#pragma unroll
                for (int k = 0; k < 6; ++k) sig1[k] = sig0[k];
#pragma unroll
                for (int a = 0; a < 3; ++a) h1[a] = h0[a];
            }
        }
        if (dbg_nan) {  // the free slot and the stress of plane p-1 are no longer read
            __syncthreads();
            nan_fill(sQ[s0], 5 * Shape::RN);
            nan_fill(const_cast<T *>(Pp), 6 * Shape::PN);
            __syncthreads();
        }
        if (more) L.store(pre, sQ[s0]);  // plane p+2 into the free slot
        __syncthreads();
        const int o = s0;
        s0 = s1;
        s1 = s2;
        s2 = s3;
        s3 = o;
    }
}

// ---------------------------------------------------------------- k_qupdate
// Predictor-corrector for the Q equation with u held at u^n (Eqs. (2)-(4)):
//   Q* = Q + R(Q, u),  Q' = [Q + Q* + R(Q*, u)] / 2   (= Q + [R(Q) + R(Q*)]/2).
// Every thread owns one point of the evaluation plane.  Per plane p: the
// predictor stage Q*(p) at the own point (in-plane stencil from the staged
// plane p, z-neighbours from the registers holding Q(p-1), u(p-1) and the
// staged plane p+1; ring points only where a tile site needs them); then on
// the tile threads the corrector at plane p-1 from Q*(p-1) in LDS and
// Q*(p-2), Q*(p) in registers, with u(p-1) and W(p-1) kept from the
// predictor of plane p-1.  FP32: Q*(p) goes into the other of two LDS
// buffers and the plane p+2, fetched into registers at the start, into the
// third staging slot, so a plane takes one barrier.  FP64 (where three slots
// and two buffers would not leave LDS for two blocks per CU): after a barrier
// Q*(p) replaces Q*(p-1) in LDS and the plane p+2 replaces plane p, and a
// second barrier ends the plane.
template <typename T>
__global__ __launch_bounds__(KernelTile<T>::NB) void k_qupdate(Geom G, Coef<T> c, TileGrid tg,
                                                       const T *__restrict__ Qin, const T *__restrict__ u,
                                                       T *__restrict__ Qout, bool dbg_nan)
{
    using Shape = KernelTile<T>;
    constexpr bool ONE = sizeof(T) == 4;      // one barrier per plane
    constexpr int NQS = ONE ? 3 : 2, NSS = ONE ? 2 : 1;
    __shared__ T sQ[NQS][5 * Shape::RN];
    __shared__ T sU[NQS][3 * Shape::RN];
    __shared__ T sS[NSS][5 * Shape::PN];
    const Block B = block_of<Shape>(G, tg);
    if (!B.ok) return;
    if (dbg_nan) {
        nan_fill(&sQ[0][0], NQS * 5 * Shape::RN);
        nan_fill(&sU[0][0], NQS * 3 * Shape::RN);
        nan_fill(&sS[0][0], NSS * 5 * Shape::PN);
        __syncthreads();
    }
    const size_t N = G.N;
    const int sxy = G.nx * G.ny;
    const int t = int(threadIdx.x);
    int pc, rc;
    const bool eval = TileMap<Shape>::point(t, pc, rc);
    const bool tile = t < Shape::NT;
    const int gx = B.x0 + t % Shape::TX, gy = B.y0 + t / Shape::TX;
    const bool mine = tile && gx < G.nx && gy < G.ny;

    PlaneLoader<Shape, 5> LQ;
    PlaneLoader<Shape, 3> LU;
    LQ.init(G, B.x0, B.y0);
    LU.init(G, B.x0, B.y0);
    int sc = 0, sn = 1, sf = NQS - 1;  // slots of planes p, p+1; FP32: the free slot
    LQ.load(Qin, N, wrapi(B.z0 - 1, G.nz) * sxy, sQ[sc]);
    LQ.load(Qin, N, wrapi(B.z0, G.nz) * sxy, sQ[sn]);
    LU.load(u, N, wrapi(B.z0 - 1, G.nz) * sxy, sU[sc]);
    LU.load(u, N, wrapi(B.z0, G.nz) * sxy, sU[sn]);
    // Plane state of the own point in two register sets: one holds Q, u and,
    // on tile sites, W of plane p-1, the other receives those of plane p.  In
    // FP32 they swap roles from one plane to the next (the loop below is
    // unrolled by two); in FP64 the new set is copied over the old.  First Q
    // and u of plane z0 - 2 (the ring's first predictor is at plane z0).
    T qA[5] = {T(0), T(0), T(0), T(0), T(0)}, uA[3] = {T(0), T(0), T(0)}, WA[3][3], qB[5], uB[3], WB[3][3];
    if (tile) {
        const int o = wrapi(B.z0 - 2, G.nz) * sxy + wrapi(B.x0 - 2 + rc % Shape::RX, G.nx)
                    + G.nx * wrapi(B.y0 - 2 + rc / Shape::RX, G.ny);
#pragma unroll
        for (int k = 0; k < 5; ++k) qA[k] = Qin[size_t(k) * N + o];
#pragma unroll
        for (int a = 0; a < 3; ++a) uA[a] = u[size_t(a) * N + o];
    }
    __syncthreads();

    T qs2[5] = {T(0), T(0), T(0), T(0), T(0)};  // Q* at the own site, plane p-2
    constexpr int NQ = PlaneLoader<Shape, 5>::NL, NU = PlaneLoader<Shape, 3>::NL;
    T preQ[NQ], preU[NU];
    auto plane = [&](int p, const T (&qmm)[5], const T (&umm)[3], const T (&Wmm)[3][3], T (&q0)[5], T (&u0)[3],
                     T (&W0)[3][3]) __attribute__((always_inline)) {
        const bool more = p + 2 <= B.z1 + 1;
        if (more) {
            LQ.fetch(Qin, N, wrapi(p + 2, G.nz) * sxy, preQ);
            LU.fetch(u, N, wrapi(p + 2, G.nz) * sxy, preU);
        }
        T qs0[5];
        T *Scur = sS[ONE ? (p & 1) : 0];         // receives Q*(p)
        const T *Sprev = sS[ONE ? (~p & 1) : 0];  // holds Q*(p-1)
        if (eval) {
#pragma unroll
            for (int k = 0; k < 5; ++k) q0[k] = sQ[sc][k * Shape::RN + rc];
#pragma unroll
            for (int a = 0; a < 3; ++a) u0[a] = sU[sc][a * Shape::RN + rc];
        }
        const bool pred = eval && (tile || (p >= B.z0 && p < B.z1));
        if (pred) {
            T q[5], d[3][5], lap[5], uc[3], R[5];
            stencil_staged<Shape>(qmm, sQ[sc], sQ[sn], rc, q, d, lap);
            velocity_staged<Shape>(umm, sU[sc], sU[sn], rc, uc, W0);
            site_rhs(c, q, d, lap, uc, W0, R);
#pragma unroll
            for (int k = 0; k < 5; ++k) qs0[k] = q[k] + R[k];
            if (ONE)
#pragma unroll
                for (int k = 0; k < 5; ++k) Scur[k * Shape::PN + pc] = qs0[k];
        }
        if (tile && p - 1 >= B.z0) {
            T q[5], d[3][5], lap[5], R[5];
            stencil_eval<Shape>(qs2, Sprev, qs0, pc, q, d, lap);
            site_rhs(c, q, d, lap, umm, Wmm, R);
            if (mine) {
                const size_t o = size_t(p - 1) * sxy + size_t(gy) * G.nx + gx;
#pragma unroll
                for (int k = 0; k < 5; ++k) Qout[k * N + o] = T(0.5) * (qmm[k] + q[k] + R[k]);
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) qs2[k] = q[k];
        } else if (tile && p == B.z0) {
            // Q*(z0 - 1) is not corrected but is the z-neighbour of the corrector at z0
#pragma unroll
            for (int k = 0; k < 5; ++k) qs2[k] = Sprev[k * Shape::PN + pc];
        }
        if constexpr (ONE) {
            if (dbg_nan) {  // the free slots and Q*(p-1) are no longer read
                __syncthreads();
                nan_fill(sQ[sf], 5 * Shape::RN);
                nan_fill(sU[sf], 3 * Shape::RN);
                nan_fill(const_cast<T *>(Sprev), 5 * Shape::PN);
                __syncthreads();
            }
            if (more) {
                LQ.store(preQ, sQ[sf]);
                LU.store(preU, sU[sf]);
            }
            __syncthreads();
            const int o = sc;
            sc = sn;
            sn = sf;
            sf = o;
        } else {
            __syncthreads();  // plane p, Q*(p-1) are no longer read
            if (dbg_nan) {
                nan_fill(sQ[sc], 5 * Shape::RN);
                nan_fill(sU[sc], 3 * Shape::RN);
                nan_fill(Scur, 5 * Shape::PN);
                __syncthreads();
            }
            if (pred)
#pragma unroll
                for (int k = 0; k < 5; ++k) Scur[k * Shape::PN + pc] = qs0[k];
            if (more) {
                LQ.store(preQ, sQ[sc]);
                LU.store(preU, sU[sc]);
            }
            __syncthreads();
            const int o = sc;
            sc = sn;
            sn = o;
        }
    };
    int p = B.z0 - 1;
    if constexpr (sizeof(T) == 4) {
        for (; p + 1 <= B.z1; p += 2) {
            plane(p, qA, uA, WA, qB, uB, WB);
            plane(p + 1, qB, uB, WB, qA, uA, WA);
        }
        if (p <= B.z1) plane(p, qA, uA, WA, qB, uB, WB);
    } else {
        // FP64: a second copy of the plane code costs more registers than the
        // copies of the plane state it saves
        for (; p <= B.z1; ++p) {
            plane(p, qA, uA, WA, qB, uB, WB);
#pragma unroll
            for (int k = 0; k < 5; ++k) qA[k] = qB[k];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                uA[a] = uB[a];
#pragma unroll
                for (int b2 = 0; b2 < 3; ++b2) WA[a][b2] = WB[a][b2];
            }
        }
    }
}

// ---------------------------------------------------------------- per-site kernels

__device__ __forceinline__ int site_index() { return logical_block() * BLK + int(threadIdx.x); }

// SPLIT: the 12 planes of the split coupling instead of the 9 of Pi.
// Occupancy floors of the per-site Q-side kernels in FP64 (blocks of 256 per
// CU): registers bounded to 128 (stress, corrector) and 96 (predictor)
// without spills, 4 and 5 waves per SIMD.  FP32 is left to the compiler
// (~60 registers, 8 waves).
template <typename T, bool SPLIT>
__global__ __launch_bounds__(BLK, sizeof(T) == 8 ? 4 : 1) void k_stress(Geom G, Coef<T> c, const T *__restrict__ Q,
                                                T *__restrict__ Pi, double *__restrict__ fpart)
{
    const int s = site_index();
    double fsum = 0.0;
    if (s < G.N) fsum = double(SPLIT ? split_at(G, c, Q, Pi, s) : stress_at(G, c, Q, Pi, s));
    if (fpart) {
        double v[1] = {fsum};
        block_sum<1, BLK>(v, fpart + logical_block());
    }
}

template <typename T, bool SPLIT>
__global__ __launch_bounds__(BLK) void k_lb(Geom G, Coef<T> c, const T *__restrict__ gin,
                                            const T *__restrict__ Pi, T *__restrict__ gout, T *__restrict__ u)
{
    const int s = site_index();
    if (s >= G.N) return;
    if (SPLIT)
        lb_split_at<T, true>(G, c, gin, Pi, gout, u, s);
    else
        lb_at<T, true>(G, c, gin, Pi, gout, u, s);
}

template <typename T>
__global__ __launch_bounds__(BLK, sizeof(T) == 8 ? 5 : 1) void k_qpred(Geom G, Coef<T> c, const T *__restrict__ Q,
                                               const T *__restrict__ u, T *__restrict__ Qs)
{
    const int s = site_index();
    if (s < G.N) pred_at(G, c, Q, u, Qs, s);
}

template <typename T>
__global__ __launch_bounds__(BLK, sizeof(T) == 8 ? 4 : 1) void k_qcorr(Geom G, Coef<T> c, T *__restrict__ Q, const T *__restrict__ Qs,
                                               const T *__restrict__ u)
{
    const int s = site_index();
    if (s < G.N) corr_at(G, c, Q, Qs, u, s);
}

// D3Q15 predictor-corrector LB, the two passes (see pc1_at, pc2_at).
template <typename T, bool SPLIT>
__global__ __launch_bounds__(BLK) void k_pc1(Geom G, Coef<T> c, const T *__restrict__ g, const T *__restrict__ Pi,
                                             T *__restrict__ P, T *__restrict__ u, T *__restrict__ bsave)
{
    const int s = site_index();
    if (s < G.N) pc1_at<T, SPLIT, true>(G, c, g, Pi, P, u, bsave, s);
}

template <typename T, bool SPLIT>
__global__ __launch_bounds__(BLK) void k_pc2(Geom G, Coef<T> c, const T *__restrict__ g, const T *__restrict__ P,
                                             const T *__restrict__ Pi, const T *__restrict__ bsave,
                                             T *__restrict__ gout)
{
    const int s = site_index();
    if (s < G.N) pc2_at<T, SPLIT, true>(G, c, g, P, Pi, bsave, gout, s);
}

// D3Q15 state from (rho, u): g_i(x) = f_i^eq(rho(x), u(x)) - A_s(rho0) in
// place, without stress or force terms; Q converted to the storage type.
template <typename T>
__global__ __launch_bounds__(BLK) void k_init15(Geom G, Coef<T> c, const double *__restrict__ rho_in,
                                                const double *__restrict__ u_in, const double *__restrict__ Q_in,
                                                T *__restrict__ g, T *__restrict__ Q)
{
    const int s = site_index();
    if (s >= G.N) return;
    const size_t N = G.N;
    const T uu3[3] = {T(u_in[s]), T(u_in[N + s]), T(u_in[2 * N + s])};
    const T uu = uu3[0] * uu3[0] + uu3[1] * uu3[1] + uu3[2] * uu3[2];
#pragma unroll
    for (int i = 0; i < 15; ++i) g[i * N + s] = lb15_eq(i, c.rho0, T(rho_in[s]), uu3, uu, static_cast<const T *>(nullptr));
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k * N + s] = T(Q_in[k * N + s]);
}

// D3Q15 readout: rho and u = sum f e / rho of the stored populations
// (Eq. (14); u == 0 with the flow off), Q in FP64, FP64 block partials.
template <typename T>
__global__ __launch_bounds__(BLK) void k_readout15(Geom G, Coef<T> c, const T *__restrict__ g, bool flow,
                                                   const T *__restrict__ Q, double *__restrict__ rho_out,
                                                   double *__restrict__ u_out, double *__restrict__ Q_out,
                                                   double *__restrict__ part)
{
    const int s = site_index();
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (s < G.N) {
        const size_t N = G.N;
        T drho = T(0), j[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int i = 0; i < 15; ++i) {
            const T f = g[i * N + s];
            drho += f;
            j[0] += T(DX15[i]) * f;
            j[1] += T(DY15[i]) * f;
            j[2] += T(DZ15[i]) * f;
        }
        const T rho = c.rho0 + drho;
        if (rho_out) rho_out[s] = double(rho);
        if (u_out)
#pragma unroll
            for (int a = 0; a < 3; ++a) u_out[a * N + s] = flow ? double(j[a] / rho) : 0.0;
        if (Q_out)
#pragma unroll
            for (int k = 0; k < 5; ++k) Q_out[k * N + s] = double(Q[k * N + s]);
        v[0] = double(drho);
        if (flow)
#pragma unroll
            for (int a = 0; a < 3; ++a) v[1 + a] = double(j[a]);
    }
    if (part) block_sum<4, BLK>(v, part + 4 * logical_block());
}

// LB with a precomputed body force (tiled schedule).
template <typename T>
__global__ __launch_bounds__(BLK) void k_lbf(Geom G, Coef<T> c, const T *__restrict__ gin,
                                             const T *__restrict__ F, T *__restrict__ gout, T *__restrict__ u)
{
    const int s = site_index();
    if (s >= G.N) return;
    const int N = G.N;
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T g[19], f[3], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 19; ++i) g[i] = pop_load<true>(plane(gin, i, N), pull_off(O, CX[i], CY[i], CZ[i]));
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = *at(plane(F, a, N), O.s);
    lb_collide(c, g, f, uu, rho);
#pragma unroll
    for (int i = 0; i < 19; ++i) pop_store<true>(plane(gout, i, N), O.s, g[i]);
#pragma unroll
    for (int a = 0; a < 3; ++a) *at(plane(u, a, N), O.s) = uu[a];
}

// Populations such that the first pull returns g^eq(rho(x), u(x)):
// g_i(y) = g_i^eq(rho(y + e_i), u(y + e_i)); Q converted to the storage type.
template <typename T>
__global__ __launch_bounds__(BLK) void k_init(Geom G, Coef<T> c, const double *__restrict__ rho_in,
                                              const double *__restrict__ u_in,
                                              const double *__restrict__ Q_in, T *__restrict__ g,
                                              T *__restrict__ Q)
{
    const int s = site_index();
    if (s >= G.N) return;
    const size_t N = G.N;
    const Nbr S = nbr_of(G, s);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const int t = pull_from(G, S, -CX[i], -CY[i], -CZ[i]);
        const T uu[3] = {T(u_in[t]), T(u_in[N + t]), T(u_in[2 * N + t])};
        g[i * N + s] = lb_geq(c, i, T(rho_in[t]), uu);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k * N + s] = T(Q_in[k * N + s]);
}

// Current-level readout: rho, u = (j + F/2)/rho with F = div Pi, or the split
// body force b (u == 0 when Pi is null, i.e. flow off) and Q in FP64; FP64
// block partials of (rho - rho0, rho u_x, rho u_y, rho u_z).
template <typename T, bool SPLIT>
__global__ __launch_bounds__(BLK) void k_readout(Geom G, Coef<T> c, const T *__restrict__ g,
                                                 const T *__restrict__ Pi, const T *__restrict__ Q,
                                                 double *__restrict__ rho_out, double *__restrict__ u_out,
                                                 double *__restrict__ Q_out, double *__restrict__ part)
{
    const int s = site_index();
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (s < G.N) {
        const size_t N = G.N;
        const Nbr S = nbr_of(G, s);
        T gg[19], drho, j[3], f[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int i = 0; i < 19; ++i) gg[i] = g[i * N + pull_from(G, S, CX[i], CY[i], CZ[i])];
        lb_moments(gg, drho, j);
        if (Pi) {
            const Off<T> O = offsets<T>(S);
            if (SPLIT)
                split_force(Pi, G.N, O, f);
            else
                divergence(Pi, G.N, O, f);
        }
        const T rho = c.rho0 + drho;
        T uu[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) uu[a] = Pi ? (j[a] + T(0.5) * f[a]) / rho : T(0);
        if (rho_out) rho_out[s] = double(rho);
        if (u_out)
#pragma unroll
            for (int a = 0; a < 3; ++a) u_out[a * N + s] = double(uu[a]);
        if (Q_out)
#pragma unroll
            for (int k = 0; k < 5; ++k) Q_out[k * N + s] = double(Q[k * N + s]);
        v[0] = double(drho);
        if (Pi)
#pragma unroll
            for (int a = 0; a < 3; ++a) v[1 + a] = double(j[a]) + 0.5 * double(f[a]);
    }
    if (part) block_sum<4, BLK>(v, part + 4 * logical_block());
}

// Second stage: out[k] = sum_b part[b*stride + k], fixed order, one block.
__global__ __launch_bounds__(BLK) void k_reduce(const double *__restrict__ part, int nblk, int nv,
                                                int stride, double *__restrict__ out)
{
    __shared__ double buf[BLK];
    for (int k = 0; k < nv; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += BLK) s += part[b * stride + k];
        buf[threadIdx.x] = s;
        __syncthreads();
        for (int w = BLK / 2; w > 0; w >>= 1) {
            if (int(threadIdx.x) < w) buf[threadIdx.x] += buf[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = buf[0];
        __syncthreads();
    }
}

// Plane sums of the free-energy density: block z sums plane z in a fixed
// order (FP64), so the profile f(z) is deterministic.
template <typename T>
__global__ __launch_bounds__(BLK) void k_fz(Geom G, Coef<T> c, const T *__restrict__ Q, double *__restrict__ fz)
{
    const int z = blockIdx.x;
    const int sxy = G.nx * G.ny;
    double acc = 0.0;
    for (int k = threadIdx.x; k < sxy; k += BLK) acc += double(fdens_at(G, c, Q, z * sxy + k));
    double v[1] = {acc};
    block_sum<1, BLK>(v, fz + z);
}

// Largest eigenvalue of a symmetric traceless 3x3 tensor and a unit
// eigenvector of it, in FP64 (local order, Sec. 2.1; director, Sec. 2.3), by
// the cyclic Jacobi method: plane rotations over the pairs (0,1), (0,2),
// (1,2), each zeroing its off-diagonal entry (tangent of the smaller rotation
// angle), repeated until the off-diagonal mass is below 1e-30 of the squared
// norm (at most 8 sweeps; 4 suffice in practice).  Unlike the closed form of
// the characteristic cubic, whose double roots lose half the digits, this
// keeps every eigenvalue within a few ulps of |Q|.  The director is the
// rotation's column of the largest diagonal entry, signed so that its last
// non-zero component is positive.  Q = 0 gives 0 and (0, 0, 1).
__device__ __forceinline__ void order_site(const double q[5], double &lam, double d[3])
{
    double A[3][3] = {{q[0], q[1], q[2]}, {q[1], q[3], q[4]}, {q[2], q[4], -q[0] - q[3]}};
    double V[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
    double nrm = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) nrm += A[a][b] * A[a][b];
    if (!(nrm > 0.0)) {
        lam = 0.0;
        d[0] = 0.0;
        d[1] = 0.0;
        d[2] = 1.0;
        return;
    }
    const int P[3] = {0, 0, 1}, R[3] = {1, 2, 2};
#pragma unroll 1
    for (int sweep = 0; sweep < 8; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        if (!(off > 1e-30 * nrm)) break;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int p = P[k], r = R[k];
            const double apr = A[p][r];
            if (apr == 0.0) continue;
            const double th = (A[r][r] - A[p][p]) / (2.0 * apr);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double amp = A[m][p], amr = A[m][r];
                A[m][p] = c * amp - sn * amr;
                A[m][r] = sn * amp + c * amr;
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double apm = A[p][m], arm = A[r][m];
                A[p][m] = c * apm - sn * arm;
                A[r][m] = sn * apm + c * arm;
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double vmp = V[m][p], vmr = V[m][r];
                V[m][p] = c * vmp - sn * vmr;
                V[m][r] = sn * vmp + c * vmr;
            }
        }
    }
    int k = 0;
    if (A[1][1] > A[k][k]) k = 1;
    if (A[2][2] > A[k][k]) k = 2;
    lam = A[k][k];
    const double v0 = V[0][k], v1 = V[1][k], v2 = V[2][k];
    const double sgn = (v2 != 0.0 ? v2 : (v1 != 0.0 ? v1 : v0)) < 0.0 ? -1.0 : 1.0;
    d[0] = sgn * v0;
    d[1] = sgn * v1;
    d[2] = sgn * v2;
}

// Local order q, director and disclination flag (q < threshold) per site;
// any output may be null.
template <typename T>
__global__ __launch_bounds__(BLK) void k_order(Geom G, const T *__restrict__ Q, double threshold,
                                               double *__restrict__ qo, double *__restrict__ dir,
                                               unsigned char *__restrict__ defect)
{
    const int s = site_index();
    if (s >= G.N) return;
    const size_t N = G.N;
    double q[5], lam, d[3];
#pragma unroll
    for (int k = 0; k < 5; ++k) q[k] = double(Q[k * N + s]);
    order_site(q, lam, d);
    if (qo) qo[s] = lam;
    if (dir)
#pragma unroll
        for (int a = 0; a < 3; ++a) dir[a * N + s] = d[a];
    if (defect) defect[s] = lam < threshold ? 1 : 0;
}

// Polarised-light texture of the current Q (Sec. 2.3), the beam along +z
// (layer z = 0 first).  Unpolarised light behind the polariser at angle
// phi_in is S = (1, cos 2phi_in, sin 2phi_in, 0)/2; each site acts as a linear
// retarder with axis angle beta to x (cos 2beta = (dx^2 - dy^2)/(dx^2 + dy^2),
// sin 2beta = 2 dx dy/(dx^2 + dy^2)) and retardance
// delta = 2 pi q h / lambda (n_o n_e / sqrt(n_o^2 sin^2 alpha + n_e^2 cos^2 alpha) - n_o),
// cos alpha = d_z, from the FP64 local order q and director d (order_site).
// A retarder leaves S0 unchanged and acts on (S1, S2, S3) by a 3x3 block; the
// analyser at phi_out passes (S0 + cos 2phi_out S1 + sin 2phi_out S2)/2.
//
// Per group of up to OPT_G wavelengths, two kernels: k_optics_seg, one thread
// per (column, z-segment), multiplies its segment's 3x3 blocks (later layers
// on the left) into T[seg][g][9][col]; k_optics_compose, one thread per
// column, applies the segments in order to the polarised input and adds the
// group's weighted analyser output to the image.  FP64 throughout.
constexpr int OPT_G = 3;

template <typename T>
__global__ __launch_bounds__(BLK) void k_optics_seg(Geom G, const T *__restrict__ Q, OpticsParams op, int wl0,
                                                    int seglen, int nseg, double *__restrict__ Tm)
{
    const int cols = G.nx * G.ny;
    const int id = blockIdx.x * BLK + int(threadIdx.x);
    if (id >= cols * nseg) return;
    const int col = id % cols, seg = id / cols;
    const int z0 = seg * seglen, z1 = min(G.nz, z0 + seglen);
    const size_t N = G.N;
    double M[OPT_G][9];
#pragma unroll
    for (int g = 0; g < OPT_G; ++g)
#pragma unroll
        for (int k = 0; k < 9; ++k) M[g][k] = (k % 4 == 0) ? 1.0 : 0.0;
    const double two_pi_h = 2.0 * 3.14159265358979323846 * op.h;
    const double no2 = op.n_o * op.n_o, ne2 = op.n_e * op.n_e, none = op.n_o * op.n_e;
#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        const size_t s = size_t(z) * cols + col;
        double q5[5], qo, d[3];
#pragma unroll
        for (int k = 0; k < 5; ++k) q5[k] = double(Q[k * N + s]);
        order_site(q5, qo, d);
        const double r2 = d[0] * d[0] + d[1] * d[1];
        double c = 1.0, sn = 0.0;
        if (r2 > 0.0) {
            c = (d[0] * d[0] - d[1] * d[1]) / r2;
            sn = 2.0 * d[0] * d[1] / r2;
        }
        const double cz = d[2] > 1.0 ? 1.0 : (d[2] < -1.0 ? -1.0 : d[2]);
        const double sin2a = 1.0 - cz * cz;
        const double base = two_pi_h * qo * (none / sqrt(no2 * sin2a + ne2 * cz * cz) - op.n_o);
        const double cc = c * c, ss = sn * sn, cs = c * sn;
#pragma unroll
        for (int g = 0; g < OPT_G; ++g) {
            if (wl0 + g >= op.nwl) break;
            double sd, cd;
            sincos(base / op.lam[wl0 + g], &sd, &cd);
            const double R[9] = {cc + ss * cd, cs * (1.0 - cd), -sn * sd,
                                 cs * (1.0 - cd), ss + cc * cd, c * sd,
                                 sn * sd, -c * sd, cd};
            double P[9];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    P[3 * a + b] = R[3 * a] * M[g][b] + R[3 * a + 1] * M[g][3 + b] + R[3 * a + 2] * M[g][6 + b];
#pragma unroll
            for (int k = 0; k < 9; ++k) M[g][k] = P[k];
        }
    }
    const int ng = min(OPT_G, op.nwl - wl0);
#pragma unroll
    for (int g = 0; g < OPT_G; ++g) {
        if (g >= ng) break;
#pragma unroll
        for (int k = 0; k < 9; ++k) Tm[((size_t(seg) * ng + g) * 9 + k) * cols + col] = M[g][k];
    }
}

__global__ __launch_bounds__(BLK) void k_optics_compose(int cols, int nseg, OpticsParams op, int wl0,
                                                        const double *__restrict__ Tm, double *__restrict__ image)
{
    const int col = blockIdx.x * BLK + int(threadIdx.x);
    if (col >= cols) return;
    const int ng = min(OPT_G, op.nwl - wl0);
    double out = 0.0;
#pragma unroll 1
    for (int g = 0; g < ng; ++g) {
        const int w = wl0 + g;
        double v[3] = {0.5 * op.c_in, 0.5 * op.s_in, 0.0};
#pragma unroll 1
        for (int seg = 0; seg < nseg; ++seg) {
            const double *t = Tm + (size_t(seg) * ng + g) * 9 * size_t(cols) + col;
            double u[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                u[a] = t[(3 * a) * size_t(cols)] * v[0] + t[(3 * a + 1) * size_t(cols)] * v[1] +
                       t[(3 * a + 2) * size_t(cols)] * v[2];
            v[0] = u[0];
            v[1] = u[1];
            v[2] = u[2];
        }
        out += op.w[w] * 0.5 * (0.5 + op.c_out * v[0] + op.s_out * v[1]);
    }
    image[col] = wl0 == 0 ? out : image[col] + out;
}

// Disclination sites per z-plane: block z counts plane z (exact integer
// counts carried in FP64).
__global__ __launch_bounds__(BLK) void k_plane_count(Geom G, const unsigned char *__restrict__ defect,
                                                     double *__restrict__ cnt)
{
    const int z = blockIdx.x;
    const int sxy = G.nx * G.ny;
    double acc = 0.0;
    for (int k = threadIdx.x; k < sxy; k += BLK) acc += double(defect[size_t(z) * sxy + k]);
    double v[1] = {acc};
    block_sum<1, BLK>(v, cnt + z);
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_fill(T *__restrict__ p, size_t n, T v)
{
    size_t i = size_t(blockIdx.x) * BLK + threadIdx.x;
    const size_t stride = size_t(gridDim.x) * BLK;
    for (; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------- launchers

inline int site_blocks(int N) { return ((N + BLK - 1) / BLK + 7) / 8 * 8; }

// Records an event pair around each launch when a timer is attached.
struct Marks {
    KernelTimer *t;
    hipStream_t s;
    template <typename Fn>
    hipError_t operator()(int kind, Fn &&launch)
    {
        if (!t) {
            launch();
            return hipSuccess;
        }
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e != hipSuccess) return e;
        (void)hipEventRecord(a, s);
        launch();
        (void)hipEventRecord(b, s);
        t->events.push_back({kind, a, b});
        return hipSuccess;
    }
};

int tile_tz(const Device &D) { return D.tz > 0 ? D.tz : 16; }
int tile_tzq(const Device &D) { return D.tzq > 0 ? D.tzq : tile_tz(D); }

// z-chunk for which the blocks of the tiled kernels fill the device's
// resident block slots `rounds` times: a launch of whole rounds leaves no CU
// idle at the end (0 if the tile columns alone exceed the slots).
template <typename T>
int tz_fill_t(const Device &D, int rounds)
{
    using S = KernelTile<T>;
    int dev = 0, cus = 0, bq = 0, bf = 0, bl = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bq, k_qupdate<T>, S::NB, 0) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bf, k_qforce<T, false>, S::NB, 0) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bl, k_qlb<T, false>, S::NB, 0) != hipSuccess) return 0;
    const long long slots = (long long)cus * std::max(1, std::min(bq, std::min(bf, bl))) * rounds;
    const long long cols = (long long)((D.G.nx + S::TX - 1) / S::TX) * ((D.G.ny + S::TY - 1) / S::TY);
    const long long chunks = slots / cols;
    if (chunks < 1) return 0;
    return int((D.G.nz + chunks - 1) / chunks);
}

template <typename T, bool SPLIT>
hipError_t steps_t(Device &D, const PhysParams &p, int nsteps, KernelTimer *timer)
{
    const bool pc = p.model == LB_D3Q15_PC;
    const int sc = D.sched;
    // the tiled stress kernels run the D3Q19 LB only, and k_qforce the whole stress only
    const bool tiled_stress = sc == SCHED_TILED || sc == SCHED_FUSED || sc == SCHED_FUSED_TILED;
    if ((pc && tiled_stress) || (SPLIT && sc == SCHED_TILED)) return hipErrorNotSupported;
    // the Q update: tiled predictor-corrector, or the per-site predictor and corrector
    const bool tiled_q = sc == SCHED_TILED || sc == SCHED_MIXED || sc == SCHED_FUSED_TILED;
    const bool dbg_nan = (D.debug & DEBUG_NAN_LDS) != 0;
    const Geom G = D.G;
    const Coef<T> c = make_coef<T>(p);
    const int nb = site_blocks(G.N);
    T *u = static_cast<T *>(D.u), *Pi = static_cast<T *>(D.Pi);
    Marks mark{timer, D.stream};
    hipError_t e = hipSuccess;
    if (!p.flow && nsteps > 0)  // pure relaxation: u == 0 (Sec. 2.1)
        k_fill<T><<<1024, BLK, 0, D.stream>>>(u, 3 * size_t(G.N), T(0));
    const TileGrid tg = tile_grid(G.nx, G.ny, G.nz, KernelTile<T>::TX, KernelTile<T>::TY, tile_tz(D));
    const TileGrid tgq = tile_grid(G.nx, G.ny, G.nz, KernelTile<T>::TX, KernelTile<T>::TY, tile_tzq(D));
    const int tb = KernelTile<T>::NB;
    for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
        T *Q = static_cast<T *>(D.Q[D.qcur]);
        T *Qs = static_cast<T *>(D.Q[D.qcur ^ 1]);  // predictor stage, or Q^{n+1} of the tiled update
        if (p.flow) {
            T *gin = static_cast<T *>(D.g[D.gcur]);
            T *gout = static_cast<T *>(D.g[D.gcur ^ 1]);
            if (sc == SCHED_FUSED || sc == SCHED_FUSED_TILED) {
                e = mark(K_QLB, [&] {
                    k_qlb<T, SPLIT><<<tg.launch, tb, 0, D.stream>>>(G, c, tg, Q, gin, gout, u, dbg_nan);
                });
            } else if (sc == SCHED_TILED) {
                e = mark(K_QFORCE, [&] {
                    k_qforce<T, false><<<tg.launch, tb, 0, D.stream>>>(G, c, tg, Q, Pi, nullptr, dbg_nan);
                });
                if (e == hipSuccess)
                    e = mark(K_LBF, [&] { k_lbf<T><<<nb, BLK, 0, D.stream>>>(G, c, gin, Pi, gout, u); });
            } else {
                e = mark(K_STRESS, [&] { k_stress<T, SPLIT><<<nb, BLK, 0, D.stream>>>(G, c, Q, Pi, nullptr); });
                if (pc) {
                    T *P = static_cast<T *>(D.aux);
                    T *bsave = gout + 15 * size_t(G.N);  // planes 15..17 of the target buffer
                    if (e == hipSuccess)
                        e = mark(K_PC1, [&] {
                            k_pc1<T, SPLIT><<<nb, BLK, 0, D.stream>>>(G, c, gin, Pi, P, u, bsave);
                        });
                    if (e == hipSuccess)
                        e = mark(K_PC2, [&] {
                            k_pc2<T, SPLIT><<<nb, BLK, 0, D.stream>>>(G, c, gin, P, Pi, bsave, gout);
                        });
                } else if (e == hipSuccess) {
                    e = mark(K_LB, [&] { k_lb<T, SPLIT><<<nb, BLK, 0, D.stream>>>(G, c, gin, Pi, gout, u); });
                }
            }
            D.gcur ^= 1;
        }
        if (tiled_q) {
            if (e == hipSuccess)
                e = mark(K_QUPDATE, [&] {
                    k_qupdate<T><<<tgq.launch, tb, 0, D.stream>>>(G, c, tgq, Q, u, Qs, dbg_nan);
                });
            D.qcur ^= 1;
        } else {
            if (e == hipSuccess)
                e = mark(K_QPRED, [&] { k_qpred<T><<<nb, BLK, 0, D.stream>>>(G, c, Q, u, Qs); });
            if (e == hipSuccess)
                e = mark(K_QCORR, [&] { k_qcorr<T><<<nb, BLK, 0, D.stream>>>(G, c, Q, Qs, u); });
        }
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <typename T>
hipError_t init_t(Device &D, const PhysParams &p, const double *stage)
{
    const Geom G = D.G;
    const Coef<T> c = make_coef<T>(p);
    const size_t N = G.N;
    const int nb = site_blocks(G.N);
    if (p.model == LB_D3Q15_PC)
        k_init15<T><<<nb, BLK, 0, D.stream>>>(G, c, stage, stage + N, stage + 4 * N,
                                              static_cast<T *>(D.g[D.gcur]), static_cast<T *>(D.Q[D.qcur]));
    else
        k_init<T><<<nb, BLK, 0, D.stream>>>(G, c, stage, stage + N, stage + 4 * N,
                                            static_cast<T *>(D.g[D.gcur]), static_cast<T *>(D.Q[D.qcur]));
    // u of the last LB step: zero until the first step (and for good with flow off)
    k_fill<T><<<1024, BLK, 0, D.stream>>>(static_cast<T *>(D.u), 3 * N, T(0));
    return hipGetLastError();
}

template <typename T, bool SPLIT>
hipError_t readout_t(Device &D, const PhysParams &p, double *stage, double *totals, double *part)
{
    const Geom G = D.G;
    const Coef<T> c = make_coef<T>(p);
    const size_t N = G.N;
    const int nb = site_blocks(G.N);
    T *Pi = static_cast<T *>(D.Pi);
    const T *Q = static_cast<const T *>(D.Q[D.qcur]);
    if (p.model == LB_D3Q15_PC) {
        // the stress sweep only for the free-energy partials
        if (totals) k_stress<T, SPLIT><<<nb, BLK, 0, D.stream>>>(G, c, Q, Pi, part + 4 * nb);
        k_readout15<T><<<nb, BLK, 0, D.stream>>>(G, c, static_cast<const T *>(D.g[D.gcur]), p.flow != 0, Q, stage,
                                                 stage ? stage + N : nullptr, stage ? stage + 4 * N : nullptr,
                                                 totals ? part : nullptr);
        if (totals) {
            k_reduce<<<1, BLK, 0, D.stream>>>(part, nb, 4, 4, totals);
            k_reduce<<<1, BLK, 0, D.stream>>>(part + 4 * nb, nb, 1, 1, totals + 4);
        }
        return hipGetLastError();
    }
    if (totals)
        k_stress<T, SPLIT><<<nb, BLK, 0, D.stream>>>(G, c, Q, Pi, part + 4 * nb);
    else if (p.flow)
        k_stress<T, SPLIT><<<nb, BLK, 0, D.stream>>>(G, c, Q, Pi, nullptr);
    k_readout<T, SPLIT><<<nb, BLK, 0, D.stream>>>(G, c, static_cast<const T *>(D.g[D.gcur]), p.flow ? Pi : nullptr,
                                                  Q, stage, stage ? stage + N : nullptr,
                                                  stage ? stage + 4 * N : nullptr, totals ? part : nullptr);
    if (totals) {
        k_reduce<<<1, BLK, 0, D.stream>>>(part, nb, 4, 4, totals);
        k_reduce<<<1, BLK, 0, D.stream>>>(part + 4 * nb, nb, 1, 1, totals + 4);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t fz_t(Device &D, const PhysParams &p, double *fz)
{
    k_fz<T><<<D.G.nz, BLK, 0, D.stream>>>(D.G, make_coef<T>(p), static_cast<const T *>(D.Q[D.qcur]), fz);
    return hipGetLastError();
}

}  // namespace

hipError_t run_order(Device &D, double threshold, double *q, double *dir, unsigned char *defect, double *cnt)
{
    const int nb = site_blocks(D.G.N);
    if (D.fp32)
        k_order<float><<<nb, BLK, 0, D.stream>>>(D.G, static_cast<const float *>(D.Q[D.qcur]), threshold, q, dir,
                                                 defect);
    else
        k_order<double><<<nb, BLK, 0, D.stream>>>(D.G, static_cast<const double *>(D.Q[D.qcur]), threshold, q,
                                                  dir, defect);
    if (cnt) k_plane_count<<<D.G.nz, BLK, 0, D.stream>>>(D.G, defect, cnt);
    return hipGetLastError();
}

int optics_segments(const Geom &G, int nwl, size_t scratch_bytes)
{
    const long long cols = (long long)G.nx * G.ny;
    const int ng = nwl < OPT_G ? nwl : OPT_G;  // wavelengths per group
    long long nseg = (262144 + cols - 1) / cols;  // enough threads to fill the device
    if (nseg > G.nz) nseg = G.nz;
    const long long cap = (long long)(scratch_bytes / (size_t(cols) * ng * 9 * 8));
    if (nseg > cap) nseg = cap;
    return int(nseg);
}

hipError_t run_optics(Device &D, const OpticsParams &op, double *Tm, size_t tm_bytes, double *image)
{
    const Geom G = D.G;
    const int cols = G.nx * G.ny;
    const int nseg = optics_segments(G, op.nwl, tm_bytes);
    if (nseg < 1) return hipErrorInvalidValue;
    const int seglen = (G.nz + nseg - 1) / nseg;
    const int nseg_used = (G.nz + seglen - 1) / seglen;
    const int nb = int((size_t(cols) * nseg_used + BLK - 1) / BLK);
    for (int wl0 = 0; wl0 < op.nwl; wl0 += OPT_G) {
        if (D.fp32)
            k_optics_seg<float><<<nb, BLK, 0, D.stream>>>(G, static_cast<const float *>(D.Q[D.qcur]), op, wl0,
                                                          seglen, nseg_used, Tm);
        else
            k_optics_seg<double><<<nb, BLK, 0, D.stream>>>(G, static_cast<const double *>(D.Q[D.qcur]), op, wl0,
                                                           seglen, nseg_used, Tm);
        k_optics_compose<<<(cols + BLK - 1) / BLK, BLK, 0, D.stream>>>(cols, nseg_used, op, wl0, Tm, image);
    }
    return hipGetLastError();
}

hipError_t run_fz(Device &D, const PhysParams &p, double *fz)
{
    return D.fp32 ? fz_t<float>(D, p, fz) : fz_t<double>(D, p, fz);
}

size_t partial_doubles(int nx, int ny, int nz)
{
    // per-site blocks x 4 (readout moments) + per-site blocks (free energy),
    // or one value per z-plane (free-energy profile)
    return size_t(5) * site_blocks(nx * ny * nz) + size_t(nz) + 16;
}

const char *kernel_name(int k)
{
    static const char *names[K_COUNT] = {"k_stress", "k_lb", "k_qpred", "k_qcorr", "k_qforce", "k_lbf",
                                         "k_qupdate", "k_pc1", "k_pc2", "k_qlb"};
    return (k >= 0 && k < K_COUNT) ? names[k] : nullptr;
}

hipError_t run_steps(Device &D, const PhysParams &p, int nsteps, KernelTimer *timer)
{
    if (p.flow == FLOW_SPLIT)
        return D.fp32 ? steps_t<float, true>(D, p, nsteps, timer) : steps_t<double, true>(D, p, nsteps, timer);
    return D.fp32 ? steps_t<float, false>(D, p, nsteps, timer) : steps_t<double, false>(D, p, nsteps, timer);
}

int tile_tz_fill(const Device &D, int rounds)
{
    return D.fp32 ? tz_fill_t<float>(D, rounds) : tz_fill_t<double>(D, rounds);
}

hipError_t run_init(Device &D, const PhysParams &p, const double *stage)
{
    return D.fp32 ? init_t<float>(D, p, stage) : init_t<double>(D, p, stage);
}

hipError_t run_readout(Device &D, const PhysParams &p, double *stage, double *totals, double *part)
{
    if (!part) part = D.part;
    if (p.flow == FLOW_SPLIT)
        return D.fp32 ? readout_t<float, true>(D, p, stage, totals, part)
                      : readout_t<double, true>(D, p, stage, totals, part);
    return D.fp32 ? readout_t<float, false>(D, p, stage, totals, part)
                  : readout_t<double, false>(D, p, stage, totals, part);
}

size_t readout_partials(const Geom &G) { return size_t(5) * site_blocks(G.N); }

}  // namespace hlb
