// sitekern.h -- one-site-per-thread work of the step, as device functions
// over a linear site index of one periodic box.  The plain kernels and the
// batched kernels all call these; neighbour values come straight from global
// memory through the L1/L2 of the executing CU.  A site index is split into
// (x, y, z) by multiply-high division (FastDiv in kernels.h), and every field
// plane is read through its wave-uniform base address plus 32-bit byte
// offsets (Off below).
//
// Buffers of one box (structure-of-arrays, component stride N, x fastest):
//   g 19 x N, Q 5 x N, Qs (predictor stage) 5 x N, u 3 x N, Pi 9 x N
//   (whole-stress coupling) or 12 x N (split coupling: sigma^xi xx, xy, xz,
//   yy, yz, zz; tau xy, xz, yz; h x, y, z).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "site.h"

namespace hlb {

struct Nbr {
    int s, x, y, z;
    int nb[6];  // x+1, x-1, y+1, y-1, z+1, z-1 (periodic)
};

// The site s = x + nx (y + ny z) at (x, y, z) and its six periodic neighbours.
__device__ __forceinline__ Nbr nbr_at(const Geom &G, int s, int x, int y, int z)
{
    Nbr S;
    const int sxy = G.nx * G.ny;
    S.s = s;
    S.x = x;
    S.y = y;
    S.z = z;
    S.nb[0] = (x == G.nx - 1) ? s - (G.nx - 1) : s + 1;
    S.nb[1] = (x == 0) ? s + (G.nx - 1) : s - 1;
    S.nb[2] = (y == G.ny - 1) ? s - G.nx * (G.ny - 1) : s + G.nx;
    S.nb[3] = (y == 0) ? s + G.nx * (G.ny - 1) : s - G.nx;
    S.nb[4] = (z == G.nz - 1) ? s - sxy * (G.nz - 1) : s + sxy;
    S.nb[5] = (z == 0) ? s + sxy * (G.nz - 1) : s - sxy;
    return S;
}

// The same from the linear site index.
__device__ __forceinline__ Nbr nbr_of(const Geom &G, int s)
{
    const int yz = int(fastdiv(unsigned(s), G.dx));
    const int z = int(fastdiv(unsigned(yz), G.dy));
    return nbr_at(G, s, s - yz * G.nx, yz - z * G.ny, z);
}

// Byte offsets of a site and of its six neighbours within one field plane of
// elements of type T.  A plane of N values is under 4 GiB (checked when a
// context is created), so 32-bit offsets from the plane's base address it;
// the base (field + c N) is the same for the whole wave, and one site's
// offsets serve every component of every field.
template <typename T>
struct Off {
    unsigned s;
    unsigned nb[6];  // x+1, x-1, y+1, y-1, z+1, z-1
};

template <typename T>
__device__ __forceinline__ Off<T> offsets(const Nbr &S)
{
    Off<T> O;
    O.s = unsigned(S.s) * unsigned(sizeof(T));
#pragma unroll
    for (int k = 0; k < 6; ++k) O.nb[k] = unsigned(S.nb[k]) * unsigned(sizeof(T));
    return O;
}

// Plane c of a component-major field of N values per component.
template <typename T>
__device__ __forceinline__ T *plane(T *f, int c, int N)
{
    return f + size_t(c) * size_t(N);
}

template <typename T>
__device__ __forceinline__ T *at(T *P, unsigned b)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(P) + b);
}

template <typename T>
__device__ __forceinline__ const T *at(const T *P, unsigned b)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(P) + b);
}

// Byte offset of the site x - e of a population with velocity e = (cx, cy,
// cz): each nonzero component adds the byte distance to the neighbour on the
// opposite side (periodic), so a pull costs one or two additions.
template <typename T>
__device__ __forceinline__ unsigned pull_off(const Off<T> &O, int cx, int cy, int cz)
{
    unsigned b = O.s;
    if (cx > 0) b += O.nb[1] - O.s;
    else if (cx < 0) b += O.nb[0] - O.s;
    if (cy > 0) b += O.nb[3] - O.s;
    else if (cy < 0) b += O.nb[2] - O.s;
    if (cz > 0) b += O.nb[5] - O.s;
    else if (cz < 0) b += O.nb[4] - O.s;
    return b;
}

// Population access.  In a sweep over one whole box every population value
// is read once and written once per step, and the next reader of the written
// value is the next step's sweep, after the Q-side kernels have moved their
// own fields; with STREAM the loads and stores are nontemporal so that the
// populations do not push Q, u and the stress out of the L2 and the
// last-level cache between the kernels of a step.  (The predicted
// populations of the first D3Q15 pass are read once, by the second pass right
// after it, but at 15 values per site they are too many to stay cached beside
// the rest: they are streamed too.)  The batched kernels stream them as
// well, so that a cache group's other fields stay in the last-level cache.
template <bool STREAM, typename T>
__device__ __forceinline__ T pop_load(const T *P, unsigned b)
{
    if constexpr (STREAM) return __builtin_nontemporal_load(at(P, b));
    else return *at(P, b);
}

template <bool STREAM, typename T>
__device__ __forceinline__ void pop_store(T *P, unsigned b, T v)
{
    if constexpr (STREAM) __builtin_nontemporal_store(v, at(P, b));
    else *at(P, b) = v;
}

// Pulled source of population i arriving at (x,y,z): site (x,y,z) - e_i.
__device__ __forceinline__ int pull_from(const Geom &G, const Nbr &S, int cx, int cy, int cz)
{
    int xs = S.x - cx, ys = S.y - cy, zs = S.z - cz;
    xs += (xs < 0) ? G.nx : ((xs >= G.nx) ? -G.nx : 0);
    ys += (ys < 0) ? G.ny : ((ys >= G.ny) ? -G.ny : 0);
    zs += (zs < 0) ? G.nz : ((zs >= G.nz) ? -G.nz : 0);
    return xs + G.nx * (ys + G.ny * zs);
}

template <typename T>
__device__ __forceinline__ void gather_q(const T *__restrict__ Q, int N, const Off<T> &O, T q[5], T d[3][5],
                                         T lap[5])
{
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const T *P = plane(Q, c, N);
        const T v = *at(P, O.s);
        const T xp = *at(P, O.nb[0]), xm = *at(P, O.nb[1]);
        const T yp = *at(P, O.nb[2]), ym = *at(P, O.nb[3]);
        const T zp = *at(P, O.nb[4]), zm = *at(P, O.nb[5]);
        q[c] = v;
        d[0][c] = T(0.5) * (xp - xm);
        d[1][c] = T(0.5) * (yp - ym);
        d[2][c] = T(0.5) * (zp - zm);
        lap[c] = ((xp + xm) + (yp + ym)) + (zp + zm) - T(6) * v;
    }
}

template <typename T>
__device__ __forceinline__ void gather_u(const T *__restrict__ u, int N, const Off<T> &O, T uc[3], T W[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T *P = plane(u, a, N);
        uc[a] = *at(P, O.s);
        W[a][0] = T(0.5) * (*at(P, O.nb[0]) - *at(P, O.nb[1]));
        W[a][1] = T(0.5) * (*at(P, O.nb[2]) - *at(P, O.nb[3]));
        W[a][2] = T(0.5) * (*at(P, O.nb[4]) - *at(P, O.nb[5]));
    }
}

// Body force F_a = sum_b [Pi_ab(x + e_b) - Pi_ab(x - e_b)] / 2 (Eq. (19)).
template <typename T>
__device__ __forceinline__ void divergence(const T *__restrict__ Pi, int N, const Off<T> &O, T F[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T *Px = plane(Pi, 3 * a + 0, N);
        const T *Py = plane(Pi, 3 * a + 1, N);
        const T *Pz = plane(Pi, 3 * a + 2, N);
        F[a] = T(0.5) * ((*at(Px, O.nb[0]) - *at(Px, O.nb[1])) + (*at(Py, O.nb[2]) - *at(Py, O.nb[3])) +
                         (*at(Pz, O.nb[4]) - *at(Pz, O.nb[5])));
    }
}

// Stress Pi(Q) at one site (Eqs. (6)-(8)); returns the free-energy density.
template <typename T>
__device__ __forceinline__ T stress_at(const Geom &G, const Coef<T> &c, const T *__restrict__ Q,
                                       T *__restrict__ Pi, int s)
{
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T q[5], d[3][5], lap[5], P[3][3], fd, H[5];
    gather_q(Q, G.N, O, q, d, lap);
    site_stress(c, q, d, lap, P, fd, H);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) *at(plane(Pi, 3 * a + b, G.N), O.s) = P[a][b];
    return fd;
}

// Pull-stream, BGK collision with the body force div Pi (Eqs. (14), (16),
// (19)) at one site; writes g' and u.
template <typename T, bool STREAM = false>
__device__ __forceinline__ void lb_at(const Geom &G, const Coef<T> &c, const T *__restrict__ gin,
                                      const T *__restrict__ Pi, T *__restrict__ gout, T *__restrict__ u, int s)
{
    const int N = G.N;
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T g[19], F[3], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 19; ++i) g[i] = pop_load<STREAM>(plane(gin, i, N), pull_off(O, CX[i], CY[i], CZ[i]));
    divergence(Pi, N, O, F);
    lb_collide(c, g, F, uu, rho);
#pragma unroll
    for (int i = 0; i < 19; ++i) pop_store<STREAM>(plane(gout, i, N), O.s, g[i]);
#pragma unroll
    for (int a = 0; a < 3; ++a) *at(plane(u, a, N), O.s) = uu[a];
}

// Split-coupling terms at one site (planes of the 12 x N layout above);
// returns the free-energy density.
template <typename T>
__device__ __forceinline__ T split_at(const Geom &G, const Coef<T> &c, const T *__restrict__ Q, T *__restrict__ P,
                                      int s)
{
    const int N = G.N;
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T q[5], d[3][5], lap[5], sig[6], tau3[3], h[3], fd;
    gather_q(Q, N, O, q, d, lap);
    site_split(c, q, d, lap, sig, tau3, h, fd);
#pragma unroll
    for (int k = 0; k < 6; ++k) *at(plane(P, k, N), O.s) = sig[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) *at(plane(P, 6 + k, N), O.s) = tau3[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) *at(plane(P, 9 + k, N), O.s) = h[k];
    return fd;
}

// Split body force b_a = d_b tau_ab + h_a (centred on the second index;
// tau antisymmetric, stored as xy, xz, yz).
template <typename T>
__device__ __forceinline__ void split_force(const T *__restrict__ P, int N, const Off<T> &O, T b[3])
{
    const T *txy = plane(P, 6, N), *txz = plane(P, 7, N), *tyz = plane(P, 8, N);
    b[0] = T(0.5) * ((*at(txy, O.nb[2]) - *at(txy, O.nb[3])) + (*at(txz, O.nb[4]) - *at(txz, O.nb[5]))) +
           *at(plane(P, 9, N), O.s);
    b[1] = T(0.5) * ((*at(tyz, O.nb[4]) - *at(tyz, O.nb[5])) - (*at(txy, O.nb[0]) - *at(txy, O.nb[1]))) +
           *at(plane(P, 10, N), O.s);
    b[2] = T(0.5) * (-(*at(txz, O.nb[0]) - *at(txz, O.nb[1])) - (*at(tyz, O.nb[2]) - *at(tyz, O.nb[3]))) +
           *at(plane(P, 11, N), O.s);
}

// LB step of the split coupling at one site: pull, collide with the stress in
// the equilibrium and the split body force; writes g' and u.
template <typename T, bool STREAM = false>
__device__ __forceinline__ void lb_split_at(const Geom &G, const Coef<T> &c, const T *__restrict__ gin,
                                            const T *__restrict__ P, T *__restrict__ gout, T *__restrict__ u, int s)
{
    const int N = G.N;
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T g[19], b[3], sig[6], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 19; ++i) g[i] = pop_load<STREAM>(plane(gin, i, N), pull_off(O, CX[i], CY[i], CZ[i]));
    split_force(P, N, O, b);
#pragma unroll
    for (int k = 0; k < 6; ++k) sig[k] = *at(plane(P, k, N), O.s);
    lb_collide_split(c, g, b, sig, uu, rho);
#pragma unroll
    for (int i = 0; i < 19; ++i) pop_store<STREAM>(plane(gout, i, N), O.s, g[i]);
#pragma unroll
    for (int a = 0; a < 3; ++a) *at(plane(u, a, N), O.s) = uu[a];
}

// D3Q15 predictor-corrector LB (Eq. (15)), first pass at one site x: the
// collision C(x, {f}) of the local populations with the stress and body force
// of this step (split: sigma^xi from the 12-plane layout and b = div tau + h;
// whole-stress coupling: no stress term and b = div Pi); writes the
// predictor populations P = f + C at x (to be streamed), the velocity u^n of
// f(x, t) and b (3 planes, read back by the second pass at the same site).
template <typename T, bool SPLIT, bool STREAM = false>
__device__ __forceinline__ void pc1_at(const Geom &G, const Coef<T> &c, const T *__restrict__ g,
                                       const T *__restrict__ Pi, T *__restrict__ P, T *__restrict__ u,
                                       T *__restrict__ bsave, int s)
{
    const int N = G.N;
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T f[15], C[15], b[3], sig[6], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 15; ++i) f[i] = *at(plane(g, i, N), O.s);
    if (SPLIT) {
        split_force(Pi, N, O, b);
#pragma unroll
        for (int k = 0; k < 6; ++k) sig[k] = *at(plane(Pi, k, N), O.s);
    } else {
        divergence(Pi, N, O, b);
    }
    lb15_collide(c, f, SPLIT ? sig : static_cast<const T *>(nullptr), b, C, uu, rho);
#pragma unroll
    for (int i = 0; i < 15; ++i) pop_store<STREAM>(plane(P, i, N), O.s, f[i] + C[i]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        *at(plane(u, a, N), O.s) = uu[a];
        *at(plane(bsave, a, N), O.s) = b[a];
    }
}

// Second pass at one site y: f*_i(y) = P_i(y - e_i), collision C(y, {f*}),
//   f_i(y, t + 1) = [f_i(y - e_i) + P_i(y - e_i)]/2 + C_i(y, {f*})/2.
template <typename T, bool SPLIT, bool STREAM = false>
__device__ __forceinline__ void pc2_at(const Geom &G, const Coef<T> &c, const T *__restrict__ g,
                                       const T *__restrict__ P, const T *__restrict__ Pi,
                                       const T *__restrict__ bsave, T *__restrict__ gout, int s)
{
    const int N = G.N;
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T fs[15], fo[15], C[15], b[3], sig[6], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 15; ++i) {
        const unsigned t = pull_off(O, DX15[i], DY15[i], DZ15[i]);
        fs[i] = pop_load<STREAM>(plane(P, i, N), t);
        fo[i] = T(0.5) * (pop_load<STREAM>(plane(g, i, N), t) + fs[i]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) b[a] = *at(plane(bsave, a, N), O.s);
    if (SPLIT)
#pragma unroll
        for (int k = 0; k < 6; ++k) sig[k] = *at(plane(Pi, k, N), O.s);
    lb15_collide(c, fs, SPLIT ? sig : static_cast<const T *>(nullptr), b, C, uu, rho);
#pragma unroll
    for (int i = 0; i < 15; ++i) pop_store<STREAM>(plane(gout, i, N), O.s, fo[i] + T(0.5) * C[i]);
}

// Predictor Q* = Q + R(Q, u) at one site (Eqs. (2)-(4)).
template <typename T>
__device__ __forceinline__ void pred_at(const Geom &G, const Coef<T> &c, const T *__restrict__ Q,
                                        const T *__restrict__ u, T *__restrict__ Qs, int s)
{
    const int N = G.N;
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T q[5], d[3][5], lap[5], uc[3], W[3][3], R[5];
    gather_q(Q, N, O, q, d, lap);
    gather_u(u, N, O, uc, W);
    site_rhs(c, q, d, lap, uc, W, R);
#pragma unroll
    for (int k = 0; k < 5; ++k) *at(plane(Qs, k, N), O.s) = q[k] + R[k];
}

// Corrector Q^{n+1} = Q^n + [R(Q^n) + R(Q*)]/2 = [Q^n + Q* + R(Q*)]/2, in
// place over Q (each site reads only its own Q^n).
template <typename T>
__device__ __forceinline__ void corr_at(const Geom &G, const Coef<T> &c, T *__restrict__ Q,
                                        const T *__restrict__ Qs, const T *__restrict__ u, int s)
{
    const int N = G.N;
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T qn[5], q[5], d[3][5], lap[5], uc[3], W[3][3], R[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) qn[k] = *at(plane(Q, k, N), O.s);  // issued with the stencil loads
    gather_q(Qs, N, O, q, d, lap);
    gather_u(u, N, O, uc, W);
    site_rhs(c, q, d, lap, uc, W, R);
#pragma unroll
    for (int k = 0; k < 5; ++k) *at(plane(Q, k, N), O.s) = T(0.5) * (qn[k] + q[k] + R[k]);
}

// Free-energy density at one site (Eq. (1) with the divergence term).
template <typename T>
__device__ __forceinline__ T fdens_at(const Geom &G, const Coef<T> &c, const T *__restrict__ Q, int s)
{
    const Off<T> O = offsets<T>(nbr_of(G, s));
    T q[5], d[3][5], lap[5], Qf[3][3], dQ[3][3][3], CQ[3][3], Q2[3][3], M[3][3], div[3];
    gather_q(Q, G.N, O, q, d, lap);
    full3(q, Qf);
    full_grad(d, dQ);
    curl(dQ, CQ);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            Q2[a][b] = Qf[a][0] * Qf[0][b] + Qf[a][1] * Qf[1][b] + Qf[a][2] * Qf[2][b];
            M[a][b] = CQ[a][b] + c.q0x2 * Qf[a][b];
        }
        div[a] = dQ[0][a][0] + dQ[1][a][1] + dQ[2][a][2];
    }
    return free_energy(c, Qf, Q2, Q2[0][0] + Q2[1][1] + Q2[2][2], div, M);
}

template <typename T>
Coef<T> make_coef(const PhysParams &p)
{
    Coef<T> c;
    c.a = T(p.A0 * (1.0 - p.gamma / 3.0));
    c.bg = T(p.A0 * p.gamma);
    c.K = T(p.K);
    c.q0x2 = T(2.0 * p.q0);
    c.Kq0x2 = T(2.0 * p.K * p.q0);
    c.Kq0sq4 = T(4.0 * p.K * p.q0 * p.q0);
    c.xi = T(p.xi);
    c.Gamma = T(p.Gamma);
    c.rho0 = T(p.rho0);
    c.omega = T(1.0 / p.tau);
    c.pref = T(1.0 - 0.5 / p.tau);
    return c;
}

}  // namespace hlb
