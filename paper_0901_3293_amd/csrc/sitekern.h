// sitekern.h -- one-site-per-thread work of the step, as device functions
// over a linear site index of one periodic box.  The plain kernels and the
// batched persistent kernel both call these; neighbour values come straight
// from global memory through the L1/L2 of the executing CU.
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

__device__ __forceinline__ Nbr nbr_of(const Geom &G, int s)
{
    Nbr S;
    S.s = s;
    S.x = s % G.nx;
    const int yz = s / G.nx;
    S.y = yz % G.ny;
    S.z = yz / G.ny;
    const int sxy = G.nx * G.ny;
    S.nb[0] = (S.x == G.nx - 1) ? s - (G.nx - 1) : s + 1;
    S.nb[1] = (S.x == 0) ? s + (G.nx - 1) : s - 1;
    S.nb[2] = (S.y == G.ny - 1) ? s - G.nx * (G.ny - 1) : s + G.nx;
    S.nb[3] = (S.y == 0) ? s + G.nx * (G.ny - 1) : s - G.nx;
    S.nb[4] = (S.z == G.nz - 1) ? s - sxy * (G.nz - 1) : s + sxy;
    S.nb[5] = (S.z == 0) ? s + sxy * (G.nz - 1) : s - sxy;
    return S;
}

// Population access.  In a sweep over one whole box every population value
// is read once and written once per step, and the next reader of the written
// value is the next step's sweep, after the Q-side kernels have moved their
// own fields; with STREAM the loads and stores are nontemporal so that the
// populations do not push Q, u and the stress out of the L2 and the
// last-level cache between the kernels of a step.  The batched kernels keep
// a cache group's populations resident on purpose and use plain accesses.
template <bool STREAM, typename T>
__device__ __forceinline__ T pop_load(const T *p)
{
    if constexpr (STREAM) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool STREAM, typename T>
__device__ __forceinline__ void pop_store(T *p, T v)
{
    if constexpr (STREAM) __builtin_nontemporal_store(v, p);
    else *p = v;
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
__device__ __forceinline__ void gather_q(const T *__restrict__ Q, size_t N, const Nbr &S, T q[5], T d[3][5],
                                         T lap[5])
{
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const T *P = Q + c * N;
        const T v = P[S.s];
        const T xp = P[S.nb[0]], xm = P[S.nb[1]];
        const T yp = P[S.nb[2]], ym = P[S.nb[3]];
        const T zp = P[S.nb[4]], zm = P[S.nb[5]];
        q[c] = v;
        d[0][c] = T(0.5) * (xp - xm);
        d[1][c] = T(0.5) * (yp - ym);
        d[2][c] = T(0.5) * (zp - zm);
        lap[c] = ((xp + xm) + (yp + ym)) + (zp + zm) - T(6) * v;
    }
}

template <typename T>
__device__ __forceinline__ void gather_u(const T *__restrict__ u, size_t N, const Nbr &S, T uc[3], T W[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T *P = u + a * N;
        uc[a] = P[S.s];
        W[a][0] = T(0.5) * (P[S.nb[0]] - P[S.nb[1]]);
        W[a][1] = T(0.5) * (P[S.nb[2]] - P[S.nb[3]]);
        W[a][2] = T(0.5) * (P[S.nb[4]] - P[S.nb[5]]);
    }
}

// Body force F_a = sum_b [Pi_ab(x + e_b) - Pi_ab(x - e_b)] / 2 (Eq. (19)).
template <typename T>
__device__ __forceinline__ void divergence(const T *__restrict__ Pi, size_t N, const Nbr &S, T F[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T *Px = Pi + (3 * a + 0) * N;
        const T *Py = Pi + (3 * a + 1) * N;
        const T *Pz = Pi + (3 * a + 2) * N;
        F[a] = T(0.5) * ((Px[S.nb[0]] - Px[S.nb[1]]) + (Py[S.nb[2]] - Py[S.nb[3]]) + (Pz[S.nb[4]] - Pz[S.nb[5]]));
    }
}

// Stress Pi(Q) at one site (Eqs. (6)-(8)); returns the free-energy density.
template <typename T>
__device__ __forceinline__ T stress_at(const Geom &G, const Coef<T> &c, const T *__restrict__ Q,
                                       T *__restrict__ Pi, int s)
{
    const size_t N = G.N;
    const Nbr S = nbr_of(G, s);
    T q[5], d[3][5], lap[5], P[3][3], fd, H[5];
    gather_q(Q, N, S, q, d, lap);
    site_stress(c, q, d, lap, P, fd, H);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Pi[(3 * a + b) * N + s] = P[a][b];
    return fd;
}

// Pull-stream, BGK collision with the body force div Pi (Eqs. (14), (16),
// (19)) at one site; writes g' and u.
template <typename T, bool STREAM = false>
__device__ __forceinline__ void lb_at(const Geom &G, const Coef<T> &c, const T *__restrict__ gin,
                                      const T *__restrict__ Pi, T *__restrict__ gout, T *__restrict__ u, int s)
{
    const size_t N = G.N;
    const Nbr S = nbr_of(G, s);
    T g[19], F[3], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 19; ++i) g[i] = pop_load<STREAM>(&gin[i * N + pull_from(G, S, CX[i], CY[i], CZ[i])]);
    divergence(Pi, N, S, F);
    lb_collide(c, g, F, uu, rho);
#pragma unroll
    for (int i = 0; i < 19; ++i) pop_store<STREAM>(&gout[i * N + s], g[i]);
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a * N + s] = uu[a];
}

// Split-coupling terms at one site (planes of the 12 x N layout above);
// returns the free-energy density.
template <typename T>
__device__ __forceinline__ T split_at(const Geom &G, const Coef<T> &c, const T *__restrict__ Q, T *__restrict__ P,
                                      int s)
{
    const size_t N = G.N;
    const Nbr S = nbr_of(G, s);
    T q[5], d[3][5], lap[5], sig[6], tau3[3], h[3], fd;
    gather_q(Q, N, S, q, d, lap);
    site_split(c, q, d, lap, sig, tau3, h, fd);
#pragma unroll
    for (int k = 0; k < 6; ++k) P[k * N + s] = sig[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) P[(6 + k) * N + s] = tau3[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) P[(9 + k) * N + s] = h[k];
    return fd;
}

// Split body force b_a = d_b tau_ab + h_a (centred on the second index;
// tau antisymmetric, stored as xy, xz, yz).
template <typename T>
__device__ __forceinline__ void split_force(const T *__restrict__ P, size_t N, const Nbr &S, T b[3])
{
    const T *txy = P + 6 * N, *txz = P + 7 * N, *tyz = P + 8 * N;
    b[0] = T(0.5) * ((txy[S.nb[2]] - txy[S.nb[3]]) + (txz[S.nb[4]] - txz[S.nb[5]])) + P[9 * N + S.s];
    b[1] = T(0.5) * ((tyz[S.nb[4]] - tyz[S.nb[5]]) - (txy[S.nb[0]] - txy[S.nb[1]])) + P[10 * N + S.s];
    b[2] = T(0.5) * (-(txz[S.nb[0]] - txz[S.nb[1]]) - (tyz[S.nb[2]] - tyz[S.nb[3]])) + P[11 * N + S.s];
}

// LB step of the split coupling at one site: pull, collide with the stress in
// the equilibrium and the split body force; writes g' and u.
template <typename T, bool STREAM = false>
__device__ __forceinline__ void lb_split_at(const Geom &G, const Coef<T> &c, const T *__restrict__ gin,
                                            const T *__restrict__ P, T *__restrict__ gout, T *__restrict__ u, int s)
{
    const size_t N = G.N;
    const Nbr S = nbr_of(G, s);
    T g[19], b[3], sig[6], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 19; ++i) g[i] = pop_load<STREAM>(&gin[i * N + pull_from(G, S, CX[i], CY[i], CZ[i])]);
    split_force(P, N, S, b);
#pragma unroll
    for (int k = 0; k < 6; ++k) sig[k] = P[k * N + s];
    lb_collide_split(c, g, b, sig, uu, rho);
#pragma unroll
    for (int i = 0; i < 19; ++i) pop_store<STREAM>(&gout[i * N + s], g[i]);
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a * N + s] = uu[a];
}

// D3Q15 predictor-corrector LB (Eq. (15)), first pass at one site x: the
// collision C(x, {f}) of the local populations with the stress and body force
// of this step (split: sigma^xi from the 12-plane layout and b = div tau + h;
// whole-stress coupling: no stress term and b = div Pi); writes the
// predictor populations P = f + C at x (to be streamed), the velocity u^n of
// f(x, t) and b (3 planes, read back by the second pass at the same site).
template <typename T, bool SPLIT>
__device__ __forceinline__ void pc1_at(const Geom &G, const Coef<T> &c, const T *__restrict__ g,
                                       const T *__restrict__ Pi, T *__restrict__ P, T *__restrict__ u,
                                       T *__restrict__ bsave, int s)
{
    const size_t N = G.N;
    const Nbr S = nbr_of(G, s);
    T f[15], C[15], b[3], sig[6], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 15; ++i) f[i] = g[i * N + s];
    if (SPLIT) {
        split_force(Pi, N, S, b);
#pragma unroll
        for (int k = 0; k < 6; ++k) sig[k] = Pi[k * N + s];
    } else {
        divergence(Pi, N, S, b);
    }
    lb15_collide(c, f, SPLIT ? sig : static_cast<const T *>(nullptr), b, C, uu, rho);
#pragma unroll
    for (int i = 0; i < 15; ++i) P[i * N + s] = f[i] + C[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a * N + s] = uu[a];
        bsave[a * N + s] = b[a];
    }
}

// Second pass at one site y: f*_i(y) = P_i(y - e_i), collision C(y, {f*}),
//   f_i(y, t + 1) = [f_i(y - e_i) + P_i(y - e_i)]/2 + C_i(y, {f*})/2.
template <typename T, bool SPLIT, bool STREAM = false>
__device__ __forceinline__ void pc2_at(const Geom &G, const Coef<T> &c, const T *__restrict__ g,
                                       const T *__restrict__ P, const T *__restrict__ Pi,
                                       const T *__restrict__ bsave, T *__restrict__ gout, int s)
{
    const size_t N = G.N;
    const Nbr S = nbr_of(G, s);
    T fs[15], fo[15], C[15], b[3], sig[6], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 15; ++i) {
        const int t = pull_from(G, S, DX15[i], DY15[i], DZ15[i]);
        fs[i] = pop_load<STREAM>(&P[i * N + t]);
        fo[i] = T(0.5) * (pop_load<STREAM>(&g[i * N + t]) + fs[i]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) b[a] = bsave[a * N + s];
    if (SPLIT)
#pragma unroll
        for (int k = 0; k < 6; ++k) sig[k] = Pi[k * N + s];
    lb15_collide(c, fs, SPLIT ? sig : static_cast<const T *>(nullptr), b, C, uu, rho);
#pragma unroll
    for (int i = 0; i < 15; ++i) pop_store<STREAM>(&gout[i * N + s], fo[i] + T(0.5) * C[i]);
}

// Predictor Q* = Q + R(Q, u) at one site (Eqs. (2)-(4)).
template <typename T>
__device__ __forceinline__ void pred_at(const Geom &G, const Coef<T> &c, const T *__restrict__ Q,
                                        const T *__restrict__ u, T *__restrict__ Qs, int s)
{
    const size_t N = G.N;
    const Nbr S = nbr_of(G, s);
    T q[5], d[3][5], lap[5], uc[3], W[3][3], R[5];
    gather_q(Q, N, S, q, d, lap);
    gather_u(u, N, S, uc, W);
    site_rhs(c, q, d, lap, uc, W, R);
#pragma unroll
    for (int k = 0; k < 5; ++k) Qs[k * N + s] = q[k] + R[k];
}

// Corrector Q^{n+1} = Q^n + [R(Q^n) + R(Q*)]/2 = [Q^n + Q* + R(Q*)]/2, in
// place over Q (each site reads only its own Q^n).
template <typename T>
__device__ __forceinline__ void corr_at(const Geom &G, const Coef<T> &c, T *__restrict__ Q,
                                        const T *__restrict__ Qs, const T *__restrict__ u, int s)
{
    const size_t N = G.N;
    const Nbr S = nbr_of(G, s);
    T q[5], d[3][5], lap[5], uc[3], W[3][3], R[5];
    gather_q(Qs, N, S, q, d, lap);
    gather_u(u, N, S, uc, W);
    site_rhs(c, q, d, lap, uc, W, R);
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k * N + s] = T(0.5) * (Q[k * N + s] + q[k] + R[k]);
}

// Free-energy density at one site (Eq. (1) with the divergence term).
template <typename T>
__device__ __forceinline__ T fdens_at(const Geom &G, const Coef<T> &c, const T *__restrict__ Q, int s)
{
    const Nbr S = nbr_of(G, s);
    T q[5], d[3][5], lap[5], Qf[3][3], dQ[3][3][3], CQ[3][3], Q2[3][3], M[3][3], div[3];
    gather_q(Q, size_t(G.N), S, q, d, lap);
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
