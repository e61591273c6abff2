// site.h -- per-site arithmetic of the hybrid step, templated on the storage
// and arithmetic type T (double or float).  Pure device functions: no memory
// access beyond their arguments, so every kernel shape (plain, LDS-tiled,
// batched) shares one definition of the physics.
//
// Tensor conventions: Q is symmetric traceless, five stored components
// (xx, xy, xz, yy, yz), Q_zz = -Q_xx - Q_yy.  d[g][c] = d_g Q_c (centred),
// lap[c] = 7-point Laplacian.  W_ab = d_b u_a.
#pragma once

#include <hip/hip_runtime.h>

namespace hlb {

// Physical constants of one run, pre-combined in the arithmetic type.
template <typename T>
struct Coef {
    T a;       // A0 (1 - gamma/3)                 bulk quadratic, Sec. 2.1 Eq. (1)
    T bg;      // A0 gamma                         bulk cubic and quartic
    T K;       // elastic constant
    T q0x2;    // 2 q0
    T Kq0x2;   // 2 K q0                           chiral term of H
    T Kq0sq4;  // 4 K q0^2
    T xi;      // flow-aligning parameter, Eqs. (4), (7)
    T Gamma;   // rotational diffusion, Eq. (2)
    T rho0;    // reference density of the deviation populations
    T omega;   // 1 / tau_LB
    T pref;    // 1 - 1/(2 tau_LB), second-order forcing prefactor
};

template <typename T>
__host__ __device__ __forceinline__ void full3(const T q[5], T Q[3][3])
{
    Q[0][0] = q[0]; Q[0][1] = q[1]; Q[0][2] = q[2];
    Q[1][0] = q[1]; Q[1][1] = q[3]; Q[1][2] = q[4];
    Q[2][0] = q[2]; Q[2][1] = q[4]; Q[2][2] = -q[0] - q[3];
}

// d_g Q_ab as a full tensor from the stored components.
template <typename T>
__host__ __device__ __forceinline__ void full_grad(const T d[3][5], T dQ[3][3][3])
{
#pragma unroll
    for (int g = 0; g < 3; ++g) full3(d[g], dQ[g]);
}

// (CQ)_ab = eps_agd d_g Q_db (the curl in Eq. (1)), written out:
//   row x: d_y Q_zb - d_z Q_yb;  row y: d_z Q_xb - d_x Q_zb;  row z: d_x Q_yb - d_y Q_xb.
template <typename T>
__host__ __device__ __forceinline__ void curl(const T dQ[3][3][3], T CQ[3][3])
{
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        CQ[0][b] = dQ[1][2][b] - dQ[2][1][b];
        CQ[1][b] = dQ[2][0][b] - dQ[0][2][b];
        CQ[2][b] = dQ[0][1][b] - dQ[1][0][b];
    }
}

// Molecular field H (Eq. (2)), symmetric traceless part of -dF/dQ for the
// free energy of Eq. (1) in its one-constant form:
//   H = -a Q + bg (Q^2 - tr(Q^2)/3 I) - bg tr(Q^2) Q + K lap Q
//       - 2 K q0 (CQ + CQ^T) - 4 K q0^2 Q.
// Returns the five stored components; also hands back Q^2 and tr(Q^2).
template <typename T>
__host__ __device__ __forceinline__ void molecular_field(const Coef<T> &c, const T Q[3][3], const T CQ[3][3],
                                                const T lap[5], T H[5], T Q2[3][3], T &trQ2)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Q2[a][b] = Q[a][0] * Q[0][b] + Q[a][1] * Q[1][b] + Q[a][2] * Q[2][b];
    trQ2 = Q2[0][0] + Q2[1][1] + Q2[2][2];
    const T third = T(1) / T(3);
    const T lin = -(c.a + c.bg * trQ2 + c.Kq0sq4);
    // (a,b) for the stored components
    const int ia[5] = {0, 0, 0, 1, 1};
    const int ib[5] = {0, 1, 2, 1, 2};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int a = ia[k], b = ib[k];
        T v = lin * Q[a][b] + c.bg * Q2[a][b] + c.K * lap[k] - c.Kq0x2 * (CQ[a][b] + CQ[b][a]);
        if (a == b) v -= c.bg * trQ2 * third;
        H[k] = v;
    }
}

// Free-energy density (Eq. (1) plus K/2 (d_b Q_ab)^2):
//   f = a/2 tr Q^2 - bg/3 tr Q^3 + bg/4 (tr Q^2)^2 + K/2 |div Q|^2 + K/2 M:M,
//   M = CQ + 2 q0 Q,  (div Q)_a = d_b Q_ab.
template <typename T>
__host__ __device__ __forceinline__ T free_energy(const Coef<T> &c, const T Q[3][3], const T Q2[3][3], T trQ2,
                                         const T div[3], const T M[3][3])
{
    T trQ3 = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) trQ3 += Q2[a][b] * Q[b][a];
    T mm = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) mm += M[a][b] * M[a][b];
    const T dd = div[0] * div[0] + div[1] * div[1] + div[2] * div[2];
    return T(0.5) * c.a * trQ2 - c.bg * trQ3 / T(3) + T(0.25) * c.bg * trQ2 * trQ2 + T(0.5) * c.K * (dd + mm);
}

// Upper triangle (xx, xy, xz, yy, yz, zz) of Q^2 for symmetric Q, and its
// trace.
template <typename T>
__host__ __device__ __forceinline__ void square_sym(const T q[5], T qzz, T s[6], T &tr)
{
    s[0] = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
    s[1] = q[0] * q[1] + q[1] * q[3] + q[2] * q[4];
    s[2] = q[0] * q[2] + q[1] * q[4] + q[2] * qzz;
    s[3] = q[1] * q[1] + q[3] * q[3] + q[4] * q[4];
    s[4] = q[1] * q[2] + q[3] * q[4] + q[4] * qzz;
    s[5] = q[2] * q[2] + q[4] * q[4] + qzz * qzz;
    tr = s[0] + s[3] + s[5];
}

// Symmetric part (stored components) of CQ + (CQ)^T, the curl term of H, from
// the derivatives of the stored components (d_g Q_zz = -(d_g Q_xx + d_g Q_yy)).
template <typename T>
__host__ __device__ __forceinline__ void curl_sym(const T d[3][5], T C[5])
{
    const T dzz0 = -(d[0][0] + d[0][3]), dzz1 = -(d[1][0] + d[1][3]);
    C[0] = T(2) * (d[1][2] - d[2][1]);                    // 2 (dy Q_zx - dz Q_yx)
    C[1] = (d[1][4] - d[2][3]) + (d[2][0] - d[0][2]);     // CQ_xy + CQ_yx
    C[2] = (dzz1 - d[2][4]) + (d[0][1] - d[1][0]);        // CQ_xz + CQ_zx
    C[3] = T(2) * (d[2][1] - d[0][4]);                    // 2 (dz Q_xy - dx Q_zy)
    C[4] = (d[2][2] - dzz0) + (d[0][3] - d[1][1]);        // CQ_yz + CQ_zy
}

// Curl (CQ)_ab = eps_agd d_g Q_db from the derivatives of the stored
// components (the full, non-symmetric tensor).
template <typename T>
__host__ __device__ __forceinline__ void curl5(const T d[3][5], const T dzz[3], T CQ[3][3])
{
    CQ[0][0] = d[1][2] - d[2][1];  // dy Q_zx - dz Q_yx
    CQ[0][1] = d[1][4] - d[2][3];  // dy Q_zy - dz Q_yy
    CQ[0][2] = dzz[1] - d[2][4];   // dy Q_zz - dz Q_yz
    CQ[1][0] = d[2][0] - d[0][2];  // dz Q_xx - dx Q_zx
    CQ[1][1] = d[2][1] - d[0][4];  // dz Q_xy - dx Q_zy
    CQ[1][2] = d[2][2] - dzz[0];   // dz Q_xz - dx Q_zz
    CQ[2][0] = d[0][1] - d[1][0];  // dx Q_yx - dy Q_xx
    CQ[2][1] = d[0][3] - d[1][1];  // dx Q_yy - dy Q_xy
    CQ[2][2] = d[0][4] - d[1][2];  // dx Q_yz - dy Q_xz
}

// Chemical stress (Eqs. (6)-(8), the rho T part of the pressure left to the
// lattice): Pi_ab = f d_ab + sigma^xi_ab - G_ab + tau_ab with
//   sigma^xi = 2 xi (Q + I/3)(Q:H) - xi (HQ + QH + 2H/3),
//   tau      = QH - HQ,
//   G_ab     = d_a Q_gn Phi_gnb,  Phi_gnb = K [d_nb (div Q)_g + eps_lbg M_ln],
// i.e. G_ab = K [ d_a Q_gb (div Q)_g + eps_bgl d_a Q_gn M_ln ], M = CQ + 2 q0 Q.
// Also returns f (Eq. (1) plus K/2 (d_b Q_ab)^2) and H (five components).
// sigma^xi is symmetric and tau antisymmetric (QH = (HQ)^T for symmetric H
// and Q), so each is formed once per pair of entries.
template <typename T>
__host__ __device__ __forceinline__ void site_stress(const Coef<T> &c, const T q[5], const T d[3][5],
                                                     const T lap[5], T Pi[3][3], T &fdens, T H5[5])
{
    const T third = T(1) / T(3);
    const T qzz = -q[0] - q[3];
    const T dzz[3] = {-(d[0][0] + d[0][3]), -(d[1][0] + d[1][3]), -(d[2][0] + d[2][3])};
    T s[6], trQ2, CQ[3][3];
    square_sym(q, qzz, s, trQ2);
    curl5(d, dzz, CQ);
    {
        const T lin = -(c.a + c.bg * trQ2 + c.Kq0sq4);
        const T diag = c.bg * trQ2 * third;
        const T C[5] = {T(2) * CQ[0][0], CQ[0][1] + CQ[1][0], CQ[0][2] + CQ[2][0], T(2) * CQ[1][1],
                        CQ[1][2] + CQ[2][1]};
        const int k2s[5] = {0, 1, 2, 3, 4};
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            T v = lin * q[k] + c.bg * s[k2s[k]] + c.K * lap[k] - c.Kq0x2 * C[k];
            if (k == 0 || k == 3) v -= diag;
            H5[k] = v;
        }
    }
    const T Q[3][3] = {{q[0], q[1], q[2]}, {q[1], q[3], q[4]}, {q[2], q[4], qzz}};
    const T hzz = -H5[0] - H5[3];
    const T H[3][3] = {{H5[0], H5[1], H5[2]}, {H5[1], H5[3], H5[4]}, {H5[2], H5[4], hzz}};
    T M[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) M[a][b] = CQ[a][b] + c.q0x2 * Q[a][b];
    const T div[3] = {d[0][0] + d[1][1] + d[2][2], d[0][1] + d[1][3] + d[2][4], d[0][2] + d[1][4] + dzz[2]};
    {
        const T trQ3 = s[0] * q[0] + s[3] * q[3] + s[5] * qzz + T(2) * (s[1] * q[1] + s[2] * q[2] + s[4] * q[4]);
        T mm = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) mm += M[a][b] * M[a][b];
        const T dd = div[0] * div[0] + div[1] * div[1] + div[2] * div[2];
        fdens = T(0.5) * c.a * trQ2 - c.bg * trQ3 * third + T(0.25) * c.bg * trQ2 * trQ2 + T(0.5) * c.K * (dd + mm);
    }
    T HQ[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) HQ[a][b] = H[a][0] * Q[0][b] + H[a][1] * Q[1][b] + H[a][2] * Q[2][b];
    const T QdH = q[0] * H5[0] + q[3] * H5[3] + qzz * hzz + T(2) * (q[1] * H5[1] + q[2] * H5[2] + q[4] * H5[4]);
    const T xq = T(2) * c.xi * QdH;
    T sig[3][3], tau[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) {
            const T v = xq * (Q[a][b] + (a == b ? third : T(0))) -
                        c.xi * (HQ[a][b] + HQ[b][a] + T(2) * third * H[a][b]);
            sig[a][b] = v;
            sig[b][a] = v;
            const T w = HQ[b][a] - HQ[a][b];
            tau[a][b] = w;
            tau[b][a] = -w;
        }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T P[3][3] = {{d[a][0], d[a][1], d[a][2]}, {d[a][1], d[a][3], d[a][4]}, {d[a][2], d[a][4], dzz[a]}};
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            // G_ab; the eps_bgl M-contraction written out per column b
            T g = P[0][b] * div[0] + P[1][b] * div[1] + P[2][b] * div[2];
            const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
#pragma unroll
            for (int n = 0; n < 3; ++n) g += P[b1][n] * M[b2][n] - P[b2][n] * M[b1][n];
            Pi[a][b] = (a == b ? fdens : T(0)) + sig[a][b] - c.K * g + tau[a][b];
        }
    }
}

// Split coupling (Sec. 2.2, Eqs. (17)-(21)) at one site: the symmetric
// xi-stress that goes into the second moment of the equilibrium,
//   sigma^xi = 2 xi (Q + I/3)(Q:H) - xi (HQ + QH + 2H/3)
// (upper triangle xx, xy, xz, yy, yz, zz), the antisymmetric stress
// tau = QH - HQ (xy, xz, yz), and h_a = -H:d_a Q, the divergence of the
// gradient and free-energy part of the stress by the identity of Eq. (21).
// The body force is b_a = d_b tau_ab + h_a.  Also returns f.
template <typename T>
__host__ __device__ __forceinline__ void site_split(const Coef<T> &c, const T q[5], const T d[3][5], const T lap[5],
                                           T sig[6], T tau3[3], T h[3], T &fdens)
{
    T Q[3][3], dQ[3][3][3], CQ[3][3], Q2[3][3], trQ2, H5[5];
    full3(q, Q);
    full_grad(d, dQ);
    curl(dQ, CQ);
    molecular_field(c, Q, CQ, lap, H5, Q2, trQ2);
    T H[3][3];
    full3(H5, H);

    T M[3][3], div[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) M[a][b] = CQ[a][b] + c.q0x2 * Q[a][b];
        div[a] = dQ[0][a][0] + dQ[1][a][1] + dQ[2][a][2];
    }
    fdens = free_energy(c, Q, Q2, trQ2, div, M);

    T HQ[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) HQ[a][b] = H[a][0] * Q[0][b] + H[a][1] * Q[1][b] + H[a][2] * Q[2][b];
    T QdH = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) QdH += Q[a][b] * H[a][b];

    const T third = T(1) / T(3);
    const int ia[6] = {0, 0, 0, 1, 1, 2};
    const int ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int a = ia[k], b = ib[k];
        sig[k] = T(2) * c.xi * (Q[a][b] + (a == b ? third : T(0))) * QdH
               - c.xi * (HQ[a][b] + HQ[b][a] + T(2) * third * H[a][b]);
    }
    // (QH)_ab = (HQ)_ba for symmetric H and Q
    tau3[0] = HQ[1][0] - HQ[0][1];
    tau3[1] = HQ[2][0] - HQ[0][2];
    tau3[2] = HQ[2][1] - HQ[1][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T v = T(0);
#pragma unroll
        for (int g = 0; g < 3; ++g)
#pragma unroll
            for (int n = 0; n < 3; ++n) v += H[g][n] * dQ[a][g][n];
        h[a] = -v;
    }
}

// Molecular field from the stored components (the same H as molecular_field,
// written for the five components).
template <typename T>
__host__ __device__ __forceinline__ void molecular_field5(const Coef<T> &c, const T q[5], const T d[3][5],
                                                          const T lap[5], T H[5])
{
    const T qzz = -q[0] - q[3];
    T s[6], trQ2, C[5];
    square_sym(q, qzz, s, trQ2);
    curl_sym(d, C);
    const T third = T(1) / T(3);
    const T lin = -(c.a + c.bg * trQ2 + c.Kq0sq4);
    const T diag = c.bg * trQ2 * third;
    const int k2s[5] = {0, 1, 2, 3, 4};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        T v = lin * q[k] + c.bg * s[k2s[k]] + c.K * lap[k] - c.Kq0x2 * C[k];
        if (k == 0 || k == 3) v -= diag;
        H[k] = v;
    }
}

// Right-hand side of the Q equation (Eqs. (2)-(4)) projected on symmetric
// traceless tensors:
//   R = P_T[ -u.grad Q + S(W,Q) + Gamma H ],
//   S = (xi D + w)(Q + I/3) + (Q + I/3)(xi D - w) - 2 xi (Q + I/3) tr(QW),
//   D = (W + W^T)/2, w = (W - W^T)/2, W_ab = d_b u_a.
// Written with M = xi D + w: the first two terms are M Q + (M Q)^T + (2 xi/3) D
// (Q symmetric, so Q M^T = (M Q)^T), tr(QW) = Q:W, and tr S = (2 xi/3) div u
// is the only trace in the bracket (u.grad Q and H are traceless), so the
// projection removes (2 xi/9) div u from the diagonal.
template <typename T>
__host__ __device__ __forceinline__ void site_rhs(const Coef<T> &c, const T q[5], const T d[3][5], const T lap[5],
                                                  const T u[3], const T W[3][3], T R[5])
{
    T H[5];
    molecular_field5(c, q, d, lap, H);
    const T qzz = -q[0] - q[3];
    const T Q[3][3] = {{q[0], q[1], q[2]}, {q[1], q[3], q[4]}, {q[2], q[4], qzz}};
    const T hp = T(0.5) * (c.xi + T(1)), hm = T(0.5) * (c.xi - T(1));
    T M[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) M[a][b] = a == b ? c.xi * W[a][a] : hp * W[a][b] + hm * W[b][a];
    // M Q, the entries the five stored components of S need
    T P[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) P[a][b] = M[a][0] * Q[0][b] + M[a][1] * Q[1][b] + M[a][2] * Q[2][b];
    const T s01 = W[0][1] + W[1][0], s02 = W[0][2] + W[2][0], s12 = W[1][2] + W[2][1];
    const T QW = q[0] * W[0][0] + q[3] * W[1][1] + qzz * W[2][2] + q[1] * s01 + q[2] * s02 + q[4] * s12;
    const T third = T(1) / T(3);
    const T t = T(-2) * c.xi * QW;
    const T x3 = c.xi * third;
    const T dtr = T(2) * x3 * (W[0][0] + W[1][1] + W[2][2]) * third;  // (2 xi/9) div u
    const T S[5] = {T(2) * P[0][0] + T(2) * x3 * W[0][0] + t * (q[0] + third) - dtr,
                    (P[0][1] + P[1][0]) + x3 * s01 + t * q[1],
                    (P[0][2] + P[2][0]) + x3 * s02 + t * q[2],
                    T(2) * P[1][1] + T(2) * x3 * W[1][1] + t * (q[3] + third) - dtr,
                    (P[1][2] + P[2][1]) + x3 * s12 + t * q[4]};
#pragma unroll
    for (int k = 0; k < 5; ++k) R[k] = -(u[0] * d[0][k] + u[1] * d[1][k] + u[2] * d[2][k]) + S[k] + c.Gamma * H[k];
}

// ---------------------------------------------------------------- D3Q19
// Velocity order (also the order of the populations in the state):
// 0 rest; 1..6 = +x -x +y -y +z -z; 7..18 = edges (+x+y)(-x-y)(+x-y)(-x+y)
// (+x+z)(-x-z)(+x-z)(-x+z)(+y+z)(-y-z)(+y-z)(-y+z).  Weights 1/3, 1/18, 1/36.
constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

template <typename T>
__host__ __device__ __forceinline__ T lb_weight(int i)
{
    return i == 0 ? T(1) / T(3) : (i <= 6 ? T(1) / T(18) : T(1) / T(36));
}

// Density deviation and bare momentum of the pulled deviations; pairs of
// opposite velocities are differenced first so the momentum keeps the
// precision of the small dynamical part.
template <typename T>
__host__ __device__ __forceinline__ void lb_moments(const T g[19], T &drho, T j[3])
{
    T s = T(0);
#pragma unroll
    for (int i = 0; i < 19; ++i) s += g[i];
    drho = s;
    j[0] = (g[1] - g[2]) + (g[7] - g[8]) + (g[9] - g[10]) + (g[11] - g[12]) + (g[13] - g[14]);
    j[1] = (g[3] - g[4]) + (g[7] - g[8]) + (g[10] - g[9]) + (g[15] - g[16]) + (g[17] - g[18]);
    j[2] = (g[5] - g[6]) + (g[11] - g[12]) + (g[14] - g[13]) + (g[15] - g[16]) + (g[18] - g[17]);
}

// a b + c with one rounding in either precision.  The collision spells out
// its fused products so that every inlined copy of it rounds alike.
template <typename T>
__host__ __device__ __forceinline__ T fmat(T a, T b, T c)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_fma(a, b, c);
}

// Update of the opposite pair (i, i+1), e_{i+1} = -e_i, from the even part s
// (the same for both) and the odd part o of omega g^eq + src:
//   s = c0 + a2 (e.u)^2 + b2 (e.u)(e.F),  o = a1 (e.u) + b1 (e.F).
template <typename T>
__host__ __device__ __forceinline__ void lb_pair(T g[19], int i, T keep, T c0, T a2, T b2, T a1, T b1, T eu, T eF)
{
    const T s = fmat(eu, fmat(a2, eu, b2 * eF), c0);
    const T o = fmat(a1, eu, b1 * eF);
    g[i] = fmat(keep, g[i], s + o);
    g[i + 1] = fmat(keep, g[i + 1], s - o);
}

// BGK collision with second-order forcing on the deviations (Eq. (16) on
// D3Q19): rho = rho0 + drho, u = (j + F/2)/rho,
//   g_i' = g_i - (g_i - g_i^eq)/tau + (1 - 1/(2 tau)) w_i [3(e_i - u) + 9 (e_i.u) e_i].F,
//   g_i^eq = w_i drho + w_i rho (3 e.u + 9/2 (e.u)^2 - 3/2 u^2)
// and, with SIG (the split coupling, Eq. (17)), the symmetric stress sig
// (xx, xy, xz, yy, yz, zz) in the second moment of the equilibrium,
//   g_i^eq += -(9/2) w_i [sig:e_i e_i - tr(sig)/3],
// a term with zero mass and momentum.  Evaluated per pair of opposite
// velocities: with keep = 1 - omega, omega g^eq + src is
//   w [omega (drho - (3/2) rho u^2) - 3 pref u.F + (9/2) omega rho (e.u)^2
//      + 9 pref (e.u)(e.F) - (9/2) omega (sig:ee - tr(sig)/3)]      (even in e)
//   + w [3 omega rho (e.u) + 3 pref (e.F)]                           (odd in e).
// g is updated in place; u and rho are returned.
template <typename T, bool SIG>
__host__ __device__ __forceinline__ void lb_update(const Coef<T> &c, T g[19], const T F[3], const T *sig, T u[3],
                                                   T &rho)
{
    T drho, j[3];
    lb_moments(g, drho, j);
    rho = c.rho0 + drho;
    const T irho = T(1) / rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + T(0.5) * F[a]) * irho;
    const T uu15 = T(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const T uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    const T keep = T(1) - c.omega;
    const T orho = c.omega * rho;
    const T base = fmat(c.omega, fmat(-rho, uu15, drho), T(-3) * c.pref * uF);
    // faces (w = 1/18) and edges (w = 1/36)
    const T c1 = (T(1) / T(18)) * base, c2 = (T(1) / T(36)) * base;
    T c0 = (T(1) / T(3)) * base;
    const T a21 = T(0.25) * orho, a22 = T(0.125) * orho;
    const T b21 = T(0.5) * c.pref, b22 = T(0.25) * c.pref;
    const T a11 = (T(1) / T(6)) * orho, a12 = (T(1) / T(12)) * orho;
    const T b11 = (T(1) / T(6)) * c.pref, b12 = (T(1) / T(12)) * c.pref;
    T cx = c1, cy = c1, cz = c1, cxy = c2, cxy_ = c2, cxz = c2, cxz_ = c2, cyz = c2, cyz_ = c2;
    if constexpr (SIG) {
        const T tr3 = (sig[0] + sig[3] + sig[5]) / T(3);
        const T m1 = T(-0.25) * c.omega, m2 = T(-0.125) * c.omega;
        c0 = fmat(T(1.5) * c.omega, tr3, c0);  // the rest velocity: sig:ee = 0
        cx = fmat(m1, sig[0] - tr3, c1);
        cy = fmat(m1, sig[3] - tr3, c1);
        cz = fmat(m1, sig[5] - tr3, c1);
        const T exy = (sig[0] + sig[3]) - tr3, exz = (sig[0] + sig[5]) - tr3, eyz = (sig[3] + sig[5]) - tr3;
        cxy = fmat(m2, fmat(T(2), sig[1], exy), c2);
        cxy_ = fmat(m2, fmat(T(-2), sig[1], exy), c2);
        cxz = fmat(m2, fmat(T(2), sig[2], exz), c2);
        cxz_ = fmat(m2, fmat(T(-2), sig[2], exz), c2);
        cyz = fmat(m2, fmat(T(2), sig[4], eyz), c2);
        cyz_ = fmat(m2, fmat(T(-2), sig[4], eyz), c2);
    }
    g[0] = fmat(keep, g[0], c0);
    lb_pair(g, 1, keep, cx, a21, b21, a11, b11, u[0], F[0]);
    lb_pair(g, 3, keep, cy, a21, b21, a11, b11, u[1], F[1]);
    lb_pair(g, 5, keep, cz, a21, b21, a11, b11, u[2], F[2]);
    lb_pair(g, 7, keep, cxy, a22, b22, a12, b12, u[0] + u[1], F[0] + F[1]);
    lb_pair(g, 9, keep, cxy_, a22, b22, a12, b12, u[0] - u[1], F[0] - F[1]);
    lb_pair(g, 11, keep, cxz, a22, b22, a12, b12, u[0] + u[2], F[0] + F[2]);
    lb_pair(g, 13, keep, cxz_, a22, b22, a12, b12, u[0] - u[2], F[0] - F[2]);
    lb_pair(g, 15, keep, cyz, a22, b22, a12, b12, u[1] + u[2], F[1] + F[2]);
    lb_pair(g, 17, keep, cyz_, a22, b22, a12, b12, u[1] - u[2], F[1] - F[2]);
}

template <typename T>
__host__ __device__ __forceinline__ void lb_collide(const Coef<T> &c, T g[19], const T F[3], T u[3], T &rho)
{
    lb_update<T, false>(c, g, F, nullptr, u, rho);
}

// The same collision in the split coupling: F is the split body force b and
// sig the symmetric stress of the equilibrium.
template <typename T>
__host__ __device__ __forceinline__ void lb_collide_split(const Coef<T> &c, T g[19], const T F[3], const T sig[6], T u[3],
                                                 T &rho)
{
    lb_update<T, true>(c, g, F, sig, u, rho);
}

// ---------------------------------------------------------------- D3Q15
// The paper's own lattice (Sec. 2.2): rest, 6 faces, 8 corners, in this
// order; populations stored as deviations g_i = f_i - A_s(rho0) at their own
// site (no pull offset).
constexpr int DX15[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
constexpr int DY15[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
constexpr int DZ15[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};

// Equilibrium deviation of velocity i, the printed polynomial
//   A_s + B_s u.e + C_s u^2 + D_s (u.e)^2 + E_s:e e
// with the printed coefficients at T = 1/3: A_1 = A_2 = rho/30,
// A_0 = rho - 14 A_2; B = (rho/3, rho/24); C = (-2rho/3, -rho/12, -rho/24);
// D = (rho/2, rho/16); E_2 = -(sig - tr(sig)/3 I)/16, E_1 = 8 E_2 (faces,
// corners).  sig: upper triangle xx, xy, xz, yy, yz, zz (null: no stress).
template <typename T>
__host__ __device__ __forceinline__ T lb15_eq(int i, T rho0, T rho, const T u[3], T uu, const T *sig)
{
    const T ex = T(DX15[i]), ey = T(DY15[i]), ez = T(DZ15[i]);
    const T eu = ex * u[0] + ey * u[1] + ez * u[2];
    const T dr = rho - rho0;
    T v;
    if (i == 0) {
        v = dr - T(14) * (dr / T(30)) - T(2) * rho / T(3) * uu;
    } else if (i <= 6) {
        v = dr / T(30) + rho / T(3) * eu - rho / T(12) * uu + rho / T(2) * eu * eu;
    } else {
        v = dr / T(30) + rho / T(24) * eu - rho / T(24) * uu + rho / T(16) * eu * eu;
    }
    if (sig && i > 0) {
        const T tr3 = (sig[0] + sig[3] + sig[5]) / T(3);
        const T see = (sig[0] - tr3) * ex * ex + (sig[3] - tr3) * ey * ey + (sig[5] - tr3) * ez * ez
                    + T(2) * (sig[1] * ex * ey + sig[2] * ex * ez + sig[4] * ey * ez);
        v -= (i <= 6 ? T(8) : T(1)) * see / T(16);
    }
    return v;
}

// Forcing term p_i = P_s b.e with P_1 = 1/3, P_2 = 1/24.
template <typename T>
__host__ __device__ __forceinline__ T lb15_force(int i, const T b[3])
{
    if (i == 0) return T(0);
    const T eb = T(DX15[i]) * b[0] + T(DY15[i]) * b[1] + T(DZ15[i]) * b[2];
    return (i <= 6 ? T(1) / T(3) : T(1) / T(24)) * eb;
}

// Collision operator of Eq. (16) on D3Q15 at one site: local moments
// (rho u = sum f e, Eq. (14)), C_i = -(g_i - g_i^eq)/tau + p_i.
template <typename T>
__host__ __device__ __forceinline__ void lb15_collide(const Coef<T> &c, const T g[15], const T *sig, const T b[3], T C[15],
                                             T u[3], T &rho)
{
    T drho = T(0), j[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < 15; ++i) {
        drho += g[i];
        j[0] += T(DX15[i]) * g[i];
        j[1] += T(DY15[i]) * g[i];
        j[2] += T(DZ15[i]) * g[i];
    }
    rho = c.rho0 + drho;
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < 15; ++i) C[i] = -(g[i] - lb15_eq(i, c.rho0, rho, u, uu, sig)) * c.omega + lb15_force(i, b);
}

// Equilibrium deviation for initialisation.
template <typename T>
__host__ __device__ __forceinline__ T lb_geq(const Coef<T> &c, int i, T rho, const T u[3])
{
    const T w = lb_weight<T>(i);
    const T eu = T(CX[i]) * u[0] + T(CY[i]) * u[1] + T(CZ[i]) * u[2];
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return w * (rho - c.rho0) + w * rho * (T(3) * eu + T(4.5) * eu * eu - T(1.5) * uu);
}

}  // namespace hlb
