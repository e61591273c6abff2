/*
 * hlb_oracle.c -- plain FP64 CPU oracle of the hybrid lattice-Boltzmann step
 * for cholesteric liquid crystals (Henrich, Marenduzzo, Stratford, Cates,
 * "Domain growth in cholesteric blue phases: hybrid lattice Boltzmann
 * simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the product library never
 * links, includes or calls it, and it shares no source with it.
 *
 * Plain loops over a periodic nx*ny*nz lattice, dx = dt = 1, OpenMP over z,
 * built with -O2 -ffp-contract=off and no fast-math.  Q is held as a full
 * 3x3 tensor per site (nine SoA planes, component (a,b) at plane 3a+b) so
 * that its symmetry and trace stay checkable.
 *
 * What each routine follows (equation numbers as printed in the paper):
 *   free-energy density f ........ Sec. 2.1, Eq. (1), plus the divergence
 *                                  term K/2 (d_b Q_ab)^2 of the one-constant
 *                                  approximation named under Eq. (1)
 *   molecular field H ............ Sec. 2.1, Eq. (2): symmetric, traceless
 *                                  part of -dF/dQ
 *   co-rotation S(W,Q) ........... Sec. 2.1, Eqs. (3)-(4), W_ab = d_b u_a
 *   stress Pi = sigma + tau ...... Sec. 2.1, Eqs. (6)-(8); the rho*T part of
 *                                  P0 = rho*T - f is the LB pressure
 *   body force b_a = d_b Pi_ab ... Sec. 2.2, Eq. (19): the whole chemical
 *                                  stress enters as a force (centred
 *                                  divergence on the second index)
 *   D3Q15 predictor-corrector LB . Sec. 2.2, Eqs. (11)-(23): the paper's own
 *                                  lattice, equilibrium and forcing terms as
 *                                  the printed polynomial with the printed
 *                                  coefficients, stepped by the trapezoidal
 *                                  (predictor-corrector) rule of Eq. (15)
 *   split coupling ............... Sec. 2.2, Eqs. (17)-(21): the symmetric
 *                                  xi-stress enters the second moment of the
 *                                  equilibrium, the body force is the
 *                                  divergence of the antisymmetric stress
 *                                  minus H : grad Q
 *   moments ...................... Sec. 2.2, Eq. (14), velocity with +F/2
 *   BGK collision + forcing ...... Sec. 2.2, Eq. (16), on D3Q19 with the
 *                                  second-order (Guo) forcing term
 *   Q update ..................... Sec. 2.2: finite-difference predictor-
 *                                  corrector (Heun) for Eq. (2) with the
 *                                  material derivative of Eq. (3)
 *   coupling order ............... Sec. 2.2: force from Q^n, LB step gives
 *                                  u^n, then Q^n -> Q^{n+1} with u^n
 *
 * LB populations are carried as deviations g_i = f_i - w_i rho0 (an exact
 * change of variable) so FP64 rounding is relative to the small dynamical
 * part, not to w_i rho0.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double tau;    /* BGK relaxation time (lattice units)                  */
    double rho0;   /* reference density; g_i = f_i - w_i rho0            */
    double A0;     /* bulk free-energy scale, Eq. (1)                     */
    double gamma;  /* temperature-like control parameter, Eq. (1)         */
    double K;      /* one elastic constant, Eq. (1)                       */
    double q0;     /* 2 pi / pitch, Eq. (1)                               */
    double Gamma;  /* collective rotational diffusion constant, Eq. (2)   */
    double xi;     /* flow-aligning parameter, Eqs. (4), (7)              */
    int flow;      /* 0: u == 0 (Sec. 2.1); 1: coupled, whole stress as a
                    * body force; 2: coupled, split coupling (Sec. 2.2)  */
    int lb_model;  /* 0: D3Q19 BGK with second-order forcing (pull);
                    * 1: D3Q15 predictor-corrector of Sec. 2.2          */
} or_params;

static int n_pop(const or_params *p) { return p->lb_model == 1 ? 15 : 19; }

/* ------------------------------------------------------------------------ */
/* D3Q19 velocity set: rest, 6 faces, 12 edges; weights 1/3, 1/18, 1/36.     */
static const int E[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight(int i)
{
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

void or_lattice(int *e, double *w)
{
    for (int i = 0; i < 19; i++) {
        for (int a = 0; a < 3; a++) e[3 * i + a] = E[i][a];
        w[i] = weight(i);
    }
}

/* ------------------------------------------------------------------------ */
static int wrap(int i, int n) { return ((i % n) + n) % n; }

static long site(int x, int y, int z, int nx, int ny, int nz)
{
    return (long)wrap(x, nx) + (long)nx * ((long)wrap(y, ny) + (long)ny * wrap(z, nz));
}

static double levi(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0.0;
    /* even permutations of (0,1,2) */
    if ((a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0)) return 1.0;
    return -1.0;
}

static void load9(const double *Q9, long N, long s, double Q[3][3])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) Q[a][b] = Q9[(3 * a + b) * N + s];
}

/* five stored components (xx, xy, xz, yy, yz) <-> full tensor */
void or_q5_to_q9(long N, const double *Q5, double *Q9)
{
    for (long s = 0; s < N; s++) {
        double xx = Q5[0 * N + s], xy = Q5[1 * N + s], xz = Q5[2 * N + s];
        double yy = Q5[3 * N + s], yz = Q5[4 * N + s];
        double zz = -xx - yy;
        double T[3][3] = {{xx, xy, xz}, {xy, yy, yz}, {xz, yz, zz}};
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Q9[(3 * a + b) * N + s] = T[a][b];
    }
}

void or_q9_to_q5(long N, const double *Q9, double *Q5)
{
    for (long s = 0; s < N; s++) {
        Q5[0 * N + s] = Q9[0 * N + s];
        Q5[1 * N + s] = Q9[1 * N + s];
        Q5[2 * N + s] = Q9[2 * N + s];
        Q5[3 * N + s] = Q9[4 * N + s];
        Q5[4 * N + s] = Q9[5 * N + s];
    }
}

/* Centred first derivatives dQ[g][a][b] = d_g Q_ab and the 7-point Laplacian
 * at one site (second-order finite differences, dx = 1). */
static void derivs(const double *Q9, int nx, int ny, int nz, int x, int y, int z,
                   double Q[3][3], double dQ[3][3][3], double lap[3][3])
{
    long N = (long)nx * ny * nz;
    long s = site(x, y, z, nx, ny, nz);
    long sp[3] = {site(x + 1, y, z, nx, ny, nz), site(x, y + 1, z, nx, ny, nz),
                  site(x, y, z + 1, nx, ny, nz)};
    long sm[3] = {site(x - 1, y, z, nx, ny, nz), site(x, y - 1, z, nx, ny, nz),
                  site(x, y, z - 1, nx, ny, nz)};
    load9(Q9, N, s, Q);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            const double *P = Q9 + (3 * a + b) * N;
            double sum = 0.0;
            for (int g = 0; g < 3; g++) {
                dQ[g][a][b] = 0.5 * (P[sp[g]] - P[sm[g]]);
                sum += P[sp[g]] + P[sm[g]];
            }
            lap[a][b] = sum - 6.0 * Q[a][b];
        }
}

/* (C Q)_ab = eps_agd d_g Q_db, the curl appearing in Eq. (1). */
static void curlQ(double dQ[3][3][3], double CQ[3][3])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double s = 0.0;
            for (int g = 0; g < 3; g++)
                for (int d = 0; d < 3; d++) s += levi(a, g, d) * dQ[g][d][b];
            CQ[a][b] = s;
        }
}

static void matmul(double A[3][3], double B[3][3], double C[3][3])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double s = 0.0;
            for (int c = 0; c < 3; c++) s += A[a][c] * B[c][b];
            C[a][b] = s;
        }
}

static double ddot(double A[3][3], double B[3][3])
{
    double s = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) s += A[a][b] * B[a][b];
    return s;
}

static double trace(double A[3][3]) { return A[0][0] + A[1][1] + A[2][2]; }

/* Free-energy density, Eq. (1) with the divergence term of the one-constant
 * approximation:
 *   f = A0/2 (1 - gamma/3) Q:Q - A0 gamma/3 tr(Q^3) + A0 gamma/4 (Q:Q)^2
 *       + K/2 (d_b Q_ab)^2 + K/2 M:M,   M_ab = eps_agd d_g Q_db + 2 q0 Q_ab. */
static double free_energy(const or_params *p, double Q[3][3], double dQ[3][3][3])
{
    double Q2[3][3], Q3[3][3], CQ[3][3], M[3][3];
    matmul(Q, Q, Q2);
    matmul(Q2, Q, Q3);
    curlQ(dQ, CQ);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) M[a][b] = CQ[a][b] + 2.0 * p->q0 * Q[a][b];
    double qq = ddot(Q, Q);
    double bulk = 0.5 * p->A0 * (1.0 - p->gamma / 3.0) * qq
                - p->A0 * p->gamma / 3.0 * trace(Q3)
                + 0.25 * p->A0 * p->gamma * qq * qq;
    double div2 = 0.0;
    for (int a = 0; a < 3; a++) {
        double d = 0.0;
        for (int b = 0; b < 3; b++) d += dQ[b][a][b];
        div2 += d * d;
    }
    return bulk + 0.5 * p->K * div2 + 0.5 * p->K * ddot(M, M);
}

/* Molecular field, Eq. (2): H = -[sym(dF/dQ) - tr(dF/dQ)/3 I].
 * Symmetric part of the functional derivative of the free energy above:
 *   sym(dF/dQ) = A0(1-gamma/3) Q - A0 gamma Q^2 + A0 gamma (Q:Q) Q
 *                - K lap Q + 2 K q0 (CQ + CQ^T) + 4 K q0^2 Q
 * (the divergence term only adds an antisymmetric part, which the
 * symmetrisation removes). */
static void molecular_field(const or_params *p, double Q[3][3], double dQ[3][3][3],
                            double lap[3][3], double H[3][3])
{
    double Q2[3][3], CQ[3][3], G[3][3];
    matmul(Q, Q, Q2);
    curlQ(dQ, CQ);
    double qq = ddot(Q, Q);
    double a = p->A0 * (1.0 - p->gamma / 3.0);
    double bg = p->A0 * p->gamma;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            G[i][j] = a * Q[i][j] - bg * Q2[i][j] + bg * qq * Q[i][j]
                    - p->K * lap[i][j]
                    + 2.0 * p->K * p->q0 * (CQ[i][j] + CQ[j][i])
                    + 4.0 * p->K * p->q0 * p->q0 * Q[i][j];
    double tr = trace(G);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            H[i][j] = -(0.5 * (G[i][j] + G[j][i]) - (i == j ? tr / 3.0 : 0.0));
}

/* Chemical stress, Eqs. (6)-(8), without the rho*T part of P0:
 *   Pi_ab = f d_ab + 2 xi A_ab (Q:H) - xi (H A)_ab - xi (A H)_ab
 *           - d_a Q_gn Phi_gnb + (Q H - H Q)_ab,
 * A = Q + I/3, Phi_gnb = df/d(d_b Q_gn) = K [d_nb (d_m Q_gm) + eps_lbg M_ln]. */
static void stress(const or_params *p, double Q[3][3], double dQ[3][3][3],
                   double H[3][3], double fd, double Pi[3][3])
{
    double CQ[3][3], M[3][3], A[3][3], HA[3][3], AH[3][3], QH[3][3], HQ[3][3];
    double divQ[3], Phi[3][3][3];
    curlQ(dQ, CQ);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            M[a][b] = CQ[a][b] + 2.0 * p->q0 * Q[a][b];
            A[a][b] = Q[a][b] + (a == b ? 1.0 / 3.0 : 0.0);
        }
    for (int g = 0; g < 3; g++) {
        double d = 0.0;
        for (int m = 0; m < 3; m++) d += dQ[m][g][m];
        divQ[g] = d;
    }
    for (int g = 0; g < 3; g++)
        for (int n = 0; n < 3; n++)
            for (int b = 0; b < 3; b++) {
                double s = (n == b) ? divQ[g] : 0.0;
                for (int l = 0; l < 3; l++) s += levi(l, b, g) * M[l][n];
                Phi[g][n][b] = p->K * s;
            }
    matmul(H, A, HA);
    matmul(A, H, AH);
    matmul(Q, H, QH);
    matmul(H, Q, HQ);
    double QdH = ddot(Q, H);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double grad = 0.0;
            for (int g = 0; g < 3; g++)
                for (int n = 0; n < 3; n++) grad += dQ[a][g][n] * Phi[g][n][b];
            Pi[a][b] = (a == b ? fd : 0.0)
                     + 2.0 * p->xi * A[a][b] * QdH
                     - p->xi * HA[a][b] - p->xi * AH[a][b]
                     - grad
                     + QH[a][b] - HQ[a][b];
        }
}

/* H (9 planes), free-energy density and stress Pi (9 planes, [3a+b]) on the
 * whole lattice; any output may be NULL. */
void or_chem(const or_params *p, int nx, int ny, int nz, const double *Q9,
             double *H9, double *fdens, double *Pi9)
{
    long N = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                double Q[3][3], dQ[3][3][3], lap[3][3], H[3][3], Pi[3][3];
                long s = site(x, y, z, nx, ny, nz);
                derivs(Q9, nx, ny, nz, x, y, z, Q, dQ, lap);
                molecular_field(p, Q, dQ, lap, H);
                double fd = free_energy(p, Q, dQ);
                if (fdens) fdens[s] = fd;
                if (H9)
                    for (int a = 0; a < 9; a++) H9[a * N + s] = H[a / 3][a % 3];
                if (Pi9) {
                    stress(p, Q, dQ, H, fd, Pi);
                    for (int a = 0; a < 9; a++) Pi9[a * N + s] = Pi[a / 3][a % 3];
                }
            }
}

/* Body force F_a = sum_b [Pi_ab(x + e_b) - Pi_ab(x - e_b)] / 2. */
void or_force(const or_params *p, int nx, int ny, int nz, const double *Q9, double *F3)
{
    long N = (long)nx * ny * nz;
    double *Pi9 = (double *)malloc(sizeof(double) * 9 * N);
    or_chem(p, nx, ny, nz, Q9, NULL, NULL, Pi9);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long s = site(x, y, z, nx, ny, nz);
                long sp[3] = {site(x + 1, y, z, nx, ny, nz), site(x, y + 1, z, nx, ny, nz),
                              site(x, y, z + 1, nx, ny, nz)};
                long sm[3] = {site(x - 1, y, z, nx, ny, nz), site(x, y - 1, z, nx, ny, nz),
                              site(x, y, z - 1, nx, ny, nz)};
                for (int a = 0; a < 3; a++) {
                    double F = 0.0;
                    for (int b = 0; b < 3; b++) {
                        const double *P = Pi9 + (3 * a + b) * N;
                        F += 0.5 * (P[sp[b]] - P[sm[b]]);
                    }
                    F3[a * N + s] = F;
                }
            }
    free(Pi9);
}

/* Split coupling, Sec. 2.2.  The stress of Eqs. (6)-(8) is divided as
 *   sigma^xi_ab = 2 xi A_ab (Q:H) - xi (H A)_ab - xi (A H)_ab   (A = Q + I/3),
 *   tau_ab      = (Q H - H Q)_ab,
 * and the remaining gradient and free-energy terms; by the identity of
 * Eq. (21) the divergence of the remainder equals -H_gn d_a Q_gn.  The
 * symmetric sigma^xi is carried by the second moment of the equilibrium
 * (Eq. (17)); the body force of Eq. (19) becomes
 *   b_a = d_b tau_ab - H_gn d_a Q_gn
 * with the divergence taken centred on the second index, as for the whole
 * stress.  sig9 (9 planes) may be NULL. */
void or_split(const or_params *p, int nx, int ny, int nz, const double *Q9, double *sig9, double *b3)
{
    long N = (long)nx * ny * nz;
    double *tau9 = (double *)malloc(sizeof(double) * 9 * N);
    double *h3 = (double *)malloc(sizeof(double) * 3 * N);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                double Q[3][3], dQ[3][3][3], lap[3][3], H[3][3], A[3][3], HA[3][3], AH[3][3], QH[3][3],
                    HQ[3][3];
                long s = site(x, y, z, nx, ny, nz);
                derivs(Q9, nx, ny, nz, x, y, z, Q, dQ, lap);
                molecular_field(p, Q, dQ, lap, H);
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) A[a][b] = Q[a][b] + (a == b ? 1.0 / 3.0 : 0.0);
                matmul(H, A, HA);
                matmul(A, H, AH);
                matmul(Q, H, QH);
                matmul(H, Q, HQ);
                double QdH = ddot(Q, H);
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) {
                        if (sig9)
                            sig9[(3 * a + b) * N + s] =
                                2.0 * p->xi * A[a][b] * QdH - p->xi * HA[a][b] - p->xi * AH[a][b];
                        tau9[(3 * a + b) * N + s] = QH[a][b] - HQ[a][b];
                    }
                for (int a = 0; a < 3; a++) h3[a * N + s] = -ddot(H, dQ[a]);
            }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long s = site(x, y, z, nx, ny, nz);
                long sp[3] = {site(x + 1, y, z, nx, ny, nz), site(x, y + 1, z, nx, ny, nz),
                              site(x, y, z + 1, nx, ny, nz)};
                long sm[3] = {site(x - 1, y, z, nx, ny, nz), site(x, y - 1, z, nx, ny, nz),
                              site(x, y, z - 1, nx, ny, nz)};
                for (int a = 0; a < 3; a++) {
                    double d = 0.0;
                    for (int b = 0; b < 3; b++) {
                        const double *T = tau9 + (3 * a + b) * N;
                        d += 0.5 * (T[sp[b]] - T[sm[b]]);
                    }
                    b3[a * N + s] = d + h3[a * N + s];
                }
            }
    free(tau9);
    free(h3);
}

/* The force the LB step takes for this coupling: the centred divergence of
 * the whole stress (flow = 1) or the split body force b (flow = 2). */
static void coupling_force(const or_params *p, int nx, int ny, int nz, const double *Q9, double *sig9,
                           double *F3)
{
    if (p->flow == 2)
        or_split(p, nx, ny, nz, Q9, sig9, F3);
    else
        or_force(p, nx, ny, nz, Q9, F3);
}

/* Right-hand side of the Q equation, Eqs. (2)-(4):
 *   dQ/dt = -u.grad Q + S(W,Q) + Gamma H,   W_ab = d_b u_a (centred),
 * projected on symmetric traceless tensors, P_T(X) = sym(X) - tr(X)/3 I. */
static void rhs_site(const or_params *p, const double *Q9, const double *u3,
                     int nx, int ny, int nz, int x, int y, int z, double R[3][3])
{
    long N = (long)nx * ny * nz;
    long s = site(x, y, z, nx, ny, nz);
    double Q[3][3], dQ[3][3][3], lap[3][3], H[3][3];
    derivs(Q9, nx, ny, nz, x, y, z, Q, dQ, lap);
    molecular_field(p, Q, dQ, lap, H);

    long sp[3] = {site(x + 1, y, z, nx, ny, nz), site(x, y + 1, z, nx, ny, nz),
                  site(x, y, z + 1, nx, ny, nz)};
    long sm[3] = {site(x - 1, y, z, nx, ny, nz), site(x, y - 1, z, nx, ny, nz),
                  site(x, y, z - 1, nx, ny, nz)};
    double u[3], W[3][3];
    for (int a = 0; a < 3; a++) {
        u[a] = u3[a * N + s];
        for (int b = 0; b < 3; b++) W[a][b] = 0.5 * (u3[a * N + sp[b]] - u3[a * N + sm[b]]);
    }
    double D[3][3], Om[3][3], A[3][3], L[3][3], Rm[3][3], T1[3][3], T2[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            D[a][b] = 0.5 * (W[a][b] + W[b][a]);
            Om[a][b] = 0.5 * (W[a][b] - W[b][a]);
            A[a][b] = Q[a][b] + (a == b ? 1.0 / 3.0 : 0.0);
        }
    double trQW = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) trQW += Q[a][b] * W[b][a];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            L[a][b] = p->xi * D[a][b] + Om[a][b];
            Rm[a][b] = p->xi * D[a][b] - Om[a][b];
        }
    matmul(L, A, T1);
    matmul(A, Rm, T2);
    double X[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double S = T1[a][b] + T2[a][b] - 2.0 * p->xi * A[a][b] * trQW;
            double adv = 0.0;
            for (int g = 0; g < 3; g++) adv += u[g] * dQ[g][a][b];
            X[a][b] = -adv + S + p->Gamma * H[a][b];
        }
    double tr = trace(X);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            R[a][b] = 0.5 * (X[a][b] + X[b][a]) - (a == b ? tr / 3.0 : 0.0);
}

void or_rhs(const or_params *p, int nx, int ny, int nz, const double *Q9,
            const double *u3, double *R9)
{
    long N = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                double R[3][3];
                rhs_site(p, Q9, u3, nx, ny, nz, x, y, z, R);
                long s = site(x, y, z, nx, ny, nz);
                for (int a = 0; a < 9; a++) R9[a * N + s] = R[a / 3][a % 3];
            }
}

/* Predictor-corrector (Heun) with the velocity held at u^n:
 *   Q* = Q + R(Q, u),   Q' = Q + [R(Q, u) + R(Q*, u)] / 2. */
void or_qupdate(const or_params *p, int nx, int ny, int nz, const double *Q9in,
                const double *u3, double *Q9out)
{
    long N = (long)nx * ny * nz;
    double *R1 = (double *)malloc(sizeof(double) * 9 * N);
    double *R2 = (double *)malloc(sizeof(double) * 9 * N);
    double *Qs = (double *)malloc(sizeof(double) * 9 * N);
    or_rhs(p, nx, ny, nz, Q9in, u3, R1);
    for (long k = 0; k < 9 * N; k++) Qs[k] = Q9in[k] + R1[k];
    or_rhs(p, nx, ny, nz, Qs, u3, R2);
    for (long k = 0; k < 9 * N; k++) Q9out[k] = Q9in[k] + 0.5 * (R1[k] + R2[k]);
    free(R1);
    free(R2);
    free(Qs);
}

/* Equilibrium deviation g_i^eq = f_i^eq - w_i rho0 with
 * f_i^eq = w_i rho [1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u^2]. */
static double geq(int i, double rho0, double rho, const double u[3])
{
    double w = weight(i);
    double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return w * (rho - rho0) + w * rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

/* Stress part of the equilibrium in the split coupling: the Hermite term
 * whose second moment is -sigma and whose zeroth and first moments vanish,
 *   -(9/2) w_i [sigma_ab e_ia e_ib - tr(sigma)/3]   (c_s^2 = 1/3). */
static double geq_stress(int i, const double sig[3][3])
{
    double see = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) see += sig[a][b] * E[i][a] * E[i][b];
    return -4.5 * weight(i) * (see - (sig[0][0] + sig[1][1] + sig[2][2]) / 3.0);
}

/* Pull the populations arriving at x: g~_i(x) = g_i(x - e_i). */
static void pull(const double *g, long N, int nx, int ny, int nz, int x, int y, int z,
                 double gt[19])
{
    for (int i = 0; i < 19; i++)
        gt[i] = g[i * N + site(x - E[i][0], y - E[i][1], z - E[i][2], nx, ny, nz)];
}

/* One LB step (pull stream, BGK collide, forcing), Eqs. (14), (16):
 *   rho = rho0 + sum g~,  rho u = sum g~ e + F/2,
 *   g' = g~ - (g~ - g^eq)/tau + (1 - 1/(2 tau)) w [3(e - u) + 9 (e.u) e].F
 * with, when sig9 is given (split coupling), the stress term of geq_stress
 * added to g^eq.  Outputs rho and u (may be NULL) are the moments used in
 * the collision. */
static void lb_step(const or_params *p, int nx, int ny, int nz, const double *g_in, const double *F3,
                    const double *sig9, double *g_out, double *rho_out, double *u3_out)
{
    long N = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long s = site(x, y, z, nx, ny, nz);
                double gt[19], F[3], u[3], j[3] = {0.0, 0.0, 0.0}, drho = 0.0;
                pull(g_in, N, nx, ny, nz, x, y, z, gt);
                for (int a = 0; a < 3; a++) F[a] = F3 ? F3[a * N + s] : 0.0;
                for (int i = 0; i < 19; i++) {
                    drho += gt[i];
                    for (int a = 0; a < 3; a++) j[a] += gt[i] * E[i][a];
                }
                double rho = p->rho0 + drho;
                for (int a = 0; a < 3; a++) u[a] = (j[a] + 0.5 * F[a]) / rho;
                double pref = 1.0 - 0.5 / p->tau;
                double sig[3][3];
                if (sig9)
                    for (int a = 0; a < 9; a++) sig[a / 3][a % 3] = sig9[a * N + s];
                for (int i = 0; i < 19; i++) {
                    double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
                    double src = 0.0;
                    for (int a = 0; a < 3; a++)
                        src += (3.0 * (E[i][a] - u[a]) + 9.0 * eu * E[i][a]) * F[a];
                    double Fi = pref * weight(i) * src;
                    double eq = geq(i, p->rho0, rho, u);
                    if (sig9) eq += geq_stress(i, sig);
                    g_out[i * N + s] = gt[i] - (gt[i] - eq) / p->tau + Fi;
                }
                if (rho_out) rho_out[s] = rho;
                if (u3_out)
                    for (int a = 0; a < 3; a++) u3_out[a * N + s] = u[a];
            }
}

void or_lb(const or_params *p, int nx, int ny, int nz, const double *g_in, const double *F3, double *g_out,
           double *rho_out, double *u3_out)
{
    lb_step(p, nx, ny, nz, g_in, F3, NULL, g_out, rho_out, u3_out);
}

/* The LB step of the split coupling: body force b3 and the symmetric stress
 * sig9 (9 planes) in the equilibrium. */
void or_lb_split(const or_params *p, int nx, int ny, int nz, const double *g_in, const double *b3,
                 const double *sig9, double *g_out, double *rho_out, double *u3_out)
{
    lb_step(p, nx, ny, nz, g_in, b3, sig9, g_out, rho_out, u3_out);
}

/* ------------------------------------------------------------------------ */
/* The paper's own LB (Sec. 2.2): D3Q15 -- rest, 6 faces, 8 corners -- with
 * the equilibrium and forcing term written as the printed polynomial
 *   f_i^eq = A_s + B_s u.e + C_s u^2 + D_s (u.e)^2 + E_s:e e,  p_i = P_s b.e,
 * s = 0, 1, 2 for |e|^2 = 0, 1, 3, and the printed coefficients (T = 1/3):
 *   A_2 = rho T/10, A_1 = A_2, A_0 = rho - 14 A_2; B_2 = rho/24, B_1 = 8 B_2;
 *   C_2 = -rho/24, C_1 = 2 C_2, C_0 = -2 rho/3; D_2 = rho/16, D_1 = 8 D_2;
 *   E_2 = -(sigma - tr(sigma)/3 I)/16, E_1 = 8 E_2; P_2 = 1/24, P_1 = 8 P_2.
 * Populations are carried as deviations g_i = f_i - A_s(rho0) and stored
 * where they are (no pull offset): f_i(x, t) at x. */
static const int E15[15][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

static const double T_LB = 1.0 / 3.0;

/* Equilibrium deviation of velocity i (sig may be NULL: no stress term). */
static double feq15(int i, double rho0, double rho, const double u[3], const double sig[3][3])
{
    const int s = i == 0 ? 0 : (i <= 6 ? 1 : 2);
    const double ex = E15[i][0], ey = E15[i][1], ez = E15[i][2];
    const double eu = ex * u[0] + ey * u[1] + ez * u[2];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double dr = rho - rho0;
    const double A2 = dr * T_LB / 10.0;
    double A, B, C, D, Es;
    if (s == 0) {
        A = dr - 14.0 * A2;
        B = 0.0;
        C = -2.0 * rho / 3.0;
        D = 0.0;
        Es = 0.0;
    } else if (s == 1) {
        A = A2;
        B = 8.0 * rho / 24.0;
        C = 2.0 * (-rho / 24.0);
        D = 8.0 * rho / 16.0;
        Es = 8.0;
    } else {
        A = A2;
        B = rho / 24.0;
        C = -rho / 24.0;
        D = rho / 16.0;
        Es = 1.0;
    }
    double v = A + B * eu + C * uu + D * eu * eu;
    if (sig && Es != 0.0) {
        const double e[3] = {ex, ey, ez};
        const double tr3 = (sig[0][0] + sig[1][1] + sig[2][2]) / 3.0;
        double see = 0.0;
        for (int a = 0; a < 3; a++)
            for (int c = 0; c < 3; c++) see += (sig[a][c] - (a == c ? tr3 : 0.0)) * e[a] * e[c];
        v += Es * (-see / 16.0);
    }
    return v;
}

/* Forcing term p_i = P_s b.e (b may be NULL). */
static double force15(int i, const double b[3])
{
    if (!b || i == 0) return 0.0;
    const double P = i <= 6 ? 8.0 / 24.0 : 1.0 / 24.0;
    return P * (E15[i][0] * b[0] + E15[i][1] * b[1] + E15[i][2] * b[2]);
}

/* Collision operator of Eq. (16) at one site for populations g (local
 * moments, rho u = sum f e as in Eq. (14)), into C; returns rho and u. */
static void collide15(const or_params *p, const double g[15], const double sig[3][3], const double b[3],
                      double C[15], double *rho_out, double u[3])
{
    double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 15; i++) {
        drho += g[i];
        for (int a = 0; a < 3; a++) j[a] += g[i] * E15[i][a];
    }
    const double rho = p->rho0 + drho;
    for (int a = 0; a < 3; a++) u[a] = j[a] / rho;
    for (int i = 0; i < 15; i++) C[i] = -(g[i] - feq15(i, p->rho0, rho, u, sig)) / p->tau + force15(i, b);
    *rho_out = rho;
}

/* One LB step of the paper's scheme, Eq. (15), with the equilibrium stress
 * sig9 (9 planes, may be NULL) and the body force b3 (may be NULL) held over
 * the step:
 *   f*_i(x + e_i) = f_i(x) + C_i(x, {f}),
 *   f_i(x + e_i, t + 1) = f_i(x) + [C_i(x, {f}) + C_i(x + e_i, {f*})] / 2.
 * rho and u (may be NULL) are the moments of f(x, t) (Eq. (14), those of the
 * first collision): the velocity u^n the Q update takes. */
void or_lb_pc(const or_params *p, int nx, int ny, int nz, const double *g_in, const double *b3,
              const double *sig9, double *g_out, double *rho_out, double *u3_out)
{
    long N = (long)nx * ny * nz;
    double *P = (double *)malloc(sizeof(double) * 15 * N);  /* f + C at the departure site */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long s = site(x, y, z, nx, ny, nz);
                double g[15], C[15], u[3], rho, sig[3][3], b[3];
                for (int i = 0; i < 15; i++) g[i] = g_in[i * N + s];
                if (sig9)
                    for (int a = 0; a < 9; a++) sig[a / 3][a % 3] = sig9[a * N + s];
                for (int a = 0; a < 3; a++) b[a] = b3 ? b3[a * N + s] : 0.0;
                collide15(p, g, sig9 ? sig : NULL, b, C, &rho, u);
                for (int i = 0; i < 15; i++) P[i * N + s] = g[i] + C[i];
                if (rho_out) rho_out[s] = rho;
                if (u3_out)
                    for (int a = 0; a < 3; a++) u3_out[a * N + s] = u[a];
            }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long s = site(x, y, z, nx, ny, nz);
                double fs[15], fo[15], C[15], u[3], rho, sig[3][3], b[3];
                for (int i = 0; i < 15; i++) {
                    long t = site(x - E15[i][0], y - E15[i][1], z - E15[i][2], nx, ny, nz);
                    fs[i] = P[i * N + t];
                    fo[i] = 0.5 * (g_in[i * N + t] + P[i * N + t]);
                }
                if (sig9)
                    for (int a = 0; a < 9; a++) sig[a / 3][a % 3] = sig9[a * N + s];
                for (int a = 0; a < 3; a++) b[a] = b3 ? b3[a * N + s] : 0.0;
                collide15(p, fs, sig9 ? sig : NULL, b, C, &rho, u);
                for (int i = 0; i < 15; i++) g_out[i * N + s] = fo[i] + 0.5 * C[i];
            }
    free(P);
}

/* Populations stored so that the first pull returns g^eq(rho(x), u(x)) at
 * every site x:  g_i(y) = g_i^eq(rho(y + e_i), u(y + e_i)).  For the D3Q15
 * scheme: g_i(x) = f_i^eq(rho(x), u(x)) - A_s(rho0) in place, without the
 * stress and force terms. */
void or_init_g(const or_params *p, int nx, int ny, int nz, const double *rho,
               const double *u3, double *g)
{
    long N = (long)nx * ny * nz;
    if (p->lb_model == 1) {
        for (long s = 0; s < N; s++) {
            double u[3] = {u3[s], u3[N + s], u3[2 * N + s]};
            for (int i = 0; i < 15; i++) g[i * N + s] = feq15(i, p->rho0, rho[s], u, NULL);
        }
        return;
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long s = site(x, y, z, nx, ny, nz);
                for (int i = 0; i < 19; i++) {
                    long t = site(x + E[i][0], y + E[i][1], z + E[i][2], nx, ny, nz);
                    double u[3] = {u3[t], u3[N + t], u3[2 * N + t]};
                    g[i * N + s] = geq(i, p->rho0, rho[t], u);
                }
            }
}

/* Density and velocity at the current time level: moments of the pulled
 * populations with the force from the current Q (u == 0 when flow is off). */
void or_readout(const or_params *p, int nx, int ny, int nz, const double *g,
                const double *Q9, double *rho_out, double *u3_out)
{
    long N = (long)nx * ny * nz;
    if (p->lb_model == 1) {  /* D3Q15: moments of the stored f(x), Eq. (14) */
        for (long s = 0; s < N; s++) {
            double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < 15; i++) {
                drho += g[i * N + s];
                for (int a = 0; a < 3; a++) j[a] += g[i * N + s] * E15[i][a];
            }
            double rho = p->rho0 + drho;
            rho_out[s] = rho;
            for (int a = 0; a < 3; a++) u3_out[a * N + s] = p->flow ? j[a] / rho : 0.0;
        }
        return;
    }
    double *F3 = (double *)calloc(3 * N, sizeof(double));
    if (p->flow) coupling_force(p, nx, ny, nz, Q9, NULL, F3);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long s = site(x, y, z, nx, ny, nz);
                double gt[19], j[3] = {0.0, 0.0, 0.0}, drho = 0.0;
                pull(g, N, nx, ny, nz, x, y, z, gt);
                for (int i = 0; i < 19; i++) {
                    drho += gt[i];
                    for (int a = 0; a < 3; a++) j[a] += gt[i] * E[i][a];
                }
                double rho = p->rho0 + drho;
                rho_out[s] = rho;
                for (int a = 0; a < 3; a++)
                    u3_out[a * N + s] = p->flow ? (j[a] + 0.5 * F3[a * N + s]) / rho : 0.0;
            }
    free(F3);
}

/* One coupled step per iteration (Sec. 2.2):
 *   F^n = div Pi(Q^n) (or b^n and sigma^xi(Q^n) in the split coupling);
 *   LB step -> g_n, u^n; Q^{n+1} = Heun(Q^n, u^n).
 * With flow off, u == 0 and the populations are left untouched. */
void or_step(const or_params *p, int nx, int ny, int nz, double *g, double *Q9, int nsteps)
{
    long N = (long)nx * ny * nz;
    double *F3 = (double *)malloc(sizeof(double) * 3 * N);
    double *sig9 = p->flow == 2 ? (double *)malloc(sizeof(double) * 9 * N) : NULL;
    double *u3 = (double *)calloc(3 * N, sizeof(double));
    double *g2 = (double *)malloc(sizeof(double) * n_pop(p) * N);
    double *Qn = (double *)malloc(sizeof(double) * 9 * N);
    for (int n = 0; n < nsteps; n++) {
        if (p->flow) {
            coupling_force(p, nx, ny, nz, Q9, sig9, F3);
            if (p->lb_model == 1)
                or_lb_pc(p, nx, ny, nz, g, F3, sig9, g2, NULL, u3);
            else
                lb_step(p, nx, ny, nz, g, F3, sig9, g2, NULL, u3);
            memcpy(g, g2, sizeof(double) * n_pop(p) * N);
        }
        or_qupdate(p, nx, ny, nz, Q9, u3, Qn);
        memcpy(Q9, Qn, sizeof(double) * 9 * N);
    }
    free(F3);
    free(sig9);
    free(u3);
    free(g2);
    free(Qn);
}

/* Pairwise (cascade) summation of a contiguous array. */
static double pairwise(const double *v, long n)
{
    if (n <= 8) {
        double s = 0.0;
        for (long k = 0; k < n; k++) s += v[k];
        return s;
    }
    long h = n / 2;
    return pairwise(v, h) + pairwise(v + h, n - h);
}

double or_sum(const double *v, long n) { return pairwise(v, n); }

/* Totals at the current level: mass sum rho, momentum sum rho u, free energy
 * sum f (each by pairwise summation). */
void or_totals(const or_params *p, int nx, int ny, int nz, const double *g,
               const double *Q9, double *mass, double *mom3, double *ftot)
{
    long N = (long)nx * ny * nz;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *u3 = (double *)malloc(sizeof(double) * 3 * N);
    double *fd = (double *)malloc(sizeof(double) * N);
    double *tmp = (double *)malloc(sizeof(double) * N);
    or_readout(p, nx, ny, nz, g, Q9, rho, u3);
    or_chem(p, nx, ny, nz, Q9, NULL, fd, NULL);
    *mass = pairwise(rho, N);
    for (int a = 0; a < 3; a++) {
        for (long s = 0; s < N; s++) tmp[s] = rho[s] * u3[a * N + s];
        mom3[a] = pairwise(tmp, N);
    }
    *ftot = pairwise(fd, N);
    free(rho);
    free(u3);
    free(fd);
    free(tmp);
}

/* Thread count of the OpenMP loops (timing runs only; results do not depend
 * on it: every loop writes disjoint sites and the sums are serial). */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int or_max_threads(void) { return omp_get_max_threads(); }
