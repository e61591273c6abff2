// Host build of the per-site physics of the HIP path (site.h), for checking
// it against the oracle on the CPU (tests/test_site_host.py).  Reads a
// periodic lattice and the parameters from a binary file, gathers the same
// centred stencils the kernels gather (first derivatives, 7-point Laplacian
// of Q; u and its centred gradient), evaluates site_stress and site_rhs at
// every site in FP64 and writes H (5), f (1), Pi (9) and R (5) per site.
//
// input  (doubles): nx ny nz, A0 gamma K q0 Gamma xi tau rho0, Q [5][N], u [3][N]
// output (doubles): H [5][N], f [N], Pi [9][N] (row-major 3x3), R [5][N]
//
// With a third argument `lb`, the D3Q19 collision instead: pulls the
// populations g_i(x - e_i) and applies lb_collide with the force F, then
// lb_collide_split with the body force F and the stress sig.
// input  (doubles): the 11 header values, g [19][N], F [3][N], sig [6][N] (xx xy xz yy yz zz)
// output (doubles): g' [19][N], rho [N], u [3][N] of lb_collide, then the same of lb_collide_split
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_0901_3293_amd/csrc/kernels.h"
#include "../../paper_0901_3293_amd/csrc/site.h"
#include "../../paper_0901_3293_amd/csrc/sitekern.h"

static int collide(const hlb::Coef<double> &c, int nx, int ny, int nz, FILE *fi, const char *outpath)
{
    const long N = long(nx) * ny * nz;
    std::vector<double> g(19 * N), F(3 * N), sig(6 * N);
    if (std::fread(g.data(), sizeof(double), 19 * N, fi) != size_t(19 * N)) return 5;
    if (std::fread(F.data(), sizeof(double), 3 * N, fi) != size_t(3 * N)) return 6;
    if (std::fread(sig.data(), sizeof(double), 6 * N, fi) != size_t(6 * N)) return 6;
    auto at = [&](int x, int y, int z) {
        x = (x + nx) % nx;
        y = (y + ny) % ny;
        z = (z + nz) % nz;
        return long(x) + nx * (long(y) + ny * long(z));
    };
    std::vector<double> out(46 * N);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long s = at(x, y, z);
                double gp[19], gs[19], f[3], sg[6], u[3], rho;
                for (int i = 0; i < 19; ++i)
                    gp[i] = gs[i] = g[i * N + at(x - hlb::CX[i], y - hlb::CY[i], z - hlb::CZ[i])];
                for (int a = 0; a < 3; ++a) f[a] = F[a * N + s];
                for (int k = 0; k < 6; ++k) sg[k] = sig[k * N + s];
                hlb::lb_collide(c, gp, f, u, rho);
                for (int i = 0; i < 19; ++i) out[i * N + s] = gp[i];
                out[19 * N + s] = rho;
                for (int a = 0; a < 3; ++a) out[(20 + a) * N + s] = u[a];
                hlb::lb_collide_split(c, gs, f, sg, u, rho);
                for (int i = 0; i < 19; ++i) out[(23 + i) * N + s] = gs[i];
                out[42 * N + s] = rho;
                for (int a = 0; a < 3; ++a) out[(43 + a) * N + s] = u[a];
            }
    FILE *fo = std::fopen(outpath, "wb");
    if (!fo) return 7;
    std::fwrite(out.data(), sizeof(double), out.size(), fo);
    std::fclose(fo);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 3 && !(argc == 4 && std::string(argv[3]) == "lb")) return 2;
    FILE *fi = std::fopen(argv[1], "rb");
    if (!fi) return 3;
    double hdr[11];
    if (std::fread(hdr, sizeof(double), 11, fi) != 11) return 4;
    const int nx = int(hdr[0]), ny = int(hdr[1]), nz = int(hdr[2]);
    const long N = long(nx) * ny * nz;
    hlb::PhysParams p{};
    p.A0 = hdr[3];
    p.gamma = hdr[4];
    p.K = hdr[5];
    p.q0 = hdr[6];
    p.Gamma = hdr[7];
    p.xi = hdr[8];
    p.tau = hdr[9];
    p.rho0 = hdr[10];
    const hlb::Coef<double> c = hlb::make_coef<double>(p);
    if (argc == 4) {
        const int rc = collide(c, nx, ny, nz, fi, argv[2]);
        std::fclose(fi);
        return rc;
    }
    std::vector<double> Q(5 * N), u(3 * N);
    if (std::fread(Q.data(), sizeof(double), 5 * N, fi) != size_t(5 * N)) return 5;
    if (std::fread(u.data(), sizeof(double), 3 * N, fi) != size_t(3 * N)) return 6;
    std::fclose(fi);
    auto at = [&](int x, int y, int z) {
        x = (x + nx) % nx;
        y = (y + ny) % ny;
        z = (z + nz) % nz;
        return long(x) + nx * (long(y) + ny * long(z));
    };
    std::vector<double> out(20 * N);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long s = at(x, y, z);
                const long nb[6] = {at(x + 1, y, z), at(x - 1, y, z), at(x, y + 1, z),
                                    at(x, y - 1, z), at(x, y, z + 1), at(x, y, z - 1)};
                double q[5], d[3][5], lap[5], uc[3], W[3][3];
                for (int k = 0; k < 5; ++k) {
                    const double *P = Q.data() + k * N;
                    q[k] = P[s];
                    d[0][k] = 0.5 * (P[nb[0]] - P[nb[1]]);
                    d[1][k] = 0.5 * (P[nb[2]] - P[nb[3]]);
                    d[2][k] = 0.5 * (P[nb[4]] - P[nb[5]]);
                    lap[k] = ((P[nb[0]] + P[nb[1]]) + (P[nb[2]] + P[nb[3]])) + (P[nb[4]] + P[nb[5]]) - 6.0 * q[k];
                }
                for (int a = 0; a < 3; ++a) {
                    const double *P = u.data() + a * N;
                    uc[a] = P[s];
                    W[a][0] = 0.5 * (P[nb[0]] - P[nb[1]]);
                    W[a][1] = 0.5 * (P[nb[2]] - P[nb[3]]);
                    W[a][2] = 0.5 * (P[nb[4]] - P[nb[5]]);
                }
                double Pi[3][3], fd, H[5], R[5];
                hlb::site_stress(c, q, d, lap, Pi, fd, H);
                hlb::site_rhs(c, q, d, lap, uc, W, R);
                for (int k = 0; k < 5; ++k) out[k * N + s] = H[k];
                out[5 * N + s] = fd;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) out[(6 + 3 * a + b) * N + s] = Pi[a][b];
                for (int k = 0; k < 5; ++k) out[(15 + k) * N + s] = R[k];
            }
    FILE *fo = std::fopen(argv[2], "wb");
    if (!fo) return 7;
    std::fwrite(out.data(), sizeof(double), out.size(), fo);
    std::fclose(fo);
    return 0;
}
