// Host build of the per-site physics of the HIP path (site.h), for checking
// it against the oracle on the CPU (tests/test_site_host.py).  Reads a
// periodic lattice and the parameters from a binary file, gathers the same
// centred stencils the kernels gather (first derivatives, 7-point Laplacian
// of Q; u and its centred gradient), evaluates site_stress and site_rhs at
// every site in FP64 and writes H (5), f (1), Pi (9) and R (5) per site.
//
// input  (doubles): nx ny nz, A0 gamma K q0 Gamma xi tau rho0, Q [5][N], u [3][N]
// output (doubles): H [5][N], f [N], Pi [9][N] (row-major 3x3), R [5][N]
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_0901_3293_amd/csrc/kernels.h"
#include "../../paper_0901_3293_amd/csrc/site.h"
#include "../../paper_0901_3293_amd/csrc/sitekern.h"

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
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
    std::vector<double> Q(5 * N), u(3 * N);
    if (std::fread(Q.data(), sizeof(double), 5 * N, fi) != size_t(5 * N)) return 5;
    if (std::fread(u.data(), sizeof(double), 3 * N, fi) != size_t(3 * N)) return 6;
    std::fclose(fi);
    const hlb::Coef<double> c = hlb::make_coef<double>(p);
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
