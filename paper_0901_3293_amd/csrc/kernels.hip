// kernels.hip -- HIP kernels of the hybrid step for gfx950 and their launchers.
//
// Data layout in HBM (all structure-of-arrays, component-major, x fastest):
//   g[2]  19 x N  deviation populations g_i = f_i - w_i rho0 (ping-pong, pull)
//   Q      5 x N  order parameter (xx, xy, xz, yy, yz)
//   Qs     5 x N  predictor stage Q*
//   u      3 x N  velocity of the last LB step
//   Pi     9 x N  chemical stress (row-major a*3+b)
// Scalars of one run are passed by value (Coef<T>); no constant memory.
//
// Step schedule (Sec. 2.2): stress(Q^n) -> lb(g, div Pi) -> pred(Q^n, u^n)
// -> corr(Q^n, Q*, u^n).  Each kernel maps one thread to one lattice site;
// neighbour values come through the L2 of the XCD that owns the block (block
// ids are remapped so each of the 8 XCDs sweeps a contiguous slab).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "site.h"

namespace hlb {

namespace {

constexpr int BLK = 256;

// Hardware hands consecutive workgroups to the 8 XCDs in turn; remap so XCD k
// sweeps blocks [k*per, (k+1)*per) of the domain and its L2 sees the stencil
// neighbours of its own sites.  gridDim.x is a multiple of 8.
__device__ __forceinline__ int logical_block()
{
    const int per = gridDim.x >> 3;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

struct Site {
    int s;       // linear index
    int nb[6];   // x+1, x-1, y+1, y-1, z+1, z-1 (periodic)
};

__device__ __forceinline__ bool site_of(const Geom &G, Site &S)
{
    const int s = logical_block() * BLK + threadIdx.x;
    if (s >= G.N) return false;
    const int x = s % G.nx;
    const int yz = s / G.nx;
    const int y = yz % G.ny;
    const int z = yz / G.ny;
    const int sxy = G.nx * G.ny;
    S.s = s;
    S.nb[0] = (x == G.nx - 1) ? s - (G.nx - 1) : s + 1;
    S.nb[1] = (x == 0) ? s + (G.nx - 1) : s - 1;
    S.nb[2] = (y == G.ny - 1) ? s - G.nx * (G.ny - 1) : s + G.nx;
    S.nb[3] = (y == 0) ? s + G.nx * (G.ny - 1) : s - G.nx;
    S.nb[4] = (z == G.nz - 1) ? s - sxy * (G.nz - 1) : s + sxy;
    S.nb[5] = (z == 0) ? s + sxy * (G.nz - 1) : s - sxy;
    return true;
}

// Pulled source of population i arriving at (x,y,z): site (x,y,z) - e_i.
__device__ __forceinline__ int pull_src(const Geom &G, int x, int y, int z, int cx, int cy, int cz)
{
    int xs = x - cx, ys = y - cy, zs = z - cz;
    xs += (xs < 0) ? G.nx : ((xs >= G.nx) ? -G.nx : 0);
    ys += (ys < 0) ? G.ny : ((ys >= G.ny) ? -G.ny : 0);
    zs += (zs < 0) ? G.nz : ((zs >= G.nz) ? -G.nz : 0);
    return xs + G.nx * (ys + G.ny * zs);
}

template <typename T>
__device__ __forceinline__ void gather_q(const T *__restrict__ Q, size_t N, const Site &S, T q[5],
                                         T d[3][5], T lap[5])
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
__device__ __forceinline__ void gather_u(const T *__restrict__ u, size_t N, const Site &S, T uc[3],
                                         T W[3][3])
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
__device__ __forceinline__ void divergence(const T *__restrict__ Pi, size_t N, const Site &S, T F[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T *Px = Pi + (3 * a + 0) * N;
        const T *Py = Pi + (3 * a + 1) * N;
        const T *Pz = Pi + (3 * a + 2) * N;
        F[a] = T(0.5) * ((Px[S.nb[0]] - Px[S.nb[1]]) + (Py[S.nb[2]] - Py[S.nb[3]]) + (Pz[S.nb[4]] - Pz[S.nb[5]]));
    }
}

// Fixed-order block reduction of NV doubles per thread into out[NV].
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV], double *out)
{
    __shared__ double buf[NV][BLK];
#pragma unroll
    for (int k = 0; k < NV; ++k) buf[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = BLK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < NV; ++k) buf[k][threadIdx.x] += buf[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = buf[k][0];
}

// ---------------------------------------------------------------- kernels

template <typename T>
__global__ __launch_bounds__(BLK) void k_stress(Geom G, Coef<T> c, const T *__restrict__ Q,
                                                T *__restrict__ Pi, double *__restrict__ fpart)
{
    Site S;
    const bool ok = site_of(G, S);
    double fsum = 0.0;
    if (ok) {
        const size_t N = G.N;
        T q[5], d[3][5], lap[5], P[3][3], fd, H[5];
        gather_q(Q, N, S, q, d, lap);
        site_stress(c, q, d, lap, P, fd, H);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) Pi[(3 * a + b) * N + S.s] = P[a][b];
        fsum = double(fd);
    }
    if (fpart) {
        double v[1] = {fsum};
        block_sum<1>(v, fpart + logical_block());
    }
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_lb(Geom G, Coef<T> c, const T *__restrict__ gin,
                                            const T *__restrict__ Pi, T *__restrict__ gout,
                                            T *__restrict__ u)
{
    Site S;
    if (!site_of(G, S)) return;
    const size_t N = G.N;
    const int x = S.s % G.nx, y = (S.s / G.nx) % G.ny, z = S.s / (G.nx * G.ny);
    T g[19], F[3], uu[3], rho;
#pragma unroll
    for (int i = 0; i < 19; ++i) g[i] = gin[i * N + pull_src(G, x, y, z, CX[i], CY[i], CZ[i])];
    divergence(Pi, N, S, F);
    lb_collide(c, g, F, uu, rho);
#pragma unroll
    for (int i = 0; i < 19; ++i) gout[i * N + S.s] = g[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a * N + S.s] = uu[a];
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_qpred(Geom G, Coef<T> c, const T *__restrict__ Q,
                                               const T *__restrict__ u, T *__restrict__ Qs)
{
    Site S;
    if (!site_of(G, S)) return;
    const size_t N = G.N;
    T q[5], d[3][5], lap[5], uc[3], W[3][3], R[5];
    gather_q(Q, N, S, q, d, lap);
    gather_u(u, N, S, uc, W);
    site_rhs(c, q, d, lap, uc, W, R);
#pragma unroll
    for (int k = 0; k < 5; ++k) Qs[k * N + S.s] = q[k] + R[k];
}

// Q^{n+1} = Q^n + [R(Q^n) + R(Q*)]/2 = [Q^n + Q* + R(Q*)]/2, written in place.
template <typename T>
__global__ __launch_bounds__(BLK) void k_qcorr(Geom G, Coef<T> c, T *__restrict__ Q,
                                               const T *__restrict__ Qs, const T *__restrict__ u)
{
    Site S;
    if (!site_of(G, S)) return;
    const size_t N = G.N;
    T q[5], d[3][5], lap[5], uc[3], W[3][3], R[5];
    gather_q(Qs, N, S, q, d, lap);
    gather_u(u, N, S, uc, W);
    site_rhs(c, q, d, lap, uc, W, R);
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k * N + S.s] = T(0.5) * (Q[k * N + S.s] + q[k] + R[k]);
}

// Populations such that the first pull returns g^eq(rho(x), u(x)):
// g_i(y) = g_i^eq(rho(y + e_i), u(y + e_i)); Q converted to the storage type.
template <typename T>
__global__ __launch_bounds__(BLK) void k_init(Geom G, Coef<T> c, const double *__restrict__ rho_in,
                                              const double *__restrict__ u_in,
                                              const double *__restrict__ Q_in, T *__restrict__ g,
                                              T *__restrict__ Q)
{
    Site S;
    if (!site_of(G, S)) return;
    const size_t N = G.N;
    const int x = S.s % G.nx, y = (S.s / G.nx) % G.ny, z = S.s / (G.nx * G.ny);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const int t = pull_src(G, x, y, z, -CX[i], -CY[i], -CZ[i]);
        const T uu[3] = {T(u_in[t]), T(u_in[N + t]), T(u_in[2 * N + t])};
        g[i * N + S.s] = lb_geq(c, i, T(rho_in[t]), uu);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k * N + S.s] = T(Q_in[k * N + S.s]);
}

// Current-level readout: rho, u = (j + F/2)/rho (F from the current stress,
// zero when Pi is null) and Q in FP64; FP64 block partials of
// (rho - rho0, rho u_x, rho u_y, rho u_z).
template <typename T>
__global__ __launch_bounds__(BLK) void k_readout(Geom G, Coef<T> c, const T *__restrict__ g,
                                                 const T *__restrict__ Pi, const T *__restrict__ Q,
                                                 double *__restrict__ rho_out, double *__restrict__ u_out,
                                                 double *__restrict__ Q_out, double *__restrict__ part)
{
    Site S;
    const bool ok = site_of(G, S);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (ok) {
        const size_t N = G.N;
        const int x = S.s % G.nx, y = (S.s / G.nx) % G.ny, z = S.s / (G.nx * G.ny);
        T gg[19], drho, j[3], F[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int i = 0; i < 19; ++i) gg[i] = g[i * N + pull_src(G, x, y, z, CX[i], CY[i], CZ[i])];
        lb_moments(gg, drho, j);
        if (Pi) divergence(Pi, N, S, F);
        const T rho = c.rho0 + drho;
        T uu[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) uu[a] = Pi ? (j[a] + T(0.5) * F[a]) / rho : T(0);
        if (rho_out) rho_out[S.s] = double(rho);
        if (u_out)
#pragma unroll
            for (int a = 0; a < 3; ++a) u_out[a * N + S.s] = double(uu[a]);
        if (Q_out)
#pragma unroll
            for (int k = 0; k < 5; ++k) Q_out[k * N + S.s] = double(Q[k * N + S.s]);
        v[0] = double(drho);
        if (Pi)
#pragma unroll
            for (int a = 0; a < 3; ++a) v[1 + a] = double(j[a]) + 0.5 * double(F[a]);
    }
    if (part) block_sum<4>(v, part + 4 * logical_block());
}

// Second stage: out[k] = sum_b part[b*nv + k], fixed order, one block.
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
            if (threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = buf[0];
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_fill(T *__restrict__ p, size_t n, T v)
{
    size_t i = size_t(blockIdx.x) * BLK + threadIdx.x;
    const size_t stride = size_t(gridDim.x) * BLK;
    for (; i < n; i += stride) p[i] = v;
}

inline int grid_blocks(int N) { return ((N + BLK - 1) / BLK + 7) / 8 * 8; }

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

// Records an event pair around each launch when a timer is attached.
struct Marks {
    KernelTimer *t;
    hipStream_t s;
    template <typename F>
    hipError_t operator()(int kind, F &&launch)
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

template <typename T>
hipError_t steps_t(const Device &D, const PhysParams &p, int nsteps, int &cur, KernelTimer *timer)
{
    const Geom G = D.G;
    const Coef<T> c = make_coef<T>(p);
    const int nb = grid_blocks(G.N);
    T *Q = static_cast<T *>(D.Q), *Qs = static_cast<T *>(D.Qs), *u = static_cast<T *>(D.u);
    T *Pi = static_cast<T *>(D.Pi);
    Marks mark{timer, D.stream};
    hipError_t e = hipSuccess;
    if (!p.flow && nsteps > 0)  // pure relaxation: u == 0 (Sec. 2.1)
        k_fill<T><<<1024, BLK, 0, D.stream>>>(u, 3 * size_t(G.N), T(0));
    for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
        if (p.flow) {
            T *gin = static_cast<T *>(D.g[cur]);
            T *gout = static_cast<T *>(D.g[cur ^ 1]);
            e = mark(K_STRESS, [&] { k_stress<T><<<nb, BLK, 0, D.stream>>>(G, c, Q, Pi, nullptr); });
            if (e == hipSuccess)
                e = mark(K_LB, [&] { k_lb<T><<<nb, BLK, 0, D.stream>>>(G, c, gin, Pi, gout, u); });
            cur ^= 1;
        }
        if (e == hipSuccess) e = mark(K_QPRED, [&] { k_qpred<T><<<nb, BLK, 0, D.stream>>>(G, c, Q, u, Qs); });
        if (e == hipSuccess) e = mark(K_QCORR, [&] { k_qcorr<T><<<nb, BLK, 0, D.stream>>>(G, c, Q, Qs, u); });
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <typename T>
hipError_t init_t(const Device &D, const PhysParams &p, const double *stage, int cur)
{
    const Geom G = D.G;
    const Coef<T> c = make_coef<T>(p);
    const size_t N = G.N;
    const int nb = grid_blocks(G.N);
    k_init<T><<<nb, BLK, 0, D.stream>>>(G, c, stage, stage + N, stage + 4 * N, static_cast<T *>(D.g[cur]),
                                        static_cast<T *>(D.Q));
    // u of the last LB step: zero until the first step (and for good with flow off)
    k_fill<T><<<1024, BLK, 0, D.stream>>>(static_cast<T *>(D.u), 3 * N, T(0));
    return hipGetLastError();
}

template <typename T>
hipError_t readout_t(const Device &D, const PhysParams &p, int cur, double *stage, double *totals)
{
    const Geom G = D.G;
    const Coef<T> c = make_coef<T>(p);
    const size_t N = G.N;
    const int nb = grid_blocks(G.N);
    T *Pi = static_cast<T *>(D.Pi);
    const bool need_stress = p.flow || totals;
    if (need_stress)
        k_stress<T><<<nb, BLK, 0, D.stream>>>(G, c, static_cast<const T *>(D.Q), Pi,
                                              totals ? D.part + 4 * nb : nullptr);
    k_readout<T><<<nb, BLK, 0, D.stream>>>(G, c, static_cast<const T *>(D.g[cur]), p.flow ? Pi : nullptr,
                                           static_cast<const T *>(D.Q), stage ? stage : nullptr,
                                           stage ? stage + N : nullptr, stage ? stage + 4 * N : nullptr,
                                           totals ? D.part : nullptr);
    if (totals) {
        k_reduce<<<1, BLK, 0, D.stream>>>(D.part, nb, 4, 4, D.res);
        k_reduce<<<1, BLK, 0, D.stream>>>(D.part + 4 * nb, nb, 1, 1, D.res + 4);
    }
    return hipGetLastError();
}

}  // namespace

size_t partial_doubles(int N) { return size_t(5) * grid_blocks(N) + 16; }

const char *kernel_name(int k)
{
    static const char *names[K_COUNT] = {"k_stress", "k_lb", "k_qpred", "k_qcorr"};
    return (k >= 0 && k < K_COUNT) ? names[k] : nullptr;
}

hipError_t run_steps(const Device &D, const PhysParams &p, int nsteps, int &cur, KernelTimer *timer)
{
    return D.fp32 ? steps_t<float>(D, p, nsteps, cur, timer) : steps_t<double>(D, p, nsteps, cur, timer);
}

hipError_t run_init(const Device &D, const PhysParams &p, const double *stage, int cur)
{
    return D.fp32 ? init_t<float>(D, p, stage, cur) : init_t<double>(D, p, stage, cur);
}

hipError_t run_readout(const Device &D, const PhysParams &p, int cur, double *stage, double *totals)
{
    return D.fp32 ? readout_t<float>(D, p, cur, stage, totals) : readout_t<double>(D, p, cur, stage, totals);
}

}  // namespace hlb
