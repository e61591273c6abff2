// nn.hip -- kernels of the 3D convolutional surrogate on BF16 matrix cores.
//
// Activations are channels-last bfloat16, act[site][C] with C padded to 16 or
// 32; weights of a layer are bfloat16 [tap][C_out][C_in] (tap = kz*9 + ky*3 +
// kx reads the input at offset (kx-1, ky-1, kz-1), periodic).  A 3x3x3
// convolution is an implicit GEMM per tile of 16x4x4 output sites:
// M = 16 sites of one x-row, N = 16 output channels, K = 16 input channels of
// one tap, on v_mfma_f32_16x16x16_bf16 with FP32 accumulation.  The input
// brick of the tile (18x6x6 sites, periodic wrap) and the layer's weights are
// staged in LDS; each of the 4 waves owns one z-plane of the tile.
#include <hip/hip_runtime.h>

#include "nn.h"

namespace hlb {
namespace nn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BLK = 256;
constexpr int TXs = 16, TYs = 4, TZs = 4;               // output tile
constexpr int BX = TXs + 2, BY = TYs + 2, BZ = TZs + 2;  // staged input brick
constexpr int BN = BX * BY * BZ;

__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                                    // round to nearest even
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(unsigned(h) << 16); }

__device__ __forceinline__ int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

__device__ __forceinline__ void tile_origin(const Grid3 &g, int t, int &x0, int &y0, int &z0)
{
    x0 = (t % g.tx) * TXs;
    const int r = t / g.tx;
    y0 = (r % g.ty) * TYs;
    z0 = (r / g.ty) * TZs;
}

// Brick of (TX+2)(TY+2)(TZ+2) sites around the tile, CIP channels each, into
// LDS rows of SP = CIP + 8 (16-byte aligned, no bank conflicts for the
// fragment reads).
template <int CIP>
__device__ __forceinline__ void stage_brick(const Grid3 &g, const unsigned short *__restrict__ act, int x0, int y0,
                                            int z0, unsigned short *sB)
{
    constexpr int SP = CIP + 8, V = CIP / 8;
    for (int e = threadIdx.x; e < BN * V; e += BLK) {
        const int site = e / V, v = e - site * V;
        const int bx = site % BX, r = site / BX, by = r % BY, bz = r / BY;
        const int x = wrap(x0 - 1 + bx, g.nx), y = wrap(y0 - 1 + by, g.ny), z = wrap(z0 - 1 + bz, g.nz);
        const size_t gs = size_t(x) + size_t(g.nx) * (size_t(y) + size_t(g.ny) * z);
        *reinterpret_cast<uint4 *>(sB + site * SP + v * 8) =
            *reinterpret_cast<const uint4 *>(act + gs * CIP + v * 8);
    }
}

template <int CIP, int COP>
__device__ __forceinline__ void stage_weights(const unsigned short *__restrict__ W, unsigned short *sW)
{
    constexpr int WP = CIP + 8, V = CIP / 8;
    for (int e = threadIdx.x; e < 27 * COP * V; e += BLK) {
        const int row = e / V, v = e - row * V;
        *reinterpret_cast<uint4 *>(sW + row * WP + v * 8) = *reinterpret_cast<const uint4 *>(W + row * CIP + v * 8);
    }
}

// Forward-style convolution with an epilogue:
//  MODE_RELU:   out_bf16[s][co] = bf16(relu(acc + b[co])), 0 for co >= co_valid
//  MODE_LINEAR: out_f32[s][co]  = acc + b[co] for co < co_valid (row stride co_valid)
//  MODE_MASK:   out_bf16[s][co] = mask[s][co] > 0 ? bf16(acc) : 0   (backward through ReLU)
//  MODE_RAW:    out_f32[s][co]  = acc (row stride COP)
template <int CIP, int COP, int MODE>
__global__ __launch_bounds__(BLK) void k_conv(Grid3 g, const unsigned short *__restrict__ X,
                                              const unsigned short *__restrict__ Wg, const float *__restrict__ bias,
                                              void *__restrict__ out, const unsigned short *__restrict__ mask,
                                              int co_valid)
{
    constexpr int SP = CIP + 8, WP = CIP + 8, NS = COP / 16, KC = CIP / 16;
    __shared__ __attribute__((aligned(16))) unsigned short sB[BN * SP];
    __shared__ __attribute__((aligned(16))) unsigned short sW[27 * COP * WP];
    stage_weights<CIP, COP>(Wg, sW);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lg = l >> 4;
    for (int t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
        int x0, y0, z0;
        tile_origin(g, t, x0, y0, z0);
        __syncthreads();
        stage_brick<CIP>(g, X, x0, y0, z0, sB);
        __syncthreads();
        f32x4 acc[4][NS];
#pragma unroll
        for (int ms = 0; ms < 4; ++ms)
#pragma unroll
            for (int ns = 0; ns < NS; ++ns) acc[ms][ns] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int tap = 0; tap < 27; ++tap) {
            const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                bf16x4 b[NS];
#pragma unroll
                for (int ns = 0; ns < NS; ++ns)
                    b[ns] = *reinterpret_cast<const bf16x4 *>(sW + (tap * COP + ns * 16 + li) * WP + kc * 16 + lg * 4);
#pragma unroll
                for (int ms = 0; ms < 4; ++ms) {
                    const int site = ((w + dz) * BY + (ms + dy)) * BX + (li + dx);
                    const bf16x4 a = *reinterpret_cast<const bf16x4 *>(sB + site * SP + kc * 16 + lg * 4);
#pragma unroll
                    for (int ns = 0; ns < NS; ++ns)
                        acc[ms][ns] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[ns], acc[ms][ns], 0, 0, 0);
                }
            }
        }
        // D[row][col]: row = site x within the x-row (4*lg + r), col = channel (li)
        const int z = z0 + w;
#pragma unroll
        for (int ms = 0; ms < 4; ++ms) {
            const int y = y0 + ms;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int x = x0 + lg * 4 + r;
                if (x >= g.nx || y >= g.ny || z >= g.nz) continue;
                const size_t s = size_t(x) + size_t(g.nx) * (size_t(y) + size_t(g.ny) * z);
#pragma unroll
                for (int ns = 0; ns < NS; ++ns) {
                    const int co = ns * 16 + li;
                    const float v = acc[ms][ns][r];
                    if (MODE == MODE_RELU) {
                        const float y1 = co < co_valid ? fmaxf(v + bias[co], 0.f) : 0.f;
                        static_cast<unsigned short *>(out)[s * COP + co] = f2bf(y1);
                    } else if (MODE == MODE_LINEAR) {
                        if (co < co_valid) static_cast<float *>(out)[s * co_valid + co] = v + bias[co];
                    } else if (MODE == MODE_MASK) {
                        const bool on = bf2f(mask[s * COP + co]) > 0.f;
                        static_cast<unsigned short *>(out)[s * COP + co] = on ? f2bf(v) : (unsigned short)0;
                    } else {
                        static_cast<float *>(out)[s * COP + co] = v;
                    }
                }
            }
        }
    }
}

// Weight gradient dW[tap][ci][co] = sum_s X[s + off(tap)][ci] dZ[s][co] and
// bias gradient db[co] = sum_s dZ[s][co]: per tile, a GEMM with M = 16 input
// channels, N = 16 output channels, K = 16 sites of one x-row; each wave owns
// a fixed set of (tap, ci block, co block) accumulators across all the tiles
// its block visits.  Per-block FP32 partials; the final sum is FP64 in a fixed
// order (k_wgrad_reduce), so the result is deterministic.
template <int CIP, int COP>
__global__ __launch_bounds__(BLK) void k_wgrad(Grid3 g, const unsigned short *__restrict__ X,
                                               const unsigned short *__restrict__ dZ, float *__restrict__ part)
{
    constexpr int SP = CIP + 8, DP = COP + 8, MS = CIP / 16, NS = COP / 16, NCOMBO = 27 * MS * NS;
    constexpr int PER = (NCOMBO + 3) / 4;
    constexpr int PS = 27 * CIP * COP + COP;
    __shared__ __attribute__((aligned(16))) unsigned short sB[BN * SP];
    __shared__ __attribute__((aligned(16))) unsigned short sD[TXs * TYs * TZs * DP];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lg = l >> 4;
    f32x4 acc[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbacc = 0.f;
    for (int t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
        int x0, y0, z0;
        tile_origin(g, t, x0, y0, z0);
        __syncthreads();
        stage_brick<CIP>(g, X, x0, y0, z0, sB);
        constexpr int V = COP / 8;
        for (int e = threadIdx.x; e < TXs * TYs * TZs * V; e += BLK) {
            const int site = e / V, v = e - site * V;
            const int tx = site % TXs, r = site / TXs, ty = r % TYs, tz = r / TYs;
            const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
            uint4 val = make_uint4(0u, 0u, 0u, 0u);
            if (x < g.nx && y < g.ny && z < g.nz) {
                const size_t gs = size_t(x) + size_t(g.nx) * (size_t(y) + size_t(g.ny) * z);
                val = *reinterpret_cast<const uint4 *>(dZ + gs * COP + v * 8);
            }
            *reinterpret_cast<uint4 *>(sD + site * DP + v * 8) = val;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int combo = w + 4 * j;
            if (combo < NCOMBO) {
                const int tap = combo / (MS * NS), rem = combo - tap * (MS * NS), ms = rem / NS, ns = rem - ms * NS;
                const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
#pragma unroll 1
                for (int kc = 0; kc < TYs * TZs; ++kc) {
                    const int yy = kc % TYs, zz = kc / TYs;
                    bf16x4 a, b;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int x = lg * 4 + q;
                        a[q] = short(sB[(((zz + dz) * BY + (yy + dy)) * BX + (x + dx)) * SP + ms * 16 + li]);
                        b[q] = short(sD[((zz * TYs + yy) * TXs + x) * DP + ns * 16 + li]);
                    }
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
                }
            }
        }
        if (int(threadIdx.x) < COP)
            for (int s = 0; s < TXs * TYs * TZs; ++s) dbacc += bf2f(sD[s * DP + threadIdx.x]);
    }
    float *P = part + size_t(blockIdx.x) * PS;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int combo = w + 4 * j;
        if (combo < NCOMBO) {
            const int tap = combo / (MS * NS), rem = combo - tap * (MS * NS), ms = rem / NS, ns = rem - ms * NS;
#pragma unroll
            for (int r = 0; r < 4; ++r) P[(tap * CIP + ms * 16 + lg * 4 + r) * COP + ns * 16 + li] = acc[j][r];
        }
    }
    if (int(threadIdx.x) < COP) P[27 * CIP * COP + threadIdx.x] = dbacc;
}

// Sum the per-block partials (FP64, block order) into the flat gradient of
// one layer: W[co][ci][tap] (ci < CI, co < CO) then b[co].
__global__ __launch_bounds__(BLK) void k_wgrad_reduce(const float *__restrict__ part, int nblk, int CIP, int COP,
                                                      int CI, int CO, float *__restrict__ grad)
{
    const int PS = 27 * CIP * COP + COP;
    const int total = CO * CI * 27 + CO;
    for (int e = blockIdx.x * BLK + threadIdx.x; e < total; e += gridDim.x * BLK) {
        int idx;
        if (e < CO * CI * 27) {
            const int co = e / (CI * 27), ci = (e / 27) % CI, tap = e % 27;
            idx = (tap * CIP + ci) * COP + co;
        } else {
            idx = 27 * CIP * COP + (e - CO * CI * 27);
        }
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += double(part[size_t(b) * PS + idx]);
        grad[e] = float(s);
    }
}

// Layer weights from the flat FP32 parameters: forward layout [tap][COP][CIP]
// and, for the backward-data convolution, the transposed layout with the
// taps reversed (offset -> -offset): [26 - tap][CIP][COP].
__global__ __launch_bounds__(BLK) void k_wprep(const float *__restrict__ W, int CI, int CO, int CIP, int COP,
                                               unsigned short *__restrict__ Wf, unsigned short *__restrict__ Wt)
{
    const int total = 27 * COP * CIP;
    for (int e = blockIdx.x * BLK + threadIdx.x; e < total; e += gridDim.x * BLK) {
        const int tap = e / (COP * CIP), co = (e / CIP) % COP, ci = e % CIP;
        const float v = (co < CO && ci < CI) ? W[(co * CI + ci) * 27 + tap] : 0.f;
        const unsigned short h = f2bf(v);
        Wf[e] = h;
        Wt[((26 - tap) * CIP + ci) * COP + co] = h;
    }
}

// Standardised input activations: raw [8][N] FP32 -> bf16 [N][16].
__global__ __launch_bounds__(BLK) void k_pack(int N, const float *__restrict__ x, const float *__restrict__ norm,
                                              unsigned short *__restrict__ A0)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
    alignas(16) unsigned short h[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) h[c] = c < 8 ? f2bf((x[size_t(c) * N + s] - norm[c]) / norm[8 + c]) : 0;
    uint4 *dst = reinterpret_cast<uint4 *>(A0 + size_t(s) * 16);
    const uint4 *src = reinterpret_cast<const uint4 *>(h);
    dst[0] = src[0];
    dst[1] = src[1];
}

// Loss and its gradient: target t = (dq_raw - mean)/std, d = y - t,
// dZ = bf16(2 d / (5 N)), block partials of sum d^2 (FP64).
__global__ __launch_bounds__(BLK) void k_lossgrad(int N, const float *__restrict__ Y, const float *__restrict__ dq,
                                                  const float *__restrict__ norm, unsigned short *__restrict__ dZ,
                                                  double *__restrict__ part)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    double acc = 0.0;
    if (s < N) {
        const float sc = 2.0f / (5.0f * float(N));
        alignas(16) unsigned short h[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k < 5) {
                const float t = (dq[size_t(k) * N + s] - norm[16 + k]) / norm[21 + k];
                const float d = Y[size_t(s) * 5 + k] - t;
                acc += double(d) * double(d);
                h[k] = f2bf(d * sc);
            } else {
                h[k] = 0;
            }
        }
        uint4 *dst = reinterpret_cast<uint4 *>(dZ + size_t(s) * 16);
        const uint4 *src = reinterpret_cast<const uint4 *>(h);
        dst[0] = src[0];
        dst[1] = src[1];
    }
    __shared__ double buf[BLK];
    buf[threadIdx.x] = acc;
    __syncthreads();
    for (int w = BLK / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = buf[0];
}

__global__ __launch_bounds__(BLK) void k_sum(const double *__restrict__ part, int n, double *__restrict__ out)
{
    __shared__ double buf[BLK];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += BLK) s += part[i];
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int w = BLK / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = buf[0];
}

// Adam (Kingma & Ba) on the flat FP32 parameters.
__global__ __launch_bounds__(BLK) void k_adam(int n, float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                                              float eps, float c1, float c2)
{
    const int i = blockIdx.x * BLK + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per-channel sums of x and x^2 over nsamples x [nch][N] FP32 (FP64 partials
// per block, grid = nch x B).
__global__ __launch_bounds__(BLK) void k_stats(const float *__restrict__ data, int nch, int N, int nsamples,
                                               double *__restrict__ part)
{
    const int c = blockIdx.y;
    double s1 = 0.0, s2 = 0.0;
    const size_t per = size_t(nsamples) * N;
    for (size_t k = size_t(blockIdx.x) * BLK + threadIdx.x; k < per; k += size_t(gridDim.x) * BLK) {
        const size_t smp = k / N, s = k - smp * N;
        const double v = data[(smp * nch + c) * N + s];
        s1 += v;
        s2 += v * v;
    }
    __shared__ double b1[BLK], b2[BLK];
    b1[threadIdx.x] = s1;
    b2[threadIdx.x] = s2;
    __syncthreads();
    for (int w = BLK / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            b1[threadIdx.x] += b1[threadIdx.x + w];
            b2[threadIdx.x] += b2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * (c * gridDim.x + blockIdx.x)] = b1[0];
        part[2 * (c * gridDim.x + blockIdx.x) + 1] = b2[0];
    }
}

// Raw network inputs from a solver state: Q (5 x N) and u (3 x N) of type T
// -> [8][N] FP32.
template <typename T>
__global__ __launch_bounds__(BLK) void k_sample(int N, const T *__restrict__ Q, const T *__restrict__ u,
                                                float *__restrict__ x)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
#pragma unroll
    for (int c = 0; c < 5; ++c) x[size_t(c) * N + s] = float(Q[size_t(c) * N + s]);
#pragma unroll
    for (int c = 0; c < 3; ++c) x[size_t(5 + c) * N + s] = float(u[size_t(c) * N + s]);
}

// Network output (standardised, [N][5]) -> raw increment; either written as
// [5][N] FP32 (dq) or added to a Q field of type T (5 x N).
template <typename T>
__global__ __launch_bounds__(BLK) void k_apply(int N, const float *__restrict__ Y, const float *__restrict__ norm,
                                               float *__restrict__ dq, T *__restrict__ Q)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const float d = Y[size_t(s) * 5 + k] * norm[21 + k] + norm[16 + k];
        if (dq) dq[size_t(k) * N + s] = d;
        if (Q) Q[size_t(k) * N + s] = T(Q[size_t(k) * N + s] + T(d));
    }
}

// Residual sums for || (Qa + dq) - Qb ||^2 and || Qb ||^2 (FP64 block partials).
template <typename T>
__global__ __launch_bounds__(BLK) void k_resid(int N, const T *__restrict__ Qa, const float *__restrict__ dq,
                                               const T *__restrict__ Qb, double *__restrict__ part)
{
    double s1 = 0.0, s2 = 0.0;
    for (size_t k = size_t(blockIdx.x) * BLK + threadIdx.x; k < size_t(5) * N; k += size_t(gridDim.x) * BLK) {
        const double b = double(Qb[k]);
        const double d = double(Qa[k]) + double(dq[k]) - b;
        s1 += d * d;
        s2 += b * b;
    }
    __shared__ double b1[BLK], b2[BLK];
    b1[threadIdx.x] = s1;
    b2[threadIdx.x] = s2;
    __syncthreads();
    for (int w = BLK / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            b1[threadIdx.x] += b1[threadIdx.x + w];
            b2[threadIdx.x] += b2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = b1[0];
        part[2 * blockIdx.x + 1] = b2[0];
    }
}

// dq = Q(t+k) - Q(t) from two network-input arrays (their first 5 planes).
__global__ __launch_bounds__(BLK) void k_diff(int N, const float *__restrict__ x0, const float *__restrict__ x1,
                                              float *__restrict__ dq)
{
    const size_t i = size_t(blockIdx.x) * BLK + threadIdx.x;
    if (i < size_t(5) * N) dq[i] = x1[i] - x0[i];
}

inline int blocks(size_t n) { return int((n + BLK - 1) / BLK); }

}  // namespace

Grid3 make_grid(int nx, int ny, int nz)
{
    Grid3 g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.N = nx * ny * nz;
    g.tx = (nx + TXs - 1) / TXs;
    g.ty = (ny + TYs - 1) / TYs;
    g.tz = (nz + TZs - 1) / TZs;
    g.ntiles = g.tx * g.ty * g.tz;
    return g;
}

int conv_grid(const Grid3 &g) { return g.ntiles < 4096 ? g.ntiles : 4096; }
int wgrad_grid(const Grid3 &g) { return g.ntiles < WGRAD_BLOCKS ? g.ntiles : WGRAD_BLOCKS; }

hipError_t conv(const Grid3 &g, int cip, int cop, int mode, const unsigned short *X, const unsigned short *W,
                const float *bias, void *out, const unsigned short *mask, int co_valid, hipStream_t st)
{
    const int gr = conv_grid(g);
#define HLB_CONV(CI_, CO_, M_) \
    k_conv<CI_, CO_, M_><<<gr, BLK, 0, st>>>(g, X, W, bias, out, mask, co_valid)
    if (cip == 16 && cop == 32 && mode == MODE_RELU) HLB_CONV(16, 32, MODE_RELU);
    else if (cip == 32 && cop == 32 && mode == MODE_RELU) HLB_CONV(32, 32, MODE_RELU);
    else if (cip == 32 && cop == 16 && mode == MODE_LINEAR) HLB_CONV(32, 16, MODE_LINEAR);
    else if (cip == 16 && cop == 32 && mode == MODE_LINEAR) HLB_CONV(16, 32, MODE_LINEAR);
    else if (cip == 32 && cop == 32 && mode == MODE_LINEAR) HLB_CONV(32, 32, MODE_LINEAR);
    else if (cip == 16 && cop == 32 && mode == MODE_MASK) HLB_CONV(16, 32, MODE_MASK);
    else if (cip == 32 && cop == 32 && mode == MODE_MASK) HLB_CONV(32, 32, MODE_MASK);
    else if (cip == 16 && cop == 32 && mode == MODE_RAW) HLB_CONV(16, 32, MODE_RAW);
    else if (cip == 32 && cop == 32 && mode == MODE_RAW) HLB_CONV(32, 32, MODE_RAW);
    else if (cip == 32 && cop == 16 && mode == MODE_RAW) HLB_CONV(32, 16, MODE_RAW);
    else if (cip == 32 && cop == 16 && mode == MODE_RELU) HLB_CONV(32, 16, MODE_RELU);
    else
        return hipErrorInvalidValue;
#undef HLB_CONV
    return hipGetLastError();
}

hipError_t wgrad(const Grid3 &g, int cip, int cop, const unsigned short *X, const unsigned short *dZ, float *part,
                 int ci, int co, float *grad, hipStream_t st)
{
    const int gr = wgrad_grid(g);
    if (cip == 16 && cop == 32)
        k_wgrad<16, 32><<<gr, BLK, 0, st>>>(g, X, dZ, part);
    else if (cip == 32 && cop == 32)
        k_wgrad<32, 32><<<gr, BLK, 0, st>>>(g, X, dZ, part);
    else if (cip == 32 && cop == 16)
        k_wgrad<32, 16><<<gr, BLK, 0, st>>>(g, X, dZ, part);
    else
        return hipErrorInvalidValue;
    k_wgrad_reduce<<<64, BLK, 0, st>>>(part, gr, cip, cop, ci, co, grad);
    return hipGetLastError();
}

hipError_t wprep(const float *W, int ci, int co, int cip, int cop, unsigned short *Wf, unsigned short *Wt,
                 hipStream_t st)
{
    k_wprep<<<64, BLK, 0, st>>>(W, ci, co, cip, cop, Wf, Wt);
    return hipGetLastError();
}

hipError_t pack(int N, const float *x, const float *norm, unsigned short *A0, hipStream_t st)
{
    k_pack<<<blocks(N), BLK, 0, st>>>(N, x, norm, A0);
    return hipGetLastError();
}

hipError_t lossgrad(int N, const float *Y, const float *dq, const float *norm, unsigned short *dZ, double *part,
                    double *out, hipStream_t st)
{
    k_lossgrad<<<blocks(N), BLK, 0, st>>>(N, Y, dq, norm, dZ, part);
    k_sum<<<1, BLK, 0, st>>>(part, blocks(N), out);
    return hipGetLastError();
}

hipError_t adam(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps, int t,
                hipStream_t st)
{
    const float c1 = 1.f - powf(b1, float(t)), c2 = 1.f - powf(b2, float(t));
    k_adam<<<blocks(n), BLK, 0, st>>>(n, p, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t stats(const float *data, int nch, int N, int nsamples, double *part, int nblk, hipStream_t st)
{
    k_stats<<<dim3(nblk, nch), BLK, 0, st>>>(data, nch, N, nsamples, part);
    return hipGetLastError();
}

hipError_t sample(bool fp32, int N, const void *Q, const void *u, float *x, hipStream_t st)
{
    if (fp32)
        k_sample<float><<<blocks(N), BLK, 0, st>>>(N, static_cast<const float *>(Q), static_cast<const float *>(u), x);
    else
        k_sample<double><<<blocks(N), BLK, 0, st>>>(N, static_cast<const double *>(Q), static_cast<const double *>(u),
                                                    x);
    return hipGetLastError();
}

hipError_t apply(bool fp32, int N, const float *Y, const float *norm, float *dq, void *Q, hipStream_t st)
{
    if (fp32)
        k_apply<float><<<blocks(N), BLK, 0, st>>>(N, Y, norm, dq, static_cast<float *>(Q));
    else
        k_apply<double><<<blocks(N), BLK, 0, st>>>(N, Y, norm, dq, static_cast<double *>(Q));
    return hipGetLastError();
}

hipError_t diff(int N, const float *x0, const float *x1, float *dq, hipStream_t st)
{
    k_diff<<<blocks(size_t(5) * N), BLK, 0, st>>>(N, x0, x1, dq);
    return hipGetLastError();
}

hipError_t resid(bool fp32, int N, const void *Qa, const float *dq, const void *Qb, double *part, int nblk,
                 hipStream_t st)
{
    if (fp32)
        k_resid<float><<<nblk, BLK, 0, st>>>(N, static_cast<const float *>(Qa), dq, static_cast<const float *>(Qb),
                                             part);
    else
        k_resid<double><<<nblk, BLK, 0, st>>>(N, static_cast<const double *>(Qa), dq,
                                              static_cast<const double *>(Qb), part);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace hlb
