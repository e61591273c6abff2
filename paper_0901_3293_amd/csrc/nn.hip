// nn.hip -- kernels of the 3D convolutional surrogate on BF16 matrix cores.
//
// Activations are channels-last bfloat16, act[site][C] with C padded to 16 or
// 32.  tap = kz*9 + ky*3 + kx of a 3x3x3 kernel reads the input at offset
// (kx-1, ky-1, kz-1), periodic.  The convolutions are implicit GEMMs on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (k_conv); the weight
// gradient is a GEMM over sites (k_wgrad) with a deterministic FP64 reduction
// of per-block partials.
#include <hip/hip_runtime.h>

#include "nn.h"
#include "tiles.h"

namespace hlb {
namespace nn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BLK = 256;
constexpr int TXs = 16, TYs = 4, TZs = 4;  // weight-gradient tile (Grid3)

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

// Periodic wrap for an index that is at most one period out of range (the
// general modulo only when it is not, i.e. on lattices smaller than a tile).
__device__ __forceinline__ int wrap_near(int v, int n)
{
    v += v < 0 ? n : 0;
    v -= v >= n ? n : 0;
    return (v >= 0 && v < n) ? v : wrap(v, n);
}

__device__ __forceinline__ void tile_origin(const Grid3 &g, int t, int &x0, int &y0, int &z0)
{
    x0 = (t % g.tx) * TXs;
    const int r = t / g.tx;
    y0 = (r % g.ty) * TYs;
    z0 = (r / g.ty) * TZs;
}

// Forward-style periodic 3x3x3 convolution of a CIN-channel activation into
// COUT channels, as an implicit GEMM on v_mfma_f32_16x16x32_bf16: M = 16
// output channels, N = 16 sites of one x-row, K = 32 (the CIN = 32 channels of
// one tap, or the 16 channels of two taps when CIN = 16).
//
// One block of 8 waves per CU owns a tile of 16 x (WY RY) x (WZ RZ) = 16 x 8
// x 4 output sites at a time; its input brick (tile plus a one-site periodic
// halo, 69 KB for 32 channels) is staged in LDS, and the brick of the block's
// next tile is fetched into registers while the current one is computed.
// The layer's weights, pre-arranged in MFMA fragment order (k_wprep, 55 KB
// for 32 -> 32), are staged in LDS once per block, so the per-kstep fragment
// reads (one kstep ahead) are LDS reads.  Each wave owns 16 x RY x RZ output
// sites with all COUT channels in its accumulators; for each x-offset of the
// stencil it reads the (RY+2)(RZ+2) brick rows it needs into registers once
// and runs all nine (y, z) taps of that offset against them.  Blocks take
// contiguous runs of tiles, and the block index is remapped so that each XCD
// (with its own L2) works on one contiguous part of the lattice.
//
// Epilogues:
//  MODE_RELU:   out_bf16[s][co] = bf16(relu(acc + b[co])), 0 for co >= co_valid
//  MODE_LINEAR: out_f32[s][co]  = acc + b[co] for co < co_valid (row stride co_valid)
//  MODE_MASK:   out_bf16[s][co] = mask[s][co] > 0 ? bf16(acc) : 0   (backward through ReLU)
//  MODE_RAW:    out_f32[s][co]  = acc (row stride COUT)
constexpr int nksteps(int cin) { return cin == 32 ? 27 : 15; }

template <int CIN, int COUT, int RY, int RZ, int WY, int WZ>
struct ConvShape {
    static constexpr int NS = COUT / 16, NKS = nksteps(CIN), KPD = NKS / 3;
    static constexpr int TY = WY * RY, TZ = WZ * RZ;              // block tile: 16 x TY x TZ
    static constexpr int BX = 18, BY = TY + 2, BZ = TZ + 2;       // brick
    static constexpr int BN = BX * BY * BZ;
    static constexpr int V = CIN / 8;                             // 16-byte chunks per site
    static constexpr int NCH = (BN * V + BLK - 1) / BLK;          // chunks staged per thread
    static constexpr size_t lds_bytes = size_t(BN) * CIN * 2;
};

// LDS position (in 16-byte chunks) of chunk v of brick site `site`: sites
// are unpadded and the chunk index is XOR-swizzled with the site so that the
// 16 lanes of a quarter-wave reading one chunk of 16 consecutive sites hit
// 16 different bank groups.
template <int V>
__device__ __forceinline__ int brick_chunk(int site, int v)
{
    return site * V + (v ^ ((site / (16 / V)) % V));
}

// Weight gradient dW[tap][ci][co] = sum_s dZ[s][co] X[s + off(tap)][ci] and
// bias gradient db[co] = sum_s dZ[s][co] on v_mfma_f32_16x16x32_bf16: per
// tile of 16x4x4 sites, M = 16 output channels, N = 16 input channels,
// K = 32 sites (two x-rows).  The tile's dZ and its input brick (18x6x6
// sites, periodic wrap) are staged channel-major in LDS (brick rows padded to
// 24 sites; each channel plane padded so that its stride is 4 dwords modulo
// the 32 LDS banks, which keeps the 16 channels a 16-byte operand read
// touches on distinct banks).  An operand of 8 consecutive sites shifted by the tap's
// x-offset comes from one aligned 16-byte read and one 4-byte read of the
// brick row, shared by the three x-offsets of a (y, z) offset pair (odd
// offsets take a 16-bit funnel shift).  With 32 output channels wave w owns
// the (co block, ci block) pair (w >> 1, w & 1) for all 27 taps; with 16, ci
// block w & 1 over half the K-chunks, the two halves summed in LDS at the end.
// The bias gradient is summed while dZ is staged (each thread keeps the
// running sums of the channels of the sites it stages; the block adds the
// threads' sums per channel in thread order at the end).
// Per-block FP32 partials; the final sum is FP64 in a fixed order
// (k_wgrad_reduce), so the result is deterministic.
template <int COP>
__global__ __launch_bounds__(BLK) void k_wgrad(Grid3 g, const unsigned short *__restrict__ X,
                                               const unsigned short *__restrict__ dZ, float *__restrict__ part)
{
    constexpr int CIP = 32;
    constexpr int XR = 24, BYs = TYs + 2, BZs = TZs + 2, ROWS = BYs * BZs;
    constexpr int TS = TXs * TYs * TZs;  // 256 sites, 8 K-chunks of 32
    constexpr int CSX = ROWS * XR + 40;  // brick channel stride (halfwords): 452 dwords, 4 mod 32
    constexpr int CSD = TS + 8;          // dZ channel stride (halfwords): 132 dwords, 4 mod 32
    static_assert((CSX / 2) % 32 == 4 && (CSD / 2) % 32 == 4, "bank-spread channel strides");
    static_assert(CSX % 8 == 0 && CSD % 8 == 0, "16-byte aligned operand rows");
    static_assert((TXs + 2) % 2 == 0 && XR % 2 == 0 && TXs % 2 == 0, "sites staged in x-pairs");
    constexpr int PS = 27 * CIP * COP + COP;
    constexpr int NBX = (TXs + 2) * ROWS;  // brick sites
    __shared__ __attribute__((aligned(16))) unsigned short sX[CIP * CSX];
    __shared__ __attribute__((aligned(16))) unsigned short sD[COP * CSD];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lg = l >> 4;
    const int mt = COP == 32 ? (w >> 1) : 0, nt = w & 1;
    const int half = COP == 32 ? 0 : (w >> 1);  // COP == 16: which K-chunks this wave takes
    const int cstep = COP == 32 ? 1 : 2;
    f32x4 acc[27];
#pragma unroll
    for (int j = 0; j < 27; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    static_assert(TS / 2 <= BLK, "one site pair of dZ per thread and tile");
    float dsum[COP];
#pragma unroll
    for (int co = 0; co < COP; ++co) dsum[co] = 0.f;
    for (int t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
        int x0, y0, z0;
        tile_origin(g, t, x0, y0, z0);
        __syncthreads();
        // input brick, channel-major: sX[ci][bz][by][bx].  A thread takes two
        // x-neighbouring sites (bx, bx + 1) with all their channels and writes
        // one 32-bit word (the two sites' values) per channel.
        unsigned *sXw = reinterpret_cast<unsigned *>(sX);
        for (int e = threadIdx.x; e < NBX / 2; e += BLK) {
            const int px = e % ((TXs + 2) / 2), r = e / ((TXs + 2) / 2), by = r % BYs, bz = r / BYs;
            const int y = wrap(y0 - 1 + by, g.ny), z = wrap(z0 - 1 + bz, g.nz);
            const size_t row = size_t(g.nx) * (size_t(y) + size_t(g.ny) * z);
            const size_t ga = row + size_t(wrap(x0 - 1 + 2 * px, g.nx));
            const size_t gb = row + size_t(wrap(x0 + 2 * px, g.nx));
            unsigned *d = sXw + r * (XR / 2) + px;
#pragma unroll
            for (int v = 0; v < CIP / 8; ++v) {
                const u32x4 a = *reinterpret_cast<const u32x4 *>(X + ga * CIP + v * 8);
                const u32x4 b = *reinterpret_cast<const u32x4 *>(X + gb * CIP + v * 8);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    d[(8 * v + 2 * c) * (CSX / 2)] = (a[c] & 0xffffu) | (b[c] << 16);
                    d[(8 * v + 2 * c + 1) * (CSX / 2)] = (a[c] >> 16) | (b[c] & 0xffff0000u);
                }
            }
        }
        // output gradient of the tile, channel-major: sD[co][site], two x-neighbouring
        // sites per thread as above (sites outside the lattice contribute zero)
        unsigned *sDw = reinterpret_cast<unsigned *>(sD);
        for (int e = threadIdx.x; e < TS / 2; e += BLK) {
            const int si = 2 * e, tx = si % TXs, r = si / TXs, ty = r % TYs, tz = r / TYs;
            const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
            const bool inyz = y < g.ny && z < g.nz;
            const bool oka = inyz && x < g.nx, okb = inyz && x + 1 < g.nx;
            const size_t ga = size_t(x) + size_t(g.nx) * (size_t(y) + size_t(g.ny) * z);
            unsigned *d = sDw + e;
#pragma unroll
            for (int v = 0; v < COP / 8; ++v) {
                const u32x4 zero4 = {0u, 0u, 0u, 0u};
                const u32x4 a = oka ? *reinterpret_cast<const u32x4 *>(dZ + ga * COP + v * 8) : zero4;
                const u32x4 b = okb ? *reinterpret_cast<const u32x4 *>(dZ + (ga + 1) * COP + v * 8) : zero4;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    d[(8 * v + 2 * c) * (CSD / 2)] = (a[c] & 0xffffu) | (b[c] << 16);
                    d[(8 * v + 2 * c + 1) * (CSD / 2)] = (a[c] >> 16) | (b[c] & 0xffff0000u);
                    dsum[8 * v + 2 * c] += bf2f((unsigned short)(a[c] & 0xffffu)) + bf2f((unsigned short)(b[c] & 0xffffu));
                    dsum[8 * v + 2 * c + 1] += bf2f((unsigned short)(a[c] >> 16)) + bf2f((unsigned short)(b[c] >> 16));
                }
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int c = half; c < TS / 32; c += cstep) {
            const int rowk = 2 * c + (lg >> 1), yy = rowk % TYs, zz = rowk / TYs, xo = 8 * (lg & 1);
            const u32x4 A = *reinterpret_cast<const u32x4 *>(sD + (16 * mt + li) * CSD + c * 32 + 8 * lg);
            const unsigned short *xrow = sX + (16 * nt + li) * CSX + xo;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int dz = q / 3, dy = q % 3;
                const unsigned short *rp = xrow + ((zz + dz) * BYs + (yy + dy)) * XR;
                const u32x4 lo = *reinterpret_cast<const u32x4 *>(rp);
                const unsigned hi = *reinterpret_cast<const unsigned *>(rp + 8);
                const u32x4 b0 = lo;
                const u32x4 b1 = {__builtin_amdgcn_alignbit(lo[1], lo[0], 16), __builtin_amdgcn_alignbit(lo[2], lo[1], 16),
                                  __builtin_amdgcn_alignbit(lo[3], lo[2], 16), __builtin_amdgcn_alignbit(hi, lo[3], 16)};
                const u32x4 b2 = {lo[1], lo[2], lo[3], hi};
                const int tap = dz * 9 + dy * 3;
                acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A),
                                                                   __builtin_bit_cast(bf16x8, b0), acc[tap], 0, 0, 0);
                acc[tap + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, A), __builtin_bit_cast(bf16x8, b1), acc[tap + 1], 0, 0, 0);
                acc[tap + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, A), __builtin_bit_cast(bf16x8, b2), acc[tap + 2], 0, 0, 0);
            }
        }
    }
    float *P = part + size_t(blockIdx.x) * PS;
    {
        // bias: channel co summed over the TS / 2 threads that stage dZ, in order
        float *sS = reinterpret_cast<float *>(sX);
        static_assert(size_t(TS / 2) * COP * sizeof(float) <= sizeof(sX), "bias sums fit the brick buffer");
        __syncthreads();
        if (int(threadIdx.x) < TS / 2)
#pragma unroll
            for (int co = 0; co < COP; ++co) sS[threadIdx.x * COP + co] = dsum[co];
        __syncthreads();
        if (int(threadIdx.x) < COP) {
            float db = 0.f;
            for (int t = 0; t < TS / 2; ++t) db += sS[t * COP + threadIdx.x];
            P[27 * CIP * COP + threadIdx.x] = db;
        }
    }
    if (COP == 16) {
        // waves 2 and 3 hand their half-sums to waves 0 and 1 through LDS
        float *sA = reinterpret_cast<float *>(sX);  // 2 x 27 x 64 x 4 floats <= sizeof(sX)
        static_assert(2 * 27 * 64 * 4 * sizeof(float) <= sizeof(sX), "exchange fits the brick buffer");
        __syncthreads();
        if (half == 1)
#pragma unroll
            for (int j = 0; j < 27; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) sA[((nt * 27 + j) * 64 + l) * 4 + r] = acc[j][r];
        __syncthreads();
        if (half == 1) return;
#pragma unroll
        for (int j = 0; j < 27; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[j][r] += sA[((nt * 27 + j) * 64 + l) * 4 + r];
    }
    // D[r] of lane (li, lg): output channel 16 mt + 4 lg + r, input channel 16 nt + li
#pragma unroll
    for (int j = 0; j < 27; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) P[(j * CIP + 16 * nt + li) * COP + 16 * mt + 4 * lg + r] = acc[j][r];
}

// Sum the per-block partials (FP64, block order) into the flat gradient of
// one layer: W[co][ci][tap] (ci < CI, co < CO) then b[co].  Threads walk the
// partial layout contiguously, so every block's partials are read coalesced.
__global__ __launch_bounds__(BLK) void k_wgrad_reduce(const float *__restrict__ part, int nblk, int CIP, int COP,
                                                      int CI, int CO, float *__restrict__ grad)
{
    const int PS = 27 * CIP * COP + COP;
    for (int idx = blockIdx.x * BLK + threadIdx.x; idx < PS; idx += gridDim.x * BLK) {
        int e;
        if (idx < 27 * CIP * COP) {
            const int co = idx % COP, ci = (idx / COP) % CIP, tap = idx / (COP * CIP);
            if (co >= CO || ci >= CI) continue;
            e = (co * CI + ci) * 27 + tap;
        } else {
            const int co = idx - 27 * CIP * COP;
            if (co >= CO) continue;
            e = CO * CI * 27 + co;
        }
        // eight interleaved partial sums (block b into sum b % 8), combined in a
        // fixed order: deterministic, with eight loads in flight per thread
        double acc8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int b = 0;
        for (; b + 8 <= nblk; b += 8)
#pragma unroll
            for (int k = 0; k < 8; ++k) acc8[k] += double(part[size_t(b + k) * PS + idx]);
        for (; b < nblk; ++b) acc8[b & 7] += double(part[size_t(b) * PS + idx]);
        const double s = ((acc8[0] + acc8[1]) + (acc8[2] + acc8[3])) + ((acc8[4] + acc8[5]) + (acc8[6] + acc8[7]));
        grad[e] = float(s);
    }
}

// Weights of one layer in MFMA fragment order for k_conv, from the flat FP32
// parameters W[co][ci][tap].  A convolution as run maps CIN input channels to
// COUT output channels; its fragment array is [kstep][COUT/16][lane][8] bf16,
// lane = 16 lg + i holding output channel 16 ns + i and the 8 input channels
// that lane group lg contributes to the K = 32 slice of the kstep.  Ksteps run
// x-offset major: for CIN = 32 kstep dx*9 + (dz*3 + dy) is one tap; for
// CIN = 16 kstep dx*5 + p pairs the (dz, dy) positions 2p (lane groups 0-1)
// and 2p + 1 (lane groups 2-3; zero past the ninth).
// Forward (transposed = 0): out channel co, in channel ci, tap as stored.
// Backward-data (transposed = 1): out channel ci, in channel co, tap reversed
// (offset -> -offset), i.e. the adjoint convolution.
__global__ __launch_bounds__(BLK) void k_wprep(const float *__restrict__ W, int CI, int CO, int cin, int cout,
                                               int transposed, unsigned short *__restrict__ F)
{
    const int nks = nksteps(cin), ns_n = cout / 16;
    const int total = nks * ns_n * 64 * 8;
    for (int e = blockIdx.x * BLK + threadIdx.x; e < total; e += gridDim.x * BLK) {
        const int j = e & 7, lane = (e >> 3) & 63, rest = e >> 9;
        const int ns = rest % ns_n, ks = rest / ns_n;
        const int lg = lane >> 4, i = lane & 15;
        int dx, q, c;
        if (cin == 32) {
            dx = ks / 9;
            q = ks % 9;
            c = 8 * lg + j;
        } else {
            dx = ks / 5;
            q = 2 * (ks % 5) + (lg >= 2 ? 1 : 0);
            c = 8 * (lg & 1) + j;
        }
        const int o = 16 * ns + i;
        float v = 0.f;
        if (q < 9) {
            const int tap = (q / 3) * 9 + (q % 3) * 3 + dx;
            if (!transposed) {
                if (o < CO && c < CI) v = W[(o * CI + c) * 27 + tap];
            } else {
                if (o < CI && c < CO) v = W[(c * CI + o) * 27 + (26 - tap)];
            }
        }
        F[e] = f2bf(v);
    }
}

// Network inputs (NIN = 18 channels): Q (5 stored components), u (3), the
// last increment d1 = Q(t) - Q(t-k) (5) and its change s2 = Q(t) - 2 Q(t-k) +
// Q(t-2k) (5).  Standardised with norm and rounded to bf16 into the first
// layer's [N][32] activation (channels 18..31 zero).
__device__ __forceinline__ void store_input_row(int N, int s, const float v[NIN], const float *__restrict__ norm,
                                                unsigned short *__restrict__ A0)
{
    alignas(16) unsigned short h[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) h[c] = c < NIN ? f2bf((v[c] - norm[NORM_IN_MEAN + c]) / norm[NORM_IN_STD + c]) : 0;
    uint4 *dst = reinterpret_cast<uint4 *>(A0 + size_t(s) * 32);
    const uint4 *src = reinterpret_cast<const uint4 *>(h);
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] = src[k];
}

// From raw inputs x [NIN][N] FP32.
__global__ __launch_bounds__(BLK) void k_pack(int N, const float *__restrict__ x, const float *__restrict__ norm,
                                              unsigned short *__restrict__ A0)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
    float v[NIN];
#pragma unroll
    for (int c = 0; c < NIN; ++c) v[c] = x[size_t(c) * N + s];
    store_input_row(N, s, v, norm, A0);
}

// From a solver state (Q, u of type T) and the history (d1, s2 FP32 [5][N]).
template <typename T>
__global__ __launch_bounds__(BLK) void k_pack_state(int N, const T *__restrict__ Q, const T *__restrict__ u,
                                                    const float *__restrict__ d1, const float *__restrict__ s2,
                                                    const float *__restrict__ norm, unsigned short *__restrict__ A0)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
    float v[NIN];
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = float(Q[size_t(c) * N + s]);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[5 + c] = float(u[size_t(c) * N + s]);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        v[8 + c] = d1[size_t(c) * N + s];
        v[13 + c] = s2[size_t(c) * N + s];
    }
    store_input_row(N, s, v, norm, A0);
}

// Raw inputs [NIN][N] from a solver state and the history.
template <typename T>
__global__ __launch_bounds__(BLK) void k_inputs(int N, const T *__restrict__ Q, const T *__restrict__ u,
                                                const float *__restrict__ d1, const float *__restrict__ s2,
                                                float *__restrict__ x)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
#pragma unroll
    for (int c = 0; c < 5; ++c) x[size_t(c) * N + s] = float(Q[size_t(c) * N + s]);
#pragma unroll
    for (int c = 0; c < 3; ++c) x[size_t(5 + c) * N + s] = float(u[size_t(c) * N + s]);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        x[size_t(8 + c) * N + s] = d1[size_t(c) * N + s];
        x[size_t(13 + c) * N + s] = s2[size_t(c) * N + s];
    }
}

// History from three snapshots of Q (type T) k steps apart, oldest A, then
// B, then the current Q: d1 = Q - B, s2 = Q - 2B + A (in T, then FP32).
template <typename T>
__global__ __launch_bounds__(BLK) void k_hist3(int N, const T *__restrict__ Q, const T *__restrict__ B,
                                               const T *__restrict__ A, float *__restrict__ d1,
                                               float *__restrict__ s2)
{
    const size_t i = size_t(blockIdx.x) * BLK + threadIdx.x;
    if (i >= size_t(5) * N) return;
    const T q = Q[i], b = B[i], a = A[i];
    d1[i] = float(q - b);
    s2[i] = float((q - b) - (b - a));
}

// History after k plain steps from the snapshot P: dq = Q - P, s2 = dq - d1, d1 = dq.
template <typename T>
__global__ __launch_bounds__(BLK) void k_hist_step(int N, const T *__restrict__ Q, const T *__restrict__ P,
                                                   float *__restrict__ d1, float *__restrict__ s2)
{
    const size_t i = size_t(blockIdx.x) * BLK + threadIdx.x;
    if (i >= size_t(5) * N) return;
    const float dq = float(Q[i] - P[i]);
    s2[i] = dq - d1[i];
    d1[i] = dq;
}

// Increment predicted by the network: dq = d1 + beta s2 + (y std + mean), y
// the standardised network output [N][5].
__device__ __forceinline__ float predicted(const float *__restrict__ Y, const float *__restrict__ norm, int N, int s,
                                           int k, float d1, float s2)
{
    return d1 + norm[NORM_BETA] * s2 + (Y[size_t(s) * 5 + k] * norm[NORM_OUT_STD + k] + norm[NORM_OUT_MEAN + k]);
}

// dq [5][N] from raw inputs x (history in its channels 8..17).
__global__ __launch_bounds__(BLK) void k_predict_out(int N, const float *__restrict__ Y, const float *__restrict__ norm,
                                                     const float *__restrict__ x, float *__restrict__ dq)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
#pragma unroll
    for (int k = 0; k < 5; ++k)
        dq[size_t(k) * N + s] =
            predicted(Y, norm, N, s, k, x[size_t(8 + k) * N + s], x[size_t(13 + k) * N + s]);
}

// One network jump on a solver state: dq from the history; either written
// out (dq != nullptr) or applied: Q += dq, s2 = dq - d1, d1 = dq.
template <typename T>
__global__ __launch_bounds__(BLK) void k_jump(int N, const float *__restrict__ Y, const float *__restrict__ norm,
                                              float *__restrict__ d1, float *__restrict__ s2, T *__restrict__ Q,
                                              float *__restrict__ dq)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const size_t i = size_t(k) * N + s;
        const float a = d1[i], b = s2[i];
        const float d = predicted(Y, norm, N, s, k, a, b);
        if (dq) {
            dq[i] = d;
        } else {
            Q[i] = T(Q[i] + T(d));
            s2[i] = d - a;
            d1[i] = d;
        }
    }
}

// Loss and its gradient: target t = (dq - d1 - beta s2 - mean) / std with the
// history from x, d = y - t, dZ = bf16(2 d / (5 N)), block partials of
// sum d^2 (FP64).
__global__ __launch_bounds__(BLK) void k_lossgrad(int N, const float *__restrict__ Y, const float *__restrict__ dq,
                                                  const float *__restrict__ x, const float *__restrict__ norm,
                                                  unsigned short *__restrict__ dZ, double *__restrict__ part)
{
    const int s = blockIdx.x * BLK + threadIdx.x;
    double acc = 0.0;
    if (s < N) {
        const float sc = 2.0f / (5.0f * float(N));
        alignas(16) unsigned short h[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k < 5) {
                const float c = dq[size_t(k) * N + s] - x[size_t(8 + k) * N + s] -
                                norm[NORM_BETA] * x[size_t(13 + k) * N + s];
                const float t = (c - norm[NORM_OUT_MEAN + k]) / norm[NORM_OUT_STD + k];
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

// Per-channel sums of the training target c = dq - d1 - beta s2 over
// nsamples pairs (x [ns][NIN][N], dq [ns][5][N]); FP64 partials, grid 5 x B.
__global__ __launch_bounds__(BLK) void k_stats_target(const float *__restrict__ x, const float *__restrict__ dq,
                                                      int N, int nsamples, float beta, double *__restrict__ part)
{
    const int c = blockIdx.y;
    double s1 = 0.0, s2 = 0.0;
    const size_t per = size_t(nsamples) * N;
    for (size_t k = size_t(blockIdx.x) * BLK + threadIdx.x; k < per; k += size_t(gridDim.x) * BLK) {
        const size_t smp = k / N, s = k - smp * N;
        const float t = dq[(smp * 5 + c) * N + s] - x[(smp * NIN + 8 + c) * N + s] -
                        beta * x[(smp * NIN + 13 + c) * N + s];
        s1 += double(t);
        s2 += double(t) * double(t);
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

int wgrad_grid(const Grid3 &g) { return g.ntiles < WGRAD_BLOCKS ? g.ntiles : WGRAD_BLOCKS; }

size_t frag_bytes(int cin, int cout) { return size_t(nksteps(cin)) * (cout / 16) * 64 * 16; }

namespace {

int device_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
    }
    return cus;
}

// One block of WBLK threads (8 waves) per CU.
constexpr int WBLK = 512;

template <int CIN, int COUT, int RY, int RZ, int WY, int WZ>
struct ConvLds {
    using S = ConvShape<CIN, COUT, RY, RZ, WY, WZ>;
    static constexpr int NCH = (S::BN * S::V + WBLK - 1) / WBLK;   // brick chunks per thread
    static constexpr int NW = S::NKS * S::NS * 64;                  // weight fragments (16 B)
    static constexpr size_t brick_bytes = size_t(S::BN) * CIN * 2;
    static constexpr size_t lds_bytes = brick_bytes + size_t(NW) * 16;
};

template <int CIN, int COUT, int MODE, int RY, int RZ, int WY, int WZ>
__global__ __launch_bounds__(WBLK, 1) void k_conv(Grid3 g, int ctx, int cty, int ntiles, int per_block,
                                                       const unsigned short *__restrict__ X,
                                                       const u32x4 *__restrict__ Wfrag,
                                                       const float *__restrict__ bias, void *__restrict__ out,
                                                       const unsigned short *__restrict__ mask, int co_valid)
{
    using S = ConvShape<CIN, COUT, RY, RZ, WY, WZ>;
    using WS = ConvLds<CIN, COUT, RY, RZ, WY, WZ>;
    constexpr int NS = S::NS, KPD = S::KPD, V = S::V, NCH = WS::NCH;
    static_assert(WY * WZ == WBLK / 64, "one wave per sub-tile");
    extern __shared__ __attribute__((aligned(16))) unsigned short smem[];
    u32x4 *sB = reinterpret_cast<u32x4 *>(smem);
    u32x4 *sW = reinterpret_cast<u32x4 *>(smem + WS::brick_bytes / 2);

    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lg = l >> 4;
    const int wy = w % WY, wz = w / WY;
    const int cv = CIN == 32 ? lg : (lg & 1);
    const bool upper = lg >= 2;
    float bv[NS][4];
#pragma unroll
    for (int ns = 0; ns < NS; ++ns)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = ns * 16 + 4 * lg + r;
            bv[ns][r] = ((MODE == MODE_RELU || MODE == MODE_LINEAR) && co < co_valid) ? bias[co] : 0.f;
        }
    const int b = xcd_logical_block();
    const int t_begin = b * per_block;
    const int t_end = min(ntiles, t_begin + per_block);
    const u32x4 zero = {0u, 0u, 0u, 0u};
    if (t_begin >= t_end) return;

    for (int e = threadIdx.x; e < WS::NW; e += WBLK) sW[e] = Wfrag[e];

    // brick of tile t into registers: chunk e = threadIdx.x + k WBLK
    u32x4 pre[NCH];
    auto fetch = [&](int t) __attribute__((always_inline)) {
        const int x0 = (t % ctx) * 16, rr = t / ctx;
        const int yb = (rr % cty) * S::TY, zb = (rr / cty) * S::TZ;
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const int e = threadIdx.x + k * WBLK;
            if (e < S::BN * V) {
                const int site = e / V, v = e - site * V;
                const int bx = site % S::BX, r2 = site / S::BX, by = r2 % S::BY, bz = r2 / S::BY;
                const int x = wrap_near(x0 - 1 + bx, g.nx), y = wrap_near(yb - 1 + by, g.ny),
                          z = wrap_near(zb - 1 + bz, g.nz);
                const size_t gs = size_t(x) + size_t(g.nx) * (size_t(y) + size_t(g.ny) * z);
                pre[k] = *reinterpret_cast<const u32x4 *>(X + gs * CIN + v * 8);
            }
        }
    };
    fetch(t_begin);

    for (int t = t_begin; t < t_end; ++t) {
        const int x0 = (t % ctx) * 16, rr = t / ctx;
        const int yb = (rr % cty) * S::TY, zb = (rr / cty) * S::TZ;
        __syncthreads();  // the previous tile's reads of the brick are done
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const int e = threadIdx.x + k * WBLK;
            if (e < S::BN * V) {
                const int site = e / V, v = e - site * V;
                sB[brick_chunk<V>(site, v)] = pre[k];
            }
        }
        __syncthreads();
        if (t + 1 < t_end) fetch(t + 1);  // in flight during this tile's MFMAs
        f32x4 acc[RZ * RY][NS];
#pragma unroll
        for (int m = 0; m < RZ * RY; ++m)
#pragma unroll
            for (int ns = 0; ns < NS; ++ns) acc[m][ns] = f32x4{0.f, 0.f, 0.f, 0.f};
        u32x4 a[NS], an[NS];
#pragma unroll
        for (int ns = 0; ns < NS; ++ns) a[ns] = sW[ns * 64 + l];
#pragma unroll 1
        for (int dx = 0; dx < 3; ++dx) {
            u32x4 f[RZ + 2][RY + 2];
#pragma unroll
            for (int zz = 0; zz < RZ + 2; ++zz)
#pragma unroll
                for (int yy = 0; yy < RY + 2; ++yy) {
                    const int site = ((wz * RZ + zz) * S::BY + (wy * RY + yy)) * S::BX + li + dx;
                    f[zz][yy] = sB[brick_chunk<V>(site, cv)];
                }
#pragma unroll
            for (int k = 0; k < KPD; ++k) {
                const int ks = dx * KPD + k;
                if (ks + 1 < S::NKS) {
#pragma unroll
                    for (int ns = 0; ns < NS; ++ns) an[ns] = sW[((ks + 1) * NS + ns) * 64 + l];
                }
#pragma unroll
                for (int zz = 0; zz < RZ; ++zz)
#pragma unroll
                    for (int yy = 0; yy < RY; ++yy) {
                        u32x4 bop;
                        if (CIN == 32) {
                            bop = f[zz + k / 3][yy + k % 3];
                        } else {
                            const int qa = 2 * k, qb = 2 * k + 1 < 9 ? 2 * k + 1 : 0;
                            const u32x4 lo = f[zz + qa / 3][yy + qa % 3];
                            const u32x4 hi = 2 * k + 1 < 9 ? f[zz + qb / 3][yy + qb % 3] : zero;
                            bop = upper ? hi : lo;
                        }
#pragma unroll
                        for (int ns = 0; ns < NS; ++ns)
                            acc[zz * RY + yy][ns] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf16x8, a[ns]), __builtin_bit_cast(bf16x8, bop),
                                acc[zz * RY + yy][ns], 0, 0, 0);
                    }
#pragma unroll
                for (int ns = 0; ns < NS; ++ns) a[ns] = an[ns];
            }
        }
        const int xo = x0 + li, y0 = yb + wy * RY, z0 = zb + wz * RZ;
#pragma unroll
        for (int zz = 0; zz < RZ; ++zz)
#pragma unroll
            for (int yy = 0; yy < RY; ++yy) {
                const int yo = y0 + yy, zo = z0 + zz;
                if (xo >= g.nx || yo >= g.ny || zo >= g.nz) continue;
                const size_t s = size_t(xo) + size_t(g.nx) * (size_t(yo) + size_t(g.ny) * zo);
#pragma unroll
                for (int ns = 0; ns < NS; ++ns) {
                    const f32x4 v = acc[zz * RY + yy][ns];
                    const int co = ns * 16 + 4 * lg;
                    if (MODE == MODE_RELU) {
                        unsigned short h[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) h[r] = co + r < co_valid ? f2bf(fmaxf(v[r] + bv[ns][r], 0.f)) : 0;
                        *reinterpret_cast<uint2 *>(static_cast<unsigned short *>(out) + s * COUT + co) =
                            make_uint2(unsigned(h[0]) | (unsigned(h[1]) << 16), unsigned(h[2]) | (unsigned(h[3]) << 16));
                    } else if (MODE == MODE_LINEAR) {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (co + r < co_valid) static_cast<float *>(out)[s * co_valid + co + r] = v[r] + bv[ns][r];
                    } else if (MODE == MODE_MASK) {
                        const uint2 mk = *reinterpret_cast<const uint2 *>(mask + s * COUT + co);
                        const unsigned short mh[4] = {(unsigned short)(mk.x & 0xffffu), (unsigned short)(mk.x >> 16),
                                                      (unsigned short)(mk.y & 0xffffu), (unsigned short)(mk.y >> 16)};
                        unsigned short h[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) h[r] = bf2f(mh[r]) > 0.f ? f2bf(v[r]) : (unsigned short)0;
                        *reinterpret_cast<uint2 *>(static_cast<unsigned short *>(out) + s * COUT + co) =
                            make_uint2(unsigned(h[0]) | (unsigned(h[1]) << 16), unsigned(h[2]) | (unsigned(h[3]) << 16));
                    } else {
                        *reinterpret_cast<float4 *>(static_cast<float *>(out) + s * COUT + co) =
                            make_float4(v[0], v[1], v[2], v[3]);
                    }
                }
            }
    }
}

template <int CIN, int COUT, int MODE>
hipError_t conv_launch(const Grid3 &g, const unsigned short *X, const unsigned short *W, const float *bias,
                            void *out, const unsigned short *mask, int co_valid, hipStream_t st)
{
    constexpr int RY = 2, RZ = 2, WY = 4, WZ = 2;
    using S = ConvShape<CIN, COUT, RY, RZ, WY, WZ>;
    using WS = ConvLds<CIN, COUT, RY, RZ, WY, WZ>;
    auto kern = k_conv<CIN, COUT, MODE, RY, RZ, WY, WZ>;
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, int(WS::lds_bytes));
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int ctx = (g.nx + 15) / 16, cty = (g.ny + S::TY - 1) / S::TY, ctz = (g.nz + S::TZ - 1) / S::TZ;
    const int ntiles = ctx * cty * ctz;
    // one resident block per CU (the LDS bound), a multiple of the 8 XCDs
    int grid = device_cus();
    grid = ntiles < grid ? ntiles : grid;
    grid = (grid + 7) & ~7;
    const int per_block = (ntiles + grid - 1) / grid;
    kern<<<grid, WBLK, WS::lds_bytes, st>>>(g, ctx, cty, ntiles, per_block, X, reinterpret_cast<const u32x4 *>(W),
                                            bias, out, mask, co_valid);
    return hipGetLastError();
}


}  // namespace

hipError_t conv(const Grid3 &g, int cin, int cout, int mode, const unsigned short *X, const unsigned short *W,
                const float *bias, void *out, const unsigned short *mask, int co_valid, hipStream_t st)
{
#define HLB_CONV(CI_, CO_, M_) \
    if (cin == CI_ && cout == CO_ && mode == M_) return conv_launch<CI_, CO_, M_>(g, X, W, bias, out, mask, co_valid, st)
    HLB_CONV(16, 32, MODE_RELU);
    HLB_CONV(32, 32, MODE_RELU);
    HLB_CONV(32, 16, MODE_LINEAR);
    HLB_CONV(16, 32, MODE_LINEAR);
    HLB_CONV(32, 32, MODE_LINEAR);
    HLB_CONV(16, 32, MODE_MASK);
    HLB_CONV(32, 32, MODE_MASK);
    HLB_CONV(16, 32, MODE_RAW);
    HLB_CONV(32, 32, MODE_RAW);
    HLB_CONV(32, 16, MODE_RAW);
#undef HLB_CONV
    return hipErrorInvalidValue;
}

hipError_t wgrad(const Grid3 &g, int cip, int cop, const unsigned short *X, const unsigned short *dZ, float *part,
                 int ci, int co, float *grad, hipStream_t st)
{
    const int gr = wgrad_grid(g);
    if (cip == 32 && cop == 32)
        k_wgrad<32><<<gr, BLK, 0, st>>>(g, X, dZ, part);
    else if (cip == 32 && cop == 16)
        k_wgrad<16><<<gr, BLK, 0, st>>>(g, X, dZ, part);
    else
        return hipErrorInvalidValue;
    k_wgrad_reduce<<<(27 * cip * cop + cop + BLK - 1) / BLK, BLK, 0, st>>>(part, gr, cip, cop, ci, co, grad);
    return hipGetLastError();
}

hipError_t wprep(const float *W, int ci, int co, int cip, int cop, unsigned short *Wf, unsigned short *Wt,
                 hipStream_t st)
{
    k_wprep<<<64, BLK, 0, st>>>(W, ci, co, cip, cop, 0, Wf);
    k_wprep<<<64, BLK, 0, st>>>(W, ci, co, cop, cip, 1, Wt);
    return hipGetLastError();
}

hipError_t pack(int N, const float *x, const float *norm, unsigned short *A0, hipStream_t st)
{
    k_pack<<<blocks(N), BLK, 0, st>>>(N, x, norm, A0);
    return hipGetLastError();
}

hipError_t pack_state(bool fp32, int N, const void *Q, const void *u, const float *d1, const float *s2,
                      const float *norm, unsigned short *A0, hipStream_t st)
{
    if (fp32)
        k_pack_state<float><<<blocks(N), BLK, 0, st>>>(N, static_cast<const float *>(Q),
                                                       static_cast<const float *>(u), d1, s2, norm, A0);
    else
        k_pack_state<double><<<blocks(N), BLK, 0, st>>>(N, static_cast<const double *>(Q),
                                                        static_cast<const double *>(u), d1, s2, norm, A0);
    return hipGetLastError();
}

hipError_t inputs(bool fp32, int N, const void *Q, const void *u, const float *d1, const float *s2, float *x,
                  hipStream_t st)
{
    if (fp32)
        k_inputs<float><<<blocks(N), BLK, 0, st>>>(N, static_cast<const float *>(Q), static_cast<const float *>(u),
                                                   d1, s2, x);
    else
        k_inputs<double><<<blocks(N), BLK, 0, st>>>(N, static_cast<const double *>(Q),
                                                    static_cast<const double *>(u), d1, s2, x);
    return hipGetLastError();
}

hipError_t hist3(bool fp32, int N, const void *Q, const void *B, const void *A, float *d1, float *s2, hipStream_t st)
{
    if (fp32)
        k_hist3<float><<<blocks(size_t(5) * N), BLK, 0, st>>>(N, static_cast<const float *>(Q),
                                                              static_cast<const float *>(B),
                                                              static_cast<const float *>(A), d1, s2);
    else
        k_hist3<double><<<blocks(size_t(5) * N), BLK, 0, st>>>(N, static_cast<const double *>(Q),
                                                               static_cast<const double *>(B),
                                                               static_cast<const double *>(A), d1, s2);
    return hipGetLastError();
}

hipError_t hist_step(bool fp32, int N, const void *Q, const void *P, float *d1, float *s2, hipStream_t st)
{
    if (fp32)
        k_hist_step<float><<<blocks(size_t(5) * N), BLK, 0, st>>>(N, static_cast<const float *>(Q),
                                                                  static_cast<const float *>(P), d1, s2);
    else
        k_hist_step<double><<<blocks(size_t(5) * N), BLK, 0, st>>>(N, static_cast<const double *>(Q),
                                                                   static_cast<const double *>(P), d1, s2);
    return hipGetLastError();
}

hipError_t predict_out(int N, const float *Y, const float *norm, const float *x, float *dq, hipStream_t st)
{
    k_predict_out<<<blocks(N), BLK, 0, st>>>(N, Y, norm, x, dq);
    return hipGetLastError();
}

hipError_t jump(bool fp32, int N, const float *Y, const float *norm, float *d1, float *s2, void *Q, float *dq,
                hipStream_t st)
{
    if (fp32)
        k_jump<float><<<blocks(N), BLK, 0, st>>>(N, Y, norm, d1, s2, static_cast<float *>(Q), dq);
    else
        k_jump<double><<<blocks(N), BLK, 0, st>>>(N, Y, norm, d1, s2, static_cast<double *>(Q), dq);
    return hipGetLastError();
}

hipError_t lossgrad(int N, const float *Y, const float *dq, const float *x, const float *norm, unsigned short *dZ,
                    double *part, double *out, hipStream_t st)
{
    k_lossgrad<<<blocks(N), BLK, 0, st>>>(N, Y, dq, x, norm, dZ, part);
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

hipError_t stats_target(const float *x, const float *dq, int N, int nsamples, float beta, double *part, int nblk,
                        hipStream_t st)
{
    k_stats_target<<<dim3(nblk, 5), BLK, 0, st>>>(x, dq, N, nsamples, beta, part);
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
