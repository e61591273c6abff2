// nn.h -- internal interface of the surrogate kernels (nn.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace hlb {
namespace nn {

struct Grid3 {
    int nx, ny, nz, N;
    int tx, ty, tz, ntiles;  // tiles of 16 x 4 x 4 sites
};

enum ConvMode { MODE_RELU = 0, MODE_LINEAR = 1, MODE_MASK = 2, MODE_RAW = 3 };

constexpr int WGRAD_BLOCKS = 512;  // persistent blocks of the weight-gradient kernel

Grid3 make_grid(int nx, int ny, int nz);
int conv_grid(const Grid3 &g);
int wgrad_grid(const Grid3 &g);

// Convolution with epilogue (see k_conv); supported (cip, cop): (16, 32),
// (32, 32), (32, 16).
hipError_t conv(const Grid3 &g, int cip, int cop, int mode, const unsigned short *X, const unsigned short *W,
                const float *bias, void *out, const unsigned short *mask, int co_valid, hipStream_t st);
// Weight and bias gradient of one layer into the flat layout W[co][ci][27], b[co].
// part: wgrad_grid(g) x (27 cip cop + cop) floats of scratch.
hipError_t wgrad(const Grid3 &g, int cip, int cop, const unsigned short *X, const unsigned short *dZ, float *part,
                 int ci, int co, float *grad, hipStream_t st);
hipError_t wprep(const float *W, int ci, int co, int cip, int cop, unsigned short *Wf, unsigned short *Wt,
                 hipStream_t st);
hipError_t pack(int N, const float *x, const float *norm, unsigned short *A0, hipStream_t st);
hipError_t lossgrad(int N, const float *Y, const float *dq, const float *norm, unsigned short *dZ, double *part,
                    double *out, hipStream_t st);
hipError_t adam(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps, int t,
                hipStream_t st);
hipError_t stats(const float *data, int nch, int N, int nsamples, double *part, int nblk, hipStream_t st);
hipError_t sample(bool fp32, int N, const void *Q, const void *u, float *x, hipStream_t st);
hipError_t apply(bool fp32, int N, const float *Y, const float *norm, float *dq, void *Q, hipStream_t st);
hipError_t diff(int N, const float *x0, const float *x1, float *dq, hipStream_t st);
hipError_t resid(bool fp32, int N, const void *Qa, const float *dq, const void *Qb, double *part, int nblk,
                 hipStream_t st);

}  // namespace nn
}  // namespace hlb
