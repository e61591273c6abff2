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

// Raw network inputs per site: Q (5), u (3), d1 (5), s2 (5).
constexpr int NIN = 18;
// Standardisation block (floats): input means and stds, output (target)
// means and stds, and beta, the weight of s2 in the extrapolation base.
constexpr int NORM_IN_MEAN = 0, NORM_IN_STD = 18, NORM_OUT_MEAN = 36, NORM_OUT_STD = 41, NORM_BETA = 46;
constexpr int NORM_SIZE = 47;

constexpr int WGRAD_BLOCKS = 512;  // persistent blocks of the weight-gradient kernel

Grid3 make_grid(int nx, int ny, int nz);
int wgrad_grid(const Grid3 &g);

// Bytes of a layer's weights in MFMA fragment order for a convolution of cin
// input and cout output channels (see k_wprep).
size_t frag_bytes(int cin, int cout);
// Convolution with epilogue (see k_conv) with weights in fragment order;
// supported (cin, cout): (16, 32), (32, 32), (32, 16).
hipError_t conv(const Grid3 &g, int cip, int cop, int mode, const unsigned short *X, const unsigned short *W,
                const float *bias, void *out, const unsigned short *mask, int co_valid, hipStream_t st);
// Weight and bias gradient of one layer into the flat layout W[co][ci][27], b[co]
// (cip = 32; cop = 32 or 16).  part: wgrad_grid(g) x (27 cip cop + cop) floats
// of scratch.
hipError_t wgrad(const Grid3 &g, int cip, int cop, const unsigned short *X, const unsigned short *dZ, float *part,
                 int ci, int co, float *grad, hipStream_t st);
// Fragment-ordered weights of one layer: Wf for the forward convolution
// (cip -> cop), Wt for the backward-data convolution (cop -> cip).
hipError_t wprep(const float *W, int ci, int co, int cip, int cop, unsigned short *Wf, unsigned short *Wt,
                 hipStream_t st);
hipError_t pack(int N, const float *x, const float *norm, unsigned short *A0, hipStream_t st);
hipError_t pack_state(bool fp32, int N, const void *Q, const void *u, const float *d1, const float *s2,
                      const float *norm, unsigned short *A0, hipStream_t st);
hipError_t inputs(bool fp32, int N, const void *Q, const void *u, const float *d1, const float *s2, float *x,
                  hipStream_t st);
hipError_t hist3(bool fp32, int N, const void *Q, const void *B, const void *A, float *d1, float *s2, hipStream_t st);
hipError_t hist_step(bool fp32, int N, const void *Q, const void *P, float *d1, float *s2, hipStream_t st);
hipError_t predict_out(int N, const float *Y, const float *norm, const float *x, float *dq, hipStream_t st);
hipError_t jump(bool fp32, int N, const float *Y, const float *norm, float *d1, float *s2, void *Q, float *dq,
                hipStream_t st);
hipError_t lossgrad(int N, const float *Y, const float *dq, const float *x, const float *norm, unsigned short *dZ,
                    double *part, double *out, hipStream_t st);
hipError_t adam(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps, int t,
                hipStream_t st);
hipError_t stats(const float *data, int nch, int N, int nsamples, double *part, int nblk, hipStream_t st);
hipError_t stats_target(const float *x, const float *dq, int N, int nsamples, float beta, double *part, int nblk,
                        hipStream_t st);
hipError_t resid(bool fp32, int N, const void *Qa, const float *dq, const void *Qb, double *part, int nblk,
                 hipStream_t st);

}  // namespace nn
}  // namespace hlb
