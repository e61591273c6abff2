// nn_api.cpp -- C-ABI of the convolutional surrogate (include/hlb.h,
// hlbnn_* and hlb_surrogate_advance): buffers, forward, training step with
// Adam, the Q history the network reads, per-layer entry points for the
// parity tests, and the surrogate-with-fallback driver.  All arithmetic runs
// in the kernels of nn.hip/kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/hlb.h"
#include "ctx.h"
#include "kernels.h"
#include "nn.h"

namespace {

using hlb::nn::NIN;
using hlb::nn::NORM_SIZE;

constexpr int NL = 4;
constexpr int CI[NL] = {NIN, 32, 32, 32};
constexpr int CO[NL] = {32, 32, 32, 5};
constexpr int CIP[NL] = {32, 32, 32, 32};
constexpr int COP[NL] = {32, 32, 32, 16};

int layer_params(int l) { return CO[l] * CI[l] * 27 + CO[l]; }
int param_total()
{
    int n = 0;
    for (int l = 0; l < NL; ++l) n += layer_params(l);
    return n;
}
int layer_offset(int l)
{
    int n = 0;
    for (int k = 0; k < l; ++k) n += layer_params(k);
    return n;
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct Sizes {
    size_t params, wbf, act, y, dz, part, red, f5, ckpt, qsnap, norm, total;
};

Sizes sizes_for(const hlb::nn::Grid3 &g)
{
    Sizes z;
    const size_t N = g.N;
    z.params = a256(size_t(param_total()) * 4);
    size_t wb = 0;
    for (int l = 0; l < NL; ++l)
        wb += a256(hlb::nn::frag_bytes(CIP[l], COP[l])) + a256(hlb::nn::frag_bytes(COP[l], CIP[l]));
    z.wbf = wb;
    z.act = a256(N * 32 * 2);
    z.y = a256(N * 5 * 4);
    z.dz = a256(N * 32 * 2);
    z.part = a256(size_t(hlb::nn::wgrad_grid(g)) * (27 * 32 * 32 + 32) * 4);
    z.red = a256((size_t((N + 255) / 256) + 64 * 2 * NIN + 4096) * 8);
    z.f5 = a256(N * 5 * 4);
    z.ckpt = a256(N * 24 * 8);  // populations + Q of an FP64 state; also two Q snapshots
    z.qsnap = a256(N * 5 * 8);
    z.norm = a256(NORM_SIZE * 4);
    z.total = 4 * z.params /* params, grads, m, v */ + z.wbf + NL * z.act + z.y + 2 * z.dz + z.part + z.red +
              3 * z.f5 /* dq, d1, s2 */ + z.ckpt + z.qsnap + z.norm;
    return z;
}

}  // namespace

struct hlbnn {
    hlb::nn::Grid3 g;
    hipStream_t stream;
    float *params, *grads, *m, *v;
    unsigned short *Wf[NL], *Wt[NL];
    unsigned short *A[NL];  // inputs of the layers, [N][32] bf16
    float *Y;               // [N][5] standardised output of the last layer
    unsigned short *dZ[2];  // [N][32]
    float *part;
    double *red;
    float *dq, *d1, *s2;    // [5][N]: predicted increment; history d1, s2
    char *ckpt, *qsnap;
    float *norm;            // NORM_SIZE floats (layout in nn.h)
    bool have_params, have_norm;
    // the history belongs to one solver context at one state version and k
    const hlb_ctx *hist_ctx;
    unsigned long long hist_version;
    int hist_k;
    int adam_t;
    int status;
    char msg[512];
};

namespace {

int nerr(hlbnn *n, int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(n->msg, sizeof(n->msg), fmt, ap);
    va_end(ap);
    n->status = code;
    return code;
}

#define N_GUARD(n)                           \
    do {                                     \
        if (!(n)) return HLB_ERR_ARG;        \
        if ((n)->status) return (n)->status; \
    } while (0)

#define N_TRY(n, call)                                                                                   \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return nerr((n), HLB_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_));     \
    } while (0)

int prep_weights(hlbnn *n)
{
    for (int l = 0; l < NL; ++l)
        N_TRY(n, hlb::nn::wprep(n->params + layer_offset(l), CI[l], CO[l], CIP[l], COP[l], n->Wf[l], n->Wt[l],
                                n->stream));
    return HLB_OK;
}

float *bias_of(hlbnn *n, int l) { return n->params + layer_offset(l) + CO[l] * CI[l] * 27; }

// Forward through the four layers from A[0]; result in Y.
int forward(hlbnn *n, hipStream_t st)
{
    using namespace hlb::nn;
    for (int l = 0; l < NL; ++l) {
        const bool last = l == NL - 1;
        N_TRY(n, conv(n->g, CIP[l], COP[l], last ? MODE_LINEAR : MODE_RELU, n->A[l], n->Wf[l], bias_of(n, l),
                      last ? static_cast<void *>(n->Y) : static_cast<void *>(n->A[l + 1]), nullptr, CO[l], st));
    }
    return HLB_OK;
}

// Backward from dZ of the last layer (in dZ[0], 16 channels); gradients into
// n->grads.  With dz_host, each layer's output gradient dZ_l is copied to
// dz_host + l N 32 (N x COP[l] values) before it is used.
int backward(hlbnn *n, unsigned short *dz_host = nullptr)
{
    using namespace hlb::nn;
    int cur = 0;
    for (int l = NL - 1; l >= 0; --l) {
        if (dz_host)
            N_TRY(n, hipMemcpyAsync(dz_host + size_t(l) * n->g.N * 32, n->dZ[cur], size_t(n->g.N) * COP[l] * 2,
                                    hipMemcpyDeviceToHost, n->stream));
        N_TRY(n, wgrad(n->g, CIP[l], COP[l], n->A[l], n->dZ[cur], n->part, CI[l], CO[l], n->grads + layer_offset(l),
                       n->stream));
        if (l > 0) {
            // dZ of layer l-1 = (W^T * dZ_l) masked by the ReLU of layer l-1's output (= A[l])
            N_TRY(n, conv(n->g, COP[l], CIP[l], MODE_MASK, n->dZ[cur], n->Wt[l], nullptr, n->dZ[cur ^ 1], n->A[l],
                          CIP[l], n->stream));
            cur ^= 1;
        }
    }
    return HLB_OK;
}

int check_solver(hlbnn *n, const hlb_ctx *c)
{
    if (!c) return nerr(n, HLB_ERR_ARG, "solver context is null");
    if (c->status) return nerr(n, c->status, "solver context in error: %s", c->msg);
    if (c->D.G.nx != n->g.nx || c->D.G.ny != n->g.ny || c->D.G.nz != n->g.nz)
        return nerr(n, HLB_ERR_ARG, "solver and network lattices differ");
    if (!c->have_fields) return nerr(n, HLB_ERR_STATE, "solver has no fields");
    return HLB_OK;
}

bool history_valid(const hlbnn *n, const hlb_ctx *c, int k)
{
    return n->hist_ctx == c && n->hist_version == c->version && n->hist_k == k;
}

// After steps_before plain steps, 2k more recording Q every k steps; the
// history from the three snapshots (the oldest two in the checkpoint area).
int record_history(hlbnn *n, hlb_ctx *c, int k, int steps_before)
{
    hlb::Device &D = c->D;
    const size_t N = D.G.N, e = D.fp32 ? 4 : 8;
    char *A = n->ckpt, *B = n->ckpt + a256(5 * N * e);
    if (steps_before > 0) N_TRY(n, hlb::run_steps(D, c->p, steps_before));
    N_TRY(n, hipMemcpyAsync(A, D.Q[D.qcur], 5 * N * e, hipMemcpyDeviceToDevice, D.stream));
    N_TRY(n, hlb::run_steps(D, c->p, k));
    N_TRY(n, hipMemcpyAsync(B, D.Q[D.qcur], 5 * N * e, hipMemcpyDeviceToDevice, D.stream));
    N_TRY(n, hlb::run_steps(D, c->p, k));
    N_TRY(n, hlb::nn::hist3(D.fp32, int(N), D.Q[D.qcur], B, A, n->d1, n->s2, D.stream));
    n->hist_ctx = c;
    n->hist_version = c->version;
    n->hist_k = k;
    return HLB_OK;
}

// Network prediction of the next increment from the solver state and the
// history: applied to Q with the history advanced (dq_out == nullptr), or
// written to dq_out.
int network_jump(hlbnn *n, hlb_ctx *c, float *dq_out)
{
    hlb::Device &D = c->D;
    const int N = int(D.G.N);
    N_TRY(n, hlb::nn::pack_state(D.fp32, N, D.Q[D.qcur], D.u, n->d1, n->s2, n->norm, n->A[0], D.stream));
    int rc = forward(n, D.stream);
    if (rc) return rc;
    N_TRY(n, hlb::nn::jump(D.fp32, N, n->Y, n->norm, n->d1, n->s2, D.Q[D.qcur], dq_out, D.stream));
    return HLB_OK;
}

}  // namespace

extern "C" {

int hlbnn_param_count(void) { return param_total(); }
int hlbnn_input_channels(void) { return NIN; }
int hlbnn_norm_size(void) { return NORM_SIZE; }

size_t hlbnn_workspace_bytes(int nx, int ny, int nz)
{
    if (nx < 4 || ny < 4 || nz < 4 || double(nx) * ny * nz >= 2147483647.0 / 32) return 0;
    return sizes_for(hlb::nn::make_grid(nx, ny, nz)).total;
}

int hlbnn_create(int nx, int ny, int nz, void *ws, size_t ws_bytes, void *stream, hlbnn **out)
{
    if (!out) return HLB_ERR_ARG;
    *out = nullptr;
    const size_t need = hlbnn_workspace_bytes(nx, ny, nz);
    if (need == 0 || !ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return HLB_ERR_ARG;
    if (ws_bytes < need) return HLB_ERR_NOMEM;
    hlbnn *n = new (std::nothrow) hlbnn();
    if (!n) return HLB_ERR_NOMEM;
    n->g = hlb::nn::make_grid(nx, ny, nz);
    n->stream = static_cast<hipStream_t>(stream);
    const Sizes z = sizes_for(n->g);
    char *p = static_cast<char *>(ws);
    n->params = reinterpret_cast<float *>(p); p += z.params;
    n->grads = reinterpret_cast<float *>(p); p += z.params;
    n->m = reinterpret_cast<float *>(p); p += z.params;
    n->v = reinterpret_cast<float *>(p); p += z.params;
    for (int l = 0; l < NL; ++l) {
        n->Wf[l] = reinterpret_cast<unsigned short *>(p); p += a256(hlb::nn::frag_bytes(CIP[l], COP[l]));
        n->Wt[l] = reinterpret_cast<unsigned short *>(p); p += a256(hlb::nn::frag_bytes(COP[l], CIP[l]));
    }
    for (int l = 0; l < NL; ++l) {
        n->A[l] = reinterpret_cast<unsigned short *>(p);
        p += z.act;
    }
    n->Y = reinterpret_cast<float *>(p); p += z.y;
    n->dZ[0] = reinterpret_cast<unsigned short *>(p); p += z.dz;
    n->dZ[1] = reinterpret_cast<unsigned short *>(p); p += z.dz;
    n->part = reinterpret_cast<float *>(p); p += z.part;
    n->red = reinterpret_cast<double *>(p); p += z.red;
    n->dq = reinterpret_cast<float *>(p); p += z.f5;
    n->d1 = reinterpret_cast<float *>(p); p += z.f5;
    n->s2 = reinterpret_cast<float *>(p); p += z.f5;
    n->ckpt = p; p += z.ckpt;
    n->qsnap = p; p += z.qsnap;
    n->norm = reinterpret_cast<float *>(p);
    *out = n;
    return HLB_OK;
}

int hlbnn_set_params(hlbnn *n, const float *host)
{
    N_GUARD(n);
    if (!host) return nerr(n, HLB_ERR_ARG, "params is null");
    const size_t bytes = size_t(param_total()) * 4;
    N_TRY(n, hipMemcpyAsync(n->params, host, bytes, hipMemcpyHostToDevice, n->stream));
    N_TRY(n, hipMemsetAsync(n->m, 0, bytes, n->stream));
    N_TRY(n, hipMemsetAsync(n->v, 0, bytes, n->stream));
    n->adam_t = 0;
    int rc = prep_weights(n);
    if (rc) return rc;
    N_TRY(n, hipStreamSynchronize(n->stream));
    n->have_params = true;
    return HLB_OK;
}

int hlbnn_get_params(hlbnn *n, float *host)
{
    N_GUARD(n);
    if (!host || !n->have_params) return nerr(n, HLB_ERR_STATE, "no parameters");
    N_TRY(n, hipMemcpyAsync(host, n->params, size_t(param_total()) * 4, hipMemcpyDeviceToHost, n->stream));
    N_TRY(n, hipStreamSynchronize(n->stream));
    return HLB_OK;
}

int hlbnn_get_grads(hlbnn *n, float *host)
{
    N_GUARD(n);
    if (!host) return nerr(n, HLB_ERR_ARG, "null");
    N_TRY(n, hipMemcpyAsync(host, n->grads, size_t(param_total()) * 4, hipMemcpyDeviceToHost, n->stream));
    N_TRY(n, hipStreamSynchronize(n->stream));
    return HLB_OK;
}

int hlbnn_set_norm(hlbnn *n, const float *norm)
{
    using namespace hlb::nn;
    N_GUARD(n);
    if (!norm) return nerr(n, HLB_ERR_ARG, "norm is null");
    for (int k = 0; k < NORM_SIZE; ++k)
        if (!std::isfinite(norm[k])) return nerr(n, HLB_ERR_PARAM, "norm[%d] not finite", k);
    for (int k = 0; k < NIN; ++k)
        if (!(norm[NORM_IN_STD + k] > 0.f)) return nerr(n, HLB_ERR_PARAM, "input std %d must be positive", k);
    for (int k = 0; k < 5; ++k)
        if (!(norm[NORM_OUT_STD + k] > 0.f)) return nerr(n, HLB_ERR_PARAM, "output std %d must be positive", k);
    N_TRY(n, hipMemcpyAsync(n->norm, norm, NORM_SIZE * 4, hipMemcpyHostToDevice, n->stream));
    N_TRY(n, hipStreamSynchronize(n->stream));
    n->have_norm = true;
    return HLB_OK;
}

int hlbnn_get_norm(hlbnn *n, float *norm)
{
    N_GUARD(n);
    if (!norm || !n->have_norm) return nerr(n, HLB_ERR_STATE, "no normalisation");
    N_TRY(n, hipMemcpyAsync(norm, n->norm, NORM_SIZE * 4, hipMemcpyDeviceToHost, n->stream));
    N_TRY(n, hipStreamSynchronize(n->stream));
    return HLB_OK;
}

int hlbnn_channel_stats(hlbnn *n, const float *data_dev, int nch, int nsamples, double *mean, double *std_out)
{
    N_GUARD(n);
    if (!data_dev || nch < 1 || nch > 64 || nsamples < 1 || !mean || !std_out)
        return nerr(n, HLB_ERR_ARG, "hlbnn_channel_stats arguments");
    const int nblk = 64;
    std::vector<double> h(size_t(2) * nch * nblk);
    N_TRY(n, hlb::nn::stats(data_dev, nch, n->g.N, nsamples, n->red, nblk, n->stream));
    N_TRY(n, hipMemcpyAsync(h.data(), n->red, h.size() * 8, hipMemcpyDeviceToHost, n->stream));
    N_TRY(n, hipStreamSynchronize(n->stream));
    const double cnt = double(n->g.N) * nsamples;
    for (int c = 0; c < nch; ++c) {
        double s1 = 0.0, s2 = 0.0;
        for (int b = 0; b < nblk; ++b) {
            s1 += h[2 * (c * nblk + b)];
            s2 += h[2 * (c * nblk + b) + 1];
        }
        mean[c] = s1 / cnt;
        std_out[c] = std::sqrt(std::fmax(s2 / cnt - mean[c] * mean[c], 0.0));
    }
    return HLB_OK;
}

int hlbnn_fit_norm(hlbnn *n, const float *x_dev, const float *dq_dev, int nsamples, float beta, float *norm_out)
{
    using namespace hlb::nn;
    N_GUARD(n);
    if (!x_dev || !dq_dev || nsamples < 1 || !std::isfinite(beta))
        return nerr(n, HLB_ERR_ARG, "hlbnn_fit_norm arguments");
    double mean[NIN], sd[NIN];
    int rc = hlbnn_channel_stats(n, x_dev, NIN, nsamples, mean, sd);
    if (rc) return rc;
    const int nblk = 64;
    std::vector<double> h(size_t(2) * 5 * nblk);
    N_TRY(n, stats_target(x_dev, dq_dev, n->g.N, nsamples, beta, n->red, nblk, n->stream));
    N_TRY(n, hipMemcpyAsync(h.data(), n->red, h.size() * 8, hipMemcpyDeviceToHost, n->stream));
    N_TRY(n, hipStreamSynchronize(n->stream));
    float norm[NORM_SIZE];
    for (int c = 0; c < NIN; ++c) {
        norm[NORM_IN_MEAN + c] = float(mean[c]);
        norm[NORM_IN_STD + c] = sd[c] > 0.0 ? float(sd[c]) : 1.f;
    }
    const double cnt = double(n->g.N) * nsamples;
    for (int c = 0; c < 5; ++c) {
        double s1 = 0.0, s2 = 0.0;
        for (int b = 0; b < nblk; ++b) {
            s1 += h[2 * (c * nblk + b)];
            s2 += h[2 * (c * nblk + b) + 1];
        }
        const double m = s1 / cnt, v = std::sqrt(std::fmax(s2 / cnt - m * m, 0.0));
        norm[NORM_OUT_MEAN + c] = float(m);
        norm[NORM_OUT_STD + c] = v > 0.0 ? float(v) : 1.f;
    }
    norm[NORM_BETA] = beta;
    if (norm_out) std::memcpy(norm_out, norm, sizeof(norm));
    return hlbnn_set_norm(n, norm);
}

int hlbnn_predict(hlbnn *n, const float *x_dev, float *dq_dev)
{
    N_GUARD(n);
    if (!n->have_params || !n->have_norm) return nerr(n, HLB_ERR_STATE, "parameters and normalisation first");
    if (!x_dev || !dq_dev) return nerr(n, HLB_ERR_ARG, "null device pointer");
    N_TRY(n, hlb::nn::pack(n->g.N, x_dev, n->norm, n->A[0], n->stream));
    int rc = forward(n, n->stream);
    if (rc) return rc;
    N_TRY(n, hlb::nn::predict_out(n->g.N, n->Y, n->norm, x_dev, dq_dev, n->stream));
    return HLB_OK;
}

int hlbnn_train_step(hlbnn *n, const float *x_dev, const float *dq_dev, float lr, double *loss)
{
    N_GUARD(n);
    if (!n->have_params || !n->have_norm) return nerr(n, HLB_ERR_STATE, "parameters and normalisation first");
    if (!x_dev || !dq_dev || !(lr >= 0.f)) return nerr(n, HLB_ERR_ARG, "hlbnn_train_step arguments");
    N_TRY(n, hlb::nn::pack(n->g.N, x_dev, n->norm, n->A[0], n->stream));
    int rc = forward(n, n->stream);
    if (rc) return rc;
    N_TRY(n, hlb::nn::lossgrad(n->g.N, n->Y, dq_dev, x_dev, n->norm, n->dZ[0], n->red, n->red + 4096, n->stream));
    if ((rc = backward(n))) return rc;
    n->adam_t += 1;
    N_TRY(n, hlb::nn::adam(param_total(), n->params, n->grads, n->m, n->v, lr, 0.9f, 0.999f, 1e-8f, n->adam_t,
                           n->stream));
    if ((rc = prep_weights(n))) return rc;
    if (loss) {
        double s = 0.0;
        N_TRY(n, hipMemcpyAsync(&s, n->red + 4096, 8, hipMemcpyDeviceToHost, n->stream));
        N_TRY(n, hipStreamSynchronize(n->stream));
        *loss = s / (5.0 * n->g.N);
        if (!std::isfinite(*loss)) return nerr(n, HLB_ERR_NONFINITE, "non-finite training loss");
    }
    return HLB_OK;
}

int hlbnn_grad_trace(hlbnn *n, const float *x_dev, const float *dq_dev, unsigned short *acts_host, float *y_host,
                     unsigned short *dz_host, float *grad_host)
{
    N_GUARD(n);
    if (!n->have_params || !n->have_norm) return nerr(n, HLB_ERR_STATE, "parameters and normalisation first");
    if (!x_dev || !dq_dev || !acts_host || !y_host || !dz_host || !grad_host)
        return nerr(n, HLB_ERR_ARG, "hlbnn_grad_trace arguments");
    const size_t N = n->g.N;
    N_TRY(n, hlb::nn::pack(n->g.N, x_dev, n->norm, n->A[0], n->stream));
    int rc = forward(n, n->stream);
    if (rc) return rc;
    N_TRY(n, hlb::nn::lossgrad(n->g.N, n->Y, dq_dev, x_dev, n->norm, n->dZ[0], n->red, n->red + 4096, n->stream));
    for (int l = 0; l < NL; ++l)
        N_TRY(n, hipMemcpyAsync(acts_host + size_t(l) * N * 32, n->A[l], N * 32 * 2, hipMemcpyDeviceToHost,
                                n->stream));
    N_TRY(n, hipMemcpyAsync(y_host, n->Y, N * 5 * 4, hipMemcpyDeviceToHost, n->stream));
    if ((rc = backward(n, dz_host))) return rc;
    N_TRY(n, hipMemcpyAsync(grad_host, n->grads, size_t(param_total()) * 4, hipMemcpyDeviceToHost, n->stream));
    N_TRY(n, hipStreamSynchronize(n->stream));
    return HLB_OK;
}

// Per-layer entry points for the parity tests: host bf16 activations in,
// host FP32 results out.
int hlbnn_layer_forward(hlbnn *n, int l, const unsigned short *x_host, float *z_host)
{
    N_GUARD(n);
    if (l < 0 || l >= NL || !x_host || !z_host) return nerr(n, HLB_ERR_ARG, "layer %d", l);
    if (!n->have_params) return nerr(n, HLB_ERR_STATE, "parameters first");
    const size_t N = n->g.N;
    N_TRY(n, hipMemcpyAsync(n->A[l], x_host, N * CIP[l] * 2, hipMemcpyHostToDevice, n->stream));
    // pre-activation with bias, FP32 [N][CO], into the checkpoint area (N*24*8 >= N*32*4 bytes)
    float *zdev = reinterpret_cast<float *>(n->ckpt);
    N_TRY(n, hlb::nn::conv(n->g, CIP[l], COP[l], hlb::nn::MODE_LINEAR, n->A[l], n->Wf[l], bias_of(n, l), zdev,
                           nullptr, CO[l], n->stream));
    N_TRY(n, hipMemcpyAsync(z_host, zdev, N * CO[l] * 4, hipMemcpyDeviceToHost, n->stream));
    N_TRY(n, hipStreamSynchronize(n->stream));
    return HLB_OK;
}

int hlbnn_layer_backward(hlbnn *n, int l, const unsigned short *x_host, const unsigned short *dz_host, float *dx_host,
                         float *grad_host)
{
    N_GUARD(n);
    if (l < 0 || l >= NL || !x_host || !dz_host || !grad_host) return nerr(n, HLB_ERR_ARG, "layer %d", l);
    if (!n->have_params) return nerr(n, HLB_ERR_STATE, "parameters first");
    const size_t N = n->g.N;
    N_TRY(n, hipMemcpyAsync(n->A[l], x_host, N * CIP[l] * 2, hipMemcpyHostToDevice, n->stream));
    N_TRY(n, hipMemcpyAsync(n->dZ[0], dz_host, N * COP[l] * 2, hipMemcpyHostToDevice, n->stream));
    N_TRY(n, hlb::nn::wgrad(n->g, CIP[l], COP[l], n->A[l], n->dZ[0], n->part, CI[l], CO[l],
                            n->grads + layer_offset(l), n->stream));
    N_TRY(n, hipMemcpyAsync(grad_host, n->grads + layer_offset(l), size_t(layer_params(l)) * 4,
                            hipMemcpyDeviceToHost, n->stream));
    if (dx_host) {
        float *dxd = reinterpret_cast<float *>(n->ckpt);  // N*24*8 bytes >= N*32*4
        N_TRY(n, hlb::nn::conv(n->g, COP[l], CIP[l], hlb::nn::MODE_RAW, n->dZ[0], n->Wt[l], nullptr, dxd, nullptr,
                               CIP[l], n->stream));
        N_TRY(n, hipMemcpyAsync(dx_host, dxd, N * CIP[l] * 4, hipMemcpyDeviceToHost, n->stream));
    }
    N_TRY(n, hipStreamSynchronize(n->stream));
    return HLB_OK;
}

int hlbnn_warmup(hlbnn *n, hlb_ctx *c, int k)
{
    N_GUARD(n);
    if (k < 1) return nerr(n, HLB_ERR_ARG, "k = %d", k);
    int rc = check_solver(n, c);
    if (rc) return rc;
    return record_history(n, c, k, 0);
}

int hlbnn_history(hlbnn *n, const hlb_ctx *c, float *d1_host, float *s2_host)
{
    N_GUARD(n);
    if (!d1_host || !s2_host) return nerr(n, HLB_ERR_ARG, "null argument");
    if (!c || !history_valid(n, c, n->hist_k)) return nerr(n, HLB_ERR_STATE, "no history for this solver state");
    const size_t N = n->g.N;
    N_TRY(n, hipMemcpyAsync(d1_host, n->d1, 5 * N * 4, hipMemcpyDeviceToHost, c->D.stream));
    N_TRY(n, hipMemcpyAsync(s2_host, n->s2, 5 * N * 4, hipMemcpyDeviceToHost, c->D.stream));
    N_TRY(n, hipStreamSynchronize(c->D.stream));
    return HLB_OK;
}

int hlbnn_inputs(hlbnn *n, const hlb_ctx *c, float *x_host)
{
    N_GUARD(n);
    if (!x_host) return nerr(n, HLB_ERR_ARG, "null argument");
    int rc = check_solver(n, c);
    if (rc) return rc;
    if (!history_valid(n, c, n->hist_k)) return nerr(n, HLB_ERR_STATE, "no history for this solver state");
    const hlb::Device &D = c->D;
    const size_t N = D.G.N;
    float *x = reinterpret_cast<float *>(n->ckpt);  // N*24*8 bytes >= NIN*N*4
    N_TRY(n, hlb::nn::inputs(D.fp32, int(N), D.Q[D.qcur], D.u, n->d1, n->s2, x, D.stream));
    N_TRY(n, hipMemcpyAsync(x_host, x, size_t(NIN) * N * 4, hipMemcpyDeviceToHost, D.stream));
    N_TRY(n, hipStreamSynchronize(D.stream));
    return HLB_OK;
}

int hlbnn_make_pair(hlbnn *n, hlb_ctx *c, int k, float *x_dev, float *dq_dev)
{
    N_GUARD(n);
    if (!x_dev || !dq_dev || k < 1) return nerr(n, HLB_ERR_ARG, "hlbnn_make_pair arguments");
    int rc = check_solver(n, c);
    if (rc) return rc;
    hlb::Device &D = c->D;
    const size_t N = D.G.N, e = D.fp32 ? 4 : 8;
    if (!history_valid(n, c, k) && (rc = record_history(n, c, k, 0))) return rc;
    N_TRY(n, hlb::nn::inputs(D.fp32, int(N), D.Q[D.qcur], D.u, n->d1, n->s2, x_dev, D.stream));
    N_TRY(n, hipMemcpyAsync(n->qsnap, D.Q[D.qcur], 5 * N * e, hipMemcpyDeviceToDevice, D.stream));
    N_TRY(n, hlb::run_steps(D, c->p, k));
    N_TRY(n, hlb::nn::hist_step(D.fp32, int(N), D.Q[D.qcur], n->qsnap, n->d1, n->s2, D.stream));
    N_TRY(n, hipMemcpyAsync(dq_dev, n->d1, 5 * N * 4, hipMemcpyDeviceToDevice, D.stream));
    return HLB_OK;
}

int hlbnn_jump(hlbnn *n, hlb_ctx *c)
{
    N_GUARD(n);
    int rc = check_solver(n, c);
    if (rc) return rc;
    if (!n->have_params || !n->have_norm) return nerr(n, HLB_ERR_STATE, "parameters and normalisation first");
    if (!history_valid(n, c, n->hist_k)) return nerr(n, HLB_ERR_STATE, "no history for this solver state");
    return network_jump(n, c, nullptr);
}

const char *hlbnn_last_error(const hlbnn *n) { return n ? n->msg : "null network"; }

void hlbnn_destroy(hlbnn *n) { delete n; }

// One surrogate cycle of M jumps of k steps (see include/hlb.h).
int hlb_surrogate_advance(hlb_ctx *c, hlbnn *n, int k, int M, double threshold, int *fell_back, double *residual)
{
    N_GUARD(n);
    if (k < 1 || M < 2 || !(threshold >= 0.0)) return nerr(n, HLB_ERR_ARG, "hlb_surrogate_advance arguments");
    int rc = check_solver(n, c);
    if (rc) return rc;
    if (!n->have_params || !n->have_norm) return nerr(n, HLB_ERR_STATE, "parameters and normalisation first");
    if (!history_valid(n, c, k)) return nerr(n, HLB_ERR_STATE, "no history for this solver state and k (warm up)");
    hlb::Device &D = c->D;
    const size_t N = D.G.N, e = D.fp32 ? 4 : 8;
    const hipStream_t st = D.stream;
    // checkpoint of the cycle start (populations and Q)
    const int g0 = D.gcur, q0 = D.qcur;
    N_TRY(n, hipMemcpyAsync(n->ckpt, D.g[D.gcur], 19 * N * e, hipMemcpyDeviceToDevice, st));
    N_TRY(n, hipMemcpyAsync(n->ckpt + 19 * N * e, D.Q[D.qcur], 5 * N * e, hipMemcpyDeviceToDevice, st));
    // M-1 unchecked jumps; the populations and u are held
    for (int j = 0; j < M - 1; ++j)
        if ((rc = network_jump(n, c, nullptr))) return rc;
    // checked jump: the network's increment and, from the same state, k plain steps
    if ((rc = network_jump(n, c, n->dq))) return rc;
    N_TRY(n, hipMemcpyAsync(n->qsnap, D.Q[D.qcur], 5 * N * e, hipMemcpyDeviceToDevice, st));
    N_TRY(n, hlb::run_steps(D, c->p, k));
    // residual || (Q_pre + dq) - Q_plain || / || Q_plain || over the five stored components
    const int nblk = 256;
    double h[2 * nblk];
    N_TRY(n, hlb::nn::resid(D.fp32, int(N), n->qsnap, n->dq, D.Q[D.qcur], n->red, nblk, st));
    N_TRY(n, hlb::nn::hist_step(D.fp32, int(N), D.Q[D.qcur], n->qsnap, n->d1, n->s2, st));
    N_TRY(n, hipMemcpyAsync(h, n->red, sizeof(h), hipMemcpyDeviceToHost, st));
    N_TRY(n, hipStreamSynchronize(st));
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
        s1 += h[2 * b];
        s2 += h[2 * b + 1];
    }
    const double r = s2 > 0.0 ? std::sqrt(s1 / s2) : std::sqrt(s1);
    if (residual) *residual = r;
    const bool bad = !(r < threshold);  // threshold 0 always falls back
    if (fell_back) *fell_back = bad ? 1 : 0;
    if (bad) {
        // roll back to the cycle start and take the whole cycle with plain
        // steps, recording the history over its last two jumps
        D.gcur = g0;
        D.qcur = q0;
        N_TRY(n, hipMemcpyAsync(D.g[D.gcur], n->ckpt, 19 * N * e, hipMemcpyDeviceToDevice, st));
        N_TRY(n, hipMemcpyAsync(D.Q[D.qcur], n->ckpt + 19 * N * e, 5 * N * e, hipMemcpyDeviceToDevice, st));
        if ((rc = record_history(n, c, k, (M - 2) * k))) return rc;
    }
    return HLB_OK;
}

}  // extern "C"
