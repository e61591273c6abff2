// nn_api.cpp -- C-ABI of the convolutional surrogate (include/hlb.h,
// hlbnn_* and hlb_surrogate_advance): buffers, forward, training step with
// Adam, per-layer entry points for the parity tests, and the surrogate-with-
// fallback driver.  All arithmetic runs in the kernels of nn.hip/kernels.hip.
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

constexpr int NL = 4;
constexpr int CI[NL] = {8, 32, 32, 32};
constexpr int CO[NL] = {32, 32, 32, 5};
constexpr int CIP[NL] = {16, 32, 32, 32};
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
    size_t params, wbf, act0, act, y, dz, part, red, xraw, dq, ckpt, total;
};

Sizes sizes_for(const hlb::nn::Grid3 &g)
{
    Sizes z;
    const size_t N = g.N;
    z.params = a256(size_t(param_total()) * 4);
    size_t wb = 0;
    for (int l = 0; l < NL; ++l) wb += 2 * a256(size_t(27) * CIP[l] * COP[l] * 2);
    z.wbf = wb;
    z.act0 = a256(N * 16 * 2);
    z.act = a256(N * 32 * 2);
    z.y = a256(N * 5 * 4);
    z.dz = a256(N * 32 * 2);
    z.part = a256(size_t(hlb::nn::wgrad_grid(g)) * (27 * 32 * 32 + 32) * 4);
    z.red = a256((size_t((N + 255) / 256) + 64 * 2 * 16 + 4096) * 8);
    z.xraw = a256(N * 8 * 4);
    z.dq = a256(N * 5 * 4);
    z.ckpt = a256(N * 24 * 8) + a256(N * 5 * 8);  // full state + one Q snapshot, FP64 worst case
    z.total = 4 * z.params /* params, grads, m, v */ + z.wbf + z.act0 + 3 * z.act + z.y + 2 * z.dz + z.part + z.red +
              z.xraw + z.dq + z.ckpt + 256 /* norm */;
    return z;
}

}  // namespace

struct hlbnn {
    hlb::nn::Grid3 g;
    hipStream_t stream;
    float *params, *grads, *m, *v;
    unsigned short *Wf[NL], *Wt[NL];
    unsigned short *A[NL];  // inputs of the layers: A[0] [N][16], A[1..3] [N][32]
    float *Y;               // [N][5]
    unsigned short *dZ[2];  // [N][32]
    float *part;
    double *red;
    float *xraw, *dq;
    char *ckpt, *qsnap;
    float *norm;  // in_mean 8, in_std 8, out_mean 5, out_std 5
    bool have_params, have_norm;
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

// Backward from dZ of the last layer (in dZ[0], 16 channels); gradients into n->grads.
int backward(hlbnn *n)
{
    using namespace hlb::nn;
    int cur = 0;
    for (int l = NL - 1; l >= 0; --l) {
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

}  // namespace

extern "C" {

int hlbnn_param_count(void) { return param_total(); }

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
        const size_t wb = a256(size_t(27) * CIP[l] * COP[l] * 2);
        n->Wf[l] = reinterpret_cast<unsigned short *>(p); p += wb;
        n->Wt[l] = reinterpret_cast<unsigned short *>(p); p += wb;
    }
    n->A[0] = reinterpret_cast<unsigned short *>(p); p += z.act0;
    for (int l = 1; l < NL; ++l) {
        n->A[l] = reinterpret_cast<unsigned short *>(p);
        p += z.act;
    }
    n->Y = reinterpret_cast<float *>(p); p += z.y;
    n->dZ[0] = reinterpret_cast<unsigned short *>(p); p += z.dz;
    n->dZ[1] = reinterpret_cast<unsigned short *>(p); p += z.dz;
    n->part = reinterpret_cast<float *>(p); p += z.part;
    n->red = reinterpret_cast<double *>(p); p += z.red;
    n->xraw = reinterpret_cast<float *>(p); p += z.xraw;
    n->dq = reinterpret_cast<float *>(p); p += z.dq;
    n->ckpt = p; p += a256(size_t(n->g.N) * 24 * 8);
    n->qsnap = p; p += a256(size_t(n->g.N) * 5 * 8);
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

int hlbnn_set_norm(hlbnn *n, const float *norm26)
{
    N_GUARD(n);
    if (!norm26) return nerr(n, HLB_ERR_ARG, "norm is null");
    for (int k = 0; k < 8; ++k)
        if (!(norm26[8 + k] > 0.f)) return nerr(n, HLB_ERR_PARAM, "input std %d must be positive", k);
    for (int k = 0; k < 5; ++k)
        if (!(norm26[21 + k] > 0.f)) return nerr(n, HLB_ERR_PARAM, "output std %d must be positive", k);
    N_TRY(n, hipMemcpyAsync(n->norm, norm26, 26 * 4, hipMemcpyHostToDevice, n->stream));
    N_TRY(n, hipStreamSynchronize(n->stream));
    n->have_norm = true;
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

int hlbnn_predict(hlbnn *n, const float *x_dev, float *dq_dev)
{
    N_GUARD(n);
    if (!n->have_params || !n->have_norm) return nerr(n, HLB_ERR_STATE, "parameters and normalisation first");
    if (!x_dev || !dq_dev) return nerr(n, HLB_ERR_ARG, "null device pointer");
    N_TRY(n, hlb::nn::pack(n->g.N, x_dev, n->norm, n->A[0], n->stream));
    int rc = forward(n, n->stream);
    if (rc) return rc;
    N_TRY(n, hlb::nn::apply(true, n->g.N, n->Y, n->norm, dq_dev, nullptr, n->stream));
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
    N_TRY(n, hlb::nn::lossgrad(n->g.N, n->Y, dq_dev, n->norm, n->dZ[0], n->red, n->red + 4096, n->stream));
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

int hlbnn_sample(hlbnn *n, hlb_ctx *c, float *x_dev)
{
    N_GUARD(n);
    if (!c || !x_dev) return nerr(n, HLB_ERR_ARG, "null argument");
    if (c->D.G.nx != n->g.nx || c->D.G.ny != n->g.ny || c->D.G.nz != n->g.nz)
        return nerr(n, HLB_ERR_ARG, "solver and network lattices differ");
    if (!c->have_fields) return nerr(n, HLB_ERR_STATE, "solver has no fields");
    N_TRY(n, hlb::nn::sample(c->D.fp32, n->g.N, c->D.Q[c->D.qcur], c->D.u, x_dev, c->D.stream));
    return HLB_OK;
}

int hlbnn_make_pair(hlbnn *n, hlb_ctx *c, int k, float *x_dev, float *dq_dev)
{
    N_GUARD(n);
    if (!c || !x_dev || !dq_dev || k < 1) return nerr(n, HLB_ERR_ARG, "hlbnn_make_pair arguments");
    if (c->status) return nerr(n, c->status, "solver context in error: %s", c->msg);
    if (c->D.G.nx != n->g.nx || c->D.G.ny != n->g.ny || c->D.G.nz != n->g.nz)
        return nerr(n, HLB_ERR_ARG, "solver and network lattices differ");
    if (!c->have_fields) return nerr(n, HLB_ERR_STATE, "solver has no fields");
    hlb::Device &D = c->D;
    N_TRY(n, hlb::nn::sample(D.fp32, n->g.N, D.Q[D.qcur], D.u, x_dev, D.stream));
    N_TRY(n, hlb::run_steps(D, c->p, k));
    N_TRY(n, hlb::nn::sample(D.fp32, n->g.N, D.Q[D.qcur], D.u, n->xraw, D.stream));
    N_TRY(n, hlb::nn::diff(n->g.N, x_dev, n->xraw, dq_dev, D.stream));
    return HLB_OK;
}

const char *hlbnn_last_error(const hlbnn *n) { return n ? n->msg : "null network"; }

void hlbnn_destroy(hlbnn *n) { delete n; }

// One surrogate cycle of M jumps of k steps (see include/hlb.h).
int hlb_surrogate_advance(hlb_ctx *c, hlbnn *n, int k, int M, double threshold, int *fell_back, double *residual)
{
    N_GUARD(n);
    if (!c || k < 1 || M < 1 || !(threshold >= 0.0)) return nerr(n, HLB_ERR_ARG, "hlb_surrogate_advance arguments");
    if (c->status) return nerr(n, c->status, "solver context in error: %s", c->msg);
    if (c->D.G.nx != n->g.nx || c->D.G.ny != n->g.ny || c->D.G.nz != n->g.nz)
        return nerr(n, HLB_ERR_ARG, "solver and network lattices differ");
    if (!c->have_fields || !n->have_params || !n->have_norm) return nerr(n, HLB_ERR_STATE, "not initialised");
    hlb::Device &D = c->D;
    const size_t N = D.G.N, e = D.fp32 ? 4 : 8;
    const hipStream_t st = D.stream;
    // checkpoint of the cycle start (populations and Q)
    const int g0 = D.gcur, q0 = D.qcur;
    N_TRY(n, hipMemcpyAsync(n->ckpt, D.g[D.gcur], 19 * N * e, hipMemcpyDeviceToDevice, st));
    N_TRY(n, hipMemcpyAsync(n->ckpt + 19 * N * e, D.Q[D.qcur], 5 * N * e, hipMemcpyDeviceToDevice, st));
    // M-1 unchecked jumps: Q += network(Q, u); populations and u held
    for (int j = 0; j < M - 1; ++j) {
        N_TRY(n, hlb::nn::sample(D.fp32, int(N), D.Q[D.qcur], D.u, n->xraw, st));
        N_TRY(n, hlb::nn::pack(int(N), n->xraw, n->norm, n->A[0], st));
        int rc = forward(n, st);
        if (rc) return rc;
        N_TRY(n, hlb::nn::apply(D.fp32, int(N), n->Y, n->norm, nullptr, D.Q[D.qcur], st));
    }
    // checked jump: network prediction from the pre-jump state, then k plain steps
    N_TRY(n, hlb::nn::sample(D.fp32, int(N), D.Q[D.qcur], D.u, n->xraw, st));
    N_TRY(n, hipMemcpyAsync(n->qsnap, D.Q[D.qcur], 5 * N * e, hipMemcpyDeviceToDevice, st));
    N_TRY(n, hlb::nn::pack(int(N), n->xraw, n->norm, n->A[0], st));
    int rc = forward(n, st);
    if (rc) return rc;
    N_TRY(n, hlb::nn::apply(true, int(N), n->Y, n->norm, n->dq, nullptr, st));
    N_TRY(n, hlb::run_steps(D, c->p, k));
    // residual || (Q_pre + dq) - Q_plain || / || Q_plain || over the five stored components
    const int nblk = 256;
    double h[2 * nblk];
    N_TRY(n, hlb::nn::resid(D.fp32, int(N), n->qsnap, n->dq, D.Q[D.qcur], n->red, nblk, st));
    N_TRY(n, hipMemcpyAsync(h, n->red, sizeof(h), hipMemcpyDeviceToHost, st));
    N_TRY(n, hipStreamSynchronize(st));
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
        s1 += h[2 * b];
        s2 += h[2 * b + 1];
    }
    const double r = s2 > 0.0 ? std::sqrt(s1 / s2) : std::sqrt(s1);
    if (residual) *residual = r;
    const bool bad = !(r <= threshold);
    if (fell_back) *fell_back = bad ? 1 : 0;
    if (bad) {
        // roll back to the cycle start and take the whole cycle with plain steps
        D.gcur = g0;
        D.qcur = q0;
        N_TRY(n, hipMemcpyAsync(D.g[D.gcur], n->ckpt, 19 * N * e, hipMemcpyDeviceToDevice, st));
        N_TRY(n, hipMemcpyAsync(D.Q[D.qcur], n->ckpt + 19 * N * e, 5 * N * e, hipMemcpyDeviceToDevice, st));
        N_TRY(n, hlb::run_steps(D, c->p, M * k));
    }
    return HLB_OK;
}

}  // extern "C"
