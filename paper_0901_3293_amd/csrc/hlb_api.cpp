// hlb_api.cpp -- the C-ABI of include/hlb.h: validation, workspace layout,
// sticky error handling and the host side of every entry point.  All
// arithmetic on the state runs in the kernels of kernels.hip.
#include <algorithm>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/hlb.h"
#include "ctx.h"
#include "kernels.h"

namespace {

static_assert(HLB_OPTICS_MAX_WAVELENGTHS == hlb::OPTICS_MAX_WL, "optics wavelength bound");
static_assert(HLB_DEBUG_NAN_LDS == hlb::DEBUG_NAN_LDS, "debug flag");

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t g, Q, u, part, res, fixed;  // the part every model uses
    size_t Pi, aux, total;             // the model's planes after it
};

// Stress planes of a coupling (the whole stress: 9; the split terms: 12) and
// the predictor populations of the D3Q15 scheme (15 planes) sit after the
// fixed part, so one context can switch models within its workspace.
int stress_planes(int flow_coupling) { return flow_coupling == HLB_FLOW_SPLIT ? 12 : 9; }
int aux_planes(int lb_model) { return lb_model == HLB_LB_D3Q15_PC ? 15 : 0; }

bool make_layout(int nx, int ny, int nz, int precision, int lb_model, int flow_coupling, Layout &L)
{
    if (nx < 4 || ny < 4 || nz < 4) return false;
    if (precision != HLB_FP64 && precision != HLB_FP32) return false;
    if (lb_model != HLB_LB_D3Q19 && lb_model != HLB_LB_D3Q15_PC) return false;
    if (flow_coupling < HLB_FLOW_OFF || flow_coupling > HLB_FLOW_SPLIT) return false;
    const double n = double(nx) * double(ny) * double(nz);
    if (n >= 2147483647.0 / 2) return false;
    const size_t N = size_t(nx) * ny * nz;
    const size_t e = precision == HLB_FP64 ? 8 : 4;
    if (N * e >= (size_t(1) << 32)) return false;  // kernels address a plane with 32-bit byte offsets
    L.g = align256(19 * N * e);
    L.Q = align256(5 * N * e);
    L.u = align256(3 * N * e);
    L.part = align256(hlb::partial_doubles(nx, ny, nz) * 8);
    L.res = 256;
    L.fixed = 2 * L.g + 2 * L.Q + L.u + L.part + L.res;
    L.Pi = align256(stress_planes(flow_coupling) * N * e);
    L.aux = align256(aux_planes(lb_model) * N * e);
    L.total = L.fixed + L.Pi + L.aux;
    return true;
}

int set_error(hlb_ctx *c, int code, const char *fmt, ...)
{
    if (!c) return code;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->msg, sizeof(c->msg), fmt, ap);
    va_end(ap);
    c->status = code;
    return code;
}

int hip_fail(hlb_ctx *c, hipError_t e, const char *what)
{
    return set_error(c, HLB_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HLB_GUARD(c)                          \
    do {                                      \
        if (!(c)) return HLB_ERR_ARG;         \
        if ((c)->status) return (c)->status;  \
    } while (0)

#define HIP_TRY(c, call)                                       \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail((c), e_, #call); \
    } while (0)

// FP64 staging area for host transfers: the population buffer that does not
// hold the state (19 x N x 4 bytes >= 9 x N doubles in both precisions).
double *stage_of(hlb_ctx *c) { return static_cast<double *>(c->D.g[c->D.gcur ^ 1]); }

// Reduction scratch of hlb_get_totals_noalloc: the reduced totals in its
// first 8 doubles, the block partials after them.  One copy per device,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in: its device address is looked up once per device and only that
// address is passed to kernels and copies.
constexpr size_t NOALLOC_DOUBLES = size_t(1) << 19;  // 4 MiB
constexpr size_t NOALLOC_TOTALS = 8;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
std::mutex scratch_mu;
double *scratch_dev[NOALLOC_MAX_DEVICES];

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with it current).
hipError_t scratch_on_current_device(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_dev[dev] = static_cast<double *>(p);
    }
    *out = scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t hlb_workspace_bytes(int nx, int ny, int nz, int precision)
{
    return hlb_workspace_bytes_for(nx, ny, nz, precision, HLB_LB_D3Q19, HLB_FLOW_FORCE);
}

size_t hlb_workspace_bytes_for(int nx, int ny, int nz, int precision, int lb_model, int flow_coupling)
{
    Layout L;
    return make_layout(nx, ny, nz, precision, lb_model, flow_coupling, L) ? L.total : 0;
}

int hlb_create(int nx, int ny, int nz, int precision, void *ws, size_t ws_bytes, void *stream,
               hlb_ctx **out)
{
    if (!out) return HLB_ERR_ARG;
    *out = nullptr;
    Layout L;
    if (!make_layout(nx, ny, nz, precision, HLB_LB_D3Q19, HLB_FLOW_FORCE, L)) return HLB_ERR_ARG;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return HLB_ERR_ARG;
    if (ws_bytes < L.total) return HLB_ERR_NOMEM;
    hlb_ctx *c = new (std::nothrow) hlb_ctx;
    if (!c) return HLB_ERR_NOMEM;
    std::memset(c, 0, sizeof(*c));
    char *p = static_cast<char *>(ws);
    c->D.G = hlb::make_geom(nx, ny, nz);
    c->D.fp32 = precision == HLB_FP32;
    c->D.g[0] = p; p += L.g;
    c->D.g[1] = p; p += L.g;
    c->D.Q[0] = p; p += L.Q;
    c->D.Q[1] = p; p += L.Q;
    c->D.u = p; p += L.u;
    c->D.part = reinterpret_cast<double *>(p); p += L.part;
    c->D.res = reinterpret_cast<double *>(p); p += L.res;
    c->D.Pi = p; p += L.Pi;
    c->D.aux = nullptr;  // placed by hlb_set_params for the D3Q15 scheme
    c->D.stream = static_cast<hipStream_t>(stream);
    c->ws = ws;
    c->ws_bytes = ws_bytes;
    const size_t e = c->D.fp32 ? 4 : 8;
    c->state_bytes = size_t(24) * c->D.G.N * e;
    *out = c;
    return HLB_OK;
}

int hlb_fe_from_reduced(double kappa, double tau_ldg, double q0, double A0, hlb_fe_params *out)
{
    if (!out) return HLB_ERR_ARG;
    if (!(q0 != 0.0) || !(A0 > 0.0) || !(tau_ldg > -9.0) || !std::isfinite(kappa)) return HLB_ERR_PARAM;
    const double gamma = 27.0 / (tau_ldg + 9.0);
    out->A0 = A0;
    out->gamma = gamma;
    out->K = kappa * kappa * A0 * gamma / (108.0 * q0 * q0);
    out->q0 = q0;
    return HLB_OK;
}

// Schedules whose stress is evaluated in LDS tiles (the D3Q19 LB only), and
// the one whose tiled stress kernel writes the whole-stress force (no split).
static bool tiled_stress(int sched)
{
    return sched == HLB_SCHED_TILED || sched == HLB_SCHED_FUSED || sched == HLB_SCHED_FUSED_TILED;
}

static bool no_split(int sched) { return sched == HLB_SCHED_TILED; }

int hlb_set_params(hlb_ctx *c, const hlb_lb_params *lb, const hlb_fe_params *fe, const hlb_be_params *be)
{
    HLB_GUARD(c);
    if (!lb || !fe || !be) return set_error(c, HLB_ERR_ARG, "null parameter struct");
    if (lb->model != HLB_LB_D3Q19 && lb->model != HLB_LB_D3Q15_PC)
        return set_error(c, HLB_ERR_PARAM, "LB model %d is not one of 0, 1", lb->model);
    if (lb->model == HLB_LB_D3Q19 && !(lb->tau > 0.5))
        return set_error(c, HLB_ERR_PARAM, "tau = %g must exceed 1/2", lb->tau);
    if (lb->model == HLB_LB_D3Q15_PC && !(lb->tau > 0.0))
        return set_error(c, HLB_ERR_PARAM, "tau = %g must be positive", lb->tau);
    if (lb->model == HLB_LB_D3Q15_PC && tiled_stress(c->D.sched))
        return set_error(c, HLB_ERR_STATE, "the D3Q15 scheme needs the sites or mixed schedule");
    if (!(lb->rho0 > 0.0)) return set_error(c, HLB_ERR_PARAM, "rho0 = %g must be positive", lb->rho0);
    if (!(fe->A0 > 0.0)) return set_error(c, HLB_ERR_PARAM, "A0 = %g must be positive", fe->A0);
    if (!(fe->gamma > 0.0)) return set_error(c, HLB_ERR_PARAM, "gamma = %g must be positive", fe->gamma);
    if (!(fe->K >= 0.0)) return set_error(c, HLB_ERR_PARAM, "K = %g must be non-negative", fe->K);
    if (!std::isfinite(fe->q0)) return set_error(c, HLB_ERR_PARAM, "q0 not finite");
    if (!(be->Gamma > 0.0)) return set_error(c, HLB_ERR_PARAM, "Gamma = %g must be positive", be->Gamma);
    if (!std::isfinite(be->xi)) return set_error(c, HLB_ERR_PARAM, "xi not finite");
    if (be->flow_coupling < HLB_FLOW_OFF || be->flow_coupling > HLB_FLOW_SPLIT)
        return set_error(c, HLB_ERR_PARAM, "flow_coupling = %d is not one of 0, 1, 2", be->flow_coupling);
    if (be->flow_coupling == HLB_FLOW_SPLIT && no_split(c->D.sched))
        return set_error(c, HLB_ERR_STATE, "the split coupling needs a schedule other than tiled");
    if (!(12.0 * be->Gamma * fe->K < 2.0))
        return set_error(c, HLB_ERR_PARAM, "12 Gamma K = %g violates the explicit diffusion bound 2",
                         12.0 * be->Gamma * fe->K);
    Layout L;
    const hlb::Geom &G = c->D.G;
    make_layout(G.nx, G.ny, G.nz, c->D.fp32 ? HLB_FP32 : HLB_FP64, lb->model, be->flow_coupling, L);
    if (c->ws_bytes < L.total)
        return set_error(c, HLB_ERR_NOMEM,
                         "workspace of %zu bytes is smaller than the %zu this LB model and coupling need "
                         "(hlb_workspace_bytes_for)", c->ws_bytes, L.total);
    c->D.aux = L.aux ? static_cast<char *>(c->ws) + L.fixed + L.Pi : nullptr;
    if (c->have_params && c->p.model != lb->model) c->have_fields = false;  // state layout differs
    c->p = {lb->tau, lb->rho0, fe->A0, fe->gamma, fe->K, fe->q0, be->Gamma, be->xi, be->flow_coupling, lb->model};
    c->have_params = true;
    ++c->version;
    return HLB_OK;
}

int hlb_set_fields(hlb_ctx *c, const double *Q5, const double *u3, const double *rho)
{
    HLB_GUARD(c);
    if (!c->have_params) return set_error(c, HLB_ERR_STATE, "hlb_set_params must come first");
    if (!Q5) return set_error(c, HLB_ERR_ARG, "Q5 is null");
    const size_t N = c->D.G.N;
    std::vector<double> host(9 * N);
    for (size_t s = 0; s < N; ++s) host[s] = rho ? rho[s] : c->p.rho0;
    if (u3)
        std::memcpy(host.data() + N, u3, 3 * N * sizeof(double));
    else
        std::fill(host.begin() + N, host.begin() + 4 * N, 0.0);
    std::memcpy(host.data() + 4 * N, Q5, 5 * N * sizeof(double));
    double *stage = stage_of(c);
    HIP_TRY(c, hipMemcpyAsync(stage, host.data(), 9 * N * sizeof(double), hipMemcpyHostToDevice, c->D.stream));
    HIP_TRY(c, hlb::run_init(c->D, c->p, stage));
    HIP_TRY(c, hipStreamSynchronize(c->D.stream));
    c->have_fields = true;
    ++c->version;
    return HLB_OK;
}

int hlb_step(hlb_ctx *c, int nsteps)
{
    HLB_GUARD(c);
    if (nsteps < 0) return set_error(c, HLB_ERR_ARG, "nsteps = %d", nsteps);
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "hlb_set_fields must come first");
    HIP_TRY(c, hlb::run_steps(c->D, c->p, nsteps));
    if (nsteps) ++c->version;
    return HLB_OK;
}

int hlb_get_fields(hlb_ctx *c, double *Q5, double *u3, double *rho)
{
    HLB_GUARD(c);
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "no fields set");
    const size_t N = c->D.G.N;
    double *stage = stage_of(c);
    HIP_TRY(c, hlb::run_readout(c->D, c->p, stage, nullptr));
    if (rho) HIP_TRY(c, hipMemcpyAsync(rho, stage, N * 8, hipMemcpyDeviceToHost, c->D.stream));
    if (u3) HIP_TRY(c, hipMemcpyAsync(u3, stage + N, 3 * N * 8, hipMemcpyDeviceToHost, c->D.stream));
    if (Q5) HIP_TRY(c, hipMemcpyAsync(Q5, stage + 4 * N, 5 * N * 8, hipMemcpyDeviceToHost, c->D.stream));
    HIP_TRY(c, hipStreamSynchronize(c->D.stream));
    return HLB_OK;
}

int hlb_get_totals(hlb_ctx *c, double *mass, double *mom3, double *free_energy)
{
    HLB_GUARD(c);
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "no fields set");
    double r[5];
    HIP_TRY(c, hlb::run_readout(c->D, c->p, nullptr, c->D.res));
    HIP_TRY(c, hipMemcpyAsync(r, c->D.res, sizeof(r), hipMemcpyDeviceToHost, c->D.stream));
    HIP_TRY(c, hipStreamSynchronize(c->D.stream));
    const double m = double(c->D.G.N) * c->p.rho0 + r[0];
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(r[k])) return set_error(c, HLB_ERR_NONFINITE, "non-finite total (component %d)", k);
    if (mass) *mass = m;
    if (mom3)
        for (int a = 0; a < 3; ++a) mom3[a] = r[1 + a];
    if (free_energy) *free_energy = r[4];
    return HLB_OK;
}

int hlb_get_totals_noalloc(hlb_ctx *c, double *mass, double *mom3, double *free_energy)
{
    HLB_GUARD(c);
    const size_t need = NOALLOC_TOTALS + hlb::readout_partials(c->D.G);
    if (need > NOALLOC_DOUBLES)
        return set_error(c, HLB_ERR_NOMEM,
                         "hlb_get_totals_noalloc: %d sites need %zu doubles of reduction scratch, more than the "
                         "%zu it holds (at most %zu sites)", c->D.G.N, need, NOALLOC_DOUBLES,
                         (NOALLOC_DOUBLES - NOALLOC_TOTALS) / 5 / 8 * 8 * 256);
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "no fields set");
    double *sp = nullptr;
    HIP_TRY(c, scratch_on_current_device(&sp));
    double r[5];
    HIP_TRY(c, hlb::run_readout(c->D, c->p, nullptr, sp, sp + NOALLOC_TOTALS));
    HIP_TRY(c, hipMemcpyAsync(r, sp, sizeof(r), hipMemcpyDeviceToHost, c->D.stream));
    HIP_TRY(c, hipStreamSynchronize(c->D.stream));
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(r[k])) return set_error(c, HLB_ERR_NONFINITE, "non-finite total (component %d)", k);
    if (mass) *mass = double(c->D.G.N) * c->p.rho0 + r[0];
    if (mom3)
        for (int a = 0; a < 3; ++a) mom3[a] = r[1 + a];
    if (free_energy) *free_energy = r[4];
    return HLB_OK;
}

int hlb_set_schedule(hlb_ctx *c, int schedule, int tz)
{
    HLB_GUARD(c);
    if (schedule < HLB_SCHED_SITES || schedule > HLB_SCHED_FUSED_TILED || tz < 0)
        return set_error(c, HLB_ERR_ARG, "schedule %d / tz %d", schedule, tz);
    if (no_split(schedule) && c->have_params && c->p.flow == HLB_FLOW_SPLIT)
        return set_error(c, HLB_ERR_STATE, "schedule %d carries the whole-stress force only", schedule);
    if (tiled_stress(schedule) && c->have_params && c->p.model == HLB_LB_D3Q15_PC)
        return set_error(c, HLB_ERR_STATE, "schedule %d runs the D3Q19 LB only", schedule);
    c->D.sched = schedule;
    c->D.tz = tz;
    c->D.tzq = 0;
    return HLB_OK;
}

int hlb_set_update_chunk(hlb_ctx *c, int tzq)
{
    HLB_GUARD(c);
    if (tzq < 0) return set_error(c, HLB_ERR_ARG, "update chunk %d", tzq);
    c->D.tzq = tzq;
    return HLB_OK;
}

int hlb_get_update_chunk(const hlb_ctx *c, int *tzq)
{
    if (!c || !tzq) return HLB_ERR_ARG;
    *tzq = c->D.tzq;
    return HLB_OK;
}

int hlb_set_debug(hlb_ctx *c, int flags)
{
    HLB_GUARD(c);
    if (flags & ~HLB_DEBUG_NAN_LDS) return set_error(c, HLB_ERR_ARG, "unknown debug flags 0x%x", flags);
    c->D.debug = flags;
    return HLB_OK;
}

int hlb_get_schedule(const hlb_ctx *c, int *schedule, int *tz)
{
    if (!c || !schedule || !tz) return HLB_ERR_ARG;
    *schedule = c->D.sched;
    *tz = c->D.tz;
    return HLB_OK;
}

int hlb_autotune(hlb_ctx *c, int trial_steps, double *best_ms_per_step)
{
    HLB_GUARD(c);
    if (trial_steps < 1) return set_error(c, HLB_ERR_ARG, "trial_steps = %d", trial_steps);
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "hlb_set_fields must come first");
    // the trials advance the state: keep a host copy and put it back after
    std::vector<char> saved(c->state_bytes);
    const int g0 = c->D.gcur, q0 = c->D.qcur;
    int rc = hlb_get_state(c, saved.data(), saved.size());
    if (rc) return rc;
    struct Cand {
        int sched, tz;
    };
    // z-chunks of 8, 16 and 32 planes, and those whose tiled launches fill the
    // device's resident block slots once or twice
    int tzs[5] = {8, 16, 32, hlb::tile_tz_fill(c->D, 1), hlb::tile_tz_fill(c->D, 2)};
    int ntz = 3;
    for (int i = 3; i < 5; ++i) {
        bool dup = tzs[i] < 1;
        for (int j = 0; j < ntz; ++j) dup = dup || tzs[j] == tzs[i];
        if (!dup) tzs[ntz++] = tzs[i];
    }
    const int tiledsc[4] = {HLB_SCHED_TILED, HLB_SCHED_MIXED, HLB_SCHED_FUSED, HLB_SCHED_FUSED_TILED};
    Cand cands[1 + 4 * 5];
    int NC = 0;
    cands[NC++] = {HLB_SCHED_SITES, 0};
    for (int sc : tiledsc)
        for (int j = 0; j < ntz; ++j) cands[NC++] = {sc, tzs[j]};
    hipEvent_t a, b;
    HIP_TRY(c, hipEventCreate(&a));
    HIP_TRY(c, hipEventCreate(&b));
    // time trial_steps steps of one setting (2 untimed steps first); ms per step
    auto trial = [&](int sched, int tz, int tzq, double &ms_step) -> hipError_t {
        c->D.sched = sched;
        c->D.tz = tz;
        c->D.tzq = tzq;
        hipError_t e = hlb::run_steps(c->D, c->p, 2);
        if (e == hipSuccess) e = hipEventRecord(a, c->D.stream);
        if (e == hipSuccess) e = hlb::run_steps(c->D, c->p, trial_steps);
        if (e == hipSuccess) e = hipEventRecord(b, c->D.stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        ms_step = double(ms) / trial_steps;
        return e;
    };
    auto fail = [&](hipError_t e) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return hip_fail(c, e, "hlb_autotune trial");
    };
    // Two passes over the candidates, each candidate scored by its faster
    // pass: the first trials of a call can run before the clocks and caches
    // have settled, which would penalise whichever candidate comes first.
    double t[1 + 4 * 5];
    for (int i = 0; i < NC; ++i) t[i] = 1e300;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i < NC; ++i) {
            const Cand &k = cands[i];
            if (k.sched != HLB_SCHED_SITES && k.tz > c->D.G.nz && k.tz != 8) continue;
            if ((tiled_stress(k.sched) && c->p.model == HLB_LB_D3Q15_PC) ||
                (no_split(k.sched) && c->p.flow == HLB_FLOW_SPLIT))
                continue;
            double ms = 0.0;
            const hipError_t e = trial(k.sched, k.tz, 0, ms);
            if (e != hipSuccess) return fail(e);
            t[i] = std::min(t[i], ms);
        }
    }
    double best = 1e300;
    Cand pick = cands[0];
    for (int i = 0; i < NC; ++i)
        if (t[i] < best) {
            best = t[i];
            pick = cands[i];
        }
    // Where a tiled stress kernel is followed by the tiled Q update, the two
    // may prefer different z-chunks: try the other chunks for the Q update.
    int pick_tzq = 0;
    if (pick.sched == HLB_SCHED_TILED || pick.sched == HLB_SCHED_FUSED_TILED) {
        double tq[5];
        for (int j = 0; j < ntz; ++j) tq[j] = 1e300;
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < ntz; ++j) {
                if (tzs[j] == pick.tz || (tzs[j] > c->D.G.nz && tzs[j] != 8)) continue;
                double ms = 0.0;
                const hipError_t e = trial(pick.sched, pick.tz, tzs[j], ms);
                if (e != hipSuccess) return fail(e);
                tq[j] = std::min(tq[j], ms);
            }
        for (int j = 0; j < ntz; ++j)
            if (tq[j] < best) {
                best = tq[j];
                pick_tzq = tzs[j];
            }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    c->D.sched = pick.sched;
    c->D.tz = pick.tz;
    c->D.tzq = pick_tzq;
    c->D.gcur = g0;
    c->D.qcur = q0;
    rc = hlb_set_state(c, saved.data(), saved.size());
    if (rc) return rc;
    if (best_ms_per_step) *best_ms_per_step = best;
    return HLB_OK;
}

int hlb_step_timed(hlb_ctx *c, int nsteps, double *kernel_ms, int nkernels)
{
    HLB_GUARD(c);
    if (nsteps < 0 || !kernel_ms || nkernels < hlb::K_COUNT)
        return set_error(c, HLB_ERR_ARG, "hlb_step_timed: bad arguments");
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "hlb_set_fields must come first");
    hlb::KernelTimer t;
    hipError_t e = hlb::run_steps(c->D, c->p, nsteps, &t);
    if (e == hipSuccess) e = hipStreamSynchronize(c->D.stream);
    for (int k = 0; k < nkernels; ++k) kernel_ms[k] = 0.0;
    for (auto &m : t.events) {
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.start, m.stop);
        kernel_ms[m.kind] += ms;
        (void)hipEventDestroy(m.start);
        (void)hipEventDestroy(m.stop);
    }
    if (e != hipSuccess) return hip_fail(c, e, "hlb_step_timed");
    if (nsteps) ++c->version;
    return hlb::K_COUNT;
}

const char *hlb_kernel_name(int k)
{
    const char *n = hlb::kernel_name(k);
    return n ? n : "";
}

int hlb_get_fz(hlb_ctx *c, double *fz)
{
    HLB_GUARD(c);
    if (!fz) return set_error(c, HLB_ERR_ARG, "fz is null");
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "no fields set");
    const int nz = c->D.G.nz;
    HIP_TRY(c, hlb::run_fz(c->D, c->p, c->D.part));
    HIP_TRY(c, hipMemcpyAsync(fz, c->D.part, nz * sizeof(double), hipMemcpyDeviceToHost, c->D.stream));
    HIP_TRY(c, hipStreamSynchronize(c->D.stream));
    for (int z = 0; z < nz; ++z)
        if (!std::isfinite(fz[z])) return set_error(c, HLB_ERR_NONFINITE, "non-finite f(z) at z = %d", z);
    return HLB_OK;
}

int hlb_get_order(hlb_ctx *c, double threshold, double *q, double *dir3, unsigned char *defect, long long *defects_z,
                  long long *n_defect)
{
    HLB_GUARD(c);
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "no fields set");
    if (!std::isfinite(threshold)) return set_error(c, HLB_ERR_ARG, "threshold not finite");
    const size_t N = c->D.G.N;
    const int nz = c->D.G.nz;
    // device staging in the population buffer that does not hold the state:
    // q [N] doubles, dir [3N] doubles, per-plane counts [nz] doubles, flags [N] bytes
    double *st = stage_of(c);
    double *dq = st, *dd = st + N, *dc = st + 4 * N;
    unsigned char *df = reinterpret_cast<unsigned char *>(st + 4 * N + nz);
    const bool want_flags = defect || defects_z || n_defect;
    HIP_TRY(c, hlb::run_order(c->D, threshold, q ? dq : nullptr, dir3 ? dd : nullptr, want_flags ? df : nullptr,
                              (defects_z || n_defect) ? dc : nullptr));
    if (q) HIP_TRY(c, hipMemcpyAsync(q, dq, N * 8, hipMemcpyDeviceToHost, c->D.stream));
    if (dir3) HIP_TRY(c, hipMemcpyAsync(dir3, dd, 3 * N * 8, hipMemcpyDeviceToHost, c->D.stream));
    if (defect) HIP_TRY(c, hipMemcpyAsync(defect, df, N, hipMemcpyDeviceToHost, c->D.stream));
    std::vector<double> cnt(defects_z || n_defect ? nz : 0);
    if (!cnt.empty()) HIP_TRY(c, hipMemcpyAsync(cnt.data(), dc, nz * 8, hipMemcpyDeviceToHost, c->D.stream));
    HIP_TRY(c, hipStreamSynchronize(c->D.stream));
    long long total = 0;
    for (int z = 0; z < int(cnt.size()); ++z) {
        const long long v = (long long)cnt[z];
        if (defects_z) defects_z[z] = v;
        total += v;
    }
    if (n_defect) *n_defect = total;
    return HLB_OK;
}

int hlb_get_optics(hlb_ctx *c, const hlb_optics_params *op, double *image)
{
    HLB_GUARD(c);
    if (!op || !image) return set_error(c, HLB_ERR_ARG, "null argument");
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "no fields set");
    if (!(op->n_o > 0.0) || !(op->n_e > 0.0) || !(op->h > 0.0) || !std::isfinite(op->n_o) ||
        !std::isfinite(op->n_e) || !std::isfinite(op->h) || !std::isfinite(op->phi_in) || !std::isfinite(op->phi_out))
        return set_error(c, HLB_ERR_ARG, "optics: indices and thickness must be positive, angles finite");
    if (op->n_wavelengths < 1 || op->n_wavelengths > HLB_OPTICS_MAX_WAVELENGTHS)
        return set_error(c, HLB_ERR_ARG, "optics: %d wavelengths (1..%d)", op->n_wavelengths,
                         HLB_OPTICS_MAX_WAVELENGTHS);
    hlb::OpticsParams p{};
    p.n_o = op->n_o;
    p.n_e = op->n_e;
    p.h = op->h;
    p.c_in = std::cos(2.0 * op->phi_in);
    p.s_in = std::sin(2.0 * op->phi_in);
    p.c_out = std::cos(2.0 * op->phi_out);
    p.s_out = std::sin(2.0 * op->phi_out);
    p.nwl = op->n_wavelengths;
    for (int k = 0; k < p.nwl; ++k) {
        if (!(op->wavelength[k] > 0.0) || !std::isfinite(op->wavelength[k]) || !std::isfinite(op->weight[k]))
            return set_error(c, HLB_ERR_ARG, "optics: wavelength %d must be positive, weight finite", k);
        p.lam[k] = op->wavelength[k];
        p.w[k] = op->weight[k];
    }
    // scratch: the population buffer that does not hold the state; the image
    // first, the per-segment transfer matrices after it
    const size_t cols = size_t(c->D.G.nx) * c->D.G.ny;
    const size_t e = c->D.fp32 ? 4 : 8;
    const size_t stage_bytes = size_t(19) * c->D.G.N * e;
    double *st = stage_of(c);
    const size_t img_bytes = (cols * 8 + 255) & ~size_t(255);
    double *Tm = st + img_bytes / 8;
    const size_t tm_bytes = stage_bytes - img_bytes;
    if (hlb::optics_segments(c->D.G, p.nwl, tm_bytes) < 1)
        return set_error(c, HLB_ERR_NOMEM, "optics: lattice too small for the transfer-matrix scratch");
    HIP_TRY(c, hlb::run_optics(c->D, p, Tm, tm_bytes, st));
    HIP_TRY(c, hipMemcpyAsync(image, st, cols * 8, hipMemcpyDeviceToHost, c->D.stream));
    HIP_TRY(c, hipStreamSynchronize(c->D.stream));
    return HLB_OK;
}

size_t hlb_state_bytes(hlb_ctx *c) { return c ? c->state_bytes : 0; }

int hlb_get_state(hlb_ctx *c, void *buf, size_t nbytes)
{
    HLB_GUARD(c);
    if (!buf || nbytes != c->state_bytes) return set_error(c, HLB_ERR_ARG, "state buffer size mismatch");
    if (!c->have_fields) return set_error(c, HLB_ERR_STATE, "no fields set");
    const size_t e = c->D.fp32 ? 4 : 8, N = c->D.G.N;
    char *b = static_cast<char *>(buf);
    HIP_TRY(c, hipMemcpyAsync(b, c->D.g[c->D.gcur], 19 * N * e, hipMemcpyDeviceToHost, c->D.stream));
    HIP_TRY(c, hipMemcpyAsync(b + 19 * N * e, c->D.Q[c->D.qcur], 5 * N * e, hipMemcpyDeviceToHost, c->D.stream));
    HIP_TRY(c, hipStreamSynchronize(c->D.stream));
    return HLB_OK;
}

int hlb_set_state(hlb_ctx *c, const void *buf, size_t nbytes)
{
    HLB_GUARD(c);
    if (!buf || nbytes != c->state_bytes) return set_error(c, HLB_ERR_ARG, "state buffer size mismatch");
    if (!c->have_params) return set_error(c, HLB_ERR_STATE, "hlb_set_params must come first");
    const size_t e = c->D.fp32 ? 4 : 8, N = c->D.G.N;
    const char *b = static_cast<const char *>(buf);
    HIP_TRY(c, hipMemcpyAsync(c->D.g[c->D.gcur], b, 19 * N * e, hipMemcpyHostToDevice, c->D.stream));
    HIP_TRY(c, hipMemcpyAsync(c->D.Q[c->D.qcur], b + 19 * N * e, 5 * N * e, hipMemcpyHostToDevice, c->D.stream));
    HIP_TRY(c, hipStreamSynchronize(c->D.stream));
    c->have_fields = true;
    ++c->version;
    return HLB_OK;
}

const char *hlb_last_error(const hlb_ctx *c) { return c ? c->msg : "null context"; }

void hlb_destroy(hlb_ctx *c) { delete c; }

}  // extern "C"
