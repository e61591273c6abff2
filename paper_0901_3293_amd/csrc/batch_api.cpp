// batch_api.cpp -- C-ABI of the batched form (include/hlb.h, hlb_batch_*):
// workspace layout of many boxes, the work list, autotuning of the chunk per
// box size, graph capture and replay, per-box readout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/hlb.h"
#include "batch.h"
#include "kernels.h"

struct hlb_batch {
    int n;
    bool fp32;
    hipStream_t stream;
    std::vector<hlb::Device> box;
    std::vector<hlb::PhysParams> par;
    std::vector<char> have_params, have_fields;
    std::vector<int> gcur;           // host mirror of the device-side ping-pong index
    std::map<int, int> chunk_of_n;   // sites per work item, per box size N
    void *d_reps;
    int *d_items;
    size_t items_cap;
    int n_items;
    unsigned *d_bar;
    int *d_err;
    int *d_misplaced;
    int *d_xlo;     // item offsets of the 8 XCD groups (9 ints)
    int *d_xcnt;    // workgroups per XCD of the running launch (8 ints)
    int *d_slo;     // item offsets of the cache groups of the persistent form (n + 9 ints)
    int *d_sgx;     // cache groups of each XCD group: [sgx[x], sgx[x + 1]) (9 ints)
    unsigned *d_gbar;  // barrier counters of the 8 XCD groups (64-byte stride)
    int xlo[9];
    int sgx[9];
    std::vector<int> slo;
    int grid;
    int bpc;                         // blocks per compute unit of the persistent grid (0: max)
    bool xcd_local = true;           // keep each box on one XCD when the launch allows it
    int launch_form = HLB_BATCH_PHASES;       // or HLB_BATCH_PERSISTENT
    long long group_sites = 1 << 21;          // cache-group budget (sites; per XCD group: 1/8 of it)
    std::vector<int> clo;                     // item offsets of the cache groups (phase form)
    bool dirty;                      // descriptor table / work list must be rebuilt
    hipGraph_t graph;
    hipGraphExec_t exec;
    int graph_steps;
    int status;
    char msg[512];
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool box_bytes(int nx, int ny, int nz, bool fp32, size_t &bytes, size_t &part)
{
    if (nx < 4 || ny < 4 || nz < 4) return false;
    const double n = double(nx) * ny * nz;
    if (n >= 2147483647.0 / 2) return false;
    const size_t N = size_t(nx) * ny * nz, e = fp32 ? 4 : 8;
    if (N * e >= (size_t(1) << 32)) return false;  // kernels address a plane with 32-bit byte offsets
    bytes = 2 * align256(19 * N * e) + 2 * align256(5 * N * e) + align256(3 * N * e) + align256(9 * N * e);
    part = align256(hlb::partial_doubles(nx, ny, nz) * 8);
    return true;
}

constexpr int kMinChunk = 256;

size_t items_upper_bound(int n, const int *dims)
{
    size_t s = 0;
    for (int i = 0; i < n; ++i) s += size_t(dims[3 * i]) * dims[3 * i + 1] * dims[3 * i + 2] / kMinChunk + 1;
    return s;
}

int bset_error(hlb_batch *b, int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(b->msg, sizeof(b->msg), fmt, ap);
    va_end(ap);
    b->status = code;
    return code;
}

#define B_GUARD(b)                           \
    do {                                     \
        if (!(b)) return HLB_ERR_ARG;        \
        if ((b)->status) return (b)->status; \
    } while (0)

#define B_TRY(b, call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return bset_error((b), HLB_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

void drop_graph(hlb_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_steps = 0;
}

int chunk_for(const hlb_batch *b, int N)
{
    auto it = b->chunk_of_n.find(N);
    return it == b->chunk_of_n.end() ? 1024 : it->second;
}

// Rebuild the device descriptor table and the work list (synchronous).
int rebuild(hlb_batch *b)
{
    for (int i = 0; i < b->n; ++i)
        if (!b->have_params[i] || !b->have_fields[i])
            return bset_error(b, HLB_ERR_STATE, "box %d has no parameters or fields", i);
    std::vector<char> blob;
    hlb::batch_pack_reps(b->fp32, b->box, b->par, b->gcur, blob);
    // boxes -> 8 XCD groups of about equal site count (largest box first to
    // the lightest group), each box whole in one group
    std::vector<int> order(b->n);
    for (int i = 0; i < b->n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->box[x].G.N > b->box[y].G.N; });
    std::vector<int> group(b->n);
    long long load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i : order) {
        int g = 0;
        for (int k = 1; k < 8; ++k)
            if (load[k] < load[g]) g = k;
        group[i] = g;
        load[g] += b->box[i].G.N;
    }
    std::vector<int> items;
    auto add_box = [&](int i) {
        const int N = b->box[i].G.N, ch = chunk_for(b, N);
        for (int s = 0; s < N; s += ch) {
            items.push_back(i);
            items.push_back(s);
            items.push_back(std::min(ch, N - s));
            items.push_back(0);
        }
    };
    b->clo.clear();
    if (b->launch_form == HLB_BATCH_PHASES) {
        // cache groups: boxes in index order, packed while the group stays
        // within group_sites sites (a larger box is a group of its own); the
        // phase form runs all steps of one group before the next
        long long in_group = 0;
        for (int i = 0; i < b->n; ++i) {
            const long long N = b->box[i].G.N;
            if (b->clo.empty() || in_group + N > b->group_sites) {
                b->clo.push_back(int(items.size() / 4));
                in_group = 0;
            }
            add_box(i);
            in_group += N;
        }
        b->clo.push_back(int(items.size() / 4));
        for (int g = 0; g <= 8; ++g) b->xlo[g] = g == 8 ? int(items.size() / 4) : 0;
    } else {
        // XCD groups, each cut into cache groups of at most group_sites / 8
        // sites (a larger box alone): the persistent kernel runs all steps of
        // one cache group of its XCD before the next
        const long long budget = std::max(1ll, b->group_sites / 8);
        b->slo.clear();
        for (int g = 0; g < 8; ++g) {
            b->xlo[g] = int(items.size() / 4);
            b->sgx[g] = int(b->slo.size());
            long long in_sub = 0;
            bool open = false;
            for (int i = 0; i < b->n; ++i) {
                if (group[i] != g) continue;
                const long long N = b->box[i].G.N;
                if (!open || in_sub + N > budget) {
                    b->slo.push_back(int(items.size() / 4));
                    in_sub = 0;
                    open = true;
                }
                add_box(i);
                in_sub += N;
            }
        }
        b->sgx[8] = int(b->slo.size());
    }
    b->n_items = int(items.size() / 4);
    b->xlo[8] = b->n_items;
    if (b->launch_form == HLB_BATCH_PHASES) {
        b->slo.clear();
        for (int g = 0; g <= 8; ++g) b->sgx[g] = 0;
    }
    b->slo.push_back(b->n_items);  // end of the last cache group
    if (b->slo.size() > size_t(b->n + 9)) return bset_error(b, HLB_ERR_ARG, "cache-group list overflow");
    if (size_t(b->n_items) > b->items_cap) return bset_error(b, HLB_ERR_ARG, "work list overflow");
    B_TRY(b, hipMemcpyAsync(b->d_reps, blob.data(), blob.size(), hipMemcpyHostToDevice, b->stream));
    B_TRY(b, hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
    B_TRY(b, hipMemcpyAsync(b->d_xlo, b->xlo, sizeof(b->xlo), hipMemcpyHostToDevice, b->stream));
    B_TRY(b, hipMemcpyAsync(b->d_sgx, b->sgx, sizeof(b->sgx), hipMemcpyHostToDevice, b->stream));
    B_TRY(b, hipMemcpyAsync(b->d_slo, b->slo.data(), b->slo.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
    B_TRY(b, hipStreamSynchronize(b->stream));
    B_TRY(b, hlb::batch_grid(b->fp32, b->n_items, b->bpc, &b->grid));
    b->dirty = false;
    drop_graph(b);
    return HLB_OK;
}

int check_err(hlb_batch *b)
{
    int err = 0;
    B_TRY(b, hipMemcpyAsync(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    B_TRY(b, hipStreamSynchronize(b->stream));
    if (err) return bset_error(b, HLB_ERR_HIP, "batched kernel: a grid barrier wait ran out (blocks not co-resident)");
    return HLB_OK;
}

void advance_host_gcur(hlb_batch *b, int nsteps)
{
    if (nsteps & 1)
        for (int i = 0; i < b->n; ++i)
            if (b->par[i].flow) b->gcur[i] ^= 1;
}

// The single-box view used for readout and initialisation: its population
// index follows the batch mirror.
hlb::Device view(hlb_batch *b, int i)
{
    hlb::Device D = b->box[i];
    D.gcur = b->gcur[i];
    D.sched = hlb::SCHED_SITES;
    return D;
}

// nsteps steps of every box in the selected launch form.
hipError_t enqueue(hlb_batch *b, int nsteps)
{
    if (b->launch_form == HLB_BATCH_PHASES)
        return hlb::batch_launch_phases(b->fp32, b->d_reps, b->n, b->d_items, b->clo.data(), int(b->clo.size()) - 1,
                                        b->d_bar, b->d_err, b->d_misplaced, b->d_xcnt, nsteps, b->stream);
    return hlb::batch_launch(b->fp32, b->d_reps, b->d_items, b->d_xlo, b->d_slo, b->d_sgx, b->d_bar, b->d_gbar,
                             b->d_err, b->d_misplaced, b->d_xcnt, b->xcd_local, nsteps, b->grid, b->stream);
}

}  // namespace

extern "C" {

size_t hlb_batch_workspace_bytes(int n, const int *dims, int precision)
{
    if (n < 1 || !dims || (precision != HLB_FP64 && precision != HLB_FP32)) return 0;
    const bool fp32 = precision == HLB_FP32;
    size_t total = 0, part_max = 0;
    for (int i = 0; i < n; ++i) {
        size_t bytes, part;
        if (!box_bytes(dims[3 * i], dims[3 * i + 1], dims[3 * i + 2], fp32, bytes, part)) return 0;
        total += bytes;
        part_max = std::max(part_max, part);
    }
    total += align256(n * hlb::batch_rep_bytes(fp32));
    total += align256(items_upper_bound(n, dims) * 16);
    total += 256 + part_max + 256;
    total += 512 + align256(size_t(n + 9) * 4) + 256;  // group barriers, cache-group offsets
    return total;
}

int hlb_batch_create(int n, const int *dims, int precision, void *ws, size_t ws_bytes, void *stream,
                     hlb_batch **out)
{
    if (!out) return HLB_ERR_ARG;
    *out = nullptr;
    const size_t need = hlb_batch_workspace_bytes(n, dims, precision);
    if (need == 0) return HLB_ERR_ARG;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return HLB_ERR_ARG;
    if (ws_bytes < need) return HLB_ERR_NOMEM;
    hlb_batch *b = new (std::nothrow) hlb_batch();
    if (!b) return HLB_ERR_NOMEM;
    b->n = n;
    b->fp32 = precision == HLB_FP32;
    b->stream = static_cast<hipStream_t>(stream);
    char *p = static_cast<char *>(ws);
    b->d_reps = p;
    p += align256(n * hlb::batch_rep_bytes(b->fp32));
    b->d_items = reinterpret_cast<int *>(p);
    b->items_cap = items_upper_bound(n, dims);
    p += align256(b->items_cap * 16);
    b->d_bar = reinterpret_cast<unsigned *>(p);
    b->d_err = reinterpret_cast<int *>(p + 64);
    b->d_misplaced = reinterpret_cast<int *>(p + 128);
    b->d_xlo = reinterpret_cast<int *>(p + 160);   // 9 ints
    b->d_xcnt = reinterpret_cast<int *>(p + 224);  // 8 ints
    p += 256;
    b->d_gbar = reinterpret_cast<unsigned *>(p);
    p += 512;
    b->d_slo = reinterpret_cast<int *>(p);
    p += align256(size_t(n + 9) * 4);
    b->d_sgx = reinterpret_cast<int *>(p);
    p += 256;
    size_t part_max = 0;
    for (int i = 0; i < n; ++i) {
        size_t bytes, part;
        box_bytes(dims[3 * i], dims[3 * i + 1], dims[3 * i + 2], b->fp32, bytes, part);
        part_max = std::max(part_max, part);
    }
    double *part = reinterpret_cast<double *>(p);
    p += part_max;
    double *res = reinterpret_cast<double *>(p);
    p += 256;
    b->box.resize(n);
    b->par.resize(n);
    b->have_params.assign(n, 0);
    b->have_fields.assign(n, 0);
    b->gcur.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        const int nx = dims[3 * i], ny = dims[3 * i + 1], nz = dims[3 * i + 2];
        const size_t N = size_t(nx) * ny * nz, e = b->fp32 ? 4 : 8;
        hlb::Device &D = b->box[i];
        std::memset(&D, 0, sizeof(D));
        D.G = hlb::make_geom(nx, ny, nz);
        D.fp32 = b->fp32;
        D.g[0] = p; p += align256(19 * N * e);
        D.g[1] = p; p += align256(19 * N * e);
        D.Q[0] = p; p += align256(5 * N * e);
        D.Q[1] = p; p += align256(5 * N * e);
        D.u = p; p += align256(3 * N * e);
        D.Pi = p; p += align256(9 * N * e);
        D.part = part;
        D.res = res;
        D.stream = b->stream;
    }
    b->dirty = true;
    *out = b;
    return HLB_OK;
}

int hlb_batch_set_params(hlb_batch *b, int i, const hlb_lb_params *lb, const hlb_fe_params *fe,
                         const hlb_be_params *be)
{
    B_GUARD(b);
    if (i < 0 || i >= b->n || !lb || !fe || !be) return bset_error(b, HLB_ERR_ARG, "box %d", i);
    if (!(lb->tau > 0.5) || !(lb->rho0 > 0.0) || !(fe->A0 > 0.0) || !(fe->gamma > 0.0) || !(fe->K >= 0.0) ||
        !(be->Gamma > 0.0) || !std::isfinite(fe->q0) || !std::isfinite(be->xi) || !(12.0 * be->Gamma * fe->K < 2.0))
        return bset_error(b, HLB_ERR_PARAM, "box %d: parameters out of range", i);
    if (be->flow_coupling != HLB_FLOW_OFF && be->flow_coupling != HLB_FLOW_FORCE)
        return bset_error(b, HLB_ERR_PARAM, "box %d: the batched kernel takes flow_coupling 0 or 1", i);
    if (lb->model != HLB_LB_D3Q19) return bset_error(b, HLB_ERR_PARAM, "box %d: the batched kernel runs D3Q19", i);
    b->par[i] = {lb->tau, lb->rho0, fe->A0, fe->gamma, fe->K, fe->q0, be->Gamma, be->xi, be->flow_coupling};
    b->have_params[i] = 1;
    b->dirty = true;
    return HLB_OK;
}

int hlb_batch_set_fields(hlb_batch *b, int i, const double *Q5, const double *u3, const double *rho)
{
    B_GUARD(b);
    if (i < 0 || i >= b->n || !Q5) return bset_error(b, HLB_ERR_ARG, "box %d", i);
    if (!b->have_params[i]) return bset_error(b, HLB_ERR_STATE, "box %d: parameters first", i);
    hlb::Device D = view(b, i);
    const size_t N = D.G.N;
    std::vector<double> host(9 * N);
    for (size_t s = 0; s < N; ++s) host[s] = rho ? rho[s] : b->par[i].rho0;
    if (u3)
        std::memcpy(host.data() + N, u3, 3 * N * sizeof(double));
    else
        std::fill(host.begin() + N, host.begin() + 4 * N, 0.0);
    std::memcpy(host.data() + 4 * N, Q5, 5 * N * sizeof(double));
    double *stage = static_cast<double *>(D.g[D.gcur ^ 1]);
    B_TRY(b, hipMemcpyAsync(stage, host.data(), 9 * N * sizeof(double), hipMemcpyHostToDevice, b->stream));
    B_TRY(b, hlb::run_init(D, b->par[i], stage));
    B_TRY(b, hipStreamSynchronize(b->stream));
    b->have_fields[i] = 1;
    return HLB_OK;
}

int hlb_batch_set_chunk(hlb_batch *b, int sites_of_box, int chunk)
{
    B_GUARD(b);
    if (chunk < kMinChunk || chunk % kMinChunk || sites_of_box < 1)
        return bset_error(b, HLB_ERR_ARG, "chunk %d must be a positive multiple of %d", chunk, kMinChunk);
    b->chunk_of_n[sites_of_box] = chunk;
    b->dirty = true;
    return HLB_OK;
}

int hlb_batch_set_launch(hlb_batch *b, int form, long long group_sites)
{
    B_GUARD(b);
    if (form != HLB_BATCH_PERSISTENT && form != HLB_BATCH_PHASES)
        return bset_error(b, HLB_ERR_ARG, "launch form %d", form);
    if (group_sites < 0) return bset_error(b, HLB_ERR_ARG, "group_sites %lld", group_sites);
    b->launch_form = form;
    if (group_sites > 0) b->group_sites = group_sites;
    b->dirty = true;
    drop_graph(b);
    return HLB_OK;
}

int hlb_batch_set_xcd_local(hlb_batch *b, int enable)
{
    B_GUARD(b);
    b->xcd_local = enable != 0;
    drop_graph(b);
    return HLB_OK;
}

int hlb_batch_step(hlb_batch *b, int nsteps)
{
    B_GUARD(b);
    if (nsteps < 0) return bset_error(b, HLB_ERR_ARG, "nsteps = %d", nsteps);
    if (b->dirty) {
        int rc = rebuild(b);
        if (rc) return rc;
    }
    if (nsteps == 0) return HLB_OK;
    B_TRY(b, enqueue(b, nsteps));
    advance_host_gcur(b, nsteps);
    return HLB_OK;
}

int hlb_batch_capture(hlb_batch *b, int nsteps)
{
    B_GUARD(b);
    if (nsteps < 1) return bset_error(b, HLB_ERR_ARG, "nsteps = %d", nsteps);
    if (!b->stream) return bset_error(b, HLB_ERR_ARG, "graph capture needs a non-null stream");
    if (b->dirty) {
        int rc = rebuild(b);
        if (rc) return rc;
    }
    drop_graph(b);
    B_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue(b, nsteps);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bset_error(b, HLB_ERR_HIP, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    B_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_steps = nsteps;
    return HLB_OK;
}

int hlb_batch_launch(hlb_batch *b)
{
    B_GUARD(b);
    if (!b->exec || b->dirty) return bset_error(b, HLB_ERR_STATE, "no captured graph (or boxes changed since)");
    B_TRY(b, hipGraphLaunch(b->exec, b->stream));
    advance_host_gcur(b, b->graph_steps);
    return HLB_OK;
}

int hlb_batch_sync(hlb_batch *b)
{
    B_GUARD(b);
    return check_err(b);
}

int hlb_batch_autotune(hlb_batch *b, int trial_steps, int *sizes_out, int *chunks_out, int max_out)
{
    B_GUARD(b);
    if (trial_steps < 1) return bset_error(b, HLB_ERR_ARG, "trial_steps = %d", trial_steps);
    if (b->dirty) {
        int rc = rebuild(b);
        if (rc) return rc;
    }
    // keep every box's state on the host; the trials advance it
    std::vector<std::vector<char>> saved(b->n);
    std::vector<int> g0 = b->gcur;
    for (int i = 0; i < b->n; ++i) {
        const hlb::Device D = view(b, i);
        const size_t N = D.G.N, e = b->fp32 ? 4 : 8;
        saved[i].resize(24 * N * e);
        B_TRY(b, hipMemcpyAsync(saved[i].data(), D.g[D.gcur], 19 * N * e, hipMemcpyDeviceToHost, b->stream));
        B_TRY(b, hipMemcpyAsync(saved[i].data() + 19 * N * e, D.Q[D.qcur], 5 * N * e, hipMemcpyDeviceToHost,
                                b->stream));
    }
    B_TRY(b, hipStreamSynchronize(b->stream));
    std::vector<int> sizes;
    for (int i = 0; i < b->n; ++i)
        if (std::find(sizes.begin(), sizes.end(), b->box[i].G.N) == sizes.end()) sizes.push_back(b->box[i].G.N);
    std::sort(sizes.begin(), sizes.end());
    const int cands[] = {256, 1024, 4096, 16384};
    hipEvent_t ea, eb;
    B_TRY(b, hipEventCreate(&ea));
    B_TRY(b, hipEventCreate(&eb));
    int rc = HLB_OK;
    // coordinate descent: the launch form (key -1), the cache-group budget
    // jointly with one chunk for every box size (key -2; the two interact
    // through the blocks per group; option k: budget 2^(19 + k % 5) sites
    // (k % 5 == 4: all boxes in one group), chunk 256 for k < 5 else 1024),
    // blocks per CU of the persistent form (key 0), then the chunk of each
    // box size in turn
    auto set_joint = [&](int k) {
        b->group_sites = (k % 5 == 4) ? (1ll << 40) : (1ll << (19 + k % 5));
        for (int N : sizes) b->chunk_of_n[N] = k < 5 ? 256 : 1024;
    };
    int joint = -1;
    std::vector<int> keys{-1, -2, 0};
    keys.insert(keys.end(), sizes.begin(), sizes.end());
    for (int N : keys) {
        if (N == 0 && b->launch_form != HLB_BATCH_PERSISTENT) continue;
        double best = 1e300;
        int pick = N == -1 ? b->launch_form
                 : N == -2 ? joint
                 : N == 0  ? b->bpc
                           : chunk_for(b, N);
        const std::vector<int> opts = N == -1 ? std::vector<int>{HLB_BATCH_PERSISTENT, HLB_BATCH_PHASES}
                                    : N == -2 ? std::vector<int>{0, 1, 2, 3, 4, 5, 6, 7, 8, 9}
                                    : N == 0  ? std::vector<int>{1, 2, 3, 4}
                                              : std::vector<int>(std::begin(cands), std::end(cands));
        for (int ch : opts) {
            if (N > 0 && ch > N && ch != 256) continue;
            if (N == -1)
                b->launch_form = ch;
            else if (N == -2)
                set_joint(ch);
            else if (N == 0)
                b->bpc = ch;
            else
                b->chunk_of_n[N] = ch;
            if ((rc = rebuild(b))) break;
            hipError_t e = enqueue(b, 1);
            advance_host_gcur(b, 1);
            if (e == hipSuccess) e = hipEventRecord(ea, b->stream);
            if (e == hipSuccess) e = enqueue(b, trial_steps);
            advance_host_gcur(b, trial_steps);
            if (e == hipSuccess) e = hipEventRecord(eb, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(eb);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
            if (e != hipSuccess) {
                rc = bset_error(b, HLB_ERR_HIP, "batch autotune: %s", hipGetErrorString(e));
                break;
            }
            if ((rc = check_err(b))) break;
            if (ms < best) {
                best = ms;
                pick = ch;
            }
        }
        if (rc) break;
        if (N == -1)
            b->launch_form = pick;
        else if (N == -2) {
            if (pick >= 0) set_joint(pick);
            joint = pick;
        } else if (N == 0)
            b->bpc = pick;
        else
            b->chunk_of_n[N] = pick;
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (rc) return rc;
    // restore the states (the device-side ping-pong index is rewritten by rebuild)
    b->gcur = g0;
    for (int i = 0; i < b->n; ++i) {
        const hlb::Device D = view(b, i);
        const size_t N = D.G.N, e = b->fp32 ? 4 : 8;
        B_TRY(b, hipMemcpyAsync(D.g[D.gcur], saved[i].data(), 19 * N * e, hipMemcpyHostToDevice, b->stream));
        B_TRY(b, hipMemcpyAsync(D.Q[D.qcur], saved[i].data() + 19 * N * e, 5 * N * e, hipMemcpyHostToDevice,
                                b->stream));
    }
    B_TRY(b, hipStreamSynchronize(b->stream));
    if ((rc = rebuild(b))) return rc;
    int k = 0;
    for (int N : sizes) {
        if (k < max_out) {
            if (sizes_out) sizes_out[k] = N;
            if (chunks_out) chunks_out[k] = b->chunk_of_n[N];
        }
        ++k;
    }
    return k;
}

int hlb_batch_get_fields(hlb_batch *b, int i, double *Q5, double *u3, double *rho)
{
    B_GUARD(b);
    if (i < 0 || i >= b->n) return bset_error(b, HLB_ERR_ARG, "box %d", i);
    if (!b->have_fields[i]) return bset_error(b, HLB_ERR_STATE, "box %d has no fields", i);
    int rc = check_err(b);
    if (rc) return rc;
    hlb::Device D = view(b, i);
    const size_t N = D.G.N;
    double *stage = static_cast<double *>(D.g[D.gcur ^ 1]);
    B_TRY(b, hlb::run_readout(D, b->par[i], stage, nullptr));
    if (rho) B_TRY(b, hipMemcpyAsync(rho, stage, N * 8, hipMemcpyDeviceToHost, b->stream));
    if (u3) B_TRY(b, hipMemcpyAsync(u3, stage + N, 3 * N * 8, hipMemcpyDeviceToHost, b->stream));
    if (Q5) B_TRY(b, hipMemcpyAsync(Q5, stage + 4 * N, 5 * N * 8, hipMemcpyDeviceToHost, b->stream));
    B_TRY(b, hipStreamSynchronize(b->stream));
    return HLB_OK;
}

int hlb_batch_get_totals(hlb_batch *b, int i, double *mass, double *mom3, double *free_energy)
{
    B_GUARD(b);
    if (i < 0 || i >= b->n) return bset_error(b, HLB_ERR_ARG, "box %d", i);
    if (!b->have_fields[i]) return bset_error(b, HLB_ERR_STATE, "box %d has no fields", i);
    int rc = check_err(b);
    if (rc) return rc;
    hlb::Device D = view(b, i);
    double r[5];
    B_TRY(b, hlb::run_readout(D, b->par[i], nullptr, D.res));
    B_TRY(b, hipMemcpyAsync(r, D.res, sizeof(r), hipMemcpyDeviceToHost, b->stream));
    B_TRY(b, hipStreamSynchronize(b->stream));
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(r[k])) return bset_error(b, HLB_ERR_NONFINITE, "box %d: non-finite total", i);
    if (mass) *mass = double(D.G.N) * b->par[i].rho0 + r[0];
    if (mom3)
        for (int a = 0; a < 3; ++a) mom3[a] = r[1 + a];
    if (free_energy) *free_energy = r[4];
    return HLB_OK;
}

int hlb_batch_info(const hlb_batch *b, int *grid, int *n_items)
{
    if (!b) return HLB_ERR_ARG;
    if (grid) *grid = b->launch_form == HLB_BATCH_PHASES ? b->n_items : b->grid;
    if (n_items) *n_items = b->n_items;
    return HLB_OK;
}

int hlb_batch_get_launch(const hlb_batch *b, int *form, long long *group_sites)
{
    if (!b || !form) return HLB_ERR_ARG;
    *form = b->launch_form;
    if (group_sites) *group_sites = b->group_sites;
    return HLB_OK;
}

int hlb_batch_xcd_local(hlb_batch *b, int *local)
{
    B_GUARD(b);
    if (!local) return bset_error(b, HLB_ERR_ARG, "null argument");
    int mis = 1;
    B_TRY(b, hipMemcpyAsync(&mis, b->d_misplaced, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    B_TRY(b, hipStreamSynchronize(b->stream));
    *local = (mis == 0 && b->launch_form == HLB_BATCH_PERSISTENT) ? 1 : 0;
    return HLB_OK;
}

const char *hlb_batch_last_error(const hlb_batch *b) { return b ? b->msg : "null batch"; }

void hlb_batch_destroy(hlb_batch *b)
{
    if (!b) return;
    drop_graph(b);
    delete b;
}

}  // extern "C"
