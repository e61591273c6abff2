// batch.hip -- many periodic boxes of uneven size, each with its own physical
// parameters, advanced by ONE persistent kernel launch per call.
//
// Work list: every box is cut into chunks of `chunk` consecutive sites; the
// boxes are packed into 8 groups of about equal site count, one per XCD.  At
// the start of a launch every workgroup reads the XCD it runs on and draws a
// rank among the workgroups of that XCD; the workgroups of an XCD then claim
// the items of its group one at a time from the group's counter, so each box
// is read and written by one XCD only (if some XCD got no workgroup, the
// launch falls back to a fixed blockIdx mapping and device-scope fences).  One step is four phases over
// the items (stress, LB, predictor, corrector -- the per-site device
// functions of sitekern.h), separated by barriers among the workgroups of
// the group: the groups hold disjoint boxes and never wait for each other.
// A group takes its boxes in cache groups, every step of the launch on one
// cache group before the next, so that its fields stay in the caches.  The
// grid never exceeds the number of co-resident blocks; every barrier wait is
// bounded so that a stall ends the kernel with an error flag instead of
// hanging it.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "sitekern.h"

namespace hlb {

namespace {

constexpr int BLK = 256;

template <typename T>
struct Rep {
    Geom G;
    Coef<T> c;
    T *g[2];
    T *Q, *Qs, *u, *Pi;
    int flow;
    int gcur;  // ping-pong index of the populations, advanced on the device
};

// Barrier over `per` workgroups (the whole grid, or the workgroups of one
// work-list group) on a monotonically increasing arrival counter.  The
// block's stores are complete at the workgroup barrier; thread 0 then
// publishes them at device scope (one L2 write-back per block), arrives,
// polls with a bounded number of sleeps, and acquires at device scope (one
// cache invalidation per block, shared by the CU's waves) so the next phase
// reads what other XCDs wrote.  Returns false (in every thread of the block)
// if the wait ran out or another block failed.
//
// With `local` (every block runs on the XCD its work-list group belongs to,
// checked at the start of the launch) a phase's results only have to reach
// the L2 of their own XCD, which all its CUs share: each wave waits until its
// own stores are acknowledged (by that L2) before the workgroup barrier, and
// the L2 write-back of the device-scope release is skipped.  The acquire
// stays at device scope: it is what is sure to drop the CU's stale L1 lines.
__device__ __forceinline__ bool group_sync(unsigned *bar, int *err, unsigned &target, unsigned per,
                                           unsigned spin_limit, bool local)
{
    if (local) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores have reached L2
    __syncthreads();
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        if (!local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        target += per;
        atomicAdd(bar, 1u);
        int ok = 1;
        unsigned spins = 0;
        // the counter and the target wrap together after 2^32 arrivals: compare
        // their difference (the group never lags by 2^31 arrivals)
        while (int(__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > spin_limit) {
                atomicMax(err, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Hardware XCD (XCC) of the executing workgroup.
__device__ __forceinline__ int xcc_id()
{
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(v));
    return int(v);
}

enum Phase { PH_STRESS, PH_LB, PH_PRED, PH_CORR };

// The work item and its box descriptor are the same for the whole block;
// moving them into scalar registers keeps the stencil addressing at one VGPR
// per access (base in SGPRs) instead of 64-bit per-lane addresses.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ double uni(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = unsigned(__builtin_amdgcn_readfirstlane(int(b & 0xffffffffll)));
    const unsigned hi = unsigned(__builtin_amdgcn_readfirstlane(int(b >> 32)));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// A device-memory pointer made wave-uniform.  It is rebuilt through a
// global-address-space pointer: rebuilt as a plain (generic) pointer, the
// compiler could no longer tell that it points to global memory and would
// address every access through flat instructions with 64-bit per-lane
// addresses instead of a scalar base and a 32-bit offset.
template <typename P>
__device__ __forceinline__ P *uni(P *p)
{
    const unsigned long long b = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = unsigned(__builtin_amdgcn_readfirstlane(int(b & 0xffffffffull)));
    const unsigned hi = unsigned(__builtin_amdgcn_readfirstlane(int(b >> 32)));
    using GP = __attribute__((address_space(1))) P *;
    return (P *)(GP)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ FastDiv uni(const FastDiv &f)
{
    return FastDiv{unsigned(__builtin_amdgcn_readfirstlane(int(f.m))), uni(f.l)};
}

template <typename T>
__device__ __forceinline__ Coef<T> uni(const Coef<T> &c)
{
    Coef<T> r;
    r.a = uni(c.a);
    r.bg = uni(c.bg);
    r.K = uni(c.K);
    r.q0x2 = uni(c.q0x2);
    r.Kq0x2 = uni(c.Kq0x2);
    r.Kq0sq4 = uni(c.Kq0sq4);
    r.xi = uni(c.xi);
    r.Gamma = uni(c.Gamma);
    r.rho0 = uni(c.rho0);
    r.omega = uni(c.omega);
    r.pref = uni(c.pref);
    return r;
}

// The items [lo, hi) of this block's group, taken by its `per` blocks in
// turn starting at `rank`.  STREAM: nontemporal population loads and stores
// in the LB phase (see pop_load in sitekern.h), which both launch forms use:
// the populations are read and written once per step, and streaming them
// leaves the last-level cache to the cache group's Q, u and stress.
template <typename T, int PH, bool STREAM = false>
__device__ __forceinline__ void run_phase(Rep<T> *__restrict__ reps, const int4 *__restrict__ items, int lo, int hi,
                                          int rank, int per, int step)
{
#pragma unroll 1
    for (int it = lo + rank; it < hi; it += per) {
        const int4 w4 = items[it];
        const int box = uni(w4.x), first = uni(w4.y), count = uni(w4.z);
        const Rep<T> &R = reps[box];
        if ((PH == PH_STRESS || PH == PH_LB) && !uni(R.flow)) continue;
        const int gc = uni(R.gcur) ^ (step & 1);
        const Geom G = {uni(R.G.nx), uni(R.G.ny), uni(R.G.nz), uni(R.G.N), uni(R.G.dx), uni(R.G.dy)};
        const Coef<T> c = uni(R.c);
        T *__restrict__ Q = uni(R.Q);
        T *__restrict__ Qs = uni(R.Qs);
        T *__restrict__ u = uni(R.u);
        T *__restrict__ Pi = uni(R.Pi);
        const T *__restrict__ gin = uni(R.g[gc]);
        T *__restrict__ gout = uni(R.g[gc ^ 1]);
#pragma unroll 1
        for (int s = first + int(threadIdx.x); s < first + count; s += BLK) {
            if (PH == PH_STRESS)
                stress_at(G, c, Q, Pi, s);
            else if (PH == PH_LB)
                lb_at<T, STREAM>(G, c, gin, Pi, gout, u, s);
            else if (PH == PH_PRED)
                pred_at(G, c, Q, u, Qs, s);
            else
                corr_at(G, c, Q, Qs, u, s);
        }
    }
}

// Barrier counters of the 8 work-list groups, one per 64-byte line; the
// group's 64-bit item counter sits in the same line, 8 bytes in.
constexpr int GBAR_STRIDE = 16;
constexpr int GCTR_OFFSET = 2;

// The items [lo, hi) of a group, claimed one at a time by the group's `per`
// blocks from the group's counter, so a block that finishes early takes more
// (the static round-robin left blocks waiting up to half their time at the
// barriers).  Phase instance m of the group owns the counter values
// [base, base + n + per): the first n claims name items, and every block
// stops after its first claim past them, so exactly `per` claims overshoot
// and the next instance starts at base + n + per.  Thread 0 claims the next
// item while the block works on the current one; the claim goes to LDS
// (two slots, one barrier per item).
template <typename T, int PH>
__device__ __forceinline__ void run_phase_claimed(Rep<T> *__restrict__ reps, const int4 *__restrict__ items, int lo,
                                                  int hi, unsigned long long *ctr, unsigned long long base,
                                                  int step, int *s_item)
{
    const unsigned long long n = (unsigned long long)(hi - lo);
    auto claim = [&]() {
        const unsigned long long v = __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return (v - base < n) ? int(v - base) : -1;
    };
    if (threadIdx.x == 0) s_item[0] = claim();
    __syncthreads();
    int slot = 0;
    int it = s_item[0];
#pragma unroll 1
    while (it >= 0) {
        int nxt = -1;
        if (threadIdx.x == 0) nxt = claim();
        run_phase<T, PH, true>(reps, items, lo + it, lo + it + 1, 0, 1, step);
        if (threadIdx.x == 0) s_item[slot ^ 1] = nxt;
        __syncthreads();
        slot ^= 1;
        it = s_item[slot];
    }
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_batch(Rep<T> *__restrict__ reps, const int4 *__restrict__ items,
                                               const int *__restrict__ xlo, const int *__restrict__ slo,
                                               const int *__restrict__ sgx, unsigned *bar, unsigned *gbar, int *err,
                                               int *misplaced, int *xcnt, int allow_local, int nsteps,
                                               unsigned spin_limit)
{
    unsigned target = 0;
    // Rank of this block among the blocks of its XCD; after one full barrier
    // every block sees the same per-XCD counts and takes the same decision.
    __shared__ int s_rank;
    const int xcd = xcc_id();
    if (threadIdx.x == 0) s_rank = xcd < 8 ? atomicAdd(&xcnt[xcd], 1) : (atomicOr(misplaced, 1), 0);
    if (!group_sync(bar, err, target, gridDim.x, spin_limit, false)) return;
    bool local = allow_local && __hip_atomic_load(misplaced, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    for (int x = 0; x < 8; ++x)
        if (__hip_atomic_load(&xcnt[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) local = false;
    int grp, rank, per;
    if (local) {
        grp = xcd;
        rank = s_rank;
        per = __hip_atomic_load(&xcnt[xcd], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        grp = blockIdx.x & 7;
        rank = blockIdx.x >> 3;
        per = gridDim.x >> 3;
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(misplaced, 1);  // report the fallback
    }
    // The groups hold disjoint boxes, so each synchronises only its own
    // workgroups; it takes its boxes in cache groups (all steps of one before
    // the next), so a cache group's fields stay in the caches across steps.
    unsigned gtarget = 0;
    unsigned *gb = gbar + grp * GBAR_STRIDE;
    auto *ctr = reinterpret_cast<unsigned long long *>(gb + GCTR_OFFSET);
    __shared__ int s_item[2];
    unsigned long long base = 0;
    for (int j = sgx[grp]; j < sgx[grp + 1]; ++j) {
        const int lo = slo[j], hi = slo[j + 1];
        const unsigned long long span = (unsigned long long)(hi - lo) + per;
        for (int n = 0; n < nsteps; ++n) {
            run_phase_claimed<T, PH_STRESS>(reps, items, lo, hi, ctr, base, n, s_item);
            base += span;
            if (!group_sync(gb, err, gtarget, per, spin_limit, local)) return;
            run_phase_claimed<T, PH_LB>(reps, items, lo, hi, ctr, base, n, s_item);
            base += span;
            if (!group_sync(gb, err, gtarget, per, spin_limit, local)) return;
            run_phase_claimed<T, PH_PRED>(reps, items, lo, hi, ctr, base, n, s_item);
            base += span;
            if (!group_sync(gb, err, gtarget, per, spin_limit, local)) return;
            run_phase_claimed<T, PH_CORR>(reps, items, lo, hi, ctr, base, n, s_item);
            base += span;
            if (!group_sync(gb, err, gtarget, per, spin_limit, local)) return;
        }
    }
    // every block of the group has read gcur of its boxes before the group's
    // last barrier: the group's first block advances it once per box
    if (rank == 0 && (nsteps & 1))
        for (int it = xlo[grp] + int(threadIdx.x); it < xlo[grp + 1]; it += BLK) {
            const int4 w = items[it];
            if (w.y == 0 && reps[w.x].flow) reps[w.x].gcur ^= 1;
        }
}

// The alternative launch form: one ordinary kernel per phase, one block per
// work item, stream order in place of the grid barriers (each phase kernel
// holds only its own registers, so more waves are resident).
// Blocks reach the XCDs round-robin; block b takes item (b % 8) * (grid / 8)
// + b / 8, so consecutive items (neighbouring site ranges of a box) run on
// one XCD and share its L2 for the stencil reads.  The grid is a multiple of
// 8; blocks past the last item return.
template <typename T, int PH>
__global__ __launch_bounds__(BLK) void k_phase(Rep<T> *__restrict__ reps, const int4 *__restrict__ items,
                                               int first, int n_items, int step)
{
    const int it = int(blockIdx.x & 7) * int(gridDim.x >> 3) + int(blockIdx.x >> 3);
    if (it >= n_items) return;
    run_phase<T, PH, true>(reps, items, first + it, first + it + 1, 0, 1, step);
}

// Advance the device ping-pong index of every box with flow after an odd
// number of steps of phase kernels.
template <typename T>
__global__ void k_flip(Rep<T> *__restrict__ reps, int n_reps)
{
    const int r = blockIdx.x * BLK + int(threadIdx.x);
    if (r < n_reps && reps[r].flow) reps[r].gcur ^= 1;
}

__global__ void k_batch_reset(unsigned *bar, int *err, int *misplaced, int *xcnt, unsigned *gbar)
{
    if (threadIdx.x == 0) {
        *bar = 0u;
        *err = 0;
        *misplaced = 0;
    }
    if (threadIdx.x < 8) {
        xcnt[threadIdx.x] = 0;
        if (gbar) {
            gbar[threadIdx.x * GBAR_STRIDE] = 0u;
            *reinterpret_cast<unsigned long long *>(gbar + threadIdx.x * GBAR_STRIDE + GCTR_OFFSET) = 0ull;
        }
    }
}

template <typename T>
void fill_reps(const std::vector<Device> &box, const std::vector<PhysParams> &par, const std::vector<int> &gcur,
               std::vector<char> &blob)
{
    blob.resize(box.size() * sizeof(Rep<T>));
    Rep<T> *r = reinterpret_cast<Rep<T> *>(blob.data());
    for (size_t i = 0; i < box.size(); ++i) {
        const Device &D = box[i];
        r[i].G = D.G;
        r[i].c = make_coef<T>(par[i]);
        r[i].g[0] = static_cast<T *>(D.g[0]);
        r[i].g[1] = static_cast<T *>(D.g[1]);
        r[i].Q = static_cast<T *>(D.Q[D.qcur]);
        r[i].Qs = static_cast<T *>(D.Q[D.qcur ^ 1]);
        r[i].u = static_cast<T *>(D.u);
        r[i].Pi = static_cast<T *>(D.Pi);
        r[i].flow = par[i].flow;
        r[i].gcur = gcur[i];
    }
}

}  // namespace

size_t batch_rep_bytes(bool fp32) { return fp32 ? sizeof(Rep<float>) : sizeof(Rep<double>); }

void batch_pack_reps(bool fp32, const std::vector<Device> &box, const std::vector<PhysParams> &par,
                     const std::vector<int> &gcur, std::vector<char> &blob)
{
    if (fp32)
        fill_reps<float>(box, par, gcur, blob);
    else
        fill_reps<double>(box, par, gcur, blob);
}

hipError_t batch_grid(bool fp32, int n_items, int blocks_per_cu, int *grid)
{
    int dev = 0, per_cu = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<float>, BLK, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<double>, BLK, 0);
    if (e != hipSuccess) return e;
    if (blocks_per_cu > 0 && blocks_per_cu < per_cu) per_cu = blocks_per_cu;
    int g = per_cu * cus;
    if (g > n_items) g = n_items;
    g = g / 8 * 8;
    if (g < 8) g = 8;
    if (g > per_cu * cus) return hipErrorInvalidConfiguration;  // fewer than 8 co-resident blocks
    *grid = g;
    return hipSuccess;
}

hipError_t batch_launch(bool fp32, void *d_reps, const int *d_items, const int *d_xlo, const int *d_slo,
                        const int *d_sgx, unsigned *d_bar, unsigned *d_gbar, int *d_err, int *d_misplaced,
                        int *d_xcnt, bool allow_local, int nsteps, int grid, hipStream_t stream)
{
    // polls per barrier before giving up: each sleeps ~50 ns and waits for one
    // device-scope load, so a stalled barrier is abandoned after about 1-10 s
    const unsigned spin_limit = 1u << 24;
    k_batch_reset<<<1, 64, 0, stream>>>(d_bar, d_err, d_misplaced, d_xcnt, d_gbar);
    const int4 *items = reinterpret_cast<const int4 *>(d_items);
    if (fp32)
        k_batch<float><<<grid, BLK, 0, stream>>>(static_cast<Rep<float> *>(d_reps), items, d_xlo, d_slo, d_sgx,
                                                 d_bar, d_gbar, d_err, d_misplaced, d_xcnt, int(allow_local),
                                                 nsteps, spin_limit);
    else
        k_batch<double><<<grid, BLK, 0, stream>>>(static_cast<Rep<double> *>(d_reps), items, d_xlo, d_slo, d_sgx,
                                                  d_bar, d_gbar, d_err, d_misplaced, d_xcnt, int(allow_local),
                                                  nsteps, spin_limit);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_phases_t(void *d_reps, int n_reps, const int *d_items, const int *clo, int ngroups, int nsteps,
                           hipStream_t st)
{
    Rep<T> *reps = static_cast<Rep<T> *>(d_reps);
    const int4 *items = reinterpret_cast<const int4 *>(d_items);
    for (int c = 0; c < ngroups; ++c) {  // every step of one cache group, then the next
        const int first = clo[c], n_items = clo[c + 1] - clo[c];
        if (n_items < 1) continue;
        const int grid = (n_items + 7) / 8 * 8;
        for (int n = 0; n < nsteps; ++n) {
            k_phase<T, PH_STRESS><<<grid, BLK, 0, st>>>(reps, items, first, n_items, n);
            k_phase<T, PH_LB><<<grid, BLK, 0, st>>>(reps, items, first, n_items, n);
            k_phase<T, PH_PRED><<<grid, BLK, 0, st>>>(reps, items, first, n_items, n);
            k_phase<T, PH_CORR><<<grid, BLK, 0, st>>>(reps, items, first, n_items, n);
        }
    }
    if (nsteps & 1) k_flip<T><<<(n_reps + BLK - 1) / BLK, BLK, 0, st>>>(reps, n_reps);
    return hipGetLastError();
}

hipError_t batch_launch_phases(bool fp32, void *d_reps, int n_reps, const int *d_items, const int *clo, int ngroups,
                               unsigned *d_bar, int *d_err, int *d_misplaced, int *d_xcnt, int nsteps,
                               hipStream_t stream)
{
    k_batch_reset<<<1, 64, 0, stream>>>(d_bar, d_err, d_misplaced, d_xcnt, nullptr);
    if (ngroups < 1 || nsteps < 1) return hipGetLastError();
    return fp32 ? launch_phases_t<float>(d_reps, n_reps, d_items, clo, ngroups, nsteps, stream)
                : launch_phases_t<double>(d_reps, n_reps, d_items, clo, ngroups, nsteps, stream);
}

}  // namespace hlb
