// batch.hip -- many periodic boxes of uneven size, each with its own physical
// parameters, advanced by ONE persistent kernel launch per call.
//
// Work list: every box is cut into chunks of `chunk` consecutive sites; the
// chunks of all boxes form one list, split into 8 contiguous segments, one
// per XCD (workgroups reach the XCDs round-robin), and the blocks of an XCD
// take the items of its segment in turn.  One step is four phases over the
// list (stress, LB, predictor, corrector -- the per-site device functions of
// sitekern.h), separated by grid barriers.  The grid never exceeds the number
// of co-resident blocks; every barrier wait is bounded so that a stall ends
// the kernel with an error flag instead of hanging it.
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

// Grid-wide barrier over a monotonically increasing arrival counter.  Every
// thread publishes its writes at device scope before arriving; thread 0 polls
// with a bounded number of sleeps; afterwards every wave invalidates its
// caches so the next phase reads what other XCDs wrote.  Returns false (in
// every thread of the block) if the wait ran out or another block failed.
__device__ __forceinline__ bool grid_sync(unsigned *bar, int *err, unsigned &target, unsigned spin_limit)
{
    __threadfence();
    __syncthreads();
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        target += gridDim.x;
        atomicAdd(bar, 1u);
        int ok = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > spin_limit) {
                atomicMax(err, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        s_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return s_ok != 0;
}

enum Phase { PH_STRESS, PH_LB, PH_PRED, PH_CORR };

template <typename T, int PH>
__device__ __forceinline__ void run_phase(Rep<T> *__restrict__ reps, const int4 *__restrict__ items,
                                          int n_items, int step)
{
    const int per = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    const int seg = (n_items + 7) >> 3;
    const int lo = xcd * seg, hi = min(n_items, lo + seg);
    for (int it = lo + local; it < hi; it += per) {
        const int4 w = items[it];
        Rep<T> &R = reps[w.x];
        if ((PH == PH_STRESS || PH == PH_LB) && !R.flow) continue;
        const int gc = R.gcur ^ (step & 1);
        for (int s = w.y + int(threadIdx.x); s < w.y + w.z; s += BLK) {
            if (PH == PH_STRESS)
                stress_at(R.G, R.c, R.Q, R.Pi, s);
            else if (PH == PH_LB)
                lb_at(R.G, R.c, R.g[gc], R.Pi, R.g[gc ^ 1], R.u, s);
            else if (PH == PH_PRED)
                pred_at(R.G, R.c, R.Q, R.u, R.Qs, s);
            else
                corr_at(R.G, R.c, R.Q, R.Qs, R.u, s);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_batch(Rep<T> *__restrict__ reps, int n_reps, const int4 *__restrict__ items,
                                               int n_items, unsigned *bar, int *err, int nsteps,
                                               unsigned spin_limit)
{
    unsigned target = 0;
    for (int n = 0; n < nsteps; ++n) {
        run_phase<T, PH_STRESS>(reps, items, n_items, n);
        if (!grid_sync(bar, err, target, spin_limit)) return;
        run_phase<T, PH_LB>(reps, items, n_items, n);
        if (!grid_sync(bar, err, target, spin_limit)) return;
        run_phase<T, PH_PRED>(reps, items, n_items, n);
        if (!grid_sync(bar, err, target, spin_limit)) return;
        run_phase<T, PH_CORR>(reps, items, n_items, n);
        if (!grid_sync(bar, err, target, spin_limit)) return;
    }
    // every block has read gcur before the last barrier: advance it once
    if (blockIdx.x == 0 && (nsteps & 1))
        for (int r = threadIdx.x; r < n_reps; r += BLK)
            if (reps[r].flow) reps[r].gcur ^= 1;
}

__global__ void k_batch_reset(unsigned *bar, int *err)
{
    if (threadIdx.x == 0) {
        *bar = 0u;
        *err = 0;
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

hipError_t batch_grid(bool fp32, int n_items, int *grid)
{
    int dev = 0, per_cu = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<float>, BLK, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<double>, BLK, 0);
    if (e != hipSuccess) return e;
    int g = per_cu * cus;
    if (g > n_items) g = n_items;
    g = g / 8 * 8;
    if (g < 8) g = 8;
    if (g > per_cu * cus) return hipErrorInvalidConfiguration;  // fewer than 8 co-resident blocks
    *grid = g;
    return hipSuccess;
}

hipError_t batch_launch(bool fp32, void *d_reps, int n_reps, const int *d_items, int n_items, unsigned *d_bar,
                        int *d_err, int nsteps, int grid, hipStream_t stream)
{
    const unsigned spin_limit = 1u << 24;  // ~1 s of polling per barrier
    k_batch_reset<<<1, 64, 0, stream>>>(d_bar, d_err);
    const int4 *items = reinterpret_cast<const int4 *>(d_items);
    if (fp32)
        k_batch<float><<<grid, BLK, 0, stream>>>(static_cast<Rep<float> *>(d_reps), n_reps, items, n_items, d_bar,
                                                 d_err, nsteps, spin_limit);
    else
        k_batch<double><<<grid, BLK, 0, stream>>>(static_cast<Rep<double> *>(d_reps), n_reps, items, n_items,
                                                  d_bar, d_err, nsteps, spin_limit);
    return hipGetLastError();
}

}  // namespace hlb
