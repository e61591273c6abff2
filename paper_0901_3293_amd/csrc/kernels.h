// kernels.h -- internal interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <vector>

namespace hlb {

struct Geom {
    int nx, ny, nz;
    int N;  // nx*ny*nz (< 2^31)
};

// Parameters of one run in FP64 (converted to the arithmetic type per launch).
struct PhysParams {
    double tau, rho0;
    double A0, gamma, K, q0;
    double Gamma, xi;
    int flow;
};

// Device buffers of one context (all inside the caller's workspace).
struct Device {
    Geom G;
    bool fp32;
    void *g[2];    // 19 x N each
    void *Q;       // 5 x N
    void *Qs;      // 5 x N
    void *u;       // 3 x N
    void *Pi;      // 9 x N
    double *part;  // partial_doubles(N)
    double *res;   // 16 doubles of reduced totals
    hipStream_t stream;
};

size_t partial_doubles(int N);

// Kernel kinds of one step, for per-kernel event timing.
enum KernelKind { K_STRESS = 0, K_LB = 1, K_QPRED = 2, K_QCORR = 3, K_COUNT = 4 };
const char *kernel_name(int k);

struct KernelTimer {
    struct Mark {
        int kind;
        hipEvent_t start, stop;
    };
    std::vector<Mark> events;
};

// Enqueue nsteps coupled steps; cur is the index of the g buffer holding the
// state and is flipped by every LB step.  With a timer, an event pair is
// recorded on the stream around every launch.
hipError_t run_steps(const Device &D, const PhysParams &p, int nsteps, int &cur,
                     KernelTimer *timer = nullptr);

// stage: device FP64 [rho N][u 3N][Q 5N]; writes g[cur] and Q, zeroes u.
hipError_t run_init(const Device &D, const PhysParams &p, const double *stage, int cur);

// Current-level readout into device FP64 stage [rho N][u 3N][Q 5N] (may be
// null) and, if totals is non-null, the reductions into D.res:
// res[0] = sum (rho - rho0), res[1..3] = sum rho u, res[4] = sum f.
hipError_t run_readout(const Device &D, const PhysParams &p, int cur, double *stage, double *totals);

}  // namespace hlb
