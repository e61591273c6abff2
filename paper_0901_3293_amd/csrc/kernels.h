// kernels.h -- internal interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <vector>

namespace hlb {

// Division of a site index by a run-time divisor d as a multiply-high and a
// shift (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, floor(n / d) = (umulhi(n, m) + n) >> l
// for every n < 2^31 (the sum then stays below 2^32).
struct FastDiv {
    unsigned m;
    int l;
};

inline FastDiv make_fastdiv(int d)
{
    int l = 0;
    while ((1ll << l) < d) ++l;
    const unsigned long long m = ((1ull << 32) * ((1ull << l) - (unsigned long long)d)) / (unsigned long long)d + 1;
    return FastDiv{unsigned(m), l};
}

__device__ __forceinline__ unsigned fastdiv(unsigned n, FastDiv f) { return (__umulhi(n, f.m) + n) >> f.l; }

struct Geom {
    int nx, ny, nz;
    int N;  // nx*ny*nz (< 2^30; one plane of N values < 4 GiB)
    FastDiv dx, dy;  // division by nx and ny
};

inline Geom make_geom(int nx, int ny, int nz)
{
    return Geom{nx, ny, nz, nx * ny * nz, make_fastdiv(nx), make_fastdiv(ny)};
}

// Fluid coupling (Sec. 2.1, 2.2): off (u == 0), the whole chemical stress as a
// body force, or the split of Eqs. (17)-(21).
enum Flow { FLOW_OFF = 0, FLOW_FORCE = 1, FLOW_SPLIT = 2 };

// Parameters of one run in FP64 (converted to the arithmetic type per launch).
// Lattice-Boltzmann scheme: D3Q19 BGK with second-order forcing (pull), or
// the paper's D3Q15 predictor-corrector (Sec. 2.2, Eq. (15)).
enum LbModel { LB_D3Q19 = 0, LB_D3Q15_PC = 1 };

struct PhysParams {
    double tau, rho0;
    double A0, gamma, K, q0;
    double Gamma, xi;
    int flow;   // Flow
    int model;  // LbModel
};

// Debug flags: fill the LDS planes of the tiled kernels with NaN before
// each plane is staged or evaluated into them, so a halo point that is never
// written surfaces as NaN in the results.
enum DebugFlags { DEBUG_NAN_LDS = 1 };

// Step schedules (see kernels.hip).
enum Schedule { SCHED_SITES = 0, SCHED_TILED = 1, SCHED_MIXED = 2, SCHED_FUSED = 3, SCHED_FUSED_TILED = 4 };

// Device buffers of one context (all inside the caller's workspace) and the
// ping-pong state indices.
struct Device {
    Geom G;
    bool fp32;
    void *g[2];    // 19 x N each; g[gcur] holds the state
    void *Q[2];    // 5 x N each; Q[qcur] holds the state
    void *u;       // 3 x N
    void *Pi;      // 12 x N: stress (9; F in its first 3 for the tiled schedule) or split terms (12)
    void *aux;     // 15 x N: predictor populations of the D3Q15 scheme (null otherwise)
    double *part;  // partial_doubles(nx, ny, nz)
    double *res;   // 16 doubles of reduced totals
    int gcur, qcur;
    int sched;     // Schedule
    int tz;        // z-chunk of the tiled kernels (0: default)
    int tzq;       // z-chunk of the tiled Q update (0: tz)
    int debug;     // debug flags (DEBUG_NAN_LDS)
    hipStream_t stream;
};

size_t partial_doubles(int nx, int ny, int nz);

// Kernel kinds of one step, for per-kernel event timing.
enum KernelKind {
    K_STRESS = 0, K_LB = 1, K_QPRED = 2, K_QCORR = 3,  // per-site schedule
    K_QFORCE = 4, K_LBF = 5, K_QUPDATE = 6,            // tiled schedule
    K_PC1 = 7, K_PC2 = 8,                              // D3Q15 predictor-corrector LB
    K_QLB = 9,                                         // stress fused with the LB step
    K_COUNT = 10
};
const char *kernel_name(int k);

struct KernelTimer {
    struct Mark {
        int kind;
        hipEvent_t start, stop;
    };
    std::vector<Mark> events;
};

// Enqueue nsteps coupled steps (flips D.gcur and D.qcur).  With a timer, an
// event pair is recorded on the stream around every launch.
hipError_t run_steps(Device &D, const PhysParams &p, int nsteps, KernelTimer *timer = nullptr);

// z-chunk of the tiled kernels whose blocks fill the current device's
// resident block slots `rounds` times over (0 if none does).
int tile_tz_fill(const Device &D, int rounds);

// stage: device FP64 [rho N][u 3N][Q 5N] (must not alias g[gcur] or Q[qcur]);
// writes g[gcur] and Q[qcur], zeroes u.
hipError_t run_init(Device &D, const PhysParams &p, const double *stage);

// Current-level readout into device FP64 stage [rho N][u 3N][Q 5N] (may be
// null) and, if totals is non-null, the reductions into totals[0..4]:
// totals[0] = sum (rho - rho0), totals[1..3] = sum rho u, totals[4] = sum f.
// The block partials of the reductions go to part (null: D.part), which
// needs readout_partials(G) doubles.
hipError_t run_readout(Device &D, const PhysParams &p, double *stage, double *totals, double *part = nullptr);
size_t readout_partials(const Geom &G);

// Plane sums of the free-energy density of the current Q into device fz[nz].
hipError_t run_fz(Device &D, const PhysParams &p, double *fz);

// Local order of the current Q into device buffers (any may be null; cnt
// needs defect): q[N] largest eigenvalue, dir[3][N] unit eigenvector,
// defect[N] = (q < threshold), cnt[nz] defect sites per z-plane (FP64).
hipError_t run_order(Device &D, double threshold, double *q, double *dir, unsigned char *defect, double *cnt);

// Polarised-light texture (Mueller retarder stack along z per column).
constexpr int OPTICS_MAX_WL = 8;
struct OpticsParams {
    double n_o, n_e, h;
    double c_in, s_in, c_out, s_out;  // cos, sin of twice the polariser / analyser angle
    int nwl;
    double lam[OPTICS_MAX_WL], w[OPTICS_MAX_WL];
};
// Segments per column for tm_bytes of transfer-matrix scratch (0: too small).
int optics_segments(const Geom &G, int nwl, size_t tm_bytes);
// image[ny][nx] (device, FP64): weighted S0 behind the analyser.  Tm: device
// scratch of tm_bytes (per-segment 3x3 transfer matrices), not aliasing image.
hipError_t run_optics(Device &D, const OpticsParams &op, double *Tm, size_t tm_bytes, double *image);

}  // namespace hlb
