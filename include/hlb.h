/*
 * hlb.h -- C-ABI of the MI355X hybrid lattice-Boltzmann solver for
 * cholesteric liquid crystals (Henrich, Marenduzzo, Stratford, Cates,
 * "Domain growth in cholesteric blue phases: hybrid lattice Boltzmann
 * simulations").
 *
 * One time step (Sec. 2.2): the finite-difference side turns Q^n into the
 * chemical stress and its divergence (Sec. 2.1, Eqs. (1), (2), (6)-(8);
 * Sec. 2.2, Eq. (19)); a D3Q19 BGK lattice-Boltzmann collide-stream step with
 * that body force gives u^n (Sec. 2.2, Eqs. (14), (16)); a predictor-corrector
 * finite-difference step of the Beris-Edwards equation with the material
 * derivative and co-rotation (Sec. 2.1, Eqs. (2)-(4)) gives Q^{n+1}.
 * Lattice units dx = dt = 1, periodic in x, y and z.
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status (hlb_status): 0 on success, < 0 on
 *    error.  No C++ exception crosses this boundary.  Errors are sticky per
 *    context: after a failure every later call on that context returns the
 *    same code until hlb_destroy; hlb_last_error() gives the message.
 *  - Host arrays are FP64, structure-of-arrays, component-major
 *    [c][z][y][x] with x fastest (site index x + nx*(y + ny*z)).  Q uses the
 *    five stored components (xx, xy, xz, yy, yz); Q_zz = -Q_xx - Q_yy.
 *  - The caller owns the device workspace (hlb_workspace_bytes bytes, 256-byte
 *    aligned device memory) and the HIP stream; both must outlive the
 *    context.  The context owns only host-side metadata.
 *  - Work is enqueued on the caller's stream.  hlb_step returns before the
 *    GPU finishes; every hlb_get_* call synchronises that stream.
 *  - One context per stream; a context must not be used from two threads at
 *    once.
 */
#ifndef HLB_H
#define HLB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HLB_OK = 0,
    HLB_ERR_ARG = -1,       /* null pointer, bad size, bad enum            */
    HLB_ERR_PARAM = -2,     /* physical parameters outside their range     */
    HLB_ERR_HIP = -3,       /* a HIP runtime call failed                   */
    HLB_ERR_NONFINITE = -4, /* a reduction found NaN or Inf in the state   */
    HLB_ERR_STATE = -5,     /* call out of order (e.g. step before fields) */
    HLB_ERR_NOMEM = -6      /* workspace smaller than required             */
} hlb_status;

typedef enum { HLB_FP64 = 0, HLB_FP32 = 1 } hlb_precision;

/* Opaque solver context. */
typedef struct hlb_ctx hlb_ctx;

/* LB parameters (Sec. 2.2, Eq. (16)): relaxation time tau, reference density
 * rho0 (> 0) and the scheme:
 *   HLB_LB_D3Q19 (0): D3Q19 BGK, collide then pull-stream, second-order
 *     (Guo) forcing with u = (sum f e + F/2)/rho; tau > 1/2, kinematic
 *     viscosity (tau - 1/2)/3; populations stored as g_i = f_i - w_i rho0.
 *   HLB_LB_D3Q15_PC (1): the paper's own scheme -- D3Q15 (rest, 6 faces, 8
 *     corners), equilibrium and forcing term as the printed polynomial with
 *     the printed coefficients (T = 1/3; the stress term carries the split
 *     sigma^xi, the forcing term P_s b.e the body force), stepped by the
 *     predictor-corrector rule of Eq. (15); u = sum f e / rho (Eq. (14));
 *     tau > 0, kinematic viscosity tau/3; populations g_i = f_i - A_s(rho0)
 *     at their own site.  Single-box contexts, sites or mixed schedule.
 * Other values are rejected with HLB_ERR_PARAM. */
enum { HLB_LB_D3Q19 = 0, HLB_LB_D3Q15_PC = 1 };
typedef struct {
    double tau;
    double rho0;
    int model;
} hlb_lb_params;

/* Landau-de Gennes free energy (Sec. 2.1, Eq. (1)): bulk scale A0 (> 0),
 * control parameter gamma (> 0), one elastic constant K (>= 0) and q0 =
 * 2 pi / pitch.  The one-constant form adds K/2 (d_b Q_ab)^2 to the printed
 * chiral term. */
typedef struct {
    double A0;
    double gamma;
    double K;
    double q0;
} hlb_fe_params;

/* Beris-Edwards kinetics (Sec. 2.1, Eqs. (2)-(4)): rotational diffusion
 * constant Gamma (> 0), flow-aligning parameter xi, and the flow switch of
 * Sec. 2.1 with the choice of coupling:
 *   HLB_FLOW_OFF   (0) imposes u == 0 (pure relaxation; the LB state is left
 *                      untouched);
 *   HLB_FLOW_FORCE (1) couples the fluid through the centred divergence of the
 *                      whole chemical stress of Eqs. (6)-(8) as a body force;
 *   HLB_FLOW_SPLIT (2) the split coupling of Sec. 2.2, Eqs. (17)-(21): the
 *                      symmetric xi-stress sigma^xi enters the second moment
 *                      of the equilibrium, the body force is
 *                      b_a = d_b tau_ab - H:d_a Q (tau the antisymmetric
 *                      stress), which vanishes with H, so an equilibrium
 *                      structure has no spurious flow.  Single-box contexts
 *                      with any schedule but HLB_SCHED_TILED.
 * Other values are rejected with HLB_ERR_PARAM. */
enum { HLB_FLOW_OFF = 0, HLB_FLOW_FORCE = 1, HLB_FLOW_SPLIT = 2 };
typedef struct {
    double Gamma;
    double xi;
    int flow_coupling;
} hlb_be_params;

/* Bytes of device workspace a context of this size and precision needs for
 * the default model: the D3Q19 LB with the fluid off or coupled through the
 * whole chemical stress -- populations 2 x 19, Q 2 x 5, u 3 and the stress 9
 * values per site (60), plus reduction partials.  hlb_workspace_bytes_for
 * gives the size for another LB model and coupling: the split coupling
 * (HLB_FLOW_SPLIT) needs 3 more values per site (63), the D3Q15 scheme
 * (HLB_LB_D3Q15_PC) 15 more for its predicted populations (75 with the whole
 * stress, 78 split) (Sec. 2.2: the hybrid scheme's small per-site state).
 * Returns 0 if the arguments are invalid (any n < 4, unknown precision, LB
 * model or coupling, or a lattice too large to index: nx*ny*nz >= 2^30
 * sites, or one field plane of nx*ny*nz values of 4 GiB or more, i.e. FP64
 * lattices of 2^29 sites and above). */
size_t hlb_workspace_bytes(int nx, int ny, int nz, int precision);
size_t hlb_workspace_bytes_for(int nx, int ny, int nz, int precision, int lb_model, int flow_coupling);

/* Create a context on the current HIP device for an nx*ny*nz periodic lattice
 * (each n >= 4).  device_workspace: caller-owned device memory of
 * workspace_bytes bytes, 256-byte aligned, at least hlb_workspace_bytes()
 * (HLB_ERR_NOMEM otherwise); the LB model and coupling later set with
 * hlb_set_params must fit in it (hlb_workspace_bytes_for).  hip_stream: a hipStream_t (may be
 * NULL for the null stream).  On success *out receives the context. */
int hlb_create(int nx, int ny, int nz, int precision, void *device_workspace,
               size_t workspace_bytes, void *hip_stream, hlb_ctx **out);

/* Map the reduced chirality kappa and reduced temperature tau of Sec. 2.1,
 * Eqs. (9)-(10), with given q0 and A0, to (A0, gamma, K, q0):
 *   gamma = 27 / (tau + 9),   K = kappa^2 A0 gamma / (108 q0^2).
 * Host arithmetic only; needs no context.  Errors: HLB_ERR_ARG for a null out,
 * HLB_ERR_PARAM for q0 == 0, A0 <= 0 or tau <= -9. */
int hlb_fe_from_reduced(double kappa, double tau_ldg, double q0, double A0,
                        hlb_fe_params *out);

/* Set all physical parameters.  Rejected with HLB_ERR_PARAM: tau <= 1/2
 * (D3Q19) or <= 0 (D3Q15), rho0 <= 0, A0 <= 0, gamma <= 0, K < 0,
 * Gamma <= 0, the explicit diffusion bound 12 Gamma K >= 2 of the
 * forward-Euler predictor, an unknown flow_coupling or LB model;
 * HLB_ERR_STATE for the split coupling while HLB_SCHED_TILED is selected, or
 * the D3Q15 scheme while HLB_SCHED_TILED, HLB_SCHED_FUSED or
 * HLB_SCHED_FUSED_TILED is; HLB_ERR_NOMEM if the context's workspace is smaller
 * than hlb_workspace_bytes_for this model and coupling.  Must be called
 * before hlb_set_fields; changing the LB model invalidates the fields (call
 * hlb_set_fields again). */
int hlb_set_params(hlb_ctx *ctx, const hlb_lb_params *lb, const hlb_fe_params *fe,
                   const hlb_be_params *be);

/* Load the state from host FP64 arrays: Q5 [5][N], u3 [3][N], rho [N].  The
 * populations are stored so that the first pull of the next step returns the
 * equilibrium f^eq(rho, u) at every site; a readout straight after this call
 * reports u + F/(2 rho) (F from Q).  u3 or rho may be NULL (fluid at rest,
 * rho = rho0).  Synchronous. */
int hlb_set_fields(hlb_ctx *ctx, const double *Q5, const double *u3, const double *rho);

/* Enqueue nsteps coupled steps on the context's stream (nsteps >= 0). */
int hlb_step(hlb_ctx *ctx, int nsteps);

/* Read the current time level into host FP64 arrays (any may be NULL):
 * Q5 [5][N]; u3 [3][N] = (sum_i f_i e_i + F/2)/rho with F from the current Q
 * (zero with flow off); rho [N].  Synchronises the stream. */
int hlb_get_fields(hlb_ctx *ctx, double *Q5, double *u3, double *rho);

/* FP64 totals at the current level: mass sum rho, momentum sum rho u (3),
 * total free energy sum f.  Fixed-order two-stage device reduction.
 * HLB_ERR_NONFINITE if any total is NaN or Inf.  Synchronises the stream. */
int hlb_get_totals(hlb_ctx *ctx, double *mass, double *mom3, double *free_energy);

/* hlb_get_totals for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same totals, reduced by the same kernels in the same order (so bitwise
 * equal to hlb_get_totals), with the block partials and totals kept in a
 * static device array of 4 MiB that the library holds per device until the
 * process ends, instead of the context's workspace.  It allocates nothing
 * (no hipMalloc, hipFree or allocating library call); the stress planes of
 * the context's own workspace still carry the force term of the momentum.
 * Lattices of at most 26,843,136 sites; larger ones fail with HLB_ERR_NOMEM
 * (sticky, like every error) before any GPU work.  The context's device must
 * be current.  All calls on one device share its array: calls that overlap
 * on one device (other threads, other streams) race and must be serialised
 * by the caller.  Synchronises the stream. */
int hlb_get_totals_noalloc(hlb_ctx *ctx, double *mass, double *mom3, double *free_energy);

/* Free-energy profile along z: fz[z] = sum over the plane z of the
 * free-energy density (Eq. (1)) of the current Q, FP64, fixed-order per-plane
 * reduction; the domain-wall position of a slab run is read off this profile.
 * fz: host array of nz doubles.  Synchronises the stream. */
int hlb_get_fz(hlb_ctx *ctx, double *fz);

/* Local order and disclinations of the current Q (Sec. 2.1): q[N] the largest
 * eigenvalue of Q (the local magnitude of order), dir3[3][N] a unit
 * eigenvector of it (the director of Sec. 2.3; sign: last non-zero component
 * positive; (0, 0, 1) where Q = 0), defect[N] = 1 where q < threshold (a
 * disclination site; the paper's runs use 0.19) else 0, defects_z[nz] the
 * number of disclination sites per z-plane, *n_defect their total.  Computed
 * on the device in FP64 from the stored Q (cyclic Jacobi rotations); host
 * outputs, any of them NULL.  Errors: HLB_ERR_ARG for a non-finite threshold,
 * HLB_ERR_STATE without fields.  Synchronises the stream. */
int hlb_get_order(hlb_ctx *ctx, double threshold, double *q, double *dir3, unsigned char *defect,
                  long long *defects_z, long long *n_defect);

/* Polarised-light texture of the current Q (Sec. 2.3, Mueller-matrix method),
 * light along +z entering at z = 0, unpolarised before the polariser: every
 * lattice site is a layer of thickness h acting as a linear retarder whose
 * axis is the projection of the director d on the (x, y) plane (angle beta
 * to x) and whose retardance is
 *   delta = 2 pi q h / lambda (n_o n_e / sqrt(n_o^2 sin^2 alpha + n_e^2 cos^2 alpha) - n_o),
 * cos alpha = d_z, q the local order (both as in hlb_get_order, FP64).
 * Polariser and analyser are linear at angles phi_in and phi_out to x
 * (0 and pi/2: crossed).  image[ny][nx] (host, FP64) receives the weighted
 * sum over the wavelengths of the first Stokes component behind the
 * analyser.  The paper's values: n_o = 1.5, n_e = 2.0, h = 1, wavelengths
 * 16, 18, 20 with weights 0.2, 0.6, 0.2.  Errors: HLB_ERR_ARG for null
 * pointers, non-positive indices, thickness or wavelengths, non-finite
 * angles or weights, or a wavelength count outside 1..8; HLB_ERR_STATE
 * without fields.  Synchronises the stream. */
#define HLB_OPTICS_MAX_WAVELENGTHS 8
typedef struct {
    double n_o, n_e;
    double h;
    double phi_in, phi_out;
    int n_wavelengths;
    double wavelength[HLB_OPTICS_MAX_WAVELENGTHS];
    double weight[HLB_OPTICS_MAX_WAVELENGTHS];
} hlb_optics_params;
int hlb_get_optics(hlb_ctx *ctx, const hlb_optics_params *params, double *image);

/* Raw checkpoint of the state (populations and Q in the context's precision).
 * hlb_state_bytes gives the size; get/set copy exactly that many bytes. */
size_t hlb_state_bytes(hlb_ctx *ctx);
int hlb_get_state(hlb_ctx *ctx, void *host_buf, size_t nbytes);
int hlb_set_state(hlb_ctx *ctx, const void *host_buf, size_t nbytes);

/* Step schedules.  HLB_SCHED_SITES: four sweeps with one lattice site per
 * thread (stress to HBM, LB with its divergence, predictor, corrector in
 * place).  HLB_SCHED_TILED: three sweeps in which 2.5D z-marching LDS tiles
 * hold the stress and the predictor stage (recomputed on a one-site halo
 * ring; tiles of 32 x 8 sites in FP32 and 16 x 12 in FP64), tz planes per
 * tile column (0: 16).  HLB_SCHED_MIXED: the per-site stress and LB sweeps,
 * then the tiled predictor-corrector.  HLB_SCHED_FUSED: the tiled stress
 * fused with the LB step (the force never leaves the CU), then the per-site
 * predictor and corrector.  HLB_SCHED_FUSED_TILED: the fused stress and LB
 * step, then the tiled predictor-corrector (two sweeps).  All give the same
 * step to rounding.  The default is HLB_SCHED_SITES.  With the D3Q15
 * scheme, HLB_SCHED_TILED, HLB_SCHED_FUSED and HLB_SCHED_FUSED_TILED are
 * rejected (HLB_ERR_STATE), with the split coupling HLB_SCHED_TILED (its
 * stress kernel writes the whole-stress force; the fused kernel evaluates
 * the split terms and the split body force in its tiles). */
enum {
    HLB_SCHED_SITES = 0,
    HLB_SCHED_TILED = 1,
    HLB_SCHED_MIXED = 2,
    HLB_SCHED_FUSED = 3,
    HLB_SCHED_FUSED_TILED = 4
};
int hlb_set_schedule(hlb_ctx *ctx, int schedule, int tz);
int hlb_get_schedule(const hlb_ctx *ctx, int *schedule, int *tz);

/* z-chunk of the tiled predictor-corrector (HLB_SCHED_TILED, HLB_SCHED_MIXED,
 * HLB_SCHED_FUSED_TILED) where it should differ from the schedule's tz
 * (0: the schedule's tz; hlb_set_schedule resets it to 0).  The step is the
 * same at any chunk to rounding (bitwise in FP64).  HLB_ERR_ARG for tzq < 0. */
int hlb_set_update_chunk(hlb_ctx *ctx, int tzq);
int hlb_get_update_chunk(const hlb_ctx *ctx, int *tzq);

/* Debug flags.  HLB_DEBUG_NAN_LDS: the tiled kernels (the tiled stress and
 * the tiled Q update of every schedule but HLB_SCHED_SITES) overwrite every
 * LDS plane with NaN before
 * staging a lattice plane into it or evaluating the stress or the predictor
 * stage into it, so a halo point the kernels fail to write surfaces as NaN
 * in Q, u and the totals (HLB_ERR_NONFINITE) instead of a stale value; the
 * results are otherwise unchanged.  For testing the tile halos only: the
 * fills cost time.  flags = 0 turns it off; HLB_ERR_ARG for unknown bits. */
enum { HLB_DEBUG_NAN_LDS = 1 };
int hlb_set_debug(hlb_ctx *ctx, int flags);

/* Autotuner: time trial_steps steps of every candidate schedule (per-site;
 * tiled, mixed, fused and fused-tiled with tz = 8, 16, 32 and the tz whose
 * tiled launch fills the device's resident block slots once or twice; only
 * the per-site and mixed schedules with the D3Q15 scheme, no tiled one with
 * the split coupling) on this context's lattice and precision with HIP events
 * on its stream, in two passes over the candidates (each scored by its faster
 * pass, 2 untimed steps before every trial), keep the fastest; if that is
 * HLB_SCHED_TILED or HLB_SCHED_FUSED_TILED, time the other chunks for the Q
 * update the same way (hlb_set_update_chunk) and keep a faster one; put the
 * state back as it was (through a host copy of hlb_state_bytes bytes).
 * *best_ms_per_step (may be NULL) receives the winner's time per step.
 * Synchronises the stream. */
int hlb_autotune(hlb_ctx *ctx, int trial_steps, double *best_ms_per_step);

/* Diagnostics: enqueue nsteps steps with a HIP event pair recorded on the
 * context's stream around every kernel launch, wait for them, and add each
 * kernel kind's elapsed milliseconds into kernel_ms[k] (zeroed first;
 * nkernels >= the number of kinds).  Returns the number of kernel kinds
 * (>= 1) on success, < 0 on error.  The state advances exactly as with
 * hlb_step.  hlb_kernel_name(k) names kind k ("" past the last). */
int hlb_step_timed(hlb_ctx *ctx, int nsteps, double *kernel_ms, int nkernels);
const char *hlb_kernel_name(int k);

/* ------------------------------------------------------------------------
 * Batched form: n periodic boxes of uneven size, each with its own
 * parameters (e.g. a scan of chirality kappa and reduced temperature tau,
 * Sec. 2.1, Eqs. (9)-(10)), advanced together: four ordinary kernels per
 * step over all boxes, or one persistent kernel per call
 * (hlb_batch_set_launch).  The step of every box is the per-site schedule
 * above (same device code), so a box gives the same result as a single
 * context on it.  Each box is cut into work items of `chunk` sites.  In the
 * persistent form the items of a group of boxes are spread over the
 * co-resident blocks of that group and the four phases of a step are
 * separated by barriers among them whose waits are bounded (a stall ends the
 * launch with an error, reported by the next hlb_batch_sync / readout as
 * HLB_ERR_HIP).
 * ------------------------------------------------------------------------ */
typedef struct hlb_batch hlb_batch;

/* dims: n triples (nx, ny, nz), each >= 4, each box within the size limits
 * of hlb_workspace_bytes.  Returns 0 for invalid input. */
size_t hlb_batch_workspace_bytes(int n, const int *dims, int precision);
int hlb_batch_create(int n, const int *dims, int precision, void *device_workspace, size_t workspace_bytes,
                     void *hip_stream, hlb_batch **out);
/* Per box i in [0, n): same validation as hlb_set_params / hlb_set_fields;
 * flow_coupling must be HLB_FLOW_OFF or HLB_FLOW_FORCE and the LB model
 * HLB_LB_D3Q19 (HLB_ERR_PARAM). */
int hlb_batch_set_params(hlb_batch *b, int i, const hlb_lb_params *lb, const hlb_fe_params *fe,
                         const hlb_be_params *be);
int hlb_batch_set_fields(hlb_batch *b, int i, const double *Q5, const double *u3, const double *rho);
/* Sites per work item for boxes of `sites_of_box` sites (multiple of 256;
 * default 1024). */
int hlb_batch_set_chunk(hlb_batch *b, int sites_of_box, int chunk);
/* Launch form of a batched step.  HLB_BATCH_PERSISTENT: one persistent
 * kernel per call; the boxes are packed into 8 groups of about
 * equal site count, one per XCD, the workgroups of a group separate the four
 * phases of a step by barriers among themselves, and each group takes its
 * boxes in cache groups of at most group_sites / 8 sites (a larger box
 * alone), all steps of the call on one cache group before the next.
 * HLB_BATCH_PHASES (default): four ordinary kernels per step (stress, LB, predictor,
 * corrector), one block per work item, ordered by the stream (meant for graph
 * capture); the boxes are packed in index order into cache groups of at most
 * group_sites sites and all steps of a call run on one group before the
 * next.  Either way a cache group's fields stay in the last-level cache
 * across steps (group_sites = 0 keeps the current budget, default 2^21).
 * Results are identical; drops a captured graph. */
enum { HLB_BATCH_PERSISTENT = 0, HLB_BATCH_PHASES = 1 };
int hlb_batch_set_launch(hlb_batch *b, int form, long long group_sites);
int hlb_batch_get_launch(const hlb_batch *b, int *form, long long *group_sites);
/* Autotuner: coordinate descent over the launch form, the cache-group
 * budget (2^19 .. 2^22 sites, or all boxes in one group) jointly with one
 * chunk (256 or 1024) for all sizes, the blocks per CU of the persistent
 * form (1..4) and, for each distinct box size, chunks of 256, 1024, 4096 and
 * 16384 sites, timing trial_steps batched steps with HIP events on the batch
 * stream and keeping the fastest; the states are put back afterwards (host
 * copies).  Writes up to max_out (size, chunk) pairs; returns the number of
 * sizes. */
int hlb_batch_autotune(hlb_batch *b, int trial_steps, int *sizes_out, int *chunks_out, int max_out);
/* enable = 1 (default): keep each box on one XCD (boxes packed into 8 groups of
 * about equal site count; the workgroups on XCD x take group x), so the phase
 * barriers need not write the XCD's L2 back to memory.  enable = 0: groups
 * follow blockIdx and every barrier uses device-scope fences.  Results are
 * identical; drops a captured graph. */
int hlb_batch_set_xcd_local(hlb_batch *b, int enable);
/* Enqueue nsteps steps of every box in the selected launch form. */
int hlb_batch_step(hlb_batch *b, int nsteps);
/* Capture the launch of nsteps steps (either form) into a HIP graph;
 * hlb_batch_launch replays it (nsteps more steps per replay).  Changing any
 * box's parameters or chunk afterwards requires a new capture.  Capture needs
 * a non-null stream (HLB_ERR_ARG otherwise). */
int hlb_batch_capture(hlb_batch *b, int nsteps);
int hlb_batch_launch(hlb_batch *b);
/* Wait for the batch stream and check the barrier error flag. */
int hlb_batch_sync(hlb_batch *b);
/* Readout of box i at the current level (as hlb_get_fields / hlb_get_totals). */
int hlb_batch_get_fields(hlb_batch *b, int i, double *Q5, double *u3, double *rho);
int hlb_batch_get_totals(hlb_batch *b, int i, double *mass, double *mom3, double *free_energy);
/* Grid size of the launch (persistent: co-resident blocks; phases: one block
 * per work item) and number of work items. */
int hlb_batch_info(const hlb_batch *b, int *grid, int *n_items);
/* After a launch (synchronises): *local = 1 if the last launch kept every box
 * on one XCD (workgroups take the group of the XCD they run on), so its phase
 * barriers skipped the L2 write-back; 0 if some XCD got no workgroup and the
 * launch fell back to a fixed mapping with device-scope fences.  Results are
 * identical either way. */
int hlb_batch_xcd_local(hlb_batch *b, int *local);
const char *hlb_batch_last_error(const hlb_batch *b);
void hlb_batch_destroy(hlb_batch *b);

/* ------------------------------------------------------------------------
 * Learned surrogate: a 3D convolutional network that advances Q by k solver
 * steps in one application.  Four 3x3x3 convolutions with periodic padding,
 * channels 18 -> 32 -> 32 -> 32 -> 5, bias, ReLU after the first three;
 * bfloat16 operands on the matrix cores, FP32 accumulation.
 *
 * Inputs per site (NIN = 18, FP32): Q (xx, xy, xz, yy, yz), u (x, y, z) of
 * the last LB step, the last increment d1 = Q(t) - Q(t-k) and its change
 * s2 = Q(t) - 2 Q(t-k) + Q(t-2k).  Output: the standardised correction c of
 * the increment over the next k steps with respect to the extrapolation base,
 *     dQ = d1 + beta s2 + (c std_out + mean_out),
 * beta = 0 (linear extrapolation base) or 1 (quadratic).  The history (d1,
 * s2) is kept by the network object for one solver context; it is recorded
 * from plain steps (hlbnn_warmup, fallbacks, checked jumps) and advanced by
 * the network's own jumps.  Any call that changes the solver's state or
 * parameters from outside (hlb_set_fields, hlb_step, ...) invalidates it.
 *
 * Parameters: one flat FP32 vector, layer by layer, each layer's weights
 * W[c_out][c_in][kz][ky][kx] (tap kz*9+ky*3+kx reads offset (kx-1,ky-1,kz-1))
 * followed by its bias; hlbnn_param_count() values (75269).
 * Standardisation block (hlbnn_norm_size() = 47 floats): [0..17] input
 * means, [18..35] input stds (> 0), [36..40] target means, [41..45] target
 * stds (> 0), [46] beta.
 * Device arrays are FP32 structure-of-arrays [c][z][y][x]: inputs x [18][N],
 * increments dq [5][N].  Training and inference calls use the network's
 * stream; calls that take a solver context run on the solver's stream.
 * Errors are reported on the network (hlbnn_last_error) and are sticky.
 * ------------------------------------------------------------------------ */
typedef struct hlbnn hlbnn;

int hlbnn_param_count(void);
int hlbnn_input_channels(void);
int hlbnn_norm_size(void);
size_t hlbnn_workspace_bytes(int nx, int ny, int nz);
/* device_workspace: caller-owned, 256-byte aligned, at least
 * hlbnn_workspace_bytes(); HLB_ERR_NOMEM if smaller, HLB_ERR_ARG for a bad
 * lattice or a misaligned or null workspace. */
int hlbnn_create(int nx, int ny, int nz, void *device_workspace, size_t workspace_bytes, void *hip_stream,
                 hlbnn **out);
/* Host FP32 parameters in / out (setting them resets the Adam moments). */
int hlbnn_set_params(hlbnn *nn, const float *params);
int hlbnn_get_params(hlbnn *nn, float *params);
/* Host FP32 gradient of the last training step (same layout as the parameters). */
int hlbnn_get_grads(hlbnn *nn, float *grads);
/* Standardisation block in / out (host, hlbnn_norm_size() floats); stds
 * must be positive and all values finite (HLB_ERR_PARAM). */
int hlbnn_set_norm(hlbnn *nn, const float *norm);
int hlbnn_get_norm(hlbnn *nn, float *norm);
/* Per-channel mean and standard deviation of nsamples device arrays
 * [nsamples][nch][N] (FP64 sums). */
int hlbnn_channel_stats(hlbnn *nn, const float *data_dev, int nch, int nsamples, double *mean, double *std_out);
/* Standardisation from nsamples training pairs x [nsamples][18][N] and dq
 * [nsamples][5][N]: input statistics of x, target statistics of
 * dq - d1 - beta s2; sets it on the network and copies it to norm_out
 * (host, may be NULL). */
int hlbnn_fit_norm(hlbnn *nn, const float *x_dev, const float *dq_dev, int nsamples, float beta, float *norm_out);
/* 2k plain steps of the solver (same lattice), recording the history for
 * jumps of k steps. */
int hlbnn_warmup(hlbnn *nn, hlb_ctx *solver, int k);
/* Host copies of the history d1, s2 ([5][N] FP32 each) for the solver's
 * current state; HLB_ERR_STATE if there is none. */
int hlbnn_history(hlbnn *nn, const hlb_ctx *solver, float *d1, float *s2);
/* Host copy x [18][N] of the network inputs for the solver's current state
 * and the history (exactly what the next jump reads); HLB_ERR_STATE without
 * a valid history. */
int hlbnn_inputs(hlbnn *nn, const hlb_ctx *solver, float *x);
/* One training pair: x_dev [18][N] = the inputs at the solver's current
 * state (after a warm-up of 2k steps when there is no valid history), then k
 * plain steps, dq_dev [5][N] = Q(t+k) - Q(t).  The history stays valid. */
int hlbnn_make_pair(hlbnn *nn, hlb_ctx *solver, int k, float *x_dev, float *dq_dev);
/* dq_dev = predicted increment for raw inputs x_dev. */
int hlbnn_predict(hlbnn *nn, const float *x_dev, float *dq_dev);
/* One unchecked network jump on the solver: Q += dQ, history advanced
 * (s2 = dQ - d1, d1 = dQ); populations and u untouched. */
int hlbnn_jump(hlbnn *nn, hlb_ctx *solver);
/* One training step on one pair: mean-squared error between the network
 * output and the standardised target (dq - d1 - beta s2 - mean) / std,
 * backward pass (bfloat16 operands, FP32 accumulation, FP64 fixed-order
 * reduction of the weight gradient), Adam (beta1 0.9, beta2 0.999, eps
 * 1e-8) with learning rate lr.  *loss (may be NULL; reading it
 * synchronises) receives the loss before the update. */
int hlbnn_train_step(hlbnn *nn, const float *x_dev, const float *dq_dev, float lr, double *loss);
/* The gradient of one training step (as hlbnn_train_step: same kernels in
 * the same order, but no Adam update and no change to the parameters), with
 * what the kernels passed between layers copied to host arrays, so each
 * layer can be checked on exactly the operands it received:
 * acts_host [4][N][32] bfloat16 bits, the input of each layer (layer 0: the
 * standardised inputs, channels 18..31 zero); y_host [N][5] FP32, the
 * standardised output of the last layer; dz_host [4][N][32] bfloat16 bits,
 * the loss gradient with respect to each layer's pre-activation output
 * (layer l uses the first N x cout_padded(l) values of its slot: 32, and 16
 * for the last layer); grad_host the flat gradient (hlbnn_param_count()
 * floats).  Synchronises the network's stream. */
int hlbnn_grad_trace(hlbnn *nn, const float *x_dev, const float *dq_dev, unsigned short *acts_host, float *y_host,
                     unsigned short *dz_host, float *grad_host);
/* Single-layer entry points (host arrays) used to check the kernels layer by
 * layer: x_bf16 [N][32] bfloat16 bits (channels beyond the layer's inputs
 * zero); z [N][c_out] FP32 = conv + bias; dz_bf16 [N][cout_padded] (32, or 16
 * for the last layer); dx [N][32] FP32 = transposed convolution of dz (may
 * be NULL); grad = the layer's flat weight and bias gradient. */
int hlbnn_layer_forward(hlbnn *nn, int layer, const unsigned short *x_bf16, float *z);
int hlbnn_layer_backward(hlbnn *nn, int layer, const unsigned short *x_bf16, const unsigned short *dz_bf16,
                         float *dx, float *grad);
const char *hlbnn_last_error(const hlbnn *nn);
void hlbnn_destroy(hlbnn *nn);

/* One surrogate cycle of M >= 2 jumps of k steps on the solver's stream,
 * the network holding a valid history for this solver and k (HLB_ERR_STATE
 * otherwise).  Keeps a checkpoint of the state; takes M-1 network jumps (the
 * populations and u are held during a jump); for the M-th jump takes the
 * network's increment dq and, from the same state, k plain steps; residual
 * r = ||Q_pre + dq - Q_plain|| / ||Q_plain|| over the five stored components
 * (FP64 sums).  r < threshold: the cycle is accepted, the state is the plain
 * result of the last jump and the history its increment.  Otherwise
 * (*fell_back = 1) the state is rolled back to the checkpoint and the whole
 * cycle is taken with M*k plain steps, the history recorded over its last
 * two jumps.  threshold = 0 therefore reproduces the plain run bit for bit.
 * Either way the simulated time advances by M*k steps.  Synchronises once
 * (to read r).  Errors are reported on nn. */
int hlb_surrogate_advance(hlb_ctx *solver, hlbnn *nn, int k, int M, double threshold, int *fell_back,
                          double *residual);

/* Message of the last error on this context ("" if none). Never NULL. */
const char *hlb_last_error(const hlb_ctx *ctx);

/* Release the context (the workspace and stream stay with the caller). */
void hlb_destroy(hlb_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* HLB_H */
