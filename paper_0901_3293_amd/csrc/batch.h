// batch.h -- internal interface of the batched persistent kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "kernels.h"

namespace hlb {

// Size of one box descriptor on the device and packing of the descriptor
// table (box views, parameters, population ping-pong indices).
size_t batch_rep_bytes(bool fp32);
void batch_pack_reps(bool fp32, const std::vector<Device> &box, const std::vector<PhysParams> &par,
                     const std::vector<int> &gcur, std::vector<char> &blob);

// Largest grid (multiple of 8, at most n_items) whose blocks are all
// co-resident on the current device, with at most blocks_per_cu blocks per
// compute unit (0: as many as fit).
hipError_t batch_grid(bool fp32, int n_items, int blocks_per_cu, int *grid);

// Enqueue: reset the barrier counters and flags (a one-block kernel, so the
// pair can be captured in a graph) and run the persistent kernel for nsteps
// steps.  d_items holds int4 {box, first site, site count, 0} per work item,
// grouped by XCD: group x is items [d_xlo[x], d_xlo[x + 1]), and every box
// lies in one group; the workgroups running on XCD x take group x.  Each
// group is cut into cache groups, items [d_slo[j], d_slo[j + 1]) for j in
// [d_sgx[x], d_sgx[x + 1]); all nsteps steps of a cache group run before the
// next, and the workgroups of a group synchronise among themselves (counter
// d_gbar[16 x]) and claim the items of each phase from the group's 64-bit
// counter (d_gbar + 16 x + 2).  d_xcnt: 8 ints of scratch (workgroups per XCD).
// d_misplaced: flag set when some XCD got no workgroup or allow_local is
// false; that launch then maps groups to blockIdx and uses device-scope
// fences throughout.
hipError_t batch_launch(bool fp32, void *d_reps, const int *d_items, const int *d_xlo, const int *d_slo,
                        const int *d_sgx, unsigned *d_bar, unsigned *d_gbar, int *d_err, int *d_misplaced,
                        int *d_xcnt, bool allow_local, int nsteps, int grid, hipStream_t stream);

// The same steps as four ordinary kernels per step (stress, LB, predictor,
// corrector), one block per work item, in stream order (no grid barriers;
// meant to be captured in a graph), plus the reset of the flags (so
// hlb_batch_sync sees a clean error flag).  The work list is cut into
// ngroups cache groups, items [clo[c], clo[c + 1]) (host array); all nsteps
// steps of group c are enqueued before group c + 1 (the boxes are
// independent), so a group's fields stay in the last-level cache.
hipError_t batch_launch_phases(bool fp32, void *d_reps, int n_reps, const int *d_items, const int *clo, int ngroups,
                               unsigned *d_bar, int *d_err, int *d_misplaced, int *d_xcnt, int nsteps,
                               hipStream_t stream);

}  // namespace hlb
