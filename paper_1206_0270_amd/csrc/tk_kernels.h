// Launch wrappers of the HIP kernels (host-callable, no HIP device code here).
#pragma once

#include <hip/hip_runtime.h>

#include "tk_internal.h"

namespace tk {

// Two-pass step (half-step array through HBM).  d_blocks[b] = {instance,
// block index within the instance}; one 256-thread block per 256 points of
// the instance's n_theta x n_r grid.
hipError_t launch_two_pass(const DevInst *d_inst, const int2 *d_blocks, int n_blocks, const DevCtl *ctl, int kstep,
                           hipStream_t s);

// Fused step: both Lax-Wendroff stages in one pass over theta-marching
// column strips.  d_work[w] = work item of wave w; waves_per_block waves of
// 64 lanes per block.
// prefetch: u^n rows in flight per wave (1 or 3); nt: non-temporal stores;
// waves: occupancy target per SIMD (1 = compiler's choice, 3, 4).  Returns
// hipErrorInvalidValue for a combination that is not compiled.
hipError_t launch_fused_fp64(const DevInst *d_inst, const WorkItem *d_work, int n_work, const DevCtl *ctl, int kstep,
                             int prefetch, bool nt, int waves, hipStream_t s);
hipError_t launch_fused_fp32c(const DevInst *d_inst, const WorkItem *d_work, int n_work, const DevCtl *ctl, int kstep,
                              int prefetch, bool nt, int waves, hipStream_t s);

// ctl->step += n
hipError_t launch_bump(DevCtl *ctl, int n, hipStream_t s);

// Output columns per fused work item (64 lanes minus the two halo lanes).
constexpr int kFusedCols = 62;
constexpr int kFusedWavesPerBlock = 4;

}  // namespace tk
