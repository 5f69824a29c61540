// Launch wrapper of the hyperboloidal layer's kernels (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include "tk_layer.h"

namespace tk {

// One step of a context holding at least one layered instance.  Fused: one
// launch of both stages (one wave per work item of 62 output columns from i0,
// its lanes holding columns i0 - 1 .. i0 + 62), else two launches, Eq. (3)
// into the half-step array and Eq. (4) (one wave per work item of 64 columns
// from i0); then the null-infinity node of each layered instance (the linear
// extrapolation of the new values at the two nodes before it).  Work items
// march rows [j0, j1); a chunk holding a pole row must be at least three rows
// long.  The coefficients are the layer's (separate outgoing and ingoing
// speeds, rescaled Pi~ equation) where d_lay[k] has a table, the plain ones
// elsewhere.  Buffers as for launch_two_pass.
// fp64: FP64 storage, else FP32-compensated storage (single pass only; the
// layer's columns are computed in FP64 on the stored values either way;
// hipErrorInvalidValue for the two passes).
hipError_t launch_layer(bool fp64, bool fused, const DevInst *d_inst, const LayerInst *d_lay, int n_inst,
                        const WorkItem *d_work, int n_work, const DevCtl *ctl, int kstep, int kflip, hipStream_t s);

// Output columns per work item of the fused and of the two-pass layer kernels.
constexpr int kLayerFusedCols = 62;
constexpr int kLayerCols = 64;

// Rows per chunk of the two-pass layer kernels' work list when the tuning
// gives none, and of the single-pass layer kernel's beside the fused kernel.
constexpr int kLayerRows = 16;
constexpr int kLayerSplitRows = 8;

}  // namespace tk
