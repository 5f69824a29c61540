// Launch wrapper of the hyperboloidal layer's kernels (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include "tk_layer.h"

namespace tk {

// One step of a context holding at least one layered instance in the
// layer's two passes (FP64): Eq. (3) into the half-step array and Eq. (4),
// one wave per work item of kLayerCols columns from i0 marching rows
// [j0, j1) (a chunk holding a pole row is at least three rows long); then
// the null-infinity node of each layered instance (the linear extrapolation
// of the new values at the two nodes before it).  The coefficients are the
// layer's (separate outgoing and ingoing speeds, rescaled Pi~ equation)
// where d_lay[k] has a table, the plain ones elsewhere.  Buffers as for
// launch_two_pass.
hipError_t launch_layer(const DevInst *d_inst, const LayerInst *d_lay, int n_inst, const WorkItem *d_work, int n_work,
                        const DevCtl *ctl, int kstep, int kflip, hipStream_t s);

// Output columns per work item of the two-pass layer kernels, and rows per
// chunk when the tuning gives none.
constexpr int kLayerCols = 64;
constexpr int kLayerRows = 16;

}  // namespace tk
