// Launch wrapper of the hyperboloidal layer's kernels (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include "tk_layer.h"

namespace tk {

// Two-pass step of a context holding at least one layered instance: Eq. (3)
// into the half-step array, then Eq. (4) with the layer's coefficients
// (separate outgoing and ingoing speeds, rescaled Pi~ equation); the last
// node of a layered instance takes the linear extrapolation of the new
// values at the two nodes before it.  Blocks and buffers as for
// launch_two_pass; d_lay[k] describes instance k.
hipError_t launch_layer(const DevInst *d_inst, const LayerInst *d_lay, const int2 *d_blocks, int n_blocks,
                        const DevCtl *ctl, int kstep, int kflip, hipStream_t s);

}  // namespace tk
