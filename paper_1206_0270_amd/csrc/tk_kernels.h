// Launch wrappers of the HIP kernels (host-callable, no HIP device code here).
#pragma once

#include <hip/hip_runtime.h>

#include "tk_internal.h"

namespace tk {

// Two-pass step (half-step array through HBM).  d_blocks[b] = {instance,
// block index within the instance}; one 256-thread block per 256 points of
// the instance's n_theta x n_r grid.  The state is read from buffer
// (ctl->cur + kflip) & 1 and written to the other one.
hipError_t launch_two_pass(const DevInst *d_inst, const int2 *d_blocks, int n_blocks, const DevCtl *ctl, int kstep,
                           int kflip, hipStream_t s);

// Launch shape of the fused kernels: u^n rows in flight per wave (1 or 3),
// non-temporal stores, occupancy target per SIMD (1 = the compiler's choice,
// the only one compiled), one or two time steps per pass, and for two steps
// whole strips or chunks of rows.
struct FusedShape {
    int prefetch;
    bool nt;
    int waves;
    bool two_step;
    bool chunked;  // two steps on chunks of rows (k_fused2c) rather than whole strips
};

// Fused step(s): both Lax-Wendroff stages in one pass over theta-marching
// column strips.  d_work[w] = work item of wave w; kFusedWavesPerBlock waves
// of 64 lanes per block.  One step: the strips are `cols` output columns
// wide (at most kFusedCols) and may be split in rows; two steps: strips of
// kFused2Cols columns over all rows.  Buffers as for the two-pass step.
// Returns hipErrorInvalidValue for a shape that is not compiled.  layered
// (FP64 only): the instances may end in hyperboloidal layers (the layer's
// coefficients beyond rho = R, the null-infinity column extrapolated inside
// the march); the work list must keep each layered instance's last column at
// least two columns into a strip's output columns.  The layered form is
// compiled with one u^n row in flight (the prefetch depth is ignored).
hipError_t launch_fused(bool fp64, const DevInst *d_inst, const WorkItem *d_work, int n_work, int cols,
                        const DevCtl *ctl, int kstep, int kflip, const FusedShape &f, hipStream_t s,
                        bool layered = false);

// One step on tiles: one block of kFusedWavesPerBlock waves per work item
// (strips of kFusedCols columns split into chunks of `rows` rows, 4 or 8),
// with the tile's u^n and half rows staged in LDS.  Bitwise the results of
// launch_fused's one-step shapes.  hipErrorInvalidValue for other row counts.
hipError_t launch_tiled(bool fp64, const DevInst *d_inst, const WorkItem *d_work, int n_work, int rows,
                        const DevCtl *ctl, int kstep, int kflip, bool nt, hipStream_t s);

// ctl->step += n; ctl->cur flips `flips` times
hipError_t launch_bump(DevCtl *ctl, int n, int flips, hipStream_t s);

// Output columns per fused work item: 64 lanes minus one halo lane per side
// and time step.
constexpr int kFusedCols = 62;
constexpr int kFused2Cols = 60;
// Rows per chunk of a marching strip that reaches a hyperboloidal layer when
// the other strips run whole.
constexpr int kLayerStripRows = 32;
constexpr int kFusedWavesPerBlock = 4;

}  // namespace tk
