// Launcher of the Symanzik gauge force / action kernel (FP64).
#pragma once
#include <hip/hip_runtime.h>

#include "smear.h"

namespace hisq {

// U: four-direction planar thin links (see smear.h).  mode 0: F (four
// planar fields) = scale * TA[U_mu(x) B_mu(x)^+], B the sum of the loop-
// closing paths from x to x+mu weighted cp (plaquettes), cr (rectangles),
// cg (parallelograms).  mode 1: part[blk] = sum over the block's links of
// Re Tr U_mu(x) B_mu(x)^+ (one value per block of gauge_force_grid).
// Every extent must be >= 4.
struct GForceArgs {
    const double2 *U;
    double2 *F;
    double *part;
    double cp, cr, cg;
    double scale;
    int ntile, tch;   // set by the launcher
};

// Grid of the kernel (and of the smearing's pass 1): ntile tiles of 64
// x-y-z sites times runs of tch time slices; nblocks (= the number of
// action partials).
void gauge_force_grid(const SmearGeom &g, int *ntile, int *tch, int *nblocks);

hipError_t launch_gauge_force(const SmearGeom &g, const GForceArgs &a, int mode, hipStream_t s);

}  // namespace hisq
