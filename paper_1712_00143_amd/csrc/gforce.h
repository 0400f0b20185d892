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

// The x-y-z tile a block of that grid takes for its tile index, a
// permutation of [0, ntile): when a tile is two whole x rows (L0 = 32) and
// L1, L2 are multiples of 8, each run of 32 consecutive tiles covers 8 y rows
// by 8 z planes instead of two whole z planes, so that the blocks an XCD
// holds at once read fewer neighbour planes of other blocks; otherwise the
// identity.
__device__ __forceinline__ int brick_tile(int tile, const SmearGeom &g)
{
    if (g.L[0] != 32 || (g.L[1] & 7) || (g.L[2] & 7)) return tile;
    const int rows = g.L[1] >> 1, nby = g.L[1] >> 3;   // tiles per z plane, y bricks
    const int b = tile >> 5, q = tile & 31;
    const int zb = b / nby, yb = b - zb * nby;
    return (zb * 8 + (q >> 2)) * rows + yb * 4 + (q & 3);
}

hipError_t launch_gauge_force(const SmearGeom &g, const GForceArgs &a, int mode, hipStream_t s);

}  // namespace hisq
