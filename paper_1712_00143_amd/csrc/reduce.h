// Deterministic per-problem reductions inside a kernel.
//
// Every tile (64 sites) writes NPART double partials; the last tile of a
// problem to finish (ticket counter in SolveState) sums that problem's
// partials in a fixed order and runs a finisher on the FP64 totals.  The sum
// order depends only on the tile count, so results are bitwise reproducible.
#pragma once
#include "hisq_dev.h"

namespace hisq {

// Block-wide sum of NV doubles per thread (result valid in thread 0).
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV], double *lds /* >= 16*NV */)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < NV; k++) lds[wave * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < NV; k++) {
            double s = 0;
            for (int w = 0; w < nw; w++) s += lds[w * NV + k];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Publish this tile's partials; returns true in every thread of the block
// that is the last tile of its problem, with totals[] (in thread 0) the
// fixed-order sum over the problem's tiles.
template <int NV>
__device__ __forceinline__ bool publish_and_reduce(double mine[NV], double *partials, int tile,
                                                   const ProbDesc &pd, SolveState *st,
                                                   double totals[NV])
{
    __shared__ double lds[16 * NV];
    __shared__ int is_last;
    block_sum<NV>(mine, lds);
    if (threadIdx.x == 0) {
        for (int k = 0; k < NV; k++) partials[(size_t)tile * NPART + k] = mine[k];
        __threadfence();
        unsigned t = atomicAdd(&st->counter, 1u);
        is_last = (t == (unsigned)pd.ntile - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) acc[k] = 0.0;
    for (int j = threadIdx.x; j < pd.ntile; j += blockDim.x) {
        const double *p = partials + (size_t)(pd.tile_begin + j) * NPART;
#pragma unroll
        for (int k = 0; k < NV; k++) acc[k] += p[k];
    }
    block_sum<NV>(acc, lds);
    if (threadIdx.x == 0) {
        for (int k = 0; k < NV; k++) totals[k] = acc[k];
        atomicExch(&st->counter, 0u);
    }
    return true;
}

}  // namespace hisq
