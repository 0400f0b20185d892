// Deterministic per-problem reductions.
//
// Every tile (64 sites) writes up to NPART double partials; a one-block-per-
// problem kernel then sums them in a fixed order and runs a finisher on the
// FP64 totals.  The order depends only on the tile count, so results are
// bitwise reproducible.
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

// Publish this tile's NV partials (block-summed, written by thread 0).  The
// per-problem totals are formed by k_finish, launched right after the kernel
// that wrote them: the kernel boundary makes the partials visible on every
// XCD without fences or atomics, and the fixed summation order keeps the
// results bitwise reproducible.
template <int NV>
__device__ __forceinline__ void publish_partials(double mine[NV], double *partials, int tile)
{
    __shared__ double lds[16 * NV];
    block_sum<NV>(mine, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; k++) partials[(size_t)tile * NPART + k] = mine[k];
}

// One block-summed value per tile in a compact array (red[tile]), for kernels
// whose consumers sum a problem's tiles themselves.
__device__ __forceinline__ void publish_compact(double mine, double *red, int tile)
{
    __shared__ double lds[16];
    double v[1] = {mine};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) red[tile] = v[0];
}

// NV block-summed values per tile in NV compact arrays stride apart
// (red[k * stride + tile]), with one block reduction.
template <int NV>
__device__ __forceinline__ void publish_compact_n(double mine[NV], double *red, int stride, int tile)
{
    __shared__ double lds[16 * NV];
    block_sum<NV>(mine, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) red[(size_t)k * stride + tile] = mine[k];
}

// Sum of red[first .. first + n) in a fixed order (each thread a strided
// subset, then the block sum), returned to every thread of the block.  Every
// block that calls it for the same range gets the same bits.
__device__ __forceinline__ double block_total(const double *red, int first, int n)
{
    __shared__ double lds[16];
    __shared__ double tot;
    double v[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += blockDim.x) v[0] += red[first + j];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) tot = v[0];
    __syncthreads();
    return tot;
}

// NV sums at once: out[k] = sum of red[k * stride + first .. + n), each in
// the order of block_total (so each total has the same bits as block_total's),
// returned to every thread of the block.  One pass and one block reduction
// instead of NV.
template <int NV>
__device__ __forceinline__ void block_totals(const double *red, int stride, int first, int n, double out[NV])
{
    __shared__ double lds[16 * NV];
    __shared__ double tot[NV];
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x)
#pragma unroll
        for (int k = 0; k < NV; k++) v[k] += red[(size_t)k * stride + first + j];
    block_sum<NV>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) tot[k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) out[k] = tot[k];
}

}  // namespace hisq
