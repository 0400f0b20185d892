// Streaming kernels that measure the device's practical HBM ceilings: a
// read-only pass (non-temporal 16-byte loads, the access the half-Dslash makes
// for its links) and a copy.  The stencil kernels are reported against these
// next to the nameplate peak.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/hisq.h"
#include "fields.h"
#include "solver.h"

namespace hisq {

constexpr int STREAM_UNROLL = 4;
constexpr unsigned STREAM_NEVER = 0x9E3779B9u;   // the xor of a zero-filled buffer is 0

__global__ void __launch_bounds__(256) k_stream_read(const u32x4 *__restrict__ a, size_t n, unsigned *sink)
{
    size_t i = (size_t)blockIdx.x * blockDim.x * STREAM_UNROLL + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x * STREAM_UNROLL;
    unsigned acc = 0;
    for (; i < n; i += stride) {
        u32x4 v[STREAM_UNROLL];
#pragma unroll
        for (int u = 0; u < STREAM_UNROLL; u++) {
            const size_t j = i + (size_t)u * blockDim.x;
            v[u] = j < n ? __builtin_nontemporal_load(a + j) : u32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < STREAM_UNROLL; u++) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    if (acc == STREAM_NEVER) sink[threadIdx.x] = acc;   // keeps the loads; never taken
}

__global__ void __launch_bounds__(256) k_stream_copy(const u32x4 *__restrict__ a, u32x4 *__restrict__ b, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) b[i] = a[i];
}

}  // namespace hisq

using namespace hisq;

extern "C" hisq_status hisq_stream_bandwidth(int device, void *stream, size_t bytes, int reps, double *read_gbs,
                                             double *copy_gbs)
{
    if (bytes < ((size_t)1 << 20) || reps < 1 || !read_gbs || !copy_gbs)
        return set_err(nullptr, HISQ_ERR_ARG, "need bytes >= 1 MiB, reps >= 1 and both outputs");
    if (hipSetDevice(device) != hipSuccess) return set_err(nullptr, HISQ_ERR_ARG, "bad device");
    hipStream_t s = (hipStream_t)stream;
    const size_t n = bytes / 16;
    void *a = nullptr, *b = nullptr, *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hisq_status st = HISQ_OK;
    float ms_read = 0, ms_copy = 0;
    const int grid_read = (int)std::min<size_t>(65536, (n + 256 * STREAM_UNROLL - 1) / (256 * STREAM_UNROLL));
    const int grid_copy = (int)std::min<size_t>(65536, (n + 255) / 256);
    if (hipMalloc(&a, n * 16) != hipSuccess || hipMalloc(&b, n * 16) != hipSuccess ||
        hipMalloc(&sink, 256 * sizeof(unsigned)) != hipSuccess) {
        st = set_err(nullptr, HISQ_ERR_OOM, "stream buffers");
        goto done;
    }
    if (hipMemsetAsync(a, 0, n * 16, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        st = set_err(nullptr, HISQ_ERR_HIP, "stream set-up");
        goto done;
    }
    hipLaunchKernelGGL(k_stream_read, dim3(grid_read), dim3(256), 0, s, (const u32x4 *)a, n, (unsigned *)sink);
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; r++)
        hipLaunchKernelGGL(k_stream_read, dim3(grid_read), dim3(256), 0, s, (const u32x4 *)a, n, (unsigned *)sink);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms_read, e0, e1) != hipSuccess) {
        st = set_err(nullptr, HISQ_ERR_HIP, "read pass");
        goto done;
    }
    hipLaunchKernelGGL(k_stream_copy, dim3(grid_copy), dim3(256), 0, s, (const u32x4 *)a, (u32x4 *)b, n);
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; r++)
        hipLaunchKernelGGL(k_stream_copy, dim3(grid_copy), dim3(256), 0, s, (const u32x4 *)a, (u32x4 *)b, n);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms_copy, e0, e1) != hipSuccess) {
        st = set_err(nullptr, HISQ_ERR_HIP, "copy pass");
        goto done;
    }
    *read_gbs = (double)n * 16 * reps / (ms_read * 1e-3) / 1e9;
    *copy_gbs = 2.0 * n * 16 * reps / (ms_copy * 1e-3) / 1e9;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (sink) (void)hipFree(sink);
    return st;
}
