// Flexible CG (truncation 1, Notay 2000) vector kernels, FP32 vectors with
// complex FP64 scalars:
//   DOTS_A: (p, q) and (p, r)        -> alpha = (p, r) / (p, q)
//   XR:     x += alpha p, r -= alpha q, |r|^2
//   DOTS_B: (q, z)                   -> beta = -(q, z) / (q, p)
//   P:      p = z + beta p
// with (a, b) = a^+ b.  beta makes the new direction A-orthogonal to the old
// one; the preconditioner z = M(r) may be any (even non-Hermitian) map.
#include "finish.h"
#include "launch.h"
#include "ptc.h"
#include "reduce.h"

namespace hisq {

__global__ void __launch_bounds__(192) k_fcg(FcgLaunch a)
{
    const int tile = blockIdx.x;
    const ProbDesc &pd = a.probs[0];
    SolveState *st = &a.states[0];
    if (st->status != a.want) return;
    const long long f = (long long)tile * TILE * 3 + threadIdx.x;
    const bool ok = f < (long long)pd.h * 3;
    double part[3] = {0.0, 0.0, 0.0};
    float2 *r = reinterpret_cast<float2 *>(a.r), *x = reinterpret_cast<float2 *>(a.x);
    float2 *p = reinterpret_cast<float2 *>(a.p), *q = reinterpret_cast<float2 *>(a.q);
    float2 *z = reinterpret_cast<float2 *>(a.z);
    if (a.op == FCG_DOTS_A) {
        if (ok) {
            float2 pv = p[f], qv = q[f], rv = r[f];
            part[0] = (double)pv.x * qv.x + (double)pv.y * qv.y;
            part[1] = (double)pv.x * rv.x + (double)pv.y * rv.y;
            part[2] = (double)pv.x * rv.y - (double)pv.y * rv.x;
        }
        publish_partials<3>(part, a.partials, tile);
    } else if (a.op == FCG_XR) {
        const float ar = (float)st->cplx[0], ai = (float)st->cplx[1];
        if (ok) {
            float2 pv = p[f], qv = q[f], rv = r[f], xv = x[f];
            xv.x += ar * pv.x - ai * pv.y;
            xv.y += ar * pv.y + ai * pv.x;
            rv.x -= ar * qv.x - ai * qv.y;
            rv.y -= ar * qv.y + ai * qv.x;
            x[f] = xv;
            r[f] = rv;
            part[0] = (double)rv.x * rv.x + (double)rv.y * rv.y;
        }
        publish_partials<1>(part, a.partials, tile);
    } else if (a.op == FCG_DOTS_B) {
        if (ok) {
            float2 qv = q[f], zv = z[f];
            part[0] = (double)qv.x * zv.x + (double)qv.y * zv.y;
            part[1] = (double)qv.x * zv.y - (double)qv.y * zv.x;
        }
        publish_partials<2>(part, a.partials, tile);
    } else {
        const float br = (float)st->cplx[2], bi = (float)st->cplx[3];
        if (ok) {
            float2 pv = p[f], zv = z[f];
            p[f] = make_float2(zv.x + br * pv.x - bi * pv.y, zv.y + br * pv.y + bi * pv.x);
        }
    }
}

hipError_t launch_fcg(const FcgLaunch &a, int ntile, hipStream_t s)
{
    hipLaunchKernelGGL(k_fcg, dim3(ntile), dim3(192), 0, s, a);
    return hipGetLastError();
}

// Adjoint weights of a layer: W'[c'][c][k'] = conj(W[c][c'][k]), k' swaps
// the +mu and -mu paths (the adjoint of a forward hop is a backward hop).
__global__ void k_ptc_adjoint(const float *w, int cin, int cout, float *wadj)
{
    const int t = threadIdx.x;
    if (t >= cin * cout * 9) return;
    const int k = t % 9, cp = (t / 9) % cin, c = t / (9 * cin);
    const int ks = k == 0 ? 0 : (((k - 1) & 1) ? k - 1 : k + 1);
    const float re = w[2 * t], im = w[2 * t + 1];
    const int o = (cp * cout + c) * 9 + ks;
    wadj[2 * o] = re;
    wadj[2 * o + 1] = -im;
}

// A gradient gp with respect to the adjoint weights W' ([cout'][cin'][9]) of
// an adjoint layer application contributes conj(gp) with the paths reversed
// to the gradient of W ([cin'][cout'][9]): W' = conj(P W), P the index map.
__global__ void k_ptc_gadj(const double *gp, int cin_p, int cout_p, double *gw)
{
    const int t = threadIdx.x;
    if (t >= cin_p * cout_p * 9) return;
    const int k = t % 9, cp = (t / 9) % cin_p, c = t / (9 * cin_p);
    const int ks = k == 0 ? 0 : (((k - 1) & 1) ? k - 1 : k + 1);
    const int o = (cp * cout_p + c) * 9 + ks;
    gw[2 * o] += gp[2 * t];
    gw[2 * o + 1] -= gp[2 * t + 1];
}

hipError_t launch_ptc_gadj(const double *gp, int cin_p, int cout_p, double *gw, hipStream_t s)
{
    hipLaunchKernelGGL(k_ptc_gadj, dim3(1), dim3(1024), 0, s, gp, cin_p, cout_p, gw);
    return hipGetLastError();
}

// z += r over n floats (the identity term of the preconditioner)
__global__ void k_add_f32(float *z, const float *r, long long n)
{
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x)
        z[j] += r[j];
}

hipError_t launch_add_f32(float *z, const float *r, long long n, hipStream_t s)
{
    long long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_add_f32, dim3((unsigned)nb), dim3(256), 0, s, z, r, n);
    return hipGetLastError();
}

__global__ void k_to_half(const float *w, __half *w16, int n)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) w16[j] = __float2half_rn(w[j]);
}

hipError_t launch_to_half(const float *w, __half *w16, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_half, dim3((n + 255) / 256), dim3(256), 0, s, w, w16, n);
    return hipGetLastError();
}

hipError_t launch_ptc_adjoint(const float *w, int cin, int cout, float *wadj, hipStream_t s)
{
    hipLaunchKernelGGL(k_ptc_adjoint, dim3(1), dim3(1024), 0, s, w, cin, cout, wadj);
    return hipGetLastError();
}

}  // namespace hisq
