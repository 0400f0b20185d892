// CG vector kernels.  One block per 64-site tile, one thread per complex
// element (192 threads), so every access is a contiguous, coalesced stream.
// Half-precision vectors keep one float scale per site, computed through LDS
// from the three colour components.  Dot products and norms are reduced
// in-kernel (FP64, fixed order) and feed the FP64 recurrences in finish.h.
#include <type_traits>

#include "finish.h"
#include "launch.h"
#include "reduce.h"

namespace hisq {

template <int M> struct ModeT {
    using R = typename std::conditional<M == 0, double, float>::type;   // r, Ap, x_lo
    using P = typename std::conditional<M == 0, double,
              typename std::conditional<M == 1, float, __half>::type>::type;  // p, t
};

template <class T>
__device__ __forceinline__ double2 ld(const void *v, const float *n, long long f)
{
    if constexpr (sizeof(T) == 8) {
        return reinterpret_cast<const double2 *>(v)[f];
    } else if constexpr (sizeof(T) == 4) {
        float2 x = reinterpret_cast<const float2 *>(v)[f];
        return make_double2(x.x, x.y);
    } else {
        float2 x = __half22float2(reinterpret_cast<const __half2 *>(v)[f]);
        float s = n[f / 3];
        return make_double2((double)(x.x * s), (double)(x.y * s));
    }
}

// store; for half, all 192 threads of the block must call it together
template <class T>
__device__ __forceinline__ void st(void *v, float *n, long long f, double2 x, bool ok, float *lds)
{
    if constexpr (sizeof(T) == 8) {
        if (ok) reinterpret_cast<double2 *>(v)[f] = x;
    } else if constexpr (sizeof(T) == 4) {
        if (ok) reinterpret_cast<float2 *>(v)[f] = make_float2((float)x.x, (float)x.y);
    } else {
        float xr = (float)x.x, xi = (float)x.y;
        lds[threadIdx.x] = ok ? fmaxf(fabsf(xr), fabsf(xi)) : 0.f;
        __syncthreads();
        int base = (threadIdx.x / 3) * 3;
        float m = fmaxf(lds[base], fmaxf(lds[base + 1], lds[base + 2]));
        __syncthreads();
        float inv = m > 0.f ? 1.f / m : 0.f;
        if (ok) {
            reinterpret_cast<__half2 *>(v)[f] = __floats2half2_rn(xr * inv, xi * inv);
            if (threadIdx.x % 3 == 0) n[f / 3] = m;
        }
    }
}

template <int M, int OP>
__global__ void __launch_bounds__(192) k_blas(BlasLaunch a)
{
    using R = typename ModeT<M>::R;
    using P = typename ModeT<M>::P;
    __shared__ float lds[192];
    const int tile = blockIdx.x;
    const int prob = a.tile2prob ? a.tile2prob[tile] : 0;
    const ProbDesc &pd = a.probs[prob];
    SolveState *st_ = a.states ? &a.states[prob] : nullptr;
    if (st_ && st_->status != a.want) return;
    const int e = threadIdx.x;
    const long long site0 = (long long)(tile - pd.tile_begin) * TILE;
    const bool ok = site0 * 3 + e < (long long)pd.h * 3;
    const long long f = (pd.voff + site0) * 3 + e;
    double part = 0.0;

    if constexpr (OP == BL_RUPDATE) {
        // v0 = r (R), v1 = Ap (R), v2 = x_lo (R), v3 = p (P)
        const double al = st_->alpha;
        if (ok) {
            double2 r = ld<R>(a.v[0], a.n[0], f), q = ld<R>(a.v[1], a.n[1], f);
            double2 x = ld<R>(a.v[2], a.n[2], f), p = ld<P>(a.v[3], a.n[3], f);
            R rr = (R)r.x - (R)al * (R)q.x, ri = (R)r.y - (R)al * (R)q.y;
            R xr = (R)x.x + (R)al * (R)p.x, xi = (R)x.y + (R)al * (R)p.y;
            st<R>(a.v[0], nullptr, f, make_double2(rr, ri), true, lds);
            st<R>(a.v[2], nullptr, f, make_double2(xr, xi), true, lds);
            part = (double)rr * (double)rr + (double)ri * (double)ri;
        }
    } else if constexpr (OP == BL_PUPDATE || OP == BL_RESUME) {
        // PUPDATE: v0 = r (R), v3 = p (P): p = r + beta p
        // RESUME:  v4 = r_hi (FP64) -> v0 = r (R); p = r + beta p
        const double be = st_->beta;
        double2 r = make_double2(0, 0), p = make_double2(0, 0);
        if (ok) {
            if constexpr (OP == BL_RESUME) {
                double2 rh = ld<double>(a.v[4], nullptr, f);
                R rr = (R)rh.x, ri = (R)rh.y;
                st<R>(a.v[0], nullptr, f, make_double2(rr, ri), true, lds);
                r = make_double2(rr, ri);
            } else {
                r = ld<R>(a.v[0], a.n[0], f);
            }
            p = ld<P>(a.v[3], a.n[3], f);
        }
        R pr = (R)r.x + (R)be * (R)p.x, pi = (R)r.y + (R)be * (R)p.y;
        st<P>(a.v[3], a.n[3], f, make_double2(pr, pi), ok, lds);
    } else if constexpr (OP == BL_XACCUM) {
        // v4 = x_hi (FP64) += v2 = x_lo (R); x_lo = 0
        if (ok) {
            double2 xh = ld<double>(a.v[4], nullptr, f), xl = ld<R>(a.v[2], a.n[2], f);
            reinterpret_cast<double2 *>(a.v[4])[f] = make_double2(xh.x + xl.x, xh.y + xl.y);
            st<R>(a.v[2], nullptr, f, make_double2(0, 0), true, lds);
        }
    } else if constexpr (OP == BL_INIT) {
        // v5 = b (FP64): r = b, p = b, x_lo = 0, x_hi = 0 (v4), partial |b|^2
        double2 b = make_double2(0, 0);
        if (ok) {
            b = ld<double>(a.v[5], nullptr, f);
            st<R>(a.v[0], nullptr, f, b, true, lds);
            st<R>(a.v[2], nullptr, f, make_double2(0, 0), true, lds);
            reinterpret_cast<double2 *>(a.v[4])[f] = make_double2(0, 0);
            part = b.x * b.x + b.y * b.y;
        }
        st<P>(a.v[3], a.n[3], f, b, ok, lds);
    } else if constexpr (OP == BL_START) {
        double2 r = make_double2(0, 0);
        if (ok) {
            r = ld<double>(a.v[4], nullptr, f);
            st<R>(a.v[0], nullptr, f, r, true, lds);
            st<R>(a.v[2], nullptr, f, make_double2(0, 0), true, lds);
        }
        st<P>(a.v[3], a.n[3], f, r, ok, lds);
    } else if constexpr (OP == BL_NORM) {
        if (ok) {
            double2 b = ld<double>(a.v[5], nullptr, f);
            part = b.x * b.x + b.y * b.y;
        }
    } else if constexpr (OP == BL_COPY_D2F) {
        double2 b = ok ? ld<double>(a.v[0], nullptr, f) : make_double2(0, 0);
        st<P>(a.v[1], a.n[1], f, b, ok, lds);
    } else if constexpr (OP == BL_COPY_F2D) {
        if (ok) reinterpret_cast<double2 *>(a.v[1])[f] = ld<P>(a.v[0], a.n[0], f);
    }

    if (a.fin != FIN_NONE) {
        double mine[1] = {part}, tot[1];
        if (publish_and_reduce<1>(mine, a.partials, tile, pd, st_, tot))
            if (threadIdx.x == 0) run_finisher(a.fin, st_, tot);
    }
}

__global__ void k_status(SolveState *states, int nprob, int from, int to)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob && states[p].status == from) states[p].status = to;
}

__global__ void k_stamp(long long *out)
{
    if (threadIdx.x == 0) *out = (long long)wall_clock64();
}

hipError_t launch_stamp(long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, out);
    return hipGetLastError();
}

template <int M>
static hipError_t launch_m(int op, const BlasLaunch &a, int nt, hipStream_t s)
{
    dim3 g(nt), b(192);
    switch (op) {
    case BL_RUPDATE: hipLaunchKernelGGL((k_blas<M, BL_RUPDATE>), g, b, 0, s, a); break;
    case BL_PUPDATE: hipLaunchKernelGGL((k_blas<M, BL_PUPDATE>), g, b, 0, s, a); break;
    case BL_XACCUM: hipLaunchKernelGGL((k_blas<M, BL_XACCUM>), g, b, 0, s, a); break;
    case BL_RESUME: hipLaunchKernelGGL((k_blas<M, BL_RESUME>), g, b, 0, s, a); break;
    case BL_NORM: hipLaunchKernelGGL((k_blas<M, BL_NORM>), g, b, 0, s, a); break;
    case BL_INIT: hipLaunchKernelGGL((k_blas<M, BL_INIT>), g, b, 0, s, a); break;
    case BL_COPY_D2F: hipLaunchKernelGGL((k_blas<M, BL_COPY_D2F>), g, b, 0, s, a); break;
    case BL_COPY_F2D: hipLaunchKernelGGL((k_blas<M, BL_COPY_F2D>), g, b, 0, s, a); break;
    case BL_START: hipLaunchKernelGGL((k_blas<M, BL_START>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_blas(int op, int prec, const BlasLaunch &a, int ntiles, int nprob, hipStream_t s)
{
    if (op == BL_STATUS) {
        hipLaunchKernelGGL(k_status, dim3((nprob + 63) / 64), dim3(64), 0, s, a.states, nprob,
                           (int)ST_RESUME, (int)ST_RUNNING);
        return hipGetLastError();
    }
    if (ntiles <= 0) return hipSuccess;
    switch (prec) {
    case 0: return launch_m<0>(op, a, ntiles, s);
    case 1: return launch_m<1>(op, a, ntiles, s);
    case 2: return launch_m<2>(op, a, ntiles, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hisq
