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
    const bool lead = tile == pd.tile_begin && threadIdx.x == 0;   // writes the problem's state
    if constexpr (OP == BL_RUPDATE_F) {
        // the state this iteration starts from, for BL_PUPDATE_F to read while
        // its leading block writes the new one
        if (lead) {
            st_->snap_status = st_->status;
            st_->snap_rr = st_->rr;
            st_->snap_maxrr = st_->maxrr;
            st_->snap_iter = st_->iter;
        }
        // the leading block may set a breakdown while other blocks start: one
        // read per block keeps every thread of a block on the same path
        __shared__ int s_status;
        if (threadIdx.x == 0) s_status = st_->status;
        __syncthreads();
        if (s_status != ST_RUNNING) return;
    } else if constexpr (OP == BL_PUPDATE_F) {
        if (st_->snap_status != ST_RUNNING) return;
    } else {
        if (st_ && st_->status != a.want) return;
    }
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
    } else if constexpr (OP == BL_RUPDATE_F) {
        // alpha = rr / (p, Ap) from the compact tile sums of the AX Dslash
        // (FP64, the same order in every block), then the update of BL_RUPDATE
        const double pap = block_total(a.red, pd.tile_begin, pd.ntile);
        if (!(pap > 0.0) || !isfinite(pap)) {
            if (lead) {
                st_->pAp = pap;
                st_->alpha = 0.0;
                st_->status = ST_BREAKDOWN;
                st_->snap_status = ST_BREAKDOWN;
            }
            return;
        }
        const double al = st_->rr / pap;
        if (lead) {
            st_->pAp = pap;
            st_->alpha = al;
        }
        if (ok) {
            double2 r = ld<R>(a.v[0], a.n[0], f), q = ld<R>(a.v[1], a.n[1], f);
            double2 x = ld<R>(a.v[2], a.n[2], f), p = ld<P>(a.v[3], a.n[3], f);
            R rr = (R)r.x - (R)al * (R)q.x, ri = (R)r.y - (R)al * (R)q.y;
            R xr = (R)x.x + (R)al * (R)p.x, xi = (R)x.y + (R)al * (R)p.y;
            st<R>(a.v[0], nullptr, f, make_double2(rr, ri), true, lds);
            st<R>(a.v[2], nullptr, f, make_double2(xr, xi), true, lds);
            part = (double)rr * (double)rr + (double)ri * (double)ri;
        }
        publish_compact(part, a.red + a.ntot, tile);
        return;
    } else if constexpr (OP == BL_PUPDATE_F) {
        // the scalar recurrence of the beta finisher, from the snapshot: every
        // block decides the same way, the leading block records it
        const double rn = block_total(a.red + a.ntot, pd.tile_begin, pd.ntile);
        const int iter1 = st_->snap_iter + 1;
        const double maxrr1 = rn > st_->snap_maxrr ? rn : st_->snap_maxrr;
        const double be = rn / st_->snap_rr;
        int stat1 = ST_RUNNING;
        if (!isfinite(rn)) stat1 = ST_BREAKDOWN;
        else if (rn <= st_->tol2 * st_->bb || rn < st_->delta2 * maxrr1 || iter1 >= st_->maxiter) stat1 = ST_RELIABLE;
        if (lead) {
            st_->iter = iter1;
            st_->beta = be;
            st_->rr_old = st_->snap_rr;
            st_->rr = rn;
            st_->maxrr = maxrr1;
            st_->status = stat1;
        }
        if (stat1 != ST_RUNNING) return;   // uniform over the block
        double2 r = make_double2(0, 0), p = make_double2(0, 0);
        if (ok) {
            r = ld<R>(a.v[0], a.n[0], f);
            p = ld<P>(a.v[3], a.n[3], f);
        }
        R pr = (R)r.x + (R)be * (R)p.x, pi = (R)r.y + (R)be * (R)p.y;
        st<P>(a.v[3], a.n[3], f, make_double2(pr, pi), ok, lds);
        return;
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
        double mine[1] = {part};
        publish_partials<1>(mine, a.partials, tile);
    }
}

// One block per problem: fixed-order sum of the problem's tile partials, then
// the finisher (FP64 scalar recurrences) on the totals.
__global__ void __launch_bounds__(1024) k_finish(const ProbDesc *probs, SolveState *states, const double *partials,
                                                int fin, int want, int nv, ShiftState *ms)
{
    __shared__ double lds[16 * NPART];
    const ProbDesc &pd = probs[blockIdx.x];
    SolveState *st_ = &states[blockIdx.x];
    if (st_->status != want) return;
    double acc[NPART];
#pragma unroll
    for (int k = 0; k < NPART; k++) acc[k] = 0.0;
    for (int j = threadIdx.x; j < pd.ntile; j += blockDim.x) {
        const double *p = partials + (size_t)(pd.tile_begin + j) * NPART;
        for (int k = 0; k < nv; k++) acc[k] += p[k];
    }
    block_sum<NPART>(acc, lds);
    if (threadIdx.x == 0) run_finisher(fin, st_, acc, ms ? &ms[blockIdx.x] : nullptr);
}

hipError_t launch_finish(const ProbDesc *probs, SolveState *states, const double *partials, int fin, int want,
                         int nv, int nprob, hipStream_t s, ShiftState *ms)
{
    // 1024 threads: a large problem's tile partials (thousands) in few loads per thread
    hipLaunchKernelGGL(k_finish, dim3(nprob), dim3(1024), 0, s, probs, states, partials, fin, want, nv, ms);
    return hipGetLastError();
}

__global__ void k_convert(const void *src, int sprec, void *dst, int dprec, long long n)
{
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        double2 v;
        if (sprec == 0) v = reinterpret_cast<const double2 *>(src)[k];
        else {
            float2 f = reinterpret_cast<const float2 *>(src)[k];
            v = make_double2(f.x, f.y);
        }
        if (dprec == 0) reinterpret_cast<double2 *>(dst)[k] = v;
        else reinterpret_cast<float2 *>(dst)[k] = make_float2((float)v.x, (float)v.y);
    }
}

hipError_t launch_convert(const void *src, int sprec, void *dst, int dprec, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_convert, dim3((unsigned)nb), dim3(256), 0, s, src, sprec, dst, dprec, n);
    return hipGetLastError();
}

// Multi-shift vector kernels (FP32 vectors, FP64 scalars).  Problem = one
// right-hand side; tiles of problem j cover its h sites.
template <int OP>
__global__ void __launch_bounds__(192) k_ms(BlasLaunch a)
{
    __shared__ float lds[192];
    const int tile = blockIdx.x;
    const int prob = a.tile2prob ? a.tile2prob[tile] : 0;
    const ProbDesc &pd = a.probs[prob];
    SolveState *st_ = &a.states[prob];
    const int stat = st_->status;
    if (OP == BL_MS_UPDATE ? (stat != ST_RUNNING && stat != ST_MS_LAST) : stat != a.want) return;
    const ShiftState *ms = &a.ms[prob];
    const int e = threadIdx.x;
    const long long site0 = (long long)(tile - pd.tile_begin) * TILE;
    const bool ok = site0 * 3 + e < (long long)pd.h * 3;
    const long long f = (pd.voff + site0) * 3 + e;       // this rhs's vectors
    const long long h3 = (long long)pd.h * 3;
    const int ns = ms->nshift;
    const int j = prob;                                   // rhs index
    double part = 0.0;
    float2 *r = reinterpret_cast<float2 *>(a.v[0]);
    float2 *p = reinterpret_cast<float2 *>(a.v[3]);
    float2 *xs = reinterpret_cast<float2 *>(a.v[2]);
    float2 *ps = reinterpret_cast<float2 *>(a.v[4]);
    const long long fk0 = (long long)j * ns * h3 + site0 * 3 + e;   // shift 0 of rhs j
    if constexpr (OP == BL_MS_INIT) {
        if (ok) {
            double2 b = reinterpret_cast<const double2 *>(a.v[5])[f];
            float2 bf = make_float2((float)b.x, (float)b.y);
            r[f] = bf;
            p[f] = bf;
            for (int k = 0; k < ns; k++) {
                ps[fk0 + k * h3] = bf;
                xs[fk0 + k * h3] = make_float2(0.f, 0.f);
            }
            part = b.x * b.x + b.y * b.y;
        }
    } else if constexpr (OP == BL_MS_RUPDATE) {
        const float al = (float)st_->alpha;
        if (ok) {
            float2 rv = r[f], q = reinterpret_cast<const float2 *>(a.v[1])[f];
            rv.x -= al * q.x;
            rv.y -= al * q.y;
            r[f] = rv;
            part = (double)rv.x * rv.x + (double)rv.y * rv.y;
        }
    } else if constexpr (OP == BL_MS_UPDATE) {
        if (ok) {
            const float2 rv = r[f];
            const float2 pv = p[f];
            for (int k = 0; k < ns; k++) {
                if (!ms->upd[k]) continue;
                const float ak = (float)ms->ak[k], bk = (float)ms->bk[k], zk = (float)ms->zeta[k];
                const long long fk = fk0 + k * h3;
                float2 pk = ps[fk], xk = xs[fk];
                xk.x += ak * pk.x;
                xk.y += ak * pk.y;
                pk.x = zk * rv.x + bk * pk.x;
                pk.y = zk * rv.y + bk * pk.y;
                xs[fk] = xk;
                ps[fk] = pk;
            }
            const float be = (float)st_->beta;
            p[f] = make_float2(rv.x + be * pv.x, rv.y + be * pv.y);
        }
    }
    (void)lds;
    if (a.fin != FIN_NONE) {
        double mine[1] = {part};
        publish_partials<1>(mine, a.partials, tile);
    }
}

hipError_t launch_ms(int op, const BlasLaunch &a, int ntiles, hipStream_t s)
{
    dim3 g(ntiles), b(192);
    switch (op) {
    case BL_MS_INIT: hipLaunchKernelGGL(k_ms<BL_MS_INIT>, g, b, 0, s, a); break;
    case BL_MS_RUPDATE: hipLaunchKernelGGL(k_ms<BL_MS_RUPDATE>, g, b, 0, s, a); break;
    case BL_MS_UPDATE: hipLaunchKernelGGL(k_ms<BL_MS_UPDATE>, g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
    case BL_RUPDATE_F: hipLaunchKernelGGL((k_blas<M, BL_RUPDATE_F>), g, b, 0, s, a); break;
    case BL_PUPDATE_F: hipLaunchKernelGGL((k_blas<M, BL_PUPDATE_F>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_blas(int op, int prec, const BlasLaunch &a, int ntiles, int nprob, hipStream_t s)
{
    if (op == BL_STATUS_MS) {
        hipLaunchKernelGGL(k_status, dim3((nprob + 63) / 64), dim3(64), 0, s, a.states, nprob,
                           (int)ST_MS_LAST, (int)ST_CONVERGED);
        return hipGetLastError();
    }
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
