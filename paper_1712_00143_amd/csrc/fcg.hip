// Flexible CG (truncation 1, Notay 2000) vector kernels, FP32 vectors with
// complex FP64 scalars, (a, b) = a^+ b:
//   alpha = (p, r) / (p, q);  x += alpha p;  r -= alpha q;  z = M(r);
//   beta = -(q, z) / (q, p);  p = z + beta p.
// beta makes the new direction A-orthogonal to the old one; the
// preconditioner may be any (even non-Hermitian) map.
//
// The iteration needs no finisher launch: the AX Dslash leaves the tile sums
// of (p, q), XR_F forms alpha from them and from the (p, r) sums of the
// previous P_F (every block sums the same tiles in the same order, so all
// blocks agree bitwise) and leaves the |r|^2 sums, the preconditioner's last
// layer leaves the (q, z) sums, and P_F takes the convergence /
// reliable-update decision and beta, updates p and leaves the (p, r) sums of
// the next iteration.  The state an iteration starts from is snapshot by XR_F
// so that P_F reads it while its leading block writes the new one.  After a
// reliable update the host-driven restart uses DOTS_B (with its finisher), P
// and DOT_PR.
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
    const bool lead = tile == 0 && threadIdx.x == 0;
    if (a.op == FCG_XR_F) {
        if (lead) {
            st->snap_status = st->status;
            st->snap_rr = st->rr;
            st->snap_maxrr = st->maxrr;
            st->snap_iter = st->iter;
        }
        // XR_F's leading block may set a breakdown while other blocks start:
        // one read per block keeps every thread of a block on the same path
        __shared__ int s_status;
        if (threadIdx.x == 0) s_status = st->status;
        __syncthreads();
        if (s_status != ST_RUNNING) return;
    } else if (a.op == FCG_P_F) {
        if (st->snap_status != ST_RUNNING) return;
    } else if (st->status != a.want) {
        return;
    }
    const long long f = (long long)tile * TILE * 3 + threadIdx.x;
    const bool ok = f < (long long)pd.h * 3;
    double part[3] = {0.0, 0.0, 0.0};
    float2 *r = reinterpret_cast<float2 *>(a.r), *x = reinterpret_cast<float2 *>(a.x);
    float2 *p = reinterpret_cast<float2 *>(a.p), *q = reinterpret_cast<float2 *>(a.q);
    float2 *z = reinterpret_cast<float2 *>(a.z);
    if (a.op == FCG_DOTS_B) {
        if (ok) {
            float2 qv = q[f], zv = z[f];
            part[0] = (double)qv.x * zv.x + (double)qv.y * zv.y;
            part[1] = (double)qv.x * zv.y - (double)qv.y * zv.x;
        }
        publish_partials<2>(part, a.partials, tile);
    } else if (a.op == FCG_P) {
        const float br = (float)st->cplx[2], bi = (float)st->cplx[3];
        if (ok) {
            float2 pv = p[f], zv = z[f];
            p[f] = make_float2(zv.x + br * pv.x - bi * pv.y, zv.y + br * pv.y + bi * pv.x);
        }
    } else if (a.op == FCG_XR_F) {
        const int nt = a.nt;
        double tot[3];   // (p, q), Re (p, r), Im (p, r)
        block_totals<3>(a.red + FRED_PQ * nt, nt, 0, nt, tot);
        const double pq = tot[0], prr = tot[1], pri = tot[2];
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(prr) || !isfinite(pri)) {
            if (lead) {
                st->pAp = pq;
                st->cplx[0] = st->cplx[1] = 0.0;
                st->status = ST_BREAKDOWN;
                st->snap_status = ST_BREAKDOWN;
            }
            return;
        }
        const double ar64 = prr / pq, ai64 = pri / pq;
        if (lead) {
            st->pAp = pq;
            st->cplx[0] = ar64;
            st->cplx[1] = ai64;
        }
        const float ar = (float)ar64, ai = (float)ai64;
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
        publish_compact(part[0], a.red + FRED_RR * nt, tile);
    } else if (a.op == FCG_P_F) {
        // the decision of the |r|^2 finisher, from the snapshot; every block
        // takes it the same way and the leading block records it
        const int nt = a.nt;
        double tot[3];   // |r|^2, Re (q, z), Im (q, z)
        block_totals<3>(a.red + FRED_RR * nt, nt, 0, nt, tot);
        const double rn = tot[0], qzr = tot[1], qzi = tot[2];
        const int iter1 = st->snap_iter + 1;
        const double maxrr1 = rn > st->snap_maxrr ? rn : st->snap_maxrr;
        const double pq = st->pAp;   // written by XR_F's leading block
        const double br64 = -qzr / pq, bi64 = -qzi / pq;
        int stat1 = ST_RUNNING;
        if (!isfinite(rn)) stat1 = ST_BREAKDOWN;
        else if (rn <= st->tol2 * st->bb || rn < st->delta2 * maxrr1 || iter1 >= st->maxiter) stat1 = ST_RELIABLE;
        else if (!isfinite(br64) || !isfinite(bi64)) stat1 = ST_BREAKDOWN;
        if (lead) {
            st->iter = iter1;
            st->rr_old = st->snap_rr;
            st->rr = rn;
            st->maxrr = maxrr1;
            st->cplx[2] = br64;
            st->cplx[3] = bi64;
            st->status = stat1;
        }
        if (stat1 != ST_RUNNING) return;   // uniform over the grid
        const float br = (float)br64, bi = (float)bi64;
        double pr = 0.0, pi = 0.0;
        if (ok) {
            float2 pv = p[f], zv = z[f], rv = r[f];
            pv = make_float2(zv.x + br * pv.x - bi * pv.y, zv.y + br * pv.y + bi * pv.x);
            p[f] = pv;
            pr = (double)pv.x * rv.x + (double)pv.y * rv.y;
            pi = (double)pv.x * rv.y - (double)pv.y * rv.x;
        }
        double pv2[2] = {pr, pi};
        publish_compact_n<2>(pv2, a.red + FRED_PR * nt, nt, tile);
    } else {   // FCG_DOT_PR: the (p, r) sums after a (re)start
        const int nt = a.nt;
        double pr = 0.0, pi = 0.0;
        if (ok) {
            float2 pv = p[f], rv = r[f];
            pr = (double)pv.x * rv.x + (double)pv.y * rv.y;
            pi = (double)pv.x * rv.y - (double)pv.y * rv.x;
        }
        double pv2[2] = {pr, pi};
        publish_compact_n<2>(pv2, a.red + FRED_PR * nt, nt, tile);
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
