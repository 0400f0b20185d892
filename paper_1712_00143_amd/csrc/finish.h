// Finishers: what the last tile of a problem does with the FP64 totals of an
// in-kernel reduction.  All CG scalar recurrences live here, in FP64 on the
// device, so the iteration loop needs no host round trip.
#pragma once
#include "hisq_dev.h"

namespace hisq {

enum : int {
    FIN_NONE = 0,
    FIN_ALPHA = 1,      // tot[0] = Re(p, Ap): alpha = rr / pAp
    FIN_BETA = 2,       // tot[0] = |r_new|^2: convergence / reliable trigger, beta
    FIN_TRUERES = 3,    // tot[0] = |b - A x_hi|^2 (FP64): converged or resume
    FIN_NORM_B = 4,     // tot[0] = |b|^2: initialise the solve state
    FIN_STORE = 5,      // store tot[0..NPART) into st->cplx
    FIN_INIT_R = 6,     // tot[0] = |b - A x0|^2 (warm start): initial residual
    FIN_MS = 7,         // tot[0] = |r_new|^2: base beta and every shift's zeta, alpha_k, beta_k
    FIN_FCG_BETA = 10,  // tot = {Re (q,z), Im (q,z)}: beta = -(q,z)/(q,p)
};

__device__ __forceinline__ long long dev_clock()
{
    return (long long)wall_clock64();
}

// Shifted CG with collinear residuals (Jegerlehner, hep-lat/9612014): with the
// base system's alpha_i, beta_i, the residual of shift k is zeta_k r and
//   zeta_{i+1} = zeta_i zeta_{i-1} alpha_{i-1} /
//                [alpha_i beta_{i-1} (zeta_{i-1} - zeta_i) + zeta_{i-1} alpha_{i-1} (1 + d_k alpha_i)],
//   alpha_k = alpha_i zeta_{i+1} / zeta_i,  beta_k = beta_i (zeta_{i+1} / zeta_i)^2,
// d_k = sigma_k - sigma_base.  A shift stops once |zeta_k| |r| <= tol |b|.
__device__ __forceinline__ void ms_finish(SolveState *st, ShiftState *ms, double rn)
{
    const double al = st->alpha, be = rn / st->rr;
    int any = 0;
    for (int k = 0; k < ms->nshift; k++) {
        ms->upd[k] = ms->active[k];
        if (!ms->active[k]) continue;
        const double z = ms->zeta[k], zo = ms->zeta_old[k];
        const double zn = z * zo * ms->alpha_old /
                          (al * ms->beta_old * (zo - z) + zo * ms->alpha_old * (1.0 + ms->shift[k] * al));
        ms->ak[k] = al * zn / z;
        ms->bk[k] = be * (zn / z) * (zn / z);
        ms->zeta_old[k] = z;
        ms->zeta[k] = zn;
        ms->iters[k] += 1;
        if (fabs(zn) * sqrt(rn) <= sqrt(st->tol2 * st->bb)) ms->active[k] = 0;
        else any = 1;
    }
    ms->alpha_old = al;
    ms->beta_old = be;
    st->beta = be;
    st->rr_old = st->rr;
    st->rr = rn;
    st->iter += 1;
    if (!any || st->iter >= st->maxiter || !isfinite(rn)) st->status = ST_MS_LAST;
}

__device__ __forceinline__ void run_finisher(int fin, SolveState *st, const double *tot, ShiftState *ms = nullptr)
{
    switch (fin) {
    case FIN_MS:
        ms_finish(st, ms, tot[0]);
        break;
    case FIN_FCG_BETA: {
        const double pq = st->pAp;
        st->cplx[2] = -tot[0] / pq;
        st->cplx[3] = -tot[1] / pq;
        if (!isfinite(st->cplx[2]) || !isfinite(st->cplx[3])) st->status = ST_BREAKDOWN;
        break;
    }
    case FIN_ALPHA: {
        double pap = tot[0];
        st->pAp = pap;
        if (!(pap > 0.0) || !isfinite(pap)) {
            st->status = ST_BREAKDOWN;
            st->alpha = 0.0;
        } else {
            st->alpha = st->rr / pap;
        }
        break;
    }
    case FIN_BETA: {
        double rn = tot[0];
        st->iter += 1;
        st->beta = rn / st->rr;
        st->rr_old = st->rr;
        st->rr = rn;
        if (rn > st->maxrr) st->maxrr = rn;
        if (!isfinite(rn)) {
            st->status = ST_BREAKDOWN;
        } else if (rn <= st->tol2 * st->bb || rn < st->delta2 * st->maxrr ||
                   st->iter >= st->maxiter) {
            st->status = ST_RELIABLE;
        }
        break;
    }
    case FIN_TRUERES: {
        double rt = tot[0];
        st->rr_true = rt;
        st->reliable += 1;
        if (rt <= st->tol2 * st->bb) {
            st->status = ST_CONVERGED;
            st->t_done = dev_clock();
        } else if (!isfinite(rt)) {
            st->status = ST_BREAKDOWN;
        } else {
            // The sloppy recursion continues from the FP64 residual.  When
            // that residual exceeds twice the sloppy one it replaces, the
            // sloppy operator's error dominates the search direction
            // (16-bit links at small mass): restart from p = r instead of
            // carrying the stale direction with a large beta.
            if (rt > 2.0 * st->rr) {
                st->beta = 0.0;
                st->restarts += 1;
            } else {
                st->beta = rt / st->rr_old;
            }
            st->rr = rt;
            st->maxrr = rt;
            st->status = ST_RESUME;
        }
        break;
    }
    case FIN_NORM_B: {
        st->bb = tot[0];
        st->rr = tot[0];
        st->rr_old = tot[0];
        st->maxrr = tot[0];
        break;
    }
    case FIN_INIT_R: {
        st->rr = tot[0];
        st->rr_old = tot[0];
        st->maxrr = tot[0];
        st->rr_true = tot[0];
        if (tot[0] <= st->tol2 * st->bb) st->status = ST_CONVERGED;
        break;
    }
    case FIN_STORE: {
        for (int k = 0; k < NPART; k++) st->cplx[k] = tot[k];
        break;
    }
    default:
        break;
    }
}

}  // namespace hisq
