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
};

__device__ __forceinline__ long long dev_clock()
{
    return (long long)wall_clock64();
}

__device__ __forceinline__ void run_finisher(int fin, SolveState *st, const double *tot)
{
    switch (fin) {
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
            st->beta = rt / st->rr_old;
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
