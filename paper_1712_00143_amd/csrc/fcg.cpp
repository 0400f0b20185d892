// Flexible CG with the learned PTC preconditioner (truncation 1, Notay
// 2000), FP32 iteration with FP64 reliable updates and the FP64 true residual
// as the stopping test; plain CG is the fallback:
//   r = b, z = M(r), p = z; repeat
//     q = A p;  alpha = (p, r) / (p, q);  x += alpha p;  r -= alpha q;
//     z = M(r); beta = -(q, z) / (q, p);  p = z + beta p.
// A breakdown ((p, q) <= 0 or a non-finite scalar) or more than maxiter / 2
// iterations hands the current iterate to hisq_cg.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <sstream>
#include <string>

#include "fcg_graph.h"
#include "finish.h"
#include "ptc.h"
#include "solver.h"

using namespace hisq;

#define HIPCHK(lat, x)                                     \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) return hip_err(lat, e_, #x); \
    } while (0)

// defined in ptc.cpp
hipError_t ptc_apply_internal(hisq_ptc n, hisq_lattice lat, int lslot, int prec, int recon, const float *r, float *z,
                              const PtcFuse *fz);
std::string ptc_graph_key(hisq_ptc n);
ChunkGraphs &ptc_fcg_graph(hisq_ptc n);

extern "C" hisq_status hisq_cg_learned(hisq_lattice lat, hisq_ptc net, double mass, const double *b, double *x,
                                       const hisq_solver_params *params, hisq_solver_info *info)
{
    if (!lat || !net || !b || !x) return set_err(lat, HISQ_ERR_ARG, "null argument");
    if (!lat->loaded) return set_err(lat, HISQ_ERR_STATE, "no links loaded");
    if (!(mass > 0)) return set_err(lat, HISQ_ERR_ARG, "mass must be > 0");
    hisq_solver_params prm;
    if (params) prm = *params;
    else hisq_default_params(&prm);
    if (!(prm.tol > 0) || prm.maxiter < 2) return set_err(lat, HISQ_ERR_ARG, "bad tol or maxiter");
    HIPCHK(lat, hipSetDevice(lat->device));
    auto t0 = std::chrono::steady_clock::now();
    const int recon = (int)prm.recon;
    const int slot = 2 + (recon == 12);   // FP32 operator
    if (!lat->ls[slot].valid) {
        hisq_status ps = hisq_prepare_links(lat, HISQ_F32, prm.recon);
        if (ps != HISQ_OK) return ps;
    }
    if (!lat->ls[2].valid) {
        hisq_status ps = hisq_prepare_links(lat, HISQ_F32, HISQ_RECON_18);
        if (ps != HISQ_OK) return ps;
    }
    // transports: the network's own link format (hisq_ptc_set_transport), the
    // one it was trained with
    int pprec = 1, precon = 18;
    {
        hisq_status ts = hisq_ptc_get_transport(net, &pprec, &precon);
        if (ts != HISQ_OK) return ts;
    }
    const int pslot = pprec * 2 + (precon == 12);
    if (!lat->ls[pslot].valid) {
        hisq_status ps = hisq_prepare_links(lat, (hisq_prec)pprec, (hisq_recon)precon);
        if (ps != HISQ_OK) return ps;
    }
    hipStream_t s = lat->s;
    const bool dev = (prm.flags & HISQ_DEVICE_PTR) != 0;

    std::vector<hisq_lattice> lats{lat};
    std::vector<double> ms{mass};
    SolveSet &S = lat->fcg;
    hisq_status st = build_set(lat, S, lats, ms, 0.0);
    if (st != HISQ_OK) return st;
    const long long h = lat->h;
    S.mode = -1;   // vectors below are FCG-specific
    for (DVec *v : {&S.b, &S.xhi, &S.rhi, &S.thi}) HIPCHK(lat, dvec_alloc(*v, 0, h));
    for (DVec *v : {&S.xlo, &S.rlo, &S.Ap, &S.p, &S.t, &S.fz}) HIPCHK(lat, dvec_alloc(*v, 1, h));
    if (!S.fred) HIPCHK(lat, hipMalloc(&S.fred, sizeof(double) * FRED_N * S.ntile));
    DVec &z = S.fz;
    const int nt = S.ntile;
    HIPCHK(lat, hipMemcpyAsync(S.b.p, b, (size_t)h * 48, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    SolveState &hs = S.hst[0];
    memset(&hs, 0, sizeof hs);
    hs.status = ST_RUNNING;
    hs.tol2 = prm.tol * prm.tol;
    hs.delta2 = prm.delta * prm.delta;
    hs.maxiter = prm.maxiter / 2 > 0 ? prm.maxiter / 2 : 1;
    HIPCHK(lat, hipMemcpyAsync(S.dst, &hs, sizeof hs, hipMemcpyHostToDevice, s));

    TuneChoice tc = pick_shape(lat, 1, recon, S.ddesc, nullptr, S.ntile, h, 1, (prm.flags & HISQ_NO_TUNE) != 0);
    auto blas = [&](int op, int want, int fin) -> hipError_t {
        BlasLaunch bl;
        memset(&bl, 0, sizeof bl);
        bl.probs = S.ddesc;
        bl.states = S.dst;
        bl.want = want;
        bl.fin = fin;
        bl.partials = S.dpart;
        bl.v[0] = S.rlo.p;
        bl.v[1] = S.Ap.p;
        bl.v[2] = S.xlo.p;
        bl.v[3] = S.p.p;
        bl.v[4] = S.xhi.p;
        bl.v[5] = S.b.p;
        hipError_t e = launch_blas(op, 1, bl, S.ntile, 1, s);
        if (e != hipSuccess || fin == FIN_NONE) return e;
        return launch_finish(S.ddesc, S.dst, S.dpart, fin, want, 1, 1, s);
    };
    auto fcg = [&](int op, int want, int fin, int nv) -> hipError_t {
        FcgLaunch f;
        memset(&f, 0, sizeof f);
        f.probs = S.ddesc;
        f.states = S.dst;
        f.want = want;
        f.op = op;
        f.partials = S.dpart;
        f.r = (float *)S.rlo.p;
        f.x = (float *)S.xlo.p;
        f.p = (float *)S.p.p;
        f.q = (float *)S.Ap.p;
        f.z = (float *)z.p;
        f.red = S.fred;
        f.nt = nt;
        hipError_t e = launch_fcg(f, S.ntile, s);
        if (e != hipSuccess || fin == FIN_NONE) return e;
        return launch_finish(S.ddesc, S.dst, S.dpart, fin, want, nv, 1, s);
    };
    auto dslash = [&](int prec, int ls, int rc, int W, int par, int epi, int fin, int want, const DVec &in, DVec &out,
                      const DVec *aux, double *red = nullptr) -> hipError_t {
        DslashLaunch a;
        memset(&a, 0, sizeof a);
        a.red = red;
        a.probs = S.ddesc;
        a.remap = tc.remap;
        a.cpol = ls == slot ? tc.cpol : 0;   // the tuned policy belongs to the FP32 operator
        a.out_par = par;
        a.lslot = ls;
        a.want = want;
        a.states = S.dst;
        a.in = in.p;
        a.out = out.p;
        if (aux) a.aux = aux->p;
        a.bvec = (const double *)S.b.p;
        a.partials = S.dpart;
        a.fin = fin;
        hipError_t e = launch_dslash(prec, rc, prec, epi, W, a, S.ntile, s);
        if (e != hipSuccess || fin == FIN_NONE) return e;
        return launch_finish(S.ddesc, S.dst, S.dpart, fin, want, 1, 1, s);
    };
    // z = M(r); fused: gated on the status, with the (q, z) tile sums
    auto precondition = [&](const PtcFuse *fz) -> hipError_t {
        return ptc_apply_internal(net, lat, pslot, pprec, precon, (const float *)S.rlo.p, (float *)z.p, fz);
    };
    const PtcFuse fuse{S.dst, ST_RUNNING, (const float *)S.Ap.p, S.fred + FRED_QZ * nt, nt};
    const PtcFuse resume_gate{S.dst, ST_RESUME, nullptr, nullptr, nt};   // gated only
    // one iteration, no finisher launches and no host decisions: q = A p with
    // the (p, q) sums; alpha, x, r and the |r|^2 sums; z = M(r) with the (q, z)
    // sums; the status decision, beta, p and the (p, r) sums
    auto iteration = [&]() -> hipError_t {
        hipError_t e;
        if ((e = dslash(1, slot, recon, tc.W, 1, EPI_PLAIN, FIN_NONE, ST_RUNNING, S.p, S.t, nullptr)) != hipSuccess)
            return e;
        if ((e = dslash(1, slot, recon, tc.W, 0, EPI_AX, FIN_NONE, ST_RUNNING, S.t, S.Ap, &S.p,
                        S.fred + FRED_PQ * nt)) != hipSuccess)
            return e;
        if ((e = fcg(FCG_XR_F, ST_RUNNING, FIN_NONE, 0)) != hipSuccess) return e;
        if ((e = precondition(&fuse)) != hipSuccess) return e;
        return fcg(FCG_P_F, ST_RUNNING, FIN_NONE, 0);
    };

    // r = b, x = 0, |b|^2; z = M(r); p = z; the (p, r) sums.  This first
    // application also settles the layer kernels' launch shapes, before any
    // capture.
    HIPCHK(lat, blas(BL_INIT, ST_RUNNING, FIN_NORM_B));
    HIPCHK(lat, precondition(nullptr));
    HIPCHK(lat, hipMemcpyAsync(S.p.p, z.p, (size_t)h * 24, hipMemcpyDeviceToDevice, s));
    HIPCHK(lat, fcg(FCG_DOT_PR, ST_RUNNING, FIN_NONE, 0));
    HIPCHK(lat, hipMemcpyAsync(&hs, S.dst, sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(lat, hipStreamSynchronize(s));
    if (hs.bb == 0.0) {
        if (dev) HIPCHK(lat, hipMemsetAsync(x, 0, (size_t)h * 48, s));
        else memset(x, 0, (size_t)h * 48);
        HIPCHK(lat, hipStreamSynchronize(s));
        if (info) {
            memset(info, 0, sizeof *info);
            info->converged = 1;
        }
        return HISQ_OK;
    }
    const int kchunk = prm.check_every > 0 ? prm.check_every : 16;
    const bool use_graph = (prm.flags & HISQ_USE_GRAPH) != 0;
    if (use_graph) {
        // every launch argument of the chunk: device pointers, shapes, formats
        std::ostringstream ks;
        ks << (const void *)lat << ":" << (const void *)lat->ddesc << ":" << S.p.p << ":" << S.t.p << ":" << S.Ap.p << ":" << S.rlo.p << ":" << S.xlo.p
           << ":" << z.p << ":" << S.fred << ":" << S.dst << ":" << S.ddesc << ":" << S.dpart << ":" << nt << ":"
           << slot << ":" << recon << ":" << tc.W << ":" << tc.remap << ":" << tc.cpol << ":" << pslot << ":" << kchunk << ":"
           << ptc_graph_key(net);
        ChunkGraphs &G = ptc_fcg_graph(net);
        if (G.key != ks.str() || !G.ready()) {
            hipError_t ce = G.capture(kchunk, s, [&](int len) -> hipError_t {
                hipError_t e = hipSuccess;
                for (int q = 0; q < len && e == hipSuccess; q++) e = iteration();
                return e;
            });
            if (ce != hipSuccess) {
                G.release();
                return hip_err(lat, ce, "flexible CG graph capture");
            }
            G.key = ks.str();
        }
    }
    const ChunkGraphs *graphs = use_graph ? &ptc_fcg_graph(net) : nullptr;
    ChunkPlanner plan(kchunk);
    plan.rebase(hs);
    int fell_back = 0;
    S.hist.assign(1, std::vector<double>());
    lat->last_solve = &S;
    for (;;) {
        const int len = plan.next(hs);
        if (graphs) HIPCHK(lat, graphs->launch(len, s));
        else
            for (int q = 0; q < len; q++) HIPCHK(lat, iteration());
        HIPCHK(lat, hipMemcpyAsync(&hs, S.dst, sizeof hs, hipMemcpyDeviceToHost, s));
        HIPCHK(lat, hipStreamSynchronize(s));
        if (hs.status == ST_RUNNING || hs.status == ST_RELIABLE) plan.observe(hs);
        if (hs.status == ST_RELIABLE) {
            // FP64 reliable update: x_hi += x_lo and the true residual, whose
            // finisher decides on the device (converged, or resume); the
            // resume runs gated on that decision, so one host read follows:
            // r = r_hi, z = M(r), the new direction and the (p, r) sums of
            // the next iteration
            HIPCHK(lat, blas(BL_XACCUM, ST_RELIABLE, FIN_NONE));
            HIPCHK(lat, dslash(0, 0, 18, 8, 1, EPI_PLAIN, FIN_NONE, ST_RELIABLE, S.xhi, S.thi, nullptr));
            HIPCHK(lat, dslash(0, 0, 18, 8, 0, EPI_RES, FIN_TRUERES, ST_RELIABLE, S.thi, S.rhi, &S.xhi));
            {
                BlasLaunch bl;
                memset(&bl, 0, sizeof bl);
                bl.probs = S.ddesc;
                bl.states = S.dst;
                bl.want = ST_RESUME;
                bl.fin = FIN_NONE;
                bl.partials = S.dpart;
                bl.v[0] = S.rhi.p;
                bl.v[1] = S.rlo.p;
                HIPCHK(lat, launch_blas(BL_COPY_D2F, 1, bl, S.ntile, 1, s));
            }
            HIPCHK(lat, precondition(&resume_gate));
            HIPCHK(lat, fcg(FCG_DOTS_B, ST_RESUME, FIN_FCG_BETA, 2));
            HIPCHK(lat, fcg(FCG_P, ST_RESUME, FIN_NONE, 0));
            HIPCHK(lat, fcg(FCG_DOT_PR, ST_RESUME, FIN_NONE, 0));
            HIPCHK(lat, blas(BL_STATUS, ST_RESUME, FIN_NONE));
            HIPCHK(lat, hipMemcpyAsync(&hs, S.dst, sizeof hs, hipMemcpyDeviceToHost, s));
            HIPCHK(lat, hipStreamSynchronize(s));
            if (hs.bb > 0) S.hist[0].push_back(std::sqrt(hs.rr_true / hs.bb));
            if (hs.status == ST_RUNNING) plan.rebase(hs);
        }
        if (hs.status == ST_CONVERGED || hs.status == ST_BREAKDOWN) break;
        if (hs.status == ST_RUNNING && hs.iter >= hs.maxiter) break;
    }
    // x = x_hi + x_lo
    int cur = hs.status;
    HIPCHK(lat, blas(BL_XACCUM, cur, FIN_NONE));
    HIPCHK(lat, hipMemcpyAsync(x, S.xhi.p, (size_t)h * 48, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    HIPCHK(lat, hipStreamSynchronize(s));
    const int it_fcg = hs.iter, rel_fcg = hs.reliable;
    double tres = hs.bb > 0 ? std::sqrt(hs.rr_true / hs.bb) : 0.0;
    hisq_status out = HISQ_OK;
    int conv = hs.status == ST_CONVERGED;
    int total_iters = it_fcg, total_rel = rel_fcg;
    if (!conv) {
        // fallback: plain (mixed) CG from the current iterate
        fell_back = 1;
        hisq_solver_params cp = prm;
        cp.flags = (prm.flags & ~HISQ_USE_GRAPH) | HISQ_X_IS_GUESS;
        cp.maxiter = prm.maxiter - it_fcg > 0 ? prm.maxiter - it_fcg : 1;
        if (cp.sloppy == HISQ_F16 && !lat->ls[4 + (recon == 12)].valid) cp.sloppy = HISQ_F32;
        hisq_solver_info ci;
        out = hisq_cg(lat, mass, b, x, &cp, &ci);
        total_iters += ci.iters;
        total_rel += ci.reliable_updates;
        tres = ci.true_residual;
        conv = ci.converged;
    }
    const double elapsed = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) {
        memset(info, 0, sizeof *info);
        info->iters = total_iters;
        info->reliable_updates = total_rel;
        info->converged = conv;
        info->status = out;
        info->true_residual = tres;
        info->time_s = elapsed;
        info->fell_back = fell_back;
        info->fcg_iters = it_fcg;
        info->dslash_bytes = (double)h * 2.0 * total_iters * (double)(link_site_bytes(1, recon) + 48);
        info->flops = 1146.0 * h * 2.0 * total_iters;
    }
    return out;
}
