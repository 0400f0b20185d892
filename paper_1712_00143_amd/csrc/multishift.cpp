// Multi-shift CG (Section 4.1: the staggered multi-shift CG is the dominant
// routine of the RHMD evolution): solve (A + sigma_k) x_{j,k} = b_j for every
// shift k and right-hand side j with one Krylov space per right-hand side.
//
// Krylov phase (FP32 vectors, FP64 scalars on the device), per iteration:
//   t_j = D_oe p_j,  Ap_j = (4m^2 + sigma_base) p_j - D_eo t_j   [multi-RHS Dslash: links read once]
//   alpha_j = rr_j / (p_j, Ap_j)                                 [k_finish]
//   r_j -= alpha_j Ap_j                                          [k_ms RUPDATE]
//   beta_j, zeta_{j,k}, alpha_{j,k}, beta_{j,k}                  [k_finish FIN_MS, FP64]
//   x_{j,k} += alpha_{j,k} p_{j,k}; p_{j,k} = zeta_{j,k} r_j + beta_{j,k} p_{j,k};
//   p_j = r_j + beta_j p_j                                       [k_ms UPDATE, one pass]
// Refinement phase: every (j, k) is finished by the batched mixed-precision
// CG with FP64 reliable updates, warm-started from x_{j,k}, until its FP64
// true residual || b_j - (A + sigma_k) x || / ||b_j|| reaches tol.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "finish.h"
#include "solver.h"

using namespace hisq;

#define HIPCHK(lat, x)                                     \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) return hip_err(lat, e_, #x); \
    } while (0)

namespace {

struct MsWork {
    int nrhs = 0, ns = 0;
    long long h = 0;
    ProbDesc *ddesc = nullptr;
    int *dt2p = nullptr;
    SolveState *dst = nullptr;
    SolveState *hst = nullptr;
    ShiftState *dms = nullptr;
    ShiftState *hms = nullptr;
    double *dpart = nullptr;
    void *r = nullptr, *p = nullptr, *Ap = nullptr, *t = nullptr, *xs = nullptr, *ps = nullptr;
    double *b64 = nullptr, *x64 = nullptr;
    void release()
    {
        for (void *q : {(void *)ddesc, (void *)dt2p, (void *)dst, (void *)dms, (void *)dpart, r, p, Ap, t, xs,
                        ps, (void *)b64, (void *)x64})
            if (q) (void)hipFree(q);
        if (hst) (void)hipHostFree(hst);
        if (hms) (void)hipHostFree(hms);
        *this = MsWork();
    }
};

}  // namespace

extern "C" hisq_status hisq_multishift_cg(hisq_lattice lat, double mass, int nshift, const double *shifts,
                                          int nrhs, const double *b, double *x,
                                          const hisq_solver_params *params, hisq_solver_info *info)
{
    if (!lat || !shifts || !b || !x) return set_err(lat, HISQ_ERR_ARG, "null argument");
    if (!lat->loaded) return set_err(lat, HISQ_ERR_STATE, "no links loaded");
    if (!(mass > 0) || nshift < 1 || nshift > MAXSHIFT || nrhs < 1 || nrhs > 64)
        return set_err(lat, HISQ_ERR_ARG, "need mass > 0, 1 <= nshift <= 64, 1 <= nrhs <= 64");
    for (int k = 0; k < nshift; k++)
        if (!(shifts[k] >= 0) || !std::isfinite(shifts[k])) return set_err(lat, HISQ_ERR_ARG, "shifts must be >= 0");
    hisq_solver_params prm;
    if (params) prm = *params;
    else hisq_default_params(&prm);
    if (!(prm.tol > 0) || prm.maxiter < 1) return set_err(lat, HISQ_ERR_ARG, "bad tol or maxiter");
    const int kprec = prm.sloppy == HISQ_F16 ? 2 : 1;   // Krylov-phase link precision (vectors FP32)
    const int recon = (int)prm.recon;
    const int slot = kprec * 2 + (recon == 12);
    if (!lat->ls[slot].valid) return set_err(lat, HISQ_ERR_STATE, "link set not prepared (hisq_prepare_links)");
    HIPCHK(lat, hipSetDevice(lat->device));
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = lat->s;
    const bool dev = (prm.flags & HISQ_DEVICE_PTR) != 0;

    int kb = 0;
    for (int k = 1; k < nshift; k++)
        if (shifts[k] < shifts[kb]) kb = k;
    const double sbase = shifts[kb];
    const long long h = lat->h;
    const int ntile = lat->ntile;

    MsWork W;
    W.nrhs = nrhs;
    W.ns = nshift;
    W.h = h;
    struct Guard {
        MsWork &w;
        ~Guard() { w.release(); }
    } guard{W};

    // one problem per right-hand side, all on this lattice
    std::vector<ProbDesc> hd(nrhs);
    std::vector<int> t2p((size_t)nrhs * ntile);
    for (int j = 0; j < nrhs; j++) {
        hd[j] = lattice_desc(lat);
        hd[j].tile_begin = j * ntile;
        hd[j].voff = (long long)j * h;
        hd[j].mass = mass;
        hd[j].diag = 4.0 * mass * mass + sbase;
        for (int q = 0; q < ntile; q++) t2p[(size_t)j * ntile + q] = j;
    }
    const size_t v32 = (size_t)nrhs * h * 24, v64 = (size_t)nrhs * h * 48;
    HIPCHK(lat, hipMalloc(&W.ddesc, sizeof(ProbDesc) * nrhs));
    HIPCHK(lat, hipMalloc(&W.dt2p, sizeof(int) * t2p.size()));
    HIPCHK(lat, hipMalloc(&W.dst, sizeof(SolveState) * nrhs));
    HIPCHK(lat, hipHostMalloc(&W.hst, sizeof(SolveState) * nrhs, hipHostMallocDefault));
    HIPCHK(lat, hipMalloc(&W.dms, sizeof(ShiftState) * nrhs));
    HIPCHK(lat, hipHostMalloc(&W.hms, sizeof(ShiftState) * nrhs, hipHostMallocDefault));
    HIPCHK(lat, hipMalloc(&W.dpart, sizeof(double) * NPART * (size_t)nrhs * ntile));
    for (void **q : {&W.r, &W.p, &W.Ap, &W.t}) HIPCHK(lat, hipMalloc(q, v32));
    HIPCHK(lat, hipMalloc(&W.xs, v32 * nshift));
    HIPCHK(lat, hipMalloc(&W.ps, v32 * nshift));
    HIPCHK(lat, hipMalloc(&W.b64, v64));
    HIPCHK(lat, hipMalloc(&W.x64, v64 * nshift));
    HIPCHK(lat, hipMemcpyAsync(W.ddesc, hd.data(), sizeof(ProbDesc) * nrhs, hipMemcpyHostToDevice, s));
    HIPCHK(lat, hipMemcpyAsync(W.dt2p, t2p.data(), sizeof(int) * t2p.size(), hipMemcpyHostToDevice, s));
    HIPCHK(lat, hipMemcpyAsync(W.b64, b, v64, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    for (int j = 0; j < nrhs; j++) {
        SolveState &st = W.hst[j];
        memset(&st, 0, sizeof st);
        st.status = ST_RUNNING;
        st.tol2 = prm.tol * prm.tol;
        st.maxiter = prm.maxiter;
        ShiftState &ms = W.hms[j];
        memset(&ms, 0, sizeof ms);
        ms.nshift = nshift;
        ms.alpha_old = 1.0;
        ms.beta_old = 0.0;
        for (int k = 0; k < nshift; k++) {
            ms.zeta[k] = ms.zeta_old[k] = 1.0;
            ms.shift[k] = shifts[k] - sbase;
            ms.active[k] = 1;
        }
    }
    HIPCHK(lat, hipMemcpyAsync(W.dst, W.hst, sizeof(SolveState) * nrhs, hipMemcpyHostToDevice, s));
    HIPCHK(lat, hipMemcpyAsync(W.dms, W.hms, sizeof(ShiftState) * nrhs, hipMemcpyHostToDevice, s));

    BlasLaunch bl;
    memset(&bl, 0, sizeof bl);
    bl.probs = W.ddesc;
    bl.tile2prob = W.dt2p;
    bl.states = W.dst;
    bl.ms = W.dms;
    bl.partials = W.dpart;
    bl.v[0] = W.r;
    bl.v[1] = W.Ap;
    bl.v[2] = W.xs;
    bl.v[3] = W.p;
    bl.v[4] = W.ps;
    bl.v[5] = W.b64;
    const int ntot = nrhs * ntile;

    // |b_j|^2 and the initial vectors
    bl.want = ST_RUNNING;
    bl.fin = FIN_NORM_B;
    HIPCHK(lat, launch_ms(BL_MS_INIT, bl, ntot, s));
    HIPCHK(lat, launch_finish(W.ddesc, W.dst, W.dpart, FIN_NORM_B, ST_RUNNING, 1, nrhs, s));

    // tuned shape of the shared-link kernel (tuning runs before any capture)
    const int group = std::min(4, nrhs);
    const TuneChoice tcm = pick_shape_mrhs(lat, kprec, recon, group, (prm.flags & HISQ_NO_TUNE) != 0);
    auto mrhs = [&](int out_par, int epi, const void *in, void *out, const void *aux) -> hipError_t {
        MrhsLaunch a;
        memset(&a, 0, sizeof a);
        a.probs = W.ddesc;
        a.desc_stride = 1;
        a.remap = tcm.remap;
        a.out_par = out_par;
        a.lslot = slot;
        a.nrhs = nrhs;
        a.vstride = h;
        a.in = in;
        a.out = out;
        a.aux = aux;
        a.partials = W.dpart;
        a.states = W.dst;
        a.epi = epi;
        a.want = ST_RUNNING;
        return launch_dslash_mrhs(kprec, recon, group, tcm.W, a, ntile, s);
    };
    auto iterate = [&]() -> hipError_t {
        hipError_t e;
        if ((e = mrhs(1, EPI_PLAIN, W.p, W.t, nullptr)) != hipSuccess) return e;
        if ((e = mrhs(0, EPI_AX, W.t, W.Ap, W.p)) != hipSuccess) return e;
        if ((e = launch_finish(W.ddesc, W.dst, W.dpart, FIN_ALPHA, ST_RUNNING, 1, nrhs, s)) != hipSuccess) return e;
        bl.want = ST_RUNNING;
        bl.fin = FIN_MS;
        if ((e = launch_ms(BL_MS_RUPDATE, bl, ntot, s)) != hipSuccess) return e;
        if ((e = launch_finish(W.ddesc, W.dst, W.dpart, FIN_MS, ST_RUNNING, 1, nrhs, s, W.dms)) != hipSuccess)
            return e;
        bl.fin = FIN_NONE;
        if ((e = launch_ms(BL_MS_UPDATE, bl, ntot, s)) != hipSuccess) return e;
        BlasLaunch st;
        memset(&st, 0, sizeof st);
        st.states = W.dst;
        return launch_blas(BL_STATUS_MS, 0, st, 0, nrhs, s);
    };

    const int kchunk = prm.check_every > 0 ? prm.check_every : 16;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const bool use_graph = (prm.flags & HISQ_USE_GRAPH) != 0;
    if (use_graph) {
        HIPCHK(lat, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t ce = hipSuccess;
        for (int q = 0; q < kchunk && ce == hipSuccess; q++) ce = iterate();
        hipError_t ee = hipStreamEndCapture(s, &graph);
        if (ce != hipSuccess) return hip_err(lat, ce, "graph capture");
        if (ee != hipSuccess) return hip_err(lat, ee, "hipStreamEndCapture");
        HIPCHK(lat, hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    }
    struct GGuard {
        hipGraph_t &g;
        hipGraphExec_t &x;
        ~GGuard()
        {
            if (x) (void)hipGraphExecDestroy(x);
            if (g) (void)hipGraphDestroy(g);
        }
    } gguard{graph, gexec};

    for (;;) {
        if (use_graph) HIPCHK(lat, hipGraphLaunch(gexec, s));
        else
            for (int q = 0; q < kchunk; q++) HIPCHK(lat, iterate());
        HIPCHK(lat, hipMemcpyAsync(W.hst, W.dst, sizeof(SolveState) * nrhs, hipMemcpyDeviceToHost, s));
        HIPCHK(lat, hipStreamSynchronize(s));
        bool any = false;
        for (int j = 0; j < nrhs; j++)
            if (W.hst[j].status == ST_RUNNING) any = true;
        if (!any) break;
    }
    HIPCHK(lat, hipMemcpyAsync(W.hms, W.dms, sizeof(ShiftState) * nrhs, hipMemcpyDeviceToHost, s));
    // x_{j,k} to FP64 for the refinement
    HIPCHK(lat, launch_convert(W.xs, 1, W.x64, 0, (long long)nrhs * nshift * h * 3, s));
    HIPCHK(lat, hipStreamSynchronize(s));
    const double t_krylov = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();

    // refinement: one batched mixed CG over all (j, k), warm start.  The
    // problems are ordered shift-major (set index k * nrhs + j): the shared-
    // link kernel groups neighbours, and one shift's sources need about the
    // same number of iterations, so a group stops reading links when its
    // shifts are done instead of waiting for the slowest shift of a source.
    const int nprob = nrhs * nshift;
    std::vector<hisq_lattice> lats(nprob, lat);
    std::vector<double> ms(nprob, mass), sig(nprob);
    std::vector<const double *> bp(nprob);
    std::vector<double *> xp(nprob);
    for (int k = 0; k < nshift; k++)
        for (int j = 0; j < nrhs; j++) {
            const int pi = k * nrhs + j, q = j * nshift + k;
            sig[pi] = shifts[k];
            bp[pi] = W.b64 + (size_t)j * h * 6;
            xp[pi] = W.x64 + (size_t)q * h * 6;
        }
    hisq_status st = build_set(lat, lat->msref, lats, ms, 0.0, &sig);
    if (st != HISQ_OK) return st;
    hisq_solver_params rp = prm;
    rp.flags = (prm.flags & (HISQ_USE_GRAPH | HISQ_NO_TUNE)) | HISQ_DEVICE_PTR | HISQ_X_IS_GUESS;
    // warm-started refinements reach a reliable update every few iterations:
    // short chunks keep problems from idling until the end of a long one
    const int ce = prm.check_every > 0 ? prm.check_every : 16;
    rp.check_every = ce < 4 ? ce : 4;
    // A warm-started refinement has one to three decades to go: a reliable
    // update per decade would be an FP64 multi-RHS Dslash pair (the costliest
    // launches of the solve) each time a group of shifts crosses a decade, so
    // the sloppy recursion is left to run two decades between them.
    rp.delta = prm.delta < 0.01 ? prm.delta : 0.01;
    if (rp.sloppy == HISQ_F64) rp.sloppy = HISQ_F32;
    if (!lat->ls[(int)rp.sloppy * 2 + (recon == 12)].valid) rp.recon = HISQ_RECON_18;
    if (!lat->ls[(int)rp.sloppy * 2 + (rp.recon == 12)].valid) {
        hisq_status ps = hisq_prepare_links(lat, rp.sloppy, rp.recon);
        if (ps != HISQ_OK) return ps;
    }
    std::vector<hisq_solver_info> rinfo(nprob);
    hisq_status rs = run_cg(lat, lat->msref, rp, bp.data(), xp.data(), rinfo.data());
    if (rs == HISQ_ERR_HIP || rs == HISQ_ERR_OOM || rs == HISQ_ERR_ARG || rs == HISQ_ERR_STATE) return rs;
    HIPCHK(lat, hipMemcpyAsync(x, W.x64, v64 * nshift, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    HIPCHK(lat, hipStreamSynchronize(s));
    const double elapsed = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) {
        for (int j = 0; j < nrhs; j++)
            for (int k = 0; k < nshift; k++) {
                const int q = j * nshift + k, pi = k * nrhs + j;
                hisq_solver_info &in = info[q];
                in = rinfo[pi];
                in.iters = W.hms[j].iters[k] + rinfo[pi].iters;
                in.refine_iters = rinfo[pi].iters;
                in.time_s = elapsed;
                in.t_done_s = t_krylov;   // end of the shared Krylov phase
                const double site = (double)(link_site_bytes(kprec, recon)) / nrhs + 2.0 * 24;
                in.dslash_bytes += (double)h * 2.0 * W.hst[j].iter * site;
                in.flops += 1146.0 * h * 2.0 * W.hst[j].iter;
            }
    }
    if (rs != HISQ_OK) return set_err(lat, rs, "multi-shift refinement did not converge");
    return HISQ_OK;
}

// hisq_dslash with nrhs > 1: FP32 colour vectors, FP32 or FP16 links.
hisq_status hisq_dslash_mrhs_impl(hisq_lattice lat, int out_parity, int prec, int recon, const void *in,
                                  void *out, int nrhs, int flags)
{
    if (prec == 0) return set_err(lat, HISQ_ERR_ARG, "multi-RHS Dslash needs FP32 or FP16 links (FP32 vectors)");
    const int slot = prec * 2 + (recon == 12);
    const long long h = lat->h;
    hipStream_t s = lat->s;
    const void *din = in;
    void *dout = out;
    void *tmp = nullptr;
    const size_t v32 = (size_t)nrhs * h * 24;
    if (!(flags & HISQ_DEVICE_PTR)) {
        HIPCHK(lat, hipMalloc(&tmp, 2 * v32 + (size_t)nrhs * h * 48));
        double *t64 = (double *)((char *)tmp + 2 * v32);
        HIPCHK(lat, hipMemcpyAsync(t64, in, (size_t)nrhs * h * 48, hipMemcpyHostToDevice, s));
        HIPCHK(lat, launch_convert(t64, 0, tmp, 1, (long long)nrhs * h * 3, s));
        din = tmp;
        dout = (char *)tmp + v32;
    }
    const int group = std::min(4, nrhs);
    const TuneChoice tc = pick_shape_mrhs(lat, prec, recon, group, (flags & HISQ_NO_TUNE) != 0);
    MrhsLaunch a;
    memset(&a, 0, sizeof a);
    a.probs = lat->ddesc;
    a.desc_stride = 0;
    a.remap = tc.remap;
    a.out_par = out_parity;
    a.lslot = slot;
    a.nrhs = nrhs;
    a.vstride = h;
    a.in = din;
    a.out = dout;
    a.epi = EPI_PLAIN;
    HIPCHK(lat, launch_dslash_mrhs(prec, recon, group, tc.W, a, lat->ntile, s));
    if (tmp) {
        double *t64 = (double *)((char *)tmp + 2 * v32);
        HIPCHK(lat, launch_convert(dout, 1, t64, 0, (long long)nrhs * h * 3, s));
        HIPCHK(lat, hipMemcpyAsync(out, t64, (size_t)nrhs * h * 48, hipMemcpyDeviceToHost, s));
        HIPCHK(lat, hipStreamSynchronize(s));
        (void)hipFree(tmp);
    }
    return HISQ_OK;
}
