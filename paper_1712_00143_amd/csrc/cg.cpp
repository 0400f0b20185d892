// Conjugate gradient on A = 4m^2 - D_eo D_oe (+ sigma), plain FP64 or mixed
// precision with reliable updates, for one lattice or a batch of lattices.
//
// The paper's solver is MILC's staggered CG (Sections 4, 4.1); mixed precision
// and reliable updates follow the QUDA description it cites (Section 3: mixed
// precision).  The iteration (Hestenes-Stiefel) per problem:
//   t = D_oe p;  Ap = diag p - D_eo t;  alpha = rr / (p, Ap)         [k_dslash x2]
//   r -= alpha Ap; x_lo += alpha p; beta = |r|^2 / rr                [k_blas RUPDATE]
//   p = r + beta p                                                   [k_blas PUPDATE]
// with every scalar in FP64 on the device.  When |r| drops below delta times
// its maximum since the last update, or the recursive residual reaches tol,
// the problem pauses and an FP64 reliable update runs:
//   x_hi += x_lo; x_lo = 0; r_hi = b - A x_hi (FP64 links); if |r_hi| <= tol |b|
//   stop, else r = r_hi, beta = |r_hi|^2 / rr_old, p = r + beta p, continue.
// Chunks of check_every iterations are launched (or replayed as a captured
// HIP graph) between host reads of the per-problem status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <sstream>

#include "finish.h"
#include "solver.h"

using namespace hisq;

#define HIPCHK(lat, x)                                     \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) return hip_err(lat, e_, #x); \
    } while (0)

namespace hisq {

size_t link_site_bytes(int prec, int recon)
{
    size_t el = prec == 0 ? 8 : prec == 1 ? 4 : 2;
    return el * (size_t)recon * NDIR;
}

static size_t spinor_site_bytes(int prec) { return prec == 0 ? 48 : prec == 1 ? 24 : 16; }

hisq_status build_set(hisq_lattice lat0, SolveSet &S, const std::vector<hisq_lattice> &lats,
                      const std::vector<double> &masses, double sigma, const std::vector<double> *sigmas)
{
    const int n = (int)lats.size();
    int ntile = 0;
    long long nsite = 0;
    std::vector<ProbDesc> hd(n);
    std::vector<int> t2p;
    for (int k = 0; k < n; k++) {
        hd[k] = lattice_desc(lats[k]);
        hd[k].tile_begin = ntile;
        hd[k].voff = nsite;
        hd[k].mass = masses[k];
        hd[k].diag = 4.0 * masses[k] * masses[k] + (sigmas ? (*sigmas)[k] : sigma);
        for (int j = 0; j < hd[k].ntile; j++) t2p.push_back(k);
        ntile += hd[k].ntile;
        nsite += hd[k].h;
    }
    bool same = S.nprob == n && S.ntile == ntile && S.nsite == nsite && S.ddesc;
    if (!same) {
        S.release();
        S.nprob = n;
        S.ntile = ntile;
        S.nsite = nsite;
        HIPCHK(lat0, hipMalloc(&S.ddesc, sizeof(ProbDesc) * n));
        if (n > 1) HIPCHK(lat0, hipMalloc(&S.dt2p, sizeof(int) * ntile));
        HIPCHK(lat0, hipMalloc(&S.dst, sizeof(SolveState) * n));
        HIPCHK(lat0, hipHostMalloc(&S.hst, sizeof(SolveState) * n, hipHostMallocDefault));
        HIPCHK(lat0, hipMalloc(&S.dpart, sizeof(double) * NPART * ntile));
        HIPCHK(lat0, hipMalloc(&S.dred, sizeof(double) * 2 * ntile));
        HIPCHK(lat0, hipMemset(S.dst, 0, sizeof(SolveState) * n));
    }
    // the tile -> problem map depends on the order of the problems, not only
    // on the totals compared above
    if (n > 1) HIPCHK(lat0, hipMemcpy(S.dt2p, t2p.data(), sizeof(int) * ntile, hipMemcpyHostToDevice));
    S.hdesc = hd;
    S.max_ntile = 0;
    for (const ProbDesc &d : hd) S.max_ntile = d.ntile > S.max_ntile ? d.ntile : S.max_ntile;
    S.one_lattice = n > 1;
    for (int k = 1; k < n; k++)
        if (lats[k] != lats[0]) S.one_lattice = false;
    HIPCHK(lat0, hipMemcpyAsync(S.ddesc, hd.data(), sizeof(ProbDesc) * n, hipMemcpyHostToDevice, lat0->s));
    HIPCHK(lat0, hipStreamSynchronize(lat0->s));
    return HISQ_OK;
}

struct CgPlan {
    int mode, recon, slot, W, remap, cpol;
    TuneChoice mrhs[5];   // shapes of the shared-link kernel per group size (one-lattice sets)
    int group64 = 0;      // one-lattice sets: FP64 shared-link group size (0: per-problem kernel)
    TuneChoice mrhs64;
};

static hipError_t enqueue_dslash(SolveSet &S, const CgPlan &pl, int prec, int lslot, int out_par, int epi,
                                 int fin, int want, const DVec &in, DVec &out, const DVec *aux,
                                 const double *bvec, int out_prec, hipStream_t s, double *red = nullptr)
{
    DslashLaunch a;
    memset(&a, 0, sizeof a);
    a.probs = S.ddesc;
    a.tile2prob = S.dt2p;
    a.remap = pl.remap;
    a.out_par = out_par;
    a.lslot = lslot;
    a.want = want;
    a.states = S.dst;
    a.in = in.p;
    a.in_nrm = in.n;
    a.out = out.p;
    a.out_nrm = out.n;
    if (aux) {
        a.aux = aux->p;
        a.aux_nrm = aux->n;
    }
    a.bvec = bvec;
    a.partials = S.dpart;
    a.fin = fin;
    a.red = red;
    // the sloppy operator uses the tuned shape; the FP64 reliable-update
    // operator (slot 0: FP64 recon-18) uses the default FP64 shape
    const bool sloppy_op = lslot == pl.slot;
    const int W = sloppy_op ? pl.W : 8;
    const int recon = sloppy_op ? pl.recon : 18;
    a.cpol = sloppy_op ? pl.cpol : 0;
    hipError_t e = launch_dslash(prec, recon, out_prec, epi, W, a, S.ntile, s);
    if (e != hipSuccess || fin == FIN_NONE) return e;
    return launch_finish(S.ddesc, S.dst, S.dpart, fin, want, 1, S.nprob, s);
}

static hipError_t enqueue_blas(SolveSet &S, int op, int mode, int want, int fin, hipStream_t s)
{
    BlasLaunch b;
    memset(&b, 0, sizeof b);
    b.probs = S.ddesc;
    b.tile2prob = S.dt2p;
    b.states = S.dst;
    b.want = want;
    b.fin = fin;
    b.partials = S.dpart;
    b.v[0] = S.rlo.p;
    b.n[0] = S.rlo.n;
    b.v[1] = S.Ap.p;
    b.n[1] = S.Ap.n;
    b.v[2] = S.xlo.p;
    b.n[2] = S.xlo.n;
    b.v[3] = S.p.p;
    b.n[3] = S.p.n;
    b.v[4] = (op == BL_RESUME || op == BL_START) ? S.rhi.p : S.xhi.p;
    b.v[5] = S.b.p;
    b.red = S.dred;
    b.ntot = S.ntile;
    hipError_t e = launch_blas(op, mode, b, S.ntile, S.nprob, s);
    if (e != hipSuccess || fin == FIN_NONE) return e;
    return launch_finish(S.ddesc, S.dst, S.dpart, fin, want, 1, S.nprob, s);
}

// Sloppy FP32 Dslash of a set whose problems all live on one lattice: one
// multi-right-hand-side launch covers every problem, four per link read, so
// the link stream is read once per four problems instead of once per problem.
static hipError_t enqueue_dslash_shared(SolveSet &S, const CgPlan &pl, int out_par, int epi, int fin,
                                        int want, const DVec &in, DVec &out, const DVec *aux, hipStream_t s,
                                        double *red = nullptr)
{
    const int group = S.nprob < 4 ? S.nprob : 4;
    const TuneChoice &tc = pl.mrhs[group];
    MrhsLaunch a;
    memset(&a, 0, sizeof a);
    a.probs = S.ddesc;
    a.desc_stride = 1;
    a.remap = tc.remap;
    a.out_par = out_par;
    a.lslot = pl.slot;
    a.nrhs = S.nprob;
    a.vstride = S.hdesc[0].h;
    a.in = in.p;
    a.out = out.p;
    a.aux = aux ? aux->p : nullptr;
    a.partials = S.dpart;
    a.states = S.dst;
    a.epi = epi;
    a.want = want;
    a.red = red;
    hipError_t e = launch_dslash_mrhs(pl.mode, pl.recon, group, tc.W, a, S.hdesc[0].ntile, s);
    if (e != hipSuccess || fin == FIN_NONE) return e;
    return launch_finish(S.ddesc, S.dst, S.dpart, fin, want, 1, S.nprob, s);
}

// FP64 recon-18 Dslash (reliable updates, initial residual) of a one-lattice
// set through the shared-link kernel: PLAIN out = D in, or RES
// out = b - diag x + D in with |out|^2 partials.
static hipError_t enqueue_dslash64_shared(SolveSet &S, const CgPlan &pl, int out_par, int epi, int fin,
                                          int want, const DVec &in, DVec &out, const DVec *x,
                                          hipStream_t s)
{
    MrhsLaunch a;
    memset(&a, 0, sizeof a);
    a.probs = S.ddesc;
    a.desc_stride = 1;
    a.remap = pl.mrhs64.remap;
    a.out_par = out_par;
    a.lslot = 0;
    a.nrhs = S.nprob;
    a.vstride = S.hdesc[0].h;
    a.in = in.p;
    a.out = out.p;
    a.aux = x ? x->p : nullptr;
    a.bvec = (const double *)S.b.p;
    a.partials = S.dpart;
    a.states = S.dst;
    a.epi = epi;
    a.want = want;
    hipError_t e = launch_dslash_mrhs(0, 18, pl.group64, pl.mrhs64.W, a, S.hdesc[0].ntile, s);
    if (e != hipSuccess || fin == FIN_NONE) return e;
    return launch_finish(S.ddesc, S.dst, S.dpart, fin, want, 1, S.nprob, s);
}

// FP64 half-Dslash pair of the reliable update / initial residual:
// t = D_oe x, r = b - diag x + D_eo t (partials of |r|^2, finisher fin).
static hipError_t enqueue_true_residual(SolveSet &S, const CgPlan &pl, int fin, int want, hipStream_t s)
{
    hipError_t e;
    if (pl.group64 > 0) {
        if ((e = enqueue_dslash64_shared(S, pl, 1, EPI_PLAIN, FIN_NONE, want, S.xhi, S.thi, nullptr, s)) !=
            hipSuccess)
            return e;
        return enqueue_dslash64_shared(S, pl, 0, EPI_RES, fin, want, S.thi, S.rhi, &S.xhi, s);
    }
    if ((e = enqueue_dslash(S, pl, 0, 0, 1, EPI_PLAIN, FIN_NONE, want, S.xhi, S.thi, nullptr, nullptr, 0, s)) !=
        hipSuccess)
        return e;
    return enqueue_dslash(S, pl, 0, 0, 0, EPI_RES, fin, want, S.thi, S.rhi, &S.xhi, (const double *)S.b.p, 0, s);
}

// Largest problem (in 64-site tiles) for which the vector kernels sum their
// problem's tile sums themselves: every block reads ntile doubles, so the
// redundant reads grow as ntile^2; beyond this a separate finisher launch is
// the cheaper way (and a small share of an iteration that large).
static constexpr int FUSE_MAX_TILES = 1024;

static bool fused_step(const SolveSet &S) { return S.max_ntile <= FUSE_MAX_TILES; }

// k CG iterations: t = D_oe p, Ap = diag p - D_eo t with p.Ap per tile, then
// the r/x and p updates.  Fused (problems up to FUSE_MAX_TILES tiles): the
// two vector kernels carry the scalar recurrences themselves from compact
// tile sums; otherwise finisher launches compute alpha and beta in between.
static hipError_t enqueue_iters(SolveSet &S, const CgPlan &pl, int k, hipStream_t s)
{
    const int ap_prec = pl.mode == 2 ? 1 : pl.mode;
    const bool shared = S.one_lattice && pl.mode == 1;
    const bool fused = fused_step(S);
    double *red = fused ? S.dred : nullptr;
    const int fin_a = fused ? FIN_NONE : FIN_ALPHA;
    for (int j = 0; j < k; j++) {
        hipError_t e;
        if (shared) {
            if ((e = enqueue_dslash_shared(S, pl, 1, EPI_PLAIN, FIN_NONE, ST_RUNNING, S.p, S.t, nullptr, s)) !=
                hipSuccess)
                return e;
            if ((e = enqueue_dslash_shared(S, pl, 0, EPI_AX, fin_a, ST_RUNNING, S.t, S.Ap, &S.p, s, red)) !=
                hipSuccess)
                return e;
        } else {
            if ((e = enqueue_dslash(S, pl, pl.mode, pl.slot, 1, EPI_PLAIN, FIN_NONE, ST_RUNNING, S.p, S.t,
                                    nullptr, nullptr, pl.mode, s)) != hipSuccess)
                return e;
            if ((e = enqueue_dslash(S, pl, pl.mode, pl.slot, 0, EPI_AX, fin_a, ST_RUNNING, S.t, S.Ap,
                                    &S.p, nullptr, ap_prec, s, red)) != hipSuccess)
                return e;
        }
        if (fused) {
            if ((e = enqueue_blas(S, BL_RUPDATE_F, pl.mode, ST_RUNNING, FIN_NONE, s)) != hipSuccess) return e;
            if ((e = enqueue_blas(S, BL_PUPDATE_F, pl.mode, ST_RUNNING, FIN_NONE, s)) != hipSuccess) return e;
        } else {
            if ((e = enqueue_blas(S, BL_RUPDATE, pl.mode, ST_RUNNING, FIN_BETA, s)) != hipSuccess) return e;
            if ((e = enqueue_blas(S, BL_PUPDATE, pl.mode, ST_RUNNING, FIN_NONE, s)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

static hipError_t enqueue_reliable(SolveSet &S, const CgPlan &pl, hipStream_t s)
{
    hipError_t e;
    if ((e = enqueue_blas(S, BL_XACCUM, pl.mode, ST_RELIABLE, FIN_NONE, s)) != hipSuccess) return e;
    if ((e = enqueue_true_residual(S, pl, FIN_TRUERES, ST_RELIABLE, s)) != hipSuccess) return e;
    if ((e = enqueue_blas(S, BL_RESUME, pl.mode, ST_RESUME, FIN_NONE, s)) != hipSuccess) return e;
    return enqueue_blas(S, BL_STATUS, pl.mode, 0, FIN_NONE, s);
}

hisq_status run_cg(hisq_lattice lat0, SolveSet &S, const hisq_solver_params &prm, const double *const *b,
                   double *const *x, hisq_solver_info *info, ChunkHook hook, void *hook_ctx)
{
    auto t0 = std::chrono::steady_clock::now();
    const int mode = (int)prm.sloppy;
    const int recon = (int)prm.recon;
    if (mode < 0 || mode > 2 || (recon != 12 && recon != 18))
        return set_err(lat0, HISQ_ERR_ARG, "bad sloppy precision or reconstruction");
    if (!(prm.tol > 0) || prm.maxiter < 1 || !(prm.delta >= 0 && prm.delta < 1))
        return set_err(lat0, HISQ_ERR_ARG, "bad tol, maxiter or delta");
    const int slot = mode * 2 + (recon == 12);
    for (auto &d : S.hdesc)
        if (!d.ls[slot].valid || !d.ls[0].valid)
            return set_err(lat0, HISQ_ERR_STATE, "link set not prepared (hisq_prepare_links)");
    hipStream_t s = lat0->s;
    const int rprec = mode == 0 ? 0 : 1;
    if (S.mode != mode) {
        S.chunks.release();
        S.mode = mode;
    }
    if (S.borrowed) {
        // the caller carved every vector out of memory it owns
        if ((prm.flags & HISQ_USE_GRAPH) || !S.dclock)
            return set_err(lat0, HISQ_ERR_ARG, "borrowed work set: no graphs, a start stamp is required");
        for (DVec *v : {&S.b, &S.xhi, &S.rhi, &S.thi})
            if (!v->p || v->prec != 0 || v->sites != S.nsite) return set_err(lat0, HISQ_ERR_STATE, "work vector");
        for (DVec *v : {&S.xlo, &S.rlo, &S.Ap})
            if (!v->p || v->prec != rprec || v->sites != S.nsite) return set_err(lat0, HISQ_ERR_STATE, "work vector");
        for (DVec *v : {&S.p, &S.t})
            if (!v->p || v->prec != mode || v->sites != S.nsite) return set_err(lat0, HISQ_ERR_STATE, "work vector");
    } else {
        for (DVec *v : {&S.b, &S.xhi, &S.rhi, &S.thi}) HIPCHK(lat0, dvec_alloc(*v, 0, S.nsite));
        for (DVec *v : {&S.xlo, &S.rlo, &S.Ap}) HIPCHK(lat0, dvec_alloc(*v, rprec, S.nsite));
        for (DVec *v : {&S.p, &S.t}) HIPCHK(lat0, dvec_alloc(*v, mode, S.nsite));
    }

    const bool dev = (prm.flags & HISQ_DEVICE_PTR) != 0;
    const bool guess = (prm.flags & HISQ_X_IS_GUESS) != 0;
    const hipMemcpyKind hk = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int k = 0; k < S.nprob; k++) {
        const size_t off = (size_t)S.hdesc[k].voff * 48, nb = (size_t)S.hdesc[k].h * 48;
        HIPCHK(lat0, hipMemcpyAsync((char *)S.b.p + off, b[k], nb, hk, s));
        if (guess) HIPCHK(lat0, hipMemcpyAsync((char *)S.xhi.p + off, x[k], nb, hk, s));
    }
    for (int k = 0; k < S.nprob; k++) {
        SolveState &st = S.hst[k];
        memset(&st, 0, sizeof st);
        st.status = ST_RUNNING;
        st.tol2 = prm.tol * prm.tol;
        st.delta2 = mode == 0 ? 0.0 : prm.delta * prm.delta;
        st.maxiter = prm.maxiter;
    }
    HIPCHK(lat0, hipMemcpyAsync(S.dst, S.hst, sizeof(SolveState) * S.nprob, hipMemcpyHostToDevice, s));

    // one-lattice FP32 sets run their sloppy operator through the shared-link
    // kernel; the single-problem kernel then serves only the FP64 updates,
    // which use the default shape, so it is not tuned for them
    const bool shared = S.one_lattice && mode == 1;
    TuneChoice tc = S.borrowed ? ((prm.flags & HISQ_NO_TUNE) ? pick_shape(lat0, mode, recon, S.ddesc, S.dt2p, S.ntile,
                                                                          S.nsite, S.nprob, true)
                                                             : lookup_shape(lat0, mode, recon, S.ntile, S.nprob))
                               : pick_shape(lat0, mode, recon, S.ddesc, S.dt2p, S.ntile, S.nsite, S.nprob,
                                            shared || (prm.flags & HISQ_NO_TUNE) != 0);
    CgPlan pl{mode, recon, slot, tc.W, tc.remap, tc.cpol, {}};
    if (shared) {
        const int group = S.nprob < 4 ? S.nprob : 4;
        pl.mrhs[group] = pick_shape_mrhs(lat0, mode, recon, group, (prm.flags & HISQ_NO_TUNE) != 0);
    }
    if (S.one_lattice) {
        // FP64 updates: up to four problems per link read (a group smaller
        // than four only when it holds the whole set, as the launch requires)
        const bool nt = (prm.flags & HISQ_NO_TUNE) != 0;
        pl.group64 = S.nprob < 4 ? S.nprob : 4;
        pl.mrhs64 = pick_shape_mrhs(lat0, 0, 18, pl.group64, nt);
    }

    long long *dclock = S.dclock;
    if (!dclock) HIPCHK(lat0, hipMalloc(&dclock, sizeof(long long)));
    HIPCHK(lat0, launch_stamp(dclock, s));
    if (guess) {
        HIPCHK(lat0, enqueue_blas(S, BL_NORM, mode, ST_RUNNING, FIN_NORM_B, s));
        HIPCHK(lat0, enqueue_true_residual(S, pl, FIN_INIT_R, ST_RUNNING, s));
        HIPCHK(lat0, enqueue_blas(S, BL_START, mode, ST_RUNNING, FIN_NONE, s));
    } else {
        HIPCHK(lat0, enqueue_blas(S, BL_INIT, mode, ST_RUNNING, FIN_NORM_B, s));
    }
    HIPCHK(lat0, hipMemcpyAsync(S.hst, S.dst, sizeof(SolveState) * S.nprob, hipMemcpyDeviceToHost, s));
    HIPCHK(lat0, hipStreamSynchronize(s));
    // zero right-hand sides: x = 0 is exact
    for (int k = 0; k < S.nprob; k++)
        if (S.hst[k].bb == 0.0 && S.hst[k].status == ST_RUNNING) {
            int v = ST_CONVERGED;
            HIPCHK(lat0, hipMemcpyAsync(&S.dst[k].status, &v, sizeof v, hipMemcpyHostToDevice, s));
            HIPCHK(lat0, hipStreamSynchronize(s));
            S.hst[k].status = ST_CONVERGED;
        }

    const int kchunk = prm.check_every > 0 ? prm.check_every : 16;
    const bool use_graph = (prm.flags & HISQ_USE_GRAPH) != 0;
    if (use_graph) {
        std::ostringstream ks;
        ks << mode << ":" << recon << ":" << tc.W << ":" << tc.remap << ":" << tc.cpol << ":" << kchunk << ":"
           << S.one_lattice;
        for (int nr = 1; nr <= 4; nr++) ks << ":" << pl.mrhs[nr].W << pl.mrhs[nr].remap;
        ks << ":" << pl.group64 << pl.mrhs64.W << pl.mrhs64.remap << ":" << fused_step(S);
        if (S.chunks.key != ks.str() || !S.chunks.ready()) {
            hipError_t ce = S.chunks.capture(kchunk, s, [&](int len) { return enqueue_iters(S, pl, len, s); });
            if (ce != hipSuccess) {
                S.chunks.release();
                return hip_err(lat0, ce, "graph capture");
            }
            S.chunks.key = ks.str();
        }
    }
    // one problem: chunks sized to end near the next pause; a batch keeps
    // fixed chunks (its paused problems' tiles exit while the others run)
    ChunkPlanner plan(kchunk);
    if (S.nprob == 1) plan.rebase(S.hst[0]);

    std::vector<int> gave_up(S.nprob, 0);
    S.hist.assign(S.nprob, std::vector<double>());
    lat0->last_solve = &S;
    auto record = [&]() {   // a reliable update ran: its FP64 true residual
        for (int k = 0; k < S.nprob; k++) {
            const SolveState &st = S.hst[k];
            if (st.reliable > (int)S.hist[k].size() && st.bb > 0)
                S.hist[k].push_back(std::sqrt(st.rr_true / st.bb));
        }
    };
    for (;;) {
        bool active = false;
        for (int k = 0; k < S.nprob; k++)
            if (S.hst[k].status == ST_RUNNING) active = true;
        if (!active) break;
        const int len = S.nprob == 1 ? plan.next(S.hst[0]) : kchunk;
        if (use_graph) HIPCHK(lat0, S.chunks.launch(len, s));
        else HIPCHK(lat0, enqueue_iters(S, pl, len, s));
        HIPCHK(lat0, hipMemcpyAsync(S.hst, S.dst, sizeof(SolveState) * S.nprob, hipMemcpyDeviceToHost, s));
        HIPCHK(lat0, hipStreamSynchronize(s));
        if (S.nprob == 1 && (S.hst[0].status == ST_RUNNING || S.hst[0].status == ST_RELIABLE)) plan.observe(S.hst[0]);
        if (hook) HIPCHK(lat0, hook(S, hook_ctx, s));
        bool rel = false;
        for (int k = 0; k < S.nprob; k++)
            if (S.hst[k].status == ST_RELIABLE) rel = true;
        if (rel) {
            HIPCHK(lat0, enqueue_reliable(S, pl, s));
            HIPCHK(lat0, hipMemcpyAsync(S.hst, S.dst, sizeof(SolveState) * S.nprob, hipMemcpyDeviceToHost, s));
            HIPCHK(lat0, hipStreamSynchronize(s));
            record();
            if (prm.flags & HISQ_STOP_STAGNATION)
                for (int k = 0; k < S.nprob; k++) {
                    // three reliable updates in a row, none below the true
                    // residual before them: stop with the current iterate
                    const std::vector<double> &hk = S.hist[k];
                    const size_t n = hk.size();
                    if (S.hst[k].status != ST_RUNNING || n < 4) continue;
                    if (std::min(hk[n - 1], std::min(hk[n - 2], hk[n - 3])) < hk[n - 4]) continue;
                    int v = ST_IDLE;
                    HIPCHK(lat0, hipMemcpyAsync(&S.dst[k].status, &v, sizeof v, hipMemcpyHostToDevice, s));
                    HIPCHK(lat0, hipStreamSynchronize(s));
                    S.hst[k].status = ST_IDLE;
                    gave_up[k] = 1;
                }
        }
        for (int k = 0; k < S.nprob; k++) {
            SolveState &st = S.hst[k];
            if (st.status == ST_RUNNING && st.iter >= st.maxiter) {
                int v = ST_IDLE;
                HIPCHK(lat0, hipMemcpyAsync(&S.dst[k].status, &v, sizeof v, hipMemcpyHostToDevice, s));
                HIPCHK(lat0, hipStreamSynchronize(s));
                st.status = ST_IDLE;
                gave_up[k] = 1;
            }
        }
        if (rel && S.nprob == 1 && S.hst[0].status == ST_RUNNING) plan.rebase(S.hst[0]);
    }

    long long clk0 = 0;
    HIPCHK(lat0, hipMemcpyAsync(&clk0, dclock, sizeof clk0, hipMemcpyDeviceToHost, s));
    for (int k = 0; k < S.nprob; k++) {
        const size_t off = (size_t)S.hdesc[k].voff * 48, nb = (size_t)S.hdesc[k].h * 48;
        HIPCHK(lat0, hipMemcpyAsync(x[k], (char *)S.xhi.p + off, nb,
                                    dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    }
    HIPCHK(lat0, hipStreamSynchronize(s));
    if (dclock != S.dclock) (void)hipFree(dclock);
    double elapsed = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int clk_khz = 100000;
    (void)hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, lat0->device);

    hisq_status worst = HISQ_OK;
    for (int k = 0; k < S.nprob; k++) {
        const SolveState &st = S.hst[k];
        hisq_status sk = HISQ_OK;
        if (st.status == ST_BREAKDOWN) sk = HISQ_ERR_BREAKDOWN;
        else if (st.status != ST_CONVERGED) sk = HISQ_ERR_NOT_CONVERGED;
        if (sk != HISQ_OK && worst == HISQ_OK) worst = sk;
        if (info) {
            hisq_solver_info &in = info[k];
            memset(&in, 0, sizeof in);
            const ProbDesc &d = S.hdesc[k];
            in.iters = st.iter;
            in.reliable_updates = st.reliable;
            in.restarts = st.restarts;
            in.converged = st.status == ST_CONVERGED;
            in.status = sk;
            in.true_residual = st.bb > 0 ? std::sqrt(st.rr_true / st.bb) : 0.0;
            in.time_s = elapsed;
            const double site_sloppy = (double)(link_site_bytes(mode, recon) + 2 * spinor_site_bytes(mode));
            const double site_hi = (double)(link_site_bytes(0, 18) + 2 * spinor_site_bytes(0));
            in.dslash_bytes = (double)d.h * (2.0 * st.iter * site_sloppy + 2.0 * st.reliable * site_hi);
            in.flops = 1146.0 * d.h * 2.0 * (st.iter + st.reliable);
            in.t_done_s = st.t_done > 0 ? (double)(st.t_done - clk0) / (clk_khz * 1000.0) : -1.0;
        }
    }
    if (worst != HISQ_OK) {
        set_err(lat0, worst, worst == HISQ_ERR_BREAKDOWN ? "CG breakdown" : "CG did not converge");
    }
    return worst;
}

}  // namespace hisq

extern "C" {

hisq_status hisq_cg(hisq_lattice lat, double mass, const double *b, double *x,
                    const hisq_solver_params *params, hisq_solver_info *info)
{
    if (!lat || !b || !x) return set_err(lat, HISQ_ERR_ARG, "null argument");
    if (!lat->loaded) return set_err(lat, HISQ_ERR_STATE, "no links loaded");
    if (!(mass > 0)) return set_err(lat, HISQ_ERR_ARG, "mass must be > 0");
    hisq_solver_params prm;
    if (params) prm = *params;
    else hisq_default_params(&prm);
    HIPCHK(lat, hipSetDevice(lat->device));
    std::vector<hisq_lattice> lats{lat};
    std::vector<double> ms{mass};
    hisq_status st = build_set(lat, lat->cg, lats, ms, 0.0);
    if (st != HISQ_OK) return st;
    const double *bb[1] = {b};
    double *xx[1] = {x};
    return run_cg(lat, lat->cg, prm, bb, xx, info);
}

hisq_status hisq_batch_cg(int nprob, const hisq_lattice *lats, const double *masses, const double *const *b,
                          double *const *x, const hisq_solver_params *params, hisq_solver_info *info)
{
    if (nprob < 1 || !lats || !masses || !b || !x) return set_err(nullptr, HISQ_ERR_ARG, "bad batch arguments");
    hisq_lattice l0 = lats[0];
    if (!l0) return set_err(nullptr, HISQ_ERR_ARG, "null handle");
    std::vector<hisq_lattice> v(lats, lats + nprob);
    std::vector<double> ms(masses, masses + nprob);
    for (int k = 0; k < nprob; k++) {
        if (!v[k] || !b[k] || !x[k]) return set_err(l0, HISQ_ERR_ARG, "null problem entry");
        if (v[k]->device != l0->device) return set_err(l0, HISQ_ERR_ARG, "handles on different devices");
        if (!v[k]->loaded) return set_err(l0, HISQ_ERR_STATE, "no links loaded");
        if (!(ms[k] > 0)) return set_err(l0, HISQ_ERR_ARG, "mass must be > 0");
    }
    hisq_solver_params prm;
    if (params) prm = *params;
    else hisq_default_params(&prm);
    HIPCHK(l0, hipSetDevice(l0->device));
    SolveSet &S = l0->batch;   // reused across calls with the same shape
    hisq_status st = build_set(l0, S, v, ms, 0.0);
    if (st != HISQ_OK) return st;
    return run_cg(l0, S, prm, b, x, info);
}

}  // extern "C"

