// HISQ link smearing, the Symanzik gauge force and the HISQ fermion force:
// host orchestration of the link kernels and the C-ABI entry points
// hisq_smear_links, hisq_fat7, hisq_unitarize, hisq_gauge_force,
// hisq_gauge_action, hisq_fermion_force_links and hisq_fermion_force.
//
// fat7(U; c1, c3, c5, c7; cL) for output direction mu is built with staple
// reuse: the three 3-staple fields T1_nu are formed once, every 5-staple is
// a staple of one of them and every 7-staple a staple of the 5-staples,
// summed over the two orders of its transverse steps before the last
// staple is taken (the staple is linear in the field it transports).
#include <vector>

#include <cmath>
#include <cstring>

#include "fforce.h"
#include "gforce.h"
#include "smear.h"
#include "solver.h"

using namespace hisq;

#define HIPCHK(lat, x)                                     \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) return hip_err(lat, e_, #x); \
    } while (0)

namespace {

constexpr double LV1[5] = {1.0 / 8, 1.0 / 16, 1.0 / 64, 1.0 / 384, 0.0};
constexpr double LV2[5] = {5.0 / 8, 1.0 / 16, 1.0 / 64, 1.0 / 384, -1.0 / 16};
constexpr double NAIK = -1.0 / 24;

SmearGeom geom_of(hisq_lattice lat)
{
    SmearGeom g;
    g.V = lat->V;
    g.P = plane_stride(lat->V);
    for (int k = 0; k < 4; k++) g.L[k] = lat->L[k];
    g.S[0] = 1;
    g.S[1] = lat->L[0];
    g.S[2] = lat->L[0] * lat->L[1];
    g.S[3] = lat->L[0] * lat->L[1] * lat->L[2];
    return g;
}

// Workspace: nf one-direction planar fields (9 P double2 each), a 256-byte
// slot for the projection's failure counter and `extra` bytes of partials.
struct Work {
    double2 *f = nullptr;   // field k at f + k * 9 P
    int *bad = nullptr;
    double *part = nullptr;
    size_t fsz = 0;         // double2 per field
    double2 *field(int k) const { return f + (size_t)k * fsz; }
};

hisq_status get_work(hisq_lattice lat, int nf, Work &w, size_t extra = 0)
{
    w.fsz = (size_t)9 * plane_stride(lat->V);
    const size_t need = (size_t)nf * w.fsz * sizeof(double2) + 256 + extra;
    if (lat->smear_ws_bytes < need) {
        if (lat->smear_ws) {
            HIPCHK(lat, hipStreamSynchronize(lat->s));
            HIPCHK(lat, hipFree(lat->smear_ws));
            lat->smear_ws = nullptr;
            lat->smear_ws_bytes = 0;
        }
        HIPCHK(lat, hipMalloc(&lat->smear_ws, need));
        lat->smear_ws_bytes = need;
    }
    w.f = (double2 *)lat->smear_ws;
    w.bad = (int *)((char *)lat->smear_ws + (size_t)nf * w.fsz * sizeof(double2));
    w.part = (double *)((char *)w.bad + 256);
    return HISQ_OK;
}

// out (4 planar fields) = fat7(U (4 planar fields)): one pass 1 for every
// direction, with a Lepage term one Lepage pass, then per output direction
// one pass 2 (its 5-staple sums) and one pass 3 (their c5 share and the
// 7-staples).  T1all: 12 fields (every direction's 3-staples).  Hall: 24
// fields for the single-sign 3-staples, needed when cL != 0 (and kept for
// the adjoint).  keep: T2all holds 12 fields and direction mu's 5-staple
// sums stay in its fields 3 mu .. 3 mu + 2 (for the adjoint); otherwise
// T2all is three fields, reused for every direction.
hipError_t run_fat7(const SmearGeom &g, const double2 *U, double2 *out, double2 *T1all, double2 *T2all,
                    double2 *Hall, const double c[5], size_t fsz, hipStream_t s, bool keep = false)
{
    const bool need5 = c[2] != 0.0 || c[3] != 0.0, lep = c[4] != 0.0;
    if (lep && !Hall) return hipErrorInvalidValue;
    Pass1Args p1{U, out, need5 ? T1all : nullptr, lep ? Hall : nullptr, c[0], c[1]};
    hipError_t e = launch_smear_pass1(g, p1, s);
    if (e == hipSuccess && lep) {
        const LepageArgs la{U, Hall, out, c[4]};
        e = launch_smear_lepage(g, la, s);
    }
    if (e != hipSuccess || !need5) return e;
    for (int mu = 0; mu < 4; mu++) {
        double2 *T2 = keep ? T2all + (size_t)3 * mu * fsz : T2all;
        const Pass2Args p2{U, T1all + (size_t)3 * mu * fsz, T2, mu};
        if ((e = launch_smear_pass2(g, p2, s)) != hipSuccess) return e;
        const Pass3Args p3{U, T2, out + (size_t)mu * fsz, c[2], c[3], mu};
        if ((e = launch_smear_pass3(g, p3, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t link_array_bytes(hisq_lattice lat) { return (size_t)lat->V * 4 * 18 * sizeof(double); }

// Bring a [V][4][3][3] array onto the device: its own pointer with
// HISQ_DEVICE_PTR, else a copy into `stage` (at least link_array_bytes).
hisq_status stage_in(hisq_lattice lat, const double *src, int flags, double2 *stage, const double2 **dev)
{
    if (flags & HISQ_DEVICE_PTR) {
        *dev = (const double2 *)src;
        return HISQ_OK;
    }
    HIPCHK(lat, hipMemcpyAsync(stage, src, link_array_bytes(lat), hipMemcpyHostToDevice, lat->s));
    *dev = stage;
    return HISQ_OK;
}

hisq_status check_projection(hisq_lattice lat, const int *bad)
{
    int h = 0;
    HIPCHK(lat, hipMemcpyAsync(&h, bad, sizeof h, hipMemcpyDeviceToHost, lat->s));
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    if (h) return set_err(lat, HISQ_ERR_BREAKDOWN, std::to_string(h) + " links have no U(3) projection (V^+ V singular or not finite)");
    return HISQ_OK;
}

}  // namespace

extern "C" {

hisq_status hisq_fat7(hisq_lattice lat, const double coef[5], const double *in, double *out, int flags)
{
    if (!lat || !coef || !in || !out) return set_err(lat, HISQ_ERR_ARG, "null argument");
    HIPCHK(lat, hipSetDevice(lat->device));
    Work w;
    hisq_status st = get_work(lat, 51, w);   // U 0-3, result 4-7, staging 8-11, T1 12-23, T2 24-26, H 27-50
    if (st != HISQ_OK) return st;
    const SmearGeom g = geom_of(lat);
    const double2 *src;
    if ((st = stage_in(lat, in, flags, w.field(8), &src)) != HISQ_OK) return st;
    HIPCHK(lat, launch_smear_to_planar(g, src, w.field(0), lat->s));
    HIPCHK(lat, run_fat7(g, w.field(0), w.field(4), w.field(12), w.field(24), w.field(27), coef, w.fsz, lat->s));
    if (flags & HISQ_DEVICE_PTR) {
        HIPCHK(lat, launch_smear_from_planar(g, w.field(4), (double2 *)out, lat->s));
    } else {
        HIPCHK(lat, launch_smear_from_planar(g, w.field(4), w.field(8), lat->s));
        HIPCHK(lat, hipMemcpyAsync(out, w.field(8), link_array_bytes(lat), hipMemcpyDeviceToHost, lat->s));
    }
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    return HISQ_OK;
}

hisq_status hisq_unitarize(hisq_lattice lat, const double *in, double *out, int flags)
{
    if (!lat || !in || !out) return set_err(lat, HISQ_ERR_ARG, "null argument");
    HIPCHK(lat, hipSetDevice(lat->device));
    Work w;
    hisq_status st = get_work(lat, 8, w);   // planar 0-3, staging 4-7
    if (st != HISQ_OK) return st;
    const SmearGeom g = geom_of(lat);
    const double2 *src;
    if ((st = stage_in(lat, in, flags, w.field(4), &src)) != HISQ_OK) return st;
    HIPCHK(lat, launch_smear_to_planar(g, src, w.field(0), lat->s));
    HIPCHK(lat, hipMemsetAsync(w.bad, 0, sizeof(int), lat->s));
    HIPCHK(lat, launch_smear_unitarize(g, w.field(0), w.bad, lat->s));
    if (flags & HISQ_DEVICE_PTR) {
        HIPCHK(lat, launch_smear_from_planar(g, w.field(0), (double2 *)out, lat->s));
    } else {
        HIPCHK(lat, launch_smear_from_planar(g, w.field(0), w.field(4), lat->s));
        HIPCHK(lat, hipMemcpyAsync(out, w.field(4), link_array_bytes(lat), hipMemcpyDeviceToHost, lat->s));
    }
    return check_projection(lat, w.bad);
}

hisq_status hisq_smear_links(hisq_lattice lat, const double *thin, double *fat, double *lng, int flags)
{
    const bool load = (flags & HISQ_LOAD_RESULT) != 0;
    if (!lat || !thin || (!load && (!fat || !lng)) || (!fat != !lng))
        return set_err(lat, HISQ_ERR_ARG, "null argument");
    HIPCHK(lat, hipSetDevice(lat->device));
    const bool dev = (flags & HISQ_DEVICE_PTR) != 0;
    // fields: thin U 0-3, level 1 / projected W 4-7, level 2 X 8-11 (also the
    // host input staging), T1 12-23, T2 24-26, H 27-50, output staging 51-58
    // for host outputs that are not loaded
    const bool stage_out = !dev && !load;
    Work w;
    hisq_status st = get_work(lat, stage_out ? 59 : 51, w);
    if (st != HISQ_OK) return st;
    const SmearGeom g = geom_of(lat);
    const double2 *src;
    if ((st = stage_in(lat, thin, flags, w.field(8), &src)) != HISQ_OK) return st;
    HIPCHK(lat, launch_smear_to_planar(g, src, w.field(0), lat->s));
    HIPCHK(lat, run_fat7(g, w.field(0), w.field(4), w.field(12), w.field(24), nullptr, LV1, w.fsz, lat->s));
    HIPCHK(lat, hipMemsetAsync(w.bad, 0, sizeof(int), lat->s));
    HIPCHK(lat, launch_smear_unitarize(g, w.field(4), w.bad, lat->s));
    HIPCHK(lat, run_fat7(g, w.field(4), w.field(8), w.field(12), w.field(24), w.field(27), LV2, w.fsz, lat->s));
    double2 *of, *ol;
    if (load) {
        const size_t bytes = link_array_bytes(lat);
        if (!lat->fat64) HIPCHK(lat, hipMalloc(&lat->fat64, bytes));
        if (!lat->lng64) HIPCHK(lat, hipMalloc(&lat->lng64, bytes));
        of = (double2 *)lat->fat64;
        ol = (double2 *)lat->lng64;
    } else if (dev) {
        of = (double2 *)fat;
        ol = (double2 *)lng;
    } else {
        of = w.field(51);
        ol = w.field(55);
    }
    HIPCHK(lat, launch_smear_output(g, w.field(8), w.field(4), NAIK, of, ol, lat->s));
    if ((st = check_projection(lat, w.bad)) != HISQ_OK) {
        if (load) {   // the FP64 copies no longer match any packed set
            for (auto &ls : lat->ls) ls = LinkSet();
            lat->cg.release();
            lat->loaded = false;
        }
        return st;
    }
    if (fat && (load || !dev)) {
        const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        HIPCHK(lat, hipMemcpyAsync(fat, of, link_array_bytes(lat), k, lat->s));
        HIPCHK(lat, hipMemcpyAsync(lng, ol, link_array_bytes(lat), k, lat->s));
    }
    if (load) return adopt_device_links(lat);
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    return HISQ_OK;
}

static hisq_status gauge_args(hisq_lattice lat, const double *U, const double coef[3], const void *out)
{
    if (!lat || !U || !coef || !out) return set_err(lat, HISQ_ERR_ARG, "null argument");
    for (int k = 0; k < 4; k++)
        if (lat->L[k] < 4) return set_err(lat, HISQ_ERR_ARG, "the gauge force and action need every extent >= 4");
    return HISQ_OK;
}

hisq_status hisq_gauge_force(hisq_lattice lat, const double *U, double beta, const double coef[3], double *F,
                             int flags)
{
    hisq_status st = gauge_args(lat, U, coef, F);
    if (st != HISQ_OK) return st;
    HIPCHK(lat, hipSetDevice(lat->device));
    Work w;
    if ((st = get_work(lat, 12, w)) != HISQ_OK) return st;   // U 0-3, F 4-7, staging 8-11
    const SmearGeom g = geom_of(lat);
    const double2 *src;
    if ((st = stage_in(lat, U, flags, w.field(8), &src)) != HISQ_OK) return st;
    HIPCHK(lat, launch_smear_to_planar(g, src, w.field(0), lat->s));
    GForceArgs a{w.field(0), w.field(4), nullptr, coef[0], coef[1], coef[2], beta / 3.0, 0, 0};
    HIPCHK(lat, launch_gauge_force(g, a, 0, lat->s));
    if (flags & HISQ_DEVICE_PTR) {
        HIPCHK(lat, launch_smear_from_planar(g, w.field(4), (double2 *)F, lat->s));
    } else {
        HIPCHK(lat, launch_smear_from_planar(g, w.field(4), w.field(8), lat->s));
        HIPCHK(lat, hipMemcpyAsync(F, w.field(8), link_array_bytes(lat), hipMemcpyDeviceToHost, lat->s));
    }
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    return HISQ_OK;
}

hisq_status hisq_gauge_action(hisq_lattice lat, const double *U, double beta, const double coef[3], double *S,
                              int flags)
{
    hisq_status st = gauge_args(lat, U, coef, S);
    if (st != HISQ_OK) return st;
    HIPCHK(lat, hipSetDevice(lat->device));
    int ntile, tch, nb;
    gauge_force_grid(geom_of(lat), &ntile, &tch, &nb);
    const size_t nblk = (size_t)nb;
    Work w;
    if ((st = get_work(lat, 8, w, nblk * sizeof(double))) != HISQ_OK) return st;   // U 0-3, staging 4-7
    const SmearGeom g = geom_of(lat);
    const double2 *src;
    if ((st = stage_in(lat, U, flags, w.field(4), &src)) != HISQ_OK) return st;
    HIPCHK(lat, launch_smear_to_planar(g, src, w.field(0), lat->s));
    // each loop is met once per link it holds: weights over the loop lengths
    GForceArgs a{w.field(0), nullptr, w.part, coef[0] / 4.0, coef[1] / 6.0, coef[2] / 6.0, 1.0, 0, 0};
    HIPCHK(lat, launch_gauge_force(g, a, 1, lat->s));
    std::vector<double> part(nblk);
    HIPCHK(lat, hipMemcpyAsync(part.data(), w.part, part.size() * sizeof(double), hipMemcpyDeviceToHost, lat->s));
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    double re = 0.0;
    for (double v : part) re += v;   // fixed order: the same bits every call
    const double V = (double)lat->V;
    *S = beta * (V * (6.0 * coef[0] + 12.0 * coef[1] + 16.0 * coef[2]) - re / 3.0);
    return HISQ_OK;
}

}  // extern "C"

// ------------------------------------------------------------ fermion force

namespace {

// Gradient of sum Re Tr(fat7(Ul; c)_mu(x) G_mu(x)) with respect to Ul, added
// to GU (four planar fields each): every pass is undone by its gather-form
// adjoint, reading the forward intermediates run_fat7 kept (T1all, T2all:
// 12 fields each; Hall: the 24 single-sign 3-staples of the Lepage term,
// needed when cL != 0).  sc: 6 scratch fields.
hipError_t fat7_adjoint(const SmearGeom &g, const double2 *Ul, const double c[5], const double2 *G, double2 *GU,
                        const double2 *T1all, const double2 *T2all, const double2 *Hall, double2 *sc, size_t fsz,
                        hipStream_t s)
{
    double2 *GT1 = sc, *GT2 = sc + 3 * fsz, *GHp = sc + 4 * fsz, *GHm = sc + 5 * fsz;
    const bool need5 = c[2] != 0.0 || c[3] != 0.0, lep = c[4] != 0.0;
    if (lep && !Hall) return hipErrorInvalidValue;
    hipError_t e;
    auto U_ = [&](int d) { return Ul + (size_t)d * fsz; };
    auto GU_ = [&](int d) { return GU + (size_t)d * fsz; };
    // both signs of the staple through d, one field M, gradient Gin; with Gb,
    // GM starts from gb Gb (gm_init) or adds it
    auto adj = [&](int mu, int d, const double2 *M, const double2 *Gin, double2 *GM, double2 *GUd, double coef,
                   const double2 *Gb = nullptr, double gb = 0.0, int init = 0) {
        StapleAdjArgs a{U_(d), {M, M}, {{Gin, nullptr}, {Gin, nullptr}}, {GM, GM}, GUd, coef, mu, d, init, {}, Gb, gb};
        const int f[2] = {d, mu};
        smear_order(f, 2, a.ord);
        return launch_staple_adjoint(g, a, s);
    };
    for (int mu = 0; mu < 4; mu++) {
        int perp[3], np = 0;
        for (int d = 0; d < 4; d++)
            if (d != mu) perp[np++] = d;
        const double2 *Gmu = G + (size_t)mu * fsz;
        // forward intermediates: the kept 3- and 5-staple fields of this
        // direction (and, for the Lepage term, its single-sign 3-staples)
        const double2 *T1 = T1all + (size_t)3 * mu * fsz, *T2 = T2all + (size_t)3 * mu * fsz;
        // reverse.  The direct shares of G_mu (c1 on U_mu, c3 on each T1,
        // c5 on each T2) enter with the first pass that writes the gradient
        // field (Gb / gb of the staple adjoint) instead of passes of their own.
        if (need5) {
            // the 3-staple gradients GT1_j are first written by the 5-staple
            // adjoints of k = 0 (j = 1, 2) and k = 1 (j = 0)
            bool gt1_set[3] = {false, false, false};
            for (int k = 0; k < 3; k++) {
                const int sig = perp[k], inu = (k + 1) % 3, irho = (k + 2) % 3;
                const int nu = perp[inu], rho = perp[irho];
                if (c[3] != 0.0) {
                    if ((e = adj(mu, sig, T2 + k * fsz, Gmu, GT2, GU_(sig), c[3], Gmu, c[2], 1)) != hipSuccess) return e;
                } else if ((e = launch_field_axpby(GT2, 0.0, Gmu, c[2], fsz, s)) != hipSuccess) {
                    return e;
                }
                for (const int j : {inu, irho}) {
                    // T1_nu is transported through rho and T1_rho through nu
                    const int dj = j == inu ? rho : nu;
                    const bool first = !gt1_set[j];
                    gt1_set[j] = true;
                    if ((e = adj(mu, dj, T1 + j * fsz, GT2, GT1 + j * fsz, GU_(dj), 1.0, first ? Gmu : nullptr,
                                 first ? c[1] : 0.0, first ? 1 : 0)) != hipSuccess)
                        return e;
                }
            }
        } else {
            for (int k = 0; k < 3; k++)
                if ((e = launch_field_axpby(GT1 + k * fsz, 0.0, Gmu, c[1], fsz, s)) != hipSuccess) return e;
        }
        for (int k = 0; k < 3; k++) {
            const int nu = perp[k];
            // the one-link share c1 G_mu joins U_mu's gradient in its first pass
            const double2 *gb = k == 0 ? Gmu : nullptr;
            const double cb = k == 0 ? c[0] : 0.0;
            if (!lep) {
                if ((e = adj(mu, nu, U_(mu), GT1 + k * fsz, GU_(mu), GU_(nu), 1.0, gb, cb)) != hipSuccess) return e;
                continue;
            }
            // Lepage = S+(H+) + S-(H-), S+- the single-sign staples through nu:
            // first the gradients of H+- (and the links' share), then every
            // staple of U_mu through nu at once (its 3-staple gradient GT1 on
            // both signs, GH+- on one each)
            const double2 *Hp = Hall + (size_t)(6 * mu + 2 * k) * fsz, *Hm = Hp + fsz;
            StapleAdjArgs a1{U_(nu), {Hp, Hm}, {{Gmu, nullptr}, {Gmu, nullptr}}, {GHp, GHm}, GU_(nu), c[4], mu, nu, 1,
                             {}};
            StapleAdjArgs a2{U_(nu), {U_(mu), U_(mu)}, {{GT1 + k * fsz, GHp}, {GT1 + k * fsz, GHm}},
                             {GU_(mu), GU_(mu)}, GU_(nu), 1.0, mu, nu, 0, {}, gb, cb};
            const int f[2] = {nu, mu};
            smear_order(f, 2, a1.ord);
            smear_order(f, 2, a2.ord);
            if ((e = launch_staple_adjoint(g, a1, s)) != hipSuccess) return e;
            if ((e = launch_staple_adjoint(g, a2, s)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hisq_status ff_check(hisq_lattice lat, int n, const double *alpha, const double *X, const void *out)
{
    if (!lat || !alpha || !X || !out) return set_err(lat, HISQ_ERR_ARG, "null argument");
    if (n < 1 || n > 64) return set_err(lat, HISQ_ERR_ARG, "the number of terms must be in [1, 64]");
    for (int k = 0; k < n; k++)
        if (!std::isfinite(alpha[k])) return set_err(lat, HISQ_ERR_ARG, "non-finite weight");
    return HISQ_OK;
}

// Y_k = D_oe X_k on the lattice's FP64 links; X, Y device [n][h][3] complex.
// One multi-right-hand-side launch: each link read serves four vectors.
hisq_status ff_solutions_odd(hisq_lattice lat, int n, const double2 *X, double2 *Y)
{
    if (n < 1) return HISQ_OK;
    const int group = n < 4 ? n : 4;
    const TuneChoice tc = pick_shape_mrhs(lat, 0, 18, group, false);
    MrhsLaunch a;
    memset(&a, 0, sizeof a);
    a.probs = lat->ddesc;
    a.desc_stride = 0;
    a.remap = tc.remap;
    a.out_par = HISQ_ODD;
    a.lslot = 0;   // FP64 recon-18
    a.nrhs = n;
    a.vstride = lat->h;
    a.in = X;
    a.out = Y;
    a.epi = EPI_PLAIN;
    hipError_t e = launch_dslash_mrhs(0, 18, group, tc.W, a, lat->ntile, lat->s);
    if (e != hipSuccess) return hip_err(lat, e, "D_oe of the solution vectors");
    return HISQ_OK;
}

}  // namespace

extern "C" {

hisq_status hisq_fermion_force_links(hisq_lattice lat, int n, const double *alpha, const double *X, double *OF,
                                     double *OL, int flags)
{
    hisq_status st = ff_check(lat, n, alpha, X, OF);
    if (st != HISQ_OK) return st;
    if (!OL) return set_err(lat, HISQ_ERR_ARG, "null argument");
    if (!lat->loaded) return set_err(lat, HISQ_ERR_STATE, "no links loaded");
    HIPCHK(lat, hipSetDevice(lat->device));
    const size_t vb = (size_t)n * lat->h * 3 * sizeof(double2);
    Work w;
    if ((st = get_work(lat, 12, w, 2 * vb + 64 * sizeof(double))) != HISQ_OK) return st;   // OF 0-3, OL 4-7, staging 8-11
    double2 *Xd = (double2 *)w.part, *Yd = Xd + (size_t)n * lat->h * 3;
    double *ad = (double *)(Yd + (size_t)n * lat->h * 3);
    const bool dev = (flags & HISQ_DEVICE_PTR) != 0;
    HIPCHK(lat, hipMemcpyAsync(Xd, X, vb, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, lat->s));
    HIPCHK(lat, hipMemcpyAsync(ad, alpha, n * sizeof(double), hipMemcpyHostToDevice, lat->s));
    if ((st = ff_solutions_odd(lat, n, Xd, Yd)) != HISQ_OK) return st;
    const SmearGeom g = geom_of(lat);
    OuterArgs oa{Xd, Yd, ad, n, lat->h, w.field(0), w.field(4), 0, 0.0};
    HIPCHK(lat, launch_ff_outer(g, oa, lat->s));
    double *outs[2] = {OF, OL};
    for (int k = 0; k < 2; k++) {
        if (dev) {
            HIPCHK(lat, launch_smear_from_planar(g, w.field(4 * k), (double2 *)outs[k], lat->s));
        } else {
            HIPCHK(lat, launch_smear_from_planar(g, w.field(4 * k), w.field(8), lat->s));
            HIPCHK(lat, hipMemcpyAsync(outs[k], w.field(8), link_array_bytes(lat), hipMemcpyDeviceToHost, lat->s));
        }
    }
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    return HISQ_OK;
}

hisq_status hisq_fermion_force(hisq_lattice lat, const double *U, int n, const double *alpha, const double *X,
                               double *F, int flags)
{
    hisq_status st = ff_check(lat, n, alpha, X, F);
    if (st != HISQ_OK) return st;
    if (!U) return set_err(lat, HISQ_ERR_ARG, "null argument");
    HIPCHK(lat, hipSetDevice(lat->device));
    const size_t vb = (size_t)n * lat->h * 3 * sizeof(double2);
    // fields: U 0-3, level-1 sum 4-7, W 8-11, level-2 sum then GX 12-15, GN
    // 16-19, GW 20-23, GU 24-27 (also the input and output staging), the
    // kept 3- and 5-staples of level 1 28-51 and of level 2 52-75, the
    // single-sign 3-staples of level 2 76-99, scratch 100-105
    Work w;
    if ((st = get_work(lat, 106, w, 2 * vb + 64 * sizeof(double))) != HISQ_OK) return st;
    const size_t fsz = w.fsz;
    const SmearGeom g = geom_of(lat);
    const bool dev = (flags & HISQ_DEVICE_PTR) != 0;
    // the smearing, keeping its level-1 sum and projection for the chain rule;
    // the smeared links become the lattice's links (the Dslash of D_oe X)
    const double2 *src;
    if ((st = stage_in(lat, U, flags, w.field(24), &src)) != HISQ_OK) return st;
    HIPCHK(lat, launch_smear_to_planar(g, src, w.field(0), lat->s));
    HIPCHK(lat, run_fat7(g, w.field(0), w.field(4), w.field(28), w.field(40), nullptr, LV1, fsz, lat->s, true));
    HIPCHK(lat, launch_field_axpby(w.field(8), 0.0, w.field(4), 1.0, 4 * fsz, lat->s));
    HIPCHK(lat, hipMemsetAsync(w.bad, 0, sizeof(int), lat->s));
    HIPCHK(lat, launch_smear_unitarize(g, w.field(8), w.bad, lat->s));
    if ((st = check_projection(lat, w.bad)) != HISQ_OK) return st;
    HIPCHK(lat, run_fat7(g, w.field(8), w.field(12), w.field(52), w.field(64), w.field(76), LV2, fsz, lat->s, true));
    {
        const size_t bytes = link_array_bytes(lat);
        if (!lat->fat64) HIPCHK(lat, hipMalloc(&lat->fat64, bytes));
        if (!lat->lng64) HIPCHK(lat, hipMalloc(&lat->lng64, bytes));
        HIPCHK(lat, launch_smear_output(g, w.field(12), w.field(8), NAIK, (double2 *)lat->fat64, (double2 *)lat->lng64,
                                        lat->s));
        if ((st = adopt_device_links(lat)) != HISQ_OK) return st;
    }
    double2 *Xd = (double2 *)w.part, *Yd = Xd + (size_t)n * lat->h * 3;
    double *ad = (double *)(Yd + (size_t)n * lat->h * 3);
    HIPCHK(lat, hipMemcpyAsync(Xd, X, vb, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, lat->s));
    HIPCHK(lat, hipMemcpyAsync(ad, alpha, n * sizeof(double), hipMemcpyHostToDevice, lat->s));
    if ((st = ff_solutions_odd(lat, n, Xd, Yd)) != HISQ_OK) return st;
    // gradients with respect to the level-2 sum (phases folded) and the Naik product
    OuterArgs oa{Xd, Yd, ad, n, lat->h, w.field(12), w.field(16), 1, NAIK};
    HIPCHK(lat, launch_ff_outer(g, oa, lat->s));
    HIPCHK(lat, hipMemsetAsync(w.field(20), 0, 4 * fsz * sizeof(double2), lat->s));
    HIPCHK(lat, launch_ff_naik_adjoint(g, w.field(8), w.field(16), w.field(20), lat->s));
    HIPCHK(lat, fat7_adjoint(g, w.field(8), LV2, w.field(12), w.field(20), w.field(52), w.field(64), w.field(76),
                             w.field(100), fsz, lat->s));
    HIPCHK(lat, launch_ff_unitarize_adjoint(g, w.field(4), w.field(20), lat->s));
    HIPCHK(lat, hipMemsetAsync(w.field(24), 0, 4 * fsz * sizeof(double2), lat->s));
    HIPCHK(lat, fat7_adjoint(g, w.field(0), LV1, w.field(20), w.field(24), w.field(28), w.field(40), nullptr,
                             w.field(100), fsz, lat->s));
    HIPCHK(lat, launch_ff_project(g, w.field(0), w.field(24), w.field(24), lat->s));
    if (dev) {
        HIPCHK(lat, launch_smear_from_planar(g, w.field(24), (double2 *)F, lat->s));
    } else {
        HIPCHK(lat, launch_smear_from_planar(g, w.field(24), w.field(12), lat->s));
        HIPCHK(lat, hipMemcpyAsync(F, w.field(12), link_array_bytes(lat), hipMemcpyDeviceToHost, lat->s));
    }
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    return HISQ_OK;
}

}  // extern "C"
