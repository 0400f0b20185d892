// Learned preconditioner: the PTC network's C ABI, training-pair harvesting
// and training (forward, backward and Adam on the GPU).
//
// The preconditioner is M = 1 + E^+ K^+ K E: E embeds an even vector on the
// full lattice, K = L_n ... L_1 is the stack of PTC layers and K^+ its exact
// adjoint (the layers with adjoint weights, in reverse order).  M is Hermitian
// positive definite by construction, like the inverse A^-1 it stands in for,
// which keeps the flexible CG that uses it well behaved; with zero weights it
// is the identity and the flexible CG is plain CG.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <random>
#include <string>
#include <vector>

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

namespace {

struct PairBlock {
    hisq_lattice lat;
    double mass;        // of the operator A the pairs belong to (A e_i = r_i)
    float *mem;         // [n][2][h][3] complex: r_i then e_i
    std::vector<double> ee;   // |e_i|^2
    std::vector<double> er;   // <e_i, r_i> = |e_i|_A^2
    int n;
};

}  // namespace

struct hisq_ptc_s {
    hisq_lattice lat = nullptr;
    int device = 0;          // kept so that destruction never touches a handle
    int nlayer = 0;
    std::vector<int> chans;
    std::vector<int> woff;   // complex offset of each layer
    int nw = 0;              // complex weights in total
    float *w32 = nullptr, *m = nullptr, *v = nullptr;
    float *wa32 = nullptr;   // adjoint weights of every layer (FP32)
    __half *w16 = nullptr, *wa16 = nullptr;
    double *gw = nullptr, *gtmp = nullptr;
    int step = 0;
    int loss = HISQ_LOSS_ENERGY;
    // link format of the transports, the same for training and inference
    int tprec = HISQ_F32, trecon = HISQ_RECON_18;
    int tslot() const { return tprec * 2 + (trecon == 12); }
    std::vector<PairBlock> pairs;
    // training workspace
    int wsB = 0;
    long long wsV = 0;
    float *act = nullptr;
    double *part = nullptr;
    size_t part_n = 0;
    double *dloss = nullptr, *dee = nullptr;
    // inference workspace
    float *inf = nullptr;
    long long infV = 0;
    // activation storage of inference (hisq_ptc_set_activations): FP32
    // [C][2][h][3] through k_ptc_layer, or FP16 [2][h][C][3] with per-site
    // scales through k_ptc_infer
    int aprec = HISQ_F32;
    __half2 *inf16 = nullptr;
    float *infsc = nullptr;
    long long inf16V = 0;
    ChunkGraphs fcg_graph;
};

namespace {

int cmax(const hisq_ptc_s *n)
{
    int c = 1;
    for (int x : n->chans) c = std::max(c, x);
    return c;
}

// the packed fat links the network's transports read, prepared on demand
hisq_status ensure_transport_links(const hisq_ptc_s *n, hisq_lattice lat)
{
    if (lat->ls[n->tslot()].valid) return HISQ_OK;
    return hisq_prepare_links(lat, (hisq_prec)n->tprec, (hisq_recon)n->trecon);
}

// adjoint weights (FP32 and FP16) of every layer from the FP32 master
hipError_t refresh_adjoint(hisq_ptc_s *n, hipStream_t s)
{
    for (int l = 0; l < n->nlayer; l++) {
        hipError_t e = launch_ptc_adjoint(n->w32 + 2 * n->woff[l], n->chans[l], n->chans[l + 1],
                                          n->wa32 + 2 * n->woff[l], s);
        if (e != hipSuccess) return e;
    }
    return launch_to_half(n->wa32, n->wa16, 2 * n->nw, s);
}

PtcLaunch base_launch(hisq_lattice lat, int lslot)
{
    PtcLaunch a;
    memset(&a, 0, sizeof a);
    a.probs = lat->ddesc;
    a.lslot = lslot;
    a.in_zero_par = -1;
    a.out_pstride = 2;
    a.g_pstride = 2;
    return a;
}

// Waves per block of the layer kernel (1, 3, 5 or 9, sharing the 9
// transport paths) for this geometry, channel pair, batch and link format:
// timed once on scratch activations, then cached.  Must not run under stream
// capture.
int pick_layer_waves(hisq_lattice lat, int lslot, int prec, int recon, bool w16, const void *w, int cin, int cout,
                     int in_zero, int npar, int batch, hipStream_t stream)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, lat->device) != hipSuccess) return 9;
    char key[256];
    snprintf(key, sizeof key, "ptc:%s:t%d:p%d:r%d:w%d:%dx%d:z%d:np%d:b%d", prop.gcnArchName, lat->ntile, prec, recon,
             (int)w16, cin, cout, in_zero, npar, batch);
    std::string k(key);
    for (auto &ch : k)
        if (ch == ' ') ch = '_';
    TuneChoice c;
    if (Tuner::get().lookup(k, c)) return c.W;
    if (Tuner::get().disabled()) return 3;
    const long long h = lat->h;
    float *in = nullptr, *out = nullptr;
    if (hipMalloc(&in, sizeof(float) * (size_t)batch * cin * 2 * h * 6) != hipSuccess ||
        hipMalloc(&out, sizeof(float) * (size_t)batch * cout * 2 * h * 6) != hipSuccess) {
        if (in) (void)hipFree(in);
        return 9;
    }
    (void)hipMemsetAsync(in, 0, sizeof(float) * (size_t)batch * cin * 2 * h * 6, stream);
    PtcLaunch a = base_launch(lat, lslot);
    a.w = w;
    a.in = in;
    a.in_bstride = (long long)cin * 2 * h * 6;
    a.in_zero_par = in_zero;
    a.out = out;
    a.out_bstride = (long long)cout * 2 * h * 6;
    a.out_pstride = 2;
    a.out_par0 = 0;
    a.par_lo = 0;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    TuneChoice best;
    best.W = 9;
    best.us = 1e30;
    // three interleaved trials of every shape, each shape's best trial counts
    // (a single short trial is at the mercy of clock ramps and neighbours)
    const int Ws[4] = {1, 3, 5, 9};
    double tbest[4] = {1e30, 1e30, 1e30, 1e30};
    bool okw[4] = {true, true, true, true};
    for (int j = 0; j < 4; j++)
        for (int r = 0; r < 2 && okw[j]; r++)
            okw[j] = launch_ptc_layer(prec, recon, w16, cin, cout, Ws[j], a, lat->ntile * npar, batch, stream) ==
                     hipSuccess;
    for (int trial = 0; trial < 3; trial++)
        for (int j = 0; j < 4; j++) {
            if (!okw[j]) continue;
            const int reps = 10;
            (void)hipEventRecord(e0, stream);
            for (int r = 0; r < reps; r++)
                (void)launch_ptc_layer(prec, recon, w16, cin, cout, Ws[j], a, lat->ntile * npar, batch, stream);
            (void)hipEventRecord(e1, stream);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tbest[j] = std::min(tbest[j], 1000.0 * ms / reps);
        }
    for (int j = 0; j < 4; j++)
        if (okw[j]) Tuner::get().note(k, Ws[j], 0, 0, tbest[j]);
    for (int j = 0; j < 4; j++)
        if (okw[j] && tbest[j] < best.us) {
            best.us = tbest[j];
            best.W = Ws[j];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(in);
    (void)hipFree(out);
    (void)hipGetLastError();
    if (best.us < 1e29) Tuner::get().store(k, best);
    return best.W;
}

// One layer application over output parities [plo, phi].  fz (may be null):
// gate the launch on the solver status; with addin, out += addin (the
// identity term of M) and the (q, out) tile sums of the flexible CG.
hipError_t run_layer(hisq_lattice lat, int lslot, int prec, int recon, bool w16, const void *w, int cin, int cout,
                     const float *in, long long in_bs, int in_zero, float *out, long long out_bs, int out_pstride,
                     int plo, int phi, int batch, hipStream_t stream, const PtcFuse *fz = nullptr,
                     const float *addin = nullptr, long long addin_bs = 0)
{
    const int W = pick_layer_waves(lat, lslot, prec, recon, w16, w, cin, cout, in_zero, phi - plo + 1, batch, stream);
    PtcLaunch a = base_launch(lat, lslot);
    if (fz) {
        a.gate = fz->gate;
        a.gate_want = fz->want;
    }
    a.addin = addin;
    a.addin_bstride = addin_bs;
    if (fz && fz->red && addin) {
        a.dotq = fz->q;
        a.dotred = fz->red;
        a.dot_nt = fz->nt;
    }
    a.w = w;
    a.in = in;
    a.in_bstride = in_bs;
    a.in_zero_par = in_zero;
    a.out = out;
    a.out_bstride = out_bs;
    a.out_pstride = out_pstride;
    a.out_par0 = plo;
    a.par_lo = plo;
    const int nblk = lat->ntile * (phi - plo + 1);
    return launch_ptc_layer(prec, recon, w16, cin, cout, W, a, nblk, batch, stream);
}

// Weight gradient of one layer application, summed over the output parities
// where g lives (g_pstride 1: even only), added into gw (FP64, the layer's
// own [cout][cin][9] layout).
hipError_t run_wgrad(hisq_ptc_s *n, hisq_lattice lat, int cin, int cout, const float *in, long long in_bs, int in_zero,
                     const float *g, long long g_bs, int g_pstride, int batch, double *gw, int accumulate,
                     hipStream_t s)
{
    PtcLaunch a = base_launch(lat, n->tslot());
    a.in = in;
    a.in_bstride = in_bs;
    a.in_zero_par = in_zero;
    a.g = g;
    a.g_bstride = g_bs;
    a.g_pstride = g_pstride;
    a.partials = n->part;
    // one partial row per block; enough blocks to fill the device, at most one
    // per work unit
    const long long units = (long long)lat->ntile * g_pstride * batch;
    const int nrow = (int)(units < WGRAD_ROWS ? units : WGRAD_ROWS);
    hipError_t e = launch_ptc_wgrad(n->tprec, n->trecon, cin, cout, a, g_pstride, batch, nrow, s);
    if (e != hipSuccess) return e;
    return launch_ptc_wsum(n->part, nrow, cin, cout, gw, accumulate, s);
}

// z = M(r) for `batch` even vectors (FP32 [batch][h][3]); `ws` holds two
// full-lattice activations of cmax channels per batch entry.  The identity
// term is added by the last layer.  fz: see run_layer (batch 1).
hipError_t apply_net(hisq_ptc_s *n, hisq_lattice lat, int lslot, int prec, int recon, bool w16, const float *r,
                     float *z, float *ws, int batch, hipStream_t s, const PtcFuse *fz = nullptr)
{
    const long long h = lat->h;
    const long long act = (long long)cmax(n) * 2 * h * 6;   // floats per batch entry
    float *bufs[2] = {ws, ws + act * batch};
    const float *cur = r;
    long long cur_bs = h * 6;
    int cur_zero = 1;   // the input is an even vector embedded with zero odd sites
    int k = 0;
    for (int l = 0; l < n->nlayer; l++) {
        const void *w = w16 ? (const void *)(n->w16 + 2 * n->woff[l]) : (const void *)(n->w32 + 2 * n->woff[l]);
        hipError_t e = run_layer(lat, lslot, prec, recon, w16, w, n->chans[l], n->chans[l + 1], cur, cur_bs, cur_zero,
                                 bufs[k], act, 2, 0, 1, batch, s, fz);
        if (e != hipSuccess) return e;
        cur = bufs[k];
        cur_bs = act;
        cur_zero = -1;
        k ^= 1;
    }
    for (int l = n->nlayer - 1; l >= 0; l--) {
        const void *w = w16 ? (const void *)(n->wa16 + 2 * n->woff[l]) : (const void *)(n->wa32 + 2 * n->woff[l]);
        const bool last = l == 0;
        hipError_t e = last ? run_layer(lat, lslot, prec, recon, w16, w, n->chans[l + 1], n->chans[l], cur, cur_bs,
                                        -1, z, h * 6, 1, 0, 0, batch, s, fz, r, h * 6)
                            : run_layer(lat, lslot, prec, recon, w16, w, n->chans[l + 1], n->chans[l], cur, cur_bs,
                                        -1, bufs[k], act, 2, 0, 1, batch, s, fz);
        if (e != hipSuccess) return e;
        cur = bufs[k];
        k ^= 1;
    }
    return hipSuccess;
}

}  // namespace

// Waves per block of the FP16-activation inference layer (1, 3 or 9, the last
// two also with matrix-core channel mixing), timed
// once per geometry, channel pair, input / output kind and link format on
// scratch activations, then cached.  Must not run under stream capture.
int pick_infer_waves(hisq_lattice lat, int lslot, int prec, int recon, const void *w16, int cin, int cout, int ik,
                     int ok, int npar, hipStream_t stream)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, lat->device) != hipSuccess) return 3;
    char key[256];
    snprintf(key, sizeof key, "ptcinf:%s:t%d:p%d:r%d:%dx%d:k%d%d:np%d", prop.gcnArchName, lat->ntile, prec, recon, cin,
             cout, ik, ok, npar);
    std::string k(key);
    for (auto &ch : k)
        if (ch == ' ') ch = '_';
    TuneChoice c;
    if (Tuner::get().lookup(k, c)) return c.W;
    if (Tuner::get().disabled()) return 3;
    const long long h = lat->h;
    const size_t act = (size_t)2 * h * 8 * 12, sc = (size_t)2 * h * 4;   // up to 8 channels
    char *buf = nullptr;
    if (hipMalloc(&buf, 2 * (act + sc) + (size_t)h * 48) != hipSuccess) return 3;
    (void)hipMemsetAsync(buf, 0, 2 * (act + sc) + (size_t)h * 48, stream);
    PtcInferLaunch a;
    memset(&a, 0, sizeof a);
    a.probs = lat->ddesc;
    a.lslot = lslot;
    a.par_lo = 0;
    a.w = w16;
    a.in16 = reinterpret_cast<const __half2 *>(buf);
    a.in_scale = reinterpret_cast<const float *>(buf + act);
    a.out16 = reinterpret_cast<__half2 *>(buf + act + sc);
    a.out_scale = reinterpret_cast<float *>(buf + 2 * act + sc);
    a.in32 = reinterpret_cast<const float *>(buf + 2 * (act + sc));
    a.out32 = reinterpret_cast<float *>(buf + 2 * (act + sc));   // read and written: timing only
    a.addin = a.in32;
    const int nblk = lat->ntile * npar;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    // vector-ALU channel mixing with 1, 3 or 9 waves, matrix-core mixing with
    // 3 or 9 (layers with at least as many outputs as inputs)
    constexpr int NWI = 5;
    const int Ws[NWI] = {1, 3, 9, 3 | PTC_MFMA, 9 | PTC_MFMA};
    double tbest[NWI] = {1e30, 1e30, 1e30, 1e30, 1e30};
    bool okw[NWI] = {true, true, true, cout >= cin, cout >= cin};
    for (int j = 0; j < NWI; j++)
        for (int r = 0; r < 2 && okw[j]; r++)
            okw[j] = launch_ptc_infer(prec, recon, cin, cout, ik, ok, Ws[j], a, nblk, stream) == hipSuccess;
    for (int trial = 0; trial < 3; trial++)
        for (int j = 0; j < NWI; j++) {
            if (!okw[j]) continue;
            const int reps = 10;
            (void)hipEventRecord(e0, stream);
            for (int r = 0; r < reps; r++) (void)launch_ptc_infer(prec, recon, cin, cout, ik, ok, Ws[j], a, nblk, stream);
            (void)hipEventRecord(e1, stream);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tbest[j] = std::min(tbest[j], 1000.0 * ms / reps);
        }
    TuneChoice best;
    best.W = 3;
    best.us = 1e30;
    for (int j = 0; j < NWI; j++)
        if (okw[j]) Tuner::get().note(k, Ws[j], 0, 0, tbest[j]);
    for (int j = 0; j < NWI; j++)
        if (okw[j] && tbest[j] < best.us) {
            best.us = tbest[j];
            best.W = Ws[j];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    (void)hipGetLastError();
    if (best.us < 1e29) Tuner::get().store(k, best);
    return best.W;
}

// z = M(r) with FP16 activation storage: the forward layers from the even
// FP32 r, the adjoint layers back, the last one writing z = r + E^+ K^+ K E r
// in FP32 with the flexible CG's (q, z) tile sums (fz).
hipError_t apply_net_infer16(hisq_ptc_s *n, hisq_lattice lat, int lslot, int prec, int recon, const float *r, float *z,
                             hipStream_t s, const PtcFuse *fz)
{
    const long long h = lat->h;
    const int C = cmax(n);
    const long long act = 2 * h * C * 3;   // half2 per activation
    if (n->inf16V < act) {
        if (n->inf16) (void)hipFree(n->inf16);
        if (n->infsc) (void)hipFree(n->infsc);
        n->inf16 = nullptr;
        n->infsc = nullptr;
        n->inf16V = 0;
        hipError_t e = hipMalloc(&n->inf16, sizeof(__half2) * 2 * act);
        if (e == hipSuccess) e = hipMalloc(&n->infsc, sizeof(float) * 2 * 2 * h);
        if (e != hipSuccess) return e;
        n->inf16V = act;
    }
    __half2 *bufs[2] = {n->inf16, n->inf16 + act};
    float *scs[2] = {n->infsc, n->infsc + 2 * h};
    auto base = [&]() {
        PtcInferLaunch a;
        memset(&a, 0, sizeof a);
        a.probs = lat->ddesc;
        a.lslot = lslot;
        if (fz) {
            a.gate = fz->gate;
            a.gate_want = fz->want;
        }
        return a;
    };
    int k = 0;
    const int L = n->nlayer;
    // forward layers: l = 0 reads the even r, the rest the previous activation
    for (int l = 0; l < L; l++) {
        const int cin = n->chans[l], cout = n->chans[l + 1], ik = l == 0 ? 0 : 1;
        const void *w = n->w16 + 2 * n->woff[l];
        const int W = pick_infer_waves(lat, lslot, prec, recon, w, cin, cout, ik, 0, 2, s);
        PtcInferLaunch a = base();
        a.w = w;
        a.in32 = r;
        a.in16 = bufs[k ^ 1];
        a.in_scale = scs[k ^ 1];
        a.out16 = bufs[k];
        a.out_scale = scs[k];
        hipError_t e = launch_ptc_infer(prec, recon, cin, cout, ik, 0, W, a, 2 * lat->ntile, s);
        if (e != hipSuccess) return e;
        k ^= 1;
    }
    // adjoint layers in reverse order; the last writes z on the even sites
    for (int l = L - 1; l >= 0; l--) {
        const int cin = n->chans[l + 1], cout = n->chans[l];
        const bool last = l == 0;
        const void *w = n->wa16 + 2 * n->woff[l];
        const int W = pick_infer_waves(lat, lslot, prec, recon, w, cin, cout, 1, last ? 1 : 0, last ? 1 : 2, s);
        PtcInferLaunch a = base();
        a.w = w;
        a.in16 = bufs[k ^ 1];
        a.in_scale = scs[k ^ 1];
        if (last) {
            a.out32 = z;
            a.addin = r;
            if (fz && fz->red) {
                a.dotq = fz->q;
                a.dotred = fz->red;
                a.dot_nt = fz->nt;
            }
        } else {
            a.out16 = bufs[k];
            a.out_scale = scs[k];
        }
        hipError_t e = launch_ptc_infer(prec, recon, cin, cout, 1, last ? 1 : 0, W, a, (last ? 1 : 2) * lat->ntile, s);
        if (e != hipSuccess) return e;
        k ^= 1;
    }
    return hipSuccess;
}

// z = M(r) for the flexible CG: FP16 weights, transports on link set `lslot`.
// fz (may be null): the flexible CG's status gate and (q, z) tile sums.
hipError_t ptc_apply_internal(hisq_ptc n, hisq_lattice lat, int lslot, int prec, int recon, const float *r, float *z,
                              const PtcFuse *fz)
{
    if (n->aprec == HISQ_F16) return apply_net_infer16(n, lat, lslot, prec, recon, r, z, lat->s, fz);
    const long long need = (long long)cmax(n) * 2 * lat->h * 6 * 2;
    if (n->infV < need) {
        if (n->inf) (void)hipFree(n->inf);
        hipError_t e = hipMalloc(&n->inf, need * 4);
        if (e != hipSuccess) return e;
        n->infV = need;
    }
    return apply_net(n, lat, lslot, prec, recon, true, r, z, n->inf, 1, lat->s, fz);
}

// Everything of the network that a captured launch of apply_net holds by
// value: the network, its weight and workspace pointers and its shape.
ChunkGraphs &ptc_fcg_graph(hisq_ptc n)
{
    return n->fcg_graph;
}

std::string ptc_graph_key(hisq_ptc n)
{
    std::string k;
    char buf[160];
    snprintf(buf, sizeof buf, "%p:%p:%p:%p:%lld:%d:%p:%p:%lld:", (const void *)n, (const void *)n->w16,
             (const void *)n->wa16, (const void *)n->inf, n->infV, n->aprec, (const void *)n->inf16,
             (const void *)n->infsc, n->inf16V);
    k = buf;
    for (int c : n->chans) k += std::to_string(c) + ",";
    return k;
}

extern "C" {

hisq_status hisq_ptc_create(hisq_lattice lat, int nlayer, const int *chans, hisq_ptc *out)
{
    if (!lat || !chans || !out || nlayer < 1 || nlayer > 8) return set_err(lat, HISQ_ERR_ARG, "bad network arguments");
    if (chans[0] != 1) return set_err(lat, HISQ_ERR_ARG, "the first channel count must be 1");
    for (int l = 0; l <= nlayer; l++)
        if (chans[l] != 1 && chans[l] != 2 && chans[l] != 4 && chans[l] != 8)
            return set_err(lat, HISQ_ERR_ARG, "channel counts must be 1, 2, 4 or 8");
    for (int l = 0; l < nlayer; l++) {
        int a = chans[l], b = chans[l + 1];
        bool ok = (a == 1 || b == 1 || a == b || (a == 2 && b == 4) || (a == 4 && b == 2));
        if (!ok || (a == 1 && b == 1 && false)) return set_err(lat, HISQ_ERR_ARG, "unsupported channel transition");
        if ((a == 8 && b != 8 && b != 1) || (b == 8 && a != 8 && a != 1))
            return set_err(lat, HISQ_ERR_ARG, "unsupported channel transition");
    }
    HIPCHK(lat, hipSetDevice(lat->device));
    hisq_ptc n = new hisq_ptc_s();
    n->lat = lat;
    n->device = lat->device;
    n->nlayer = nlayer;
    n->chans.assign(chans, chans + nlayer + 1);
    int maxw = 0;
    for (int l = 0; l < nlayer; l++) {
        n->woff.push_back(n->nw);
        n->nw += 9 * chans[l] * chans[l + 1];
        maxw = std::max(maxw, 9 * chans[l] * chans[l + 1]);
    }
    const size_t nf = (size_t)2 * n->nw;
    if (hipMalloc(&n->w32, nf * 4) != hipSuccess || hipMalloc(&n->m, nf * 4) != hipSuccess ||
        hipMalloc(&n->v, nf * 4) != hipSuccess || hipMalloc(&n->wa32, nf * 4) != hipSuccess ||
        hipMalloc(&n->w16, nf * 2) != hipSuccess || hipMalloc(&n->wa16, nf * 2) != hipSuccess ||
        hipMalloc(&n->gw, nf * 8) != hipSuccess || hipMalloc(&n->gtmp, (size_t)2 * maxw * 8) != hipSuccess ||
        hipMalloc(&n->dloss, 8 * 65536) != hipSuccess) {
        hisq_ptc_destroy(n);
        return set_err(lat, HISQ_ERR_OOM, "network allocation failed");
    }
    for (void *p : {(void *)n->w32, (void *)n->m, (void *)n->v, (void *)n->wa32}) (void)hipMemset(p, 0, nf * 4);
    (void)hipMemset(n->w16, 0, nf * 2);
    (void)hipMemset(n->wa16, 0, nf * 2);
    (void)hipMemset(n->gw, 0, nf * 8);
    *out = n;
    return HISQ_OK;
}

hisq_status hisq_ptc_destroy(hisq_ptc n)
{
    if (!n) return HISQ_ERR_ARG;
    // the lattice handles may already be gone: touch only the device
    (void)hipSetDevice(n->device);
    (void)hipDeviceSynchronize();
    n->fcg_graph.release();
    for (void *p : {(void *)n->w32, (void *)n->m, (void *)n->v, (void *)n->wa32, (void *)n->w16, (void *)n->wa16,
                    (void *)n->gw, (void *)n->gtmp, (void *)n->act, (void *)n->part, (void *)n->dloss,
                    (void *)n->dee, (void *)n->inf, (void *)n->inf16, (void *)n->infsc})
        if (p) (void)hipFree(p);
    for (auto &pb : n->pairs)
        if (pb.mem) (void)hipFree(pb.mem);
    delete n;
    return HISQ_OK;
}

hisq_status hisq_ptc_set_weights(hisq_ptc n, const double *w)
{
    if (!n || !w) return HISQ_ERR_ARG;
    hisq_lattice lat = n->lat;
    std::vector<float> f(2 * n->nw);
    for (int j = 0; j < 2 * n->nw; j++) f[j] = (float)w[j];
    HIPCHK(lat, hipMemcpy(n->w32, f.data(), f.size() * 4, hipMemcpyHostToDevice));
    // the FP16 inference copies are rounded from the FP32 master on the device
    // (round to nearest even), as after every Adam step
    HIPCHK(lat, launch_to_half(n->w32, n->w16, 2 * n->nw, lat->s));
    HIPCHK(lat, refresh_adjoint(n, lat->s));
    HIPCHK(lat, hipMemsetAsync(n->m, 0, f.size() * 4, lat->s));
    HIPCHK(lat, hipMemsetAsync(n->v, 0, f.size() * 4, lat->s));
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    n->step = 0;
    return HISQ_OK;
}

hisq_status hisq_ptc_get_weights(hisq_ptc n, double *w)
{
    if (!n || !w) return HISQ_ERR_ARG;
    std::vector<float> f(2 * n->nw);
    HIPCHK(n->lat, hipStreamSynchronize(n->lat->s));
    HIPCHK(n->lat, hipMemcpy(f.data(), n->w32, f.size() * 4, hipMemcpyDeviceToHost));
    for (int j = 0; j < 2 * n->nw; j++) w[j] = f[j];
    return HISQ_OK;
}

// Polynomial starting point.  With D_f the one-hop (fat-link) part of D, the
// stack is set to K = a (1 + D_f^2 / lambda): the first layer copies r into
// channel 0 and D_f r into channel 1, the next hop layer applies D_f to
// channel 1 once more, any further layers pass both channels through, and the
// last layer sums a * ch0 + (a c / lambda) * ch1, i.e. K = a (1 + c D_f^2 /
// lambda).  D_f is anti-Hermitian, so on an eigenvector of -D_f^2 with
// eigenvalue t the preconditioner is M = 1 + a^2 (1 - c t / lambda)^2: the
// low modes, which set the condition number of A, are enlarged up to 1 + a^2
// times against the upper part of the spectrum.  lambda, the largest eigenvalue of -D_f^2 on even sites, is
// estimated by power iteration on D_f^4 (a two-layer K = D_f^2 network, so
// that M - 1 = D_f^4), with FP32 transports.
hisq_status hisq_ptc_init_polynomial(hisq_ptc n, double a, double c, int iters, double *lambda)
{
    if (!n) return HISQ_ERR_ARG;
    hisq_lattice lat = n->lat;
    if (!(a > 0.0) || !std::isfinite(a) || !(c > 0.0) || !(c <= 4.0) || iters < 1 || iters > 1000)
        return set_err(lat, HISQ_ERR_ARG, "polynomial start: a > 0, 0 < c <= 4 and 1 <= iters <= 1000 required");
    if (n->nlayer < 2) return set_err(lat, HISQ_ERR_ARG, "polynomial start needs at least two layers");
    for (int l = 1; l < n->nlayer; l++)
        if (n->chans[l] < 2) return set_err(lat, HISQ_ERR_ARG, "polynomial start needs two inner channels");
    HIPCHK(lat, hipSetDevice(lat->device));
    hisq_status st = ensure_transport_links(n, lat);
    if (st != HISQ_OK) return st;

    // one hop: weight +1 on the forward paths, -1 on the backward ones
    auto hop = [](double *w9) {
        for (int mu = 0; mu < 4; mu++) {
            w9[2 * (1 + 2 * mu)] = 1.0;
            w9[2 * (2 + 2 * mu)] = -1.0;
        }
    };

    // power iteration
    const long long h = lat->h, nf = h * 6;
    hisq_ptc t = nullptr;
    const int tch[3] = {1, 1, 1};
    st = hisq_ptc_create(lat, 2, tch, &t);
    if (st != HISQ_OK) return st;
    std::vector<double> tw(2 * t->nw, 0.0);
    hop(&tw[0]);
    hop(&tw[18]);
    float *dv = nullptr;
    double lam2 = 0.0;
    st = hisq_ptc_set_weights(t, tw.data());
    if (st == HISQ_OK && hipMalloc(&dv, sizeof(float) * 2 * nf) != hipSuccess)
        st = set_err(lat, HISQ_ERR_OOM, "polynomial start: vector allocation failed");
    if (st == HISQ_OK) {
        std::vector<float> v(nf), z(nf);
        std::mt19937_64 gen(0x9e3779b97f4a7c15ull);
        std::normal_distribution<float> nd(0.f, 1.f);
        for (auto &x : v) x = nd(gen);
        for (int it = 0; it < iters && st == HISQ_OK; it++) {
            double vv = 0.0, vz = 0.0;
            for (long long j = 0; j < nf; j++) vv += (double)v[j] * v[j];
            if (!(vv > 0.0)) {
                st = set_err(lat, HISQ_ERR_BREAKDOWN, "polynomial start: power iteration reached zero");
                break;
            }
            hipError_t e = hipMemcpy(dv, v.data(), sizeof(float) * nf, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = ptc_apply_internal(t, lat, n->tslot(), n->tprec, n->trecon, dv, dv + nf, nullptr);
            if (e == hipSuccess) e = hipStreamSynchronize(lat->s);
            if (e == hipSuccess) e = hipMemcpy(z.data(), dv + nf, sizeof(float) * nf, hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                st = hip_err(lat, e, "polynomial start power iteration");
                break;
            }
            // M v - v = D_f^4 v; Re<v, D_f^4 v> is the Rayleigh quotient's numerator
            const double inv = 1.0 / std::sqrt(vv);
            for (long long j = 0; j < nf; j++) {
                const double d = (double)z[j] - (double)v[j];
                vz += (double)v[j] * d;
                z[j] = (float)(d * inv);
            }
            lam2 = vz / vv;
            v.swap(z);
        }
    }
    if (dv) (void)hipFree(dv);
    hisq_ptc_destroy(t);
    if (st != HISQ_OK) return st;
    if (!(lam2 > 0.0) || !std::isfinite(lam2))
        return set_err(lat, HISQ_ERR_BREAKDOWN, "polynomial start: no positive spectrum estimate");
    const double lam = std::sqrt(lam2);

    std::vector<double> w(2 * n->nw, 0.0);
    for (int l = 0; l < n->nlayer; l++) {
        const int ci = n->chans[l], co = n->chans[l + 1];
        double *wl = &w[2 * n->woff[l]];
        auto at = [&](int c, int cp) { return wl + 2 * 9 * (c * ci + cp); };
        const bool last = l == n->nlayer - 1;
        if (l == 0) {
            at(0, 0)[0] = 1.0;
            hop(at(1, 0));
        } else if (!last) {
            at(0, 0)[0] = 1.0;
            if (l == 1) hop(at(1, 1));
            else at(1, 1)[0] = 1.0;
        }
        if (last) {
            at(0, 0)[0] = a;
            if (l == 1) {
                // two layers: the second hop is taken here
                double *p = at(0, 1);
                hop(p);
                for (int k = 0; k < 18; k++) p[k] *= a * c / lam;
            } else {
                at(0, 1)[0] = a * c / lam;
            }
        }
    }
    st = hisq_ptc_set_weights(n, w.data());
    if (st != HISQ_OK) return st;
    if (lambda) *lambda = lam;
    return HISQ_OK;
}

hisq_status hisq_ptc_layer_forward(hisq_ptc n, int layer, const void *in, void *out, int flags)
{
    if (!n || !in || !out || layer < 0 || layer >= n->nlayer) return HISQ_ERR_ARG;
    hisq_lattice lat = n->lat;
    if (!(flags & HISQ_DEVICE_PTR)) return set_err(lat, HISQ_ERR_ARG, "layer calls take device pointers");
    HIPCHK(lat, hipSetDevice(lat->device));
    hisq_status st = ensure_transport_links(n, lat);
    if (st != HISQ_OK) return st;
    const int cin = n->chans[layer], cout = n->chans[layer + 1];
    HIPCHK(lat, run_layer(lat, n->tslot(), n->tprec, n->trecon, false, n->w32 + 2 * n->woff[layer], cin, cout, (const float *)in, 0, -1,
                          (float *)out, 0, 2, 0, 1, 1, lat->s));
    return HISQ_OK;
}

hisq_status hisq_ptc_layer_backward(hisq_ptc n, int layer, const void *in, const void *gout, void *gin, double *gw,
                                    int flags)
{
    if (!n || !in || !gout || layer < 0 || layer >= n->nlayer) return HISQ_ERR_ARG;
    hisq_lattice lat = n->lat;
    if (!(flags & HISQ_DEVICE_PTR)) return set_err(lat, HISQ_ERR_ARG, "layer calls take device pointers");
    HIPCHK(lat, hipSetDevice(lat->device));
    hisq_status st = ensure_transport_links(n, lat);
    if (st != HISQ_OK) return st;
    const int cin = n->chans[layer], cout = n->chans[layer + 1];
    hipStream_t s = lat->s;
    if (gin)
        HIPCHK(lat, run_layer(lat, n->tslot(), n->tprec, n->trecon, false, n->wa32 + 2 * n->woff[layer], cout, cin, (const float *)gout, 0,
                              -1, (float *)gin, 0, 2, 0, 1, 1, s));
    if (gw) {
        const size_t need = ((size_t)2 * lat->ntile + 256) * 9 * cin * cout * 2;
        if (n->part_n < need) {
            if (n->part) (void)hipFree(n->part);
            HIPCHK(lat, hipMalloc(&n->part, need * 8));
            n->part_n = need;
        }
        HIPCHK(lat, run_wgrad(n, lat, cin, cout, (const float *)in, 0, -1, (const float *)gout, 0, 2, 1, n->gtmp, 0, s));
        HIPCHK(lat, hipMemcpyAsync(gw, n->gtmp, sizeof(double) * 2 * 9 * cin * cout, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(lat, hipStreamSynchronize(s));
    return HISQ_OK;
}

hisq_status hisq_ptc_apply(hisq_ptc n, const void *r, void *z, int flags)
{
    if (!n || !r || !z) return HISQ_ERR_ARG;
    hisq_lattice lat = n->lat;
    if (!(flags & HISQ_DEVICE_PTR)) return set_err(lat, HISQ_ERR_ARG, "hisq_ptc_apply takes device pointers");
    HIPCHK(lat, hipSetDevice(lat->device));
    hisq_status st = ensure_transport_links(n, lat);
    if (st != HISQ_OK) return st;
    HIPCHK(lat, ptc_apply_internal(n, lat, n->tslot(), n->tprec, n->trecon, (const float *)r, (float *)z, nullptr));
    return HISQ_OK;
}

// Plain FP64 CG on b (to 1e-12), snapshotting x_i every `every` iterations;
// pairs r_i = b - A x_i (FP64) and e_i = x* - x_i, kept on the device in FP32.
hisq_status hisq_ptc_harvest(hisq_ptc n, hisq_lattice lat, double mass, const double *b, int every, int maxpairs,
                             int *npairs)
{
    if (!n || !lat || !b || every < 1 || maxpairs < 1) return HISQ_ERR_ARG;
    if (npairs) *npairs = 0;
    if (!lat->loaded) return set_err(lat, HISQ_ERR_STATE, "no links loaded");
    HIPCHK(lat, hipSetDevice(lat->device));
    hisq_status st = ensure_transport_links(n, lat);   // the pairs are trained on with these transports
    if (st != HISQ_OK) return st;
    const long long h = lat->h;
    hipStream_t s = lat->s;
    std::vector<hisq_lattice> lats{lat};
    std::vector<double> ms{mass};
    SolveSet &S = lat->cg;
    st = build_set(lat, S, lats, ms, 0.0);
    if (st != HISQ_OK) return st;
    double *xs = nullptr, *x_cur = nullptr, *bd = nullptr;
    HIPCHK(lat, hipMalloc(&xs, (size_t)maxpairs * h * 48));
    HIPCHK(lat, hipMalloc(&x_cur, (size_t)h * 48));
    HIPCHK(lat, hipMalloc(&bd, (size_t)h * 48));
    HIPCHK(lat, hipMemcpy(bd, b, (size_t)h * 48, hipMemcpyHostToDevice));
    hisq_solver_params prm;
    hisq_default_params(&prm);
    prm.sloppy = HISQ_F64;
    prm.check_every = every;
    prm.flags = HISQ_DEVICE_PTR;
    // The reference x* is solved well beyond the 1e-10 target so that
    // e_i = x* - x_i is accurate: A e_i = r_i - r*, with |r*| <= 1e-12 |b|.
    prm.tol = 1e-12;
    // Plain FP64 CG: with no intermediate reliable update the iterate lives in
    // x_lo, which the chunk hook copies out every `every` iterations.
    struct Snap {
        double *xs;
        long long h;
        int max, taken;
    } snap{xs, h, maxpairs, 1};
    HIPCHK(lat, hipMemsetAsync(xs, 0, (size_t)h * 48, s));   // x_0 = 0
    auto hook = [](SolveSet &S, void *ctx, hipStream_t st) -> hipError_t {
        Snap *sn = (Snap *)ctx;
        if (sn->taken >= sn->max || S.hst[0].status != ST_RUNNING) return hipSuccess;
        hipError_t e = hipMemcpyAsync(sn->xs + (size_t)sn->taken * sn->h * 6, S.xlo.p, (size_t)sn->h * 48,
                                      hipMemcpyDeviceToDevice, st);
        sn->taken++;
        return e;
    };
    hisq_solver_info info;
    const double *bb[1] = {bd};
    double *xx[1] = {x_cur};
    st = run_cg(lat, S, prm, bb, xx, &info, hook, &snap);
    if (st != HISQ_OK) {
        (void)hipFree(xs); (void)hipFree(x_cur); (void)hipFree(bd);
        return st;
    }
    const int taken = snap.taken;
    PairBlock pb;
    pb.lat = lat;
    pb.mass = mass;
    pb.n = taken;
    HIPCHK(lat, hipMalloc(&pb.mem, (size_t)taken * 2 * h * 24));
    std::vector<double> xh((size_t)h * 6), xsh((size_t)h * 6), rh((size_t)h * 6);
    HIPCHK(lat, hipMemcpy(xsh.data(), x_cur, (size_t)h * 48, hipMemcpyDeviceToHost));
    double *t_odd = nullptr, *r_hi = nullptr;
    HIPCHK(lat, hipMalloc(&t_odd, (size_t)h * 48));
    HIPCHK(lat, hipMalloc(&r_hi, (size_t)h * 48));
    ProbDesc d = lattice_desc(lat);
    d.diag = 4.0 * mass * mass;
    ProbDesc *dd = nullptr;
    HIPCHK(lat, hipMalloc(&dd, sizeof d));
    HIPCHK(lat, hipMemcpy(dd, &d, sizeof d, hipMemcpyHostToDevice));
    pb.ee.resize(taken);
    pb.er.resize(taken);
    std::vector<double> rr(taken, 0.0);
    double b2 = 0.0;
    for (int i = 0; i < taken; i++) {
        double *xi = xs + (size_t)i * h * 6;
        // r_i = b - A x_i with the FP64 operator
        DslashLaunch a;
        memset(&a, 0, sizeof a);
        a.probs = dd;
        a.out_par = 1;
        a.lslot = 0;
        a.in = xi;
        a.out = t_odd;
        HIPCHK(lat, launch_dslash(0, 18, 0, EPI_PLAIN, 8, a, lat->ntile, s));
        a.out_par = 0;
        a.in = t_odd;
        a.out = r_hi;
        a.aux = xi;
        a.bvec = bd;
        HIPCHK(lat, launch_dslash(0, 18, 0, EPI_RES, 8, a, lat->ntile, s));
        HIPCHK(lat, hipStreamSynchronize(s));
        HIPCHK(lat, hipMemcpy(xh.data(), xi, (size_t)h * 48, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < xh.size(); k++) xh[k] = xsh[k] - xh[k];      // e_i in FP64
        double ee = 0;
        for (double v : xh) ee += v * v;
        pb.ee[i] = ee;
        std::vector<float> ef(xh.begin(), xh.end());
        HIPCHK(lat, hipMemcpy(pb.mem + ((size_t)2 * i + 1) * h * 6, ef.data(), ef.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(lat, launch_convert(r_hi, 0, pb.mem + (size_t)2 * i * h * 6, 1, h * 3, s));
        HIPCHK(lat, hipStreamSynchronize(s));
        HIPCHK(lat, hipMemcpy(rh.data(), r_hi, (size_t)h * 48, hipMemcpyDeviceToHost));
        double r2 = 0, er = 0;
        for (double v : rh) r2 += v * v;
        for (size_t k = 0; k < rh.size(); k++) er += xh[k] * rh[k];   // Re <e_i, r_i>
        rr[i] = r2;
        pb.er[i] = er;
        if (i == 0) b2 = r2;   // x_0 = 0: r_0 = b
    }
    (void)hipFree(dd); (void)hipFree(t_odd); (void)hipFree(r_hi);
    (void)hipFree(xs); (void)hipFree(x_cur); (void)hipFree(bd);
    // keep the pairs whose residual is well above the reference's own
    // (|r_i| >= 1e-9 |b|, i.e. 1e3 times |r*|), compacted in order
    int keep = 0;
    for (int i = 0; i < taken; i++) {
        if (!(rr[i] >= 1e-18 * b2) || pb.ee[i] == 0.0 || !(pb.er[i] > 0.0)) continue;
        if (keep != i)
            HIPCHK(lat, hipMemcpy(pb.mem + (size_t)2 * keep * h * 6, pb.mem + (size_t)2 * i * h * 6, (size_t)h * 48,
                                  hipMemcpyDeviceToDevice));
        pb.ee[keep] = pb.ee[i];
        pb.er[keep++] = pb.er[i];
    }
    pb.n = keep;
    pb.ee.resize(keep);
    pb.er.resize(keep);
    if (keep > 0) n->pairs.push_back(pb);
    else (void)hipFree(pb.mem);
    if (npairs) *npairs = keep;
    return HISQ_OK;
}

// Checkpoint file: magic, int32 header, then the FP32 weights and the Adam
// moments as stored on the device (host byte order: little-endian).
static const char PTC_MAGIC[8] = {'H', 'I', 'S', 'Q', 'P', 'T', 'C', '1'};

hisq_status hisq_ptc_save(hisq_ptc n, const char *path)
{
    if (!n || !path) return HISQ_ERR_ARG;
    hisq_lattice lat = n->lat;
    const size_t nf = (size_t)2 * n->nw;
    std::vector<float> w(nf), m(nf), v(nf);
    HIPCHK(lat, hipSetDevice(n->device));
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    HIPCHK(lat, hipMemcpy(w.data(), n->w32, nf * 4, hipMemcpyDeviceToHost));
    HIPCHK(lat, hipMemcpy(m.data(), n->m, nf * 4, hipMemcpyDeviceToHost));
    HIPCHK(lat, hipMemcpy(v.data(), n->v, nf * 4, hipMemcpyDeviceToHost));
    std::vector<int32_t> hdr{1, n->nlayer};
    for (int c : n->chans) hdr.push_back(c);
    hdr.push_back(n->nw);
    hdr.push_back(n->step);
    FILE *f = std::fopen(path, "wb");
    if (!f) return set_err(lat, HISQ_ERR_IO, std::string("cannot open for writing: ") + path);
    bool ok = std::fwrite(PTC_MAGIC, 1, 8, f) == 8 &&
              std::fwrite(hdr.data(), 4, hdr.size(), f) == hdr.size() &&
              std::fwrite(w.data(), 4, nf, f) == nf && std::fwrite(m.data(), 4, nf, f) == nf &&
              std::fwrite(v.data(), 4, nf, f) == nf;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return set_err(lat, HISQ_ERR_IO, std::string("write failed: ") + path);
    return HISQ_OK;
}

hisq_status hisq_ptc_load(hisq_ptc n, const char *path)
{
    if (!n || !path) return HISQ_ERR_ARG;
    hisq_lattice lat = n->lat;
    FILE *f = std::fopen(path, "rb");
    if (!f) return set_err(lat, HISQ_ERR_IO, std::string("cannot open for reading: ") + path);
    const size_t nf = (size_t)2 * n->nw;
    char magic[8];
    std::vector<int32_t> hdr((size_t)n->nlayer + 5);
    std::vector<float> w(nf), m(nf), v(nf);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, PTC_MAGIC, 8) == 0;
    // version and nlayer first, so that another shape is told apart before
    // reading a header of the wrong length
    ok = ok && std::fread(hdr.data(), 4, 2, f) == 2 && hdr[0] == 1 && hdr[1] == n->nlayer;
    ok = ok && std::fread(hdr.data() + 2, 4, hdr.size() - 2, f) == hdr.size() - 2;
    if (ok)
        for (int l = 0; l <= n->nlayer; l++) ok = ok && hdr[2 + l] == n->chans[l];
    ok = ok && hdr[3 + n->nlayer] == n->nw && hdr[4 + n->nlayer] >= 0;
    ok = ok && std::fread(w.data(), 4, nf, f) == nf && std::fread(m.data(), 4, nf, f) == nf &&
         std::fread(v.data(), 4, nf, f) == nf;
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;   // nothing after the moments
    std::fclose(f);
    if (!ok) return set_err(lat, HISQ_ERR_IO, std::string("not a checkpoint of a network of this shape: ") + path);
    HIPCHK(lat, hipSetDevice(n->device));
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    HIPCHK(lat, hipMemcpy(n->w32, w.data(), nf * 4, hipMemcpyHostToDevice));
    HIPCHK(lat, hipMemcpy(n->m, m.data(), nf * 4, hipMemcpyHostToDevice));
    HIPCHK(lat, hipMemcpy(n->v, v.data(), nf * 4, hipMemcpyHostToDevice));
    HIPCHK(lat, launch_to_half(n->w32, n->w16, (int)nf, lat->s));
    HIPCHK(lat, refresh_adjoint(n, lat->s));
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    n->step = hdr[4 + n->nlayer];
    return HISQ_OK;
}

hisq_status hisq_ptc_set_loss(hisq_ptc n, int loss)
{
    if (!n) return HISQ_ERR_ARG;
    if (loss != HISQ_LOSS_ENERGY && loss != HISQ_LOSS_EUCLIDEAN)
        return set_err(n->lat, HISQ_ERR_ARG, "unknown training loss");
    n->loss = loss;
    return HISQ_OK;
}

hisq_status hisq_ptc_set_transport(hisq_ptc n, hisq_prec prec, hisq_recon recon)
{
    if (!n) return HISQ_ERR_ARG;
    const bool ok = (prec == HISQ_F32 && recon == HISQ_RECON_18) || (prec == HISQ_F16 && recon == HISQ_RECON_12);
    if (!ok) return set_err(n->lat, HISQ_ERR_ARG, "transports: FP32 recon-18 or FP16 recon-12");
    if (n->tprec != (int)prec || n->trecon != (int)recon) n->fcg_graph.release();
    n->tprec = prec;
    n->trecon = recon;
    return HISQ_OK;
}

hisq_status hisq_ptc_set_activations(hisq_ptc n, hisq_prec prec)
{
    if (!n) return HISQ_ERR_ARG;
    if (prec != HISQ_F32 && prec != HISQ_F16)
        return set_err(n->lat, HISQ_ERR_ARG, "inference activations: FP32 or FP16");
    if (n->aprec != (int)prec) n->fcg_graph.release();
    n->aprec = prec;
    return HISQ_OK;
}

hisq_status hisq_ptc_get_transport(hisq_ptc n, int *prec, int *recon)
{
    if (!n || !prec || !recon) return HISQ_ERR_ARG;
    *prec = n->tprec;
    *recon = n->trecon;
    return HISQ_OK;
}

hisq_status hisq_ptc_pair_count(hisq_ptc n, int *count)
{
    if (!n || !count) return HISQ_ERR_ARG;
    int c = 0;
    for (auto &pb : n->pairs) c += pb.n;
    *count = c;
    return HISQ_OK;
}

hisq_status hisq_ptc_get_pair(hisq_ptc n, int index, double *r, double *e)
{
    if (!n || !r || !e || index < 0) return HISQ_ERR_ARG;
    for (auto &pb : n->pairs) {
        if (index >= pb.n) {
            index -= pb.n;
            continue;
        }
        const long long h = pb.lat->h;
        std::vector<float> f((size_t)h * 12);
        HIPCHK(pb.lat, hipStreamSynchronize(pb.lat->s));
        HIPCHK(pb.lat, hipMemcpy(f.data(), pb.mem + (size_t)2 * index * h * 6, (size_t)h * 48, hipMemcpyDeviceToHost));
        for (long long k = 0; k < h * 6; k++) {
            r[k] = f[k];
            e[k] = f[h * 6 + k];
        }
        return HISQ_OK;
    }
    return HISQ_ERR_ARG;
}

// Training step on a minibatch (all pairs of one lattice):
//   forward   a_0 = E r, a_l = L_l a_{l-1} (l = 1..n), b_n = a_n,
//             b_{l-1} = L_l^+ b_l, z = E^+ b_0;
//   loss      scale-invariant (k_ptc_loss_*), g_{b_0} on even sites;
//   backward  through the adjoint half (l = 1..n): the weight gradient of the
//             adjoint application, mapped back to W_l by the adjoint-weight
//             transform, and g_{b_l} = L_l g_{b_{l-1}}; then through the
//             forward half (l = n..1) with g_{a_n} = g_{b_n}:
//             the weight gradient and g_{a_{l-1}} = L_l^+ g_{a_l};
//   update    Adam on the FP32 master, refreshed FP16 and adjoint copies.
hisq_status hisq_ptc_train(hisq_ptc n, int steps, int batch, double lr, unsigned long long seed, double *losses)
{
    if (!n || steps < 0 || batch < 1 || !(lr > 0)) return HISQ_ERR_ARG;
    hisq_lattice lat0 = n->lat;
    if (n->pairs.empty()) return set_err(lat0, HISQ_ERR_STATE, "no training pairs (hisq_ptc_harvest)");
    if (steps > 65536) return set_err(lat0, HISQ_ERR_ARG, "at most 65536 steps per call");
    HIPCHK(lat0, hipSetDevice(lat0->device));
    hipStream_t s = lat0->s;
    const int C = cmax(n);
    long long V = 0;
    for (auto &pb : n->pairs) {
        V = std::max(V, pb.lat->V);
        if (pb.lat->s != s) HIPCHK(lat0, hipStreamSynchronize(pb.lat->s));
    }
    const long long h = V / 2;
    const int nl = n->nlayer;
    // workspace per batch entry: a_1..a_n and b_1..b_{n-1} (full, C channels),
    // two gradient buffers (full), and z, g_{b_0}, r, e (even)
    const long long actf = (long long)C * 2 * h * 6;
    const size_t nbuf = (size_t)(2 * nl + 1);
    const size_t need = (size_t)batch * (actf * nbuf + h * 6 * 6);
    if (n->wsB != batch || n->wsV != V) {
        if (n->act) (void)hipFree(n->act);
        if (n->dee) (void)hipFree(n->dee);
        n->act = nullptr;
        n->dee = nullptr;
        HIPCHK(lat0, hipMalloc(&n->act, need * 4));
        HIPCHK(lat0, hipMalloc(&n->dee, sizeof(double) * batch));
        n->wsB = batch;
        n->wsV = V;
    }
    const size_t ntl = (size_t)((h + 63) / 64);
    // weight-gradient rows plus the second-pass rows of the sum
    const size_t pneed = ((size_t)batch * 2 * ntl + 256) * 9 * C * C * 2 + 64;
    const size_t lneed = (size_t)batch * ntl * NPART + 4 * (size_t)batch + 4;
    if (n->part_n < std::max(pneed, lneed)) {
        if (n->part) (void)hipFree(n->part);
        n->part_n = std::max(pneed, lneed);
        HIPCHK(lat0, hipMalloc(&n->part, n->part_n * 8));
    }
    float *A = n->act;
    auto full = [&](size_t k) { return A + (size_t)batch * actf * k; };
    std::vector<float *> acts(nl + 1), bs(nl + 1);
    for (int l = 1; l <= nl; l++) acts[l] = full(l - 1);
    for (int l = 1; l < nl; l++) bs[l] = full(nl + l - 1);
    bs[nl] = acts[nl];
    float *gbuf[2] = {full(2 * nl - 1), full(2 * nl)};
    float *zb = full(nbuf);
    float *g0 = zb + (size_t)batch * h * 6;
    float *rb = g0 + (size_t)batch * h * 6;
    float *eb = rb + (size_t)batch * h * 6;
    float *tb = eb + (size_t)batch * h * 6;   // energy norm: D_oe z (odd sites)
    float *ub = tb + (size_t)batch * h * 6;   // energy norm: D_eo D_oe z
    long long total = 0;
    for (auto &pb : n->pairs) total += pb.n;
    std::mt19937_64 rng(seed);
    for (int it = 0; it < steps; it++) {
        // draw a lattice (weighted by its pair count), then `batch` pairs of it
        long long pick = (long long)(rng() % (unsigned long long)total);
        size_t g = 0;
        while (pick >= n->pairs[g].n) pick -= n->pairs[g++].n;
        PairBlock &pb = n->pairs[g];
        hisq_lattice lat = pb.lat;
        hisq_status st = ensure_transport_links(n, lat);
        // the energy-norm loss applies the FP32 recon-18 operator of the pairs' lattice
        if (st == HISQ_OK && !lat->ls[2].valid) st = hisq_prepare_links(lat, HISQ_F32, HISQ_RECON_18);
        if (st != HISQ_OK) return st;
        const long long hl = lat->h;
        const long long af = (long long)C * 2 * hl * 6;
        std::vector<double> ee(batch);
        for (int b = 0; b < batch; b++) {
            const int i = (int)(rng() % (unsigned long long)pb.n);
            HIPCHK(lat0, hipMemcpyAsync(rb + (size_t)b * hl * 6, pb.mem + (size_t)2 * i * hl * 6, hl * 24,
                                        hipMemcpyDeviceToDevice, s));
            HIPCHK(lat0, hipMemcpyAsync(eb + (size_t)b * hl * 6, pb.mem + ((size_t)2 * i + 1) * hl * 6, hl * 24,
                                        hipMemcpyDeviceToDevice, s));
            ee[b] = n->loss == HISQ_LOSS_ENERGY ? pb.er[i] : pb.ee[i];
        }
        HIPCHK(lat0, hipMemcpyAsync(n->dee, ee.data(), sizeof(double) * batch, hipMemcpyHostToDevice, s));
        // forward half
        for (int l = 1; l <= nl; l++) {
            const bool first = l == 1;
            HIPCHK(lat0, run_layer(lat, n->tslot(), n->tprec, n->trecon, false, n->w32 + 2 * n->woff[l - 1], n->chans[l - 1], n->chans[l],
                                   first ? rb : acts[l - 1], first ? hl * 6 : af, first ? 1 : -1, acts[l], af, 2, 0, 1,
                                   batch, s));
        }
        // adjoint half
        for (int l = nl; l >= 1; l--) {
            const float *w = n->wa32 + 2 * n->woff[l - 1];
            if (l == 1)
                HIPCHK(lat0, run_layer(lat, n->tslot(), n->tprec, n->trecon, false, w, n->chans[l], n->chans[l - 1], bs[1], af, -1, zb,
                                       hl * 6, 1, 0, 0, batch, s));
            else
                HIPCHK(lat0, run_layer(lat, n->tslot(), n->tprec, n->trecon, false, w, n->chans[l], n->chans[l - 1], bs[l], af, -1, bs[l - 1],
                                       af, 2, 0, 1, batch, s));
        }
        // z = r + E^+ b_0, then the loss and g_z = g_{b_0}
        HIPCHK(lat0, launch_add_f32(zb, rb, (long long)batch * hl * 6, s));
        const bool energy = n->loss == HISQ_LOSS_ENERGY;
        if (energy) {
            // D_eo D_oe z for A z = 4 m^2 z - D_eo D_oe z, on the FP32 operator
            // of the pairs' lattice (its own stream, ordered by the host)
            if (lat->s != s) HIPCHK(lat0, hipStreamSynchronize(s));
            st = hisq_dslash(lat, HISQ_ODD, HISQ_F32, HISQ_RECON_18, zb, tb, batch, HISQ_DEVICE_PTR);
            if (st == HISQ_OK) st = hisq_dslash(lat, HISQ_EVEN, HISQ_F32, HISQ_RECON_18, tb, ub, batch, HISQ_DEVICE_PTR);
            if (st != HISQ_OK) return st;
            if (lat->s != s) HIPCHK(lat0, hipStreamSynchronize(lat->s));
        }
        PtcLaunch la = base_launch(lat, 2);
        la.in = zb;
        la.in_bstride = hl * 6;
        la.tgt = energy ? rb : eb;
        la.tgt_bstride = hl * 6;
        la.wvec = energy ? ub : nullptr;
        la.wdiag = 4.0 * pb.mass * pb.mass;
        la.out = g0;
        la.out_bstride = hl * 6;
        la.ee = n->dee;
        la.partials = n->part;
        HIPCHK(lat0, launch_ptc_loss(la, lat->ntile, batch, n->dloss + it, s));
        HIPCHK(lat0, hipMemsetAsync(n->gw, 0, sizeof(double) * 2 * n->nw, s));
        // backward through the adjoint half
        const float *gcur = g0;
        long long g_bs = hl * 6;
        int g_pstride = 1;
        int k = 0;
        for (int l = 1; l <= nl; l++) {
            const int ci = n->chans[l], co = n->chans[l - 1];   // the adjoint application maps ci -> co
            HIPCHK(lat0, run_wgrad(n, lat, ci, co, bs[l], af, -1, gcur, g_bs, g_pstride, batch, n->gtmp, 0, s));
            HIPCHK(lat0, launch_ptc_gadj(n->gtmp, ci, co, n->gw + 2 * n->woff[l - 1], s));
            HIPCHK(lat0, run_layer(lat, n->tslot(), n->tprec, n->trecon, false, n->w32 + 2 * n->woff[l - 1], co, ci, gcur, g_bs,
                                   g_pstride == 1 ? 1 : -1, gbuf[k], af, 2, 0, 1, batch, s));
            gcur = gbuf[k];
            g_bs = af;
            g_pstride = 2;
            k ^= 1;
        }
        // backward through the forward half
        for (int l = nl; l >= 1; l--) {
            const int ci = n->chans[l - 1], co = n->chans[l];
            const bool first = l == 1;
            HIPCHK(lat0, run_wgrad(n, lat, ci, co, first ? rb : acts[l - 1], first ? hl * 6 : af, first ? 1 : -1, gcur,
                                   af, 2, batch, n->gw + 2 * n->woff[l - 1], 1, s));
            if (!first) {
                HIPCHK(lat0, run_layer(lat, n->tslot(), n->tprec, n->trecon, false, n->wa32 + 2 * n->woff[l - 1], co, ci, gcur, af, -1,
                                       gbuf[k], af, 2, 0, 1, batch, s));
                gcur = gbuf[k];
                k ^= 1;
            }
        }
        n->step += 1;
        HIPCHK(lat0, launch_adam(n->w32, n->m, n->v, n->gw, 2 * n->nw, n->step, (float)lr, n->w16, s));
        HIPCHK(lat0, refresh_adjoint(n, s));
    }
    if (losses && steps > 0)
        HIPCHK(lat0, hipMemcpyAsync(losses, n->dloss, sizeof(double) * steps, hipMemcpyDeviceToHost, s));
    HIPCHK(lat0, hipStreamSynchronize(s));
    return HISQ_OK;
}

}  // extern "C"
