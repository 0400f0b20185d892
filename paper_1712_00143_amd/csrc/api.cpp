// C ABI: lattice handles, link loading / packing, Dslash, CG and batched CG.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <vector>

#include "engine.h"
#include "solver.h"

using namespace hisq;

static std::string g_create_err;

namespace hisq {

size_t vec_bytes(int prec, long long sites)
{
    switch (prec) {
    case 0: return (size_t)sites * 48;
    case 1: return (size_t)sites * 24;
    case 2: return (size_t)sites * 16;
    }
    return 0;
}

hipError_t dvec_alloc(DVec &v, int prec, long long sites)
{
    if (v.p && v.prec == prec && v.sites == sites) return hipSuccess;
    dvec_free(v);
    size_t b = vec_bytes(prec, sites);
    if (b == 0) b = 64;
    hipError_t e = hipMalloc(&v.p, b);
    if (e != hipSuccess) {
        v.p = nullptr;
        return e;
    }
    v.bytes = b;
    v.prec = prec;
    v.sites = sites;
    v.n = prec == 2 ? reinterpret_cast<float *>((char *)v.p + (size_t)sites * 12) : nullptr;
    return hipMemset(v.p, 0, b);
}

void dvec_free(DVec &v)
{
    if (v.p) (void)hipFree(v.p);
    v = DVec();
}

void SolveSet::release()
{
    if (borrowed) {   // nothing here is owned: forget the pointers
        for (DVec *v : {&b, &xhi, &rhi, &thi, &xlo, &rlo, &Ap, &p, &t, &fz}) *v = DVec();
        ddesc = nullptr;
        dt2p = nullptr;
        dst = nullptr;
        hst = nullptr;
        dpart = nullptr;
        dred = nullptr;
        fred = nullptr;
        dclock = nullptr;
        nprob = ntile = 0;
        nsite = 0;
        mode = -1;
        hdesc.clear();
        hist.clear();
        return;
    }
    chunks.release();
    if (fred) (void)hipFree(fred);
    fred = nullptr;
    for (DVec *v : {&b, &xhi, &rhi, &thi, &xlo, &rlo, &Ap, &p, &t, &fz}) dvec_free(*v);
    if (ddesc) (void)hipFree(ddesc);
    if (dt2p) (void)hipFree(dt2p);
    if (dst) (void)hipFree(dst);
    if (hst) (void)hipHostFree(hst);
    if (dpart) (void)hipFree(dpart);
    if (dred) (void)hipFree(dred);
    dred = nullptr;
    ddesc = nullptr;
    dt2p = nullptr;
    dst = nullptr;
    hst = nullptr;
    dpart = nullptr;
    nprob = ntile = 0;
    nsite = 0;
    mode = -1;
    hdesc.clear();
    hist.clear();
}

SolveSet::~SolveSet() { release(); }

Tuner &Tuner::get()
{
    static Tuner t;
    return t;
}

Tuner::Tuner()
{
    const char *t = getenv("HISQ_TUNE");
    disabled_ = t && std::string(t) == "0";
    const char *v = getenv("HISQ_TUNE_VERBOSE");
    verbose_ = v && std::string(v) == "1";
    const char *p = getenv("HISQ_TUNE_CACHE");
    if (p && *p) {
        path_ = p;
        std::ifstream f(path_);
        std::string key;
        TuneChoice c;
        while (f >> key >> c.W >> c.remap >> c.cpol >> c.us) cache_[key] = c;
    }
}

void Tuner::note(const std::string &key, int W, int remap, int cpol, double us)
{
    if (!verbose_) return;
    std::lock_guard<std::mutex> g(mu_);
    fprintf(stderr, "[hisq tune] %s W %d remap %d cpol %d: %.3f us\n", key.c_str(), W, remap, cpol, us);
}

bool Tuner::lookup(const std::string &key, TuneChoice &c)
{
    std::lock_guard<std::mutex> g(mu_);
    auto it = cache_.find(key);
    if (it == cache_.end()) return false;
    c = it->second;
    return true;
}

void Tuner::store(const std::string &key, const TuneChoice &c)
{
    std::lock_guard<std::mutex> g(mu_);
    cache_[key] = c;
    if (!path_.empty()) {
        std::ofstream f(path_, std::ios::app);
        f << key << " " << c.W << " " << c.remap << " " << c.cpol << " " << c.us << "\n";
    }
}

}  // namespace hisq

// ------------------------------------------------------------------ errors

hisq_status set_err(hisq_lattice lat, hisq_status st, const std::string &msg)
{
    if (lat) lat->err = msg;
    else g_create_err = msg;
    return st;
}

hisq_status hip_err(hisq_lattice lat, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_err(lat, e == hipErrorOutOfMemory ? HISQ_ERR_OOM : HISQ_ERR_HIP, m);
}

#define HIPCHK(lat, x)                                     \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) return hip_err(lat, e_, #x); \
    } while (0)

extern "C" {

void hisq_default_params(hisq_solver_params *p)
{
    if (!p) return;
    p->tol = 1e-10;
    p->maxiter = 100000;
    p->sloppy = HISQ_F64;
    p->recon = HISQ_RECON_18;
    p->delta = 0.1;
    p->check_every = 16;
    p->flags = 0;
}

const char *hisq_status_string(hisq_status s)
{
    switch (s) {
    case HISQ_OK: return "ok";
    case HISQ_ERR_ARG: return "invalid argument";
    case HISQ_ERR_HIP: return "HIP runtime error";
    case HISQ_ERR_OOM: return "out of device memory";
    case HISQ_ERR_STATE: return "call out of order";
    case HISQ_ERR_RECON: return "links cannot be reconstructed from 12 reals";
    case HISQ_ERR_NOT_CONVERGED: return "not converged";
    case HISQ_ERR_BREAKDOWN: return "solver breakdown";
    case HISQ_ERR_IO: return "file error";
    }
    return "unknown status";
}

hisq_status hisq_last_error(hisq_lattice lat, char *buf, size_t n)
{
    if (!buf || n == 0) return HISQ_ERR_ARG;
    const std::string &m = lat ? lat->err : g_create_err;
    snprintf(buf, n, "%s", m.c_str());
    return HISQ_OK;
}

hisq_status hisq_create(const int dims[4], int device, void *stream, hisq_lattice *out)
{
    if (!out || !dims) return set_err(nullptr, HISQ_ERR_ARG, "null argument");
    *out = nullptr;
    long long V = 1;
    for (int k = 0; k < 4; k++) {
        if (dims[k] < 2 || dims[k] % 2)
            return set_err(nullptr, HISQ_ERR_ARG, "lattice extents must be even and >= 2");
        V *= dims[k];
    }
    if (V / 2 > (1LL << 30)) return set_err(nullptr, HISQ_ERR_ARG, "lattice too large");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) return set_err(nullptr, HISQ_ERR_HIP, "no HIP device");
    if (device < 0 || device >= ndev) return set_err(nullptr, HISQ_ERR_ARG, "bad device index");
    e = hipSetDevice(device);
    if (e != hipSuccess) return set_err(nullptr, HISQ_ERR_HIP, "hipSetDevice failed");
    hisq_lattice lat = new hisq_lattice_s();
    for (int k = 0; k < 4; k++) lat->L[k] = dims[k];
    lat->V = V;
    lat->h = V / 2;
    lat->ntile = (int)((lat->h + TILE - 1) / TILE);
    lat->device = device;
    if (stream) {
        lat->s = (hipStream_t)stream;
    } else {
        e = hipStreamCreateWithFlags(&lat->s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete lat;
            return set_err(nullptr, HISQ_ERR_HIP, "stream creation failed");
        }
        lat->own_stream = true;
    }
    if (hipMalloc(&lat->ddesc, sizeof(ProbDesc)) != hipSuccess ||
        hipMalloc(&lat->dpart, sizeof(double) * NPART * (size_t)lat->ntile) != hipSuccess) {
        hisq_destroy(lat);
        return set_err(nullptr, HISQ_ERR_OOM, "descriptor allocation failed");
    }
    *out = lat;
    return HISQ_OK;
}

hisq_status hisq_destroy(hisq_lattice lat)
{
    if (!lat) return HISQ_ERR_ARG;
    (void)hipSetDevice(lat->device);
    if (lat->s) (void)hipStreamSynchronize(lat->s);
    lat->cg.release();
    lat->batch.release();
    lat->msref.release();
    lat->fcg.release();
    for (auto &pp : lat->lk)
        for (auto &q : pp)
            if (q) (void)hipFree(q);
    if (lat->fat64) (void)hipFree(lat->fat64);
    if (lat->lng64) (void)hipFree(lat->lng64);
    for (DVec *v : {&lat->tmp_in, &lat->tmp_out, &lat->tmp64a, &lat->tmp64b}) dvec_free(*v);
    if (lat->ddesc) (void)hipFree(lat->ddesc);
    if (lat->dpart) (void)hipFree(lat->dpart);
    if (lat->smear_ws) (void)hipFree(lat->smear_ws);
    if (lat->own_stream && lat->s) (void)hipStreamDestroy(lat->s);
    delete lat;
    return HISQ_OK;
}

}  // extern "C"

namespace hisq {

static size_t link_bytes(int prec, int recon)
{
    size_t el = prec == 0 ? 8 : prec == 1 ? 4 : 2;
    return el * (size_t)recon;
}

ProbDesc lattice_desc(hisq_lattice lat)
{
    ProbDesc d;
    memset(&d, 0, sizeof d);
    for (int k = 0; k < 4; k++) d.L[k] = lat->L[k];
    d.h = (int)lat->h;
    d.tile_begin = 0;
    d.ntile = lat->ntile;
    d.voff = 0;
    int lmax = 0;
    for (int k = 0; k < 3; k++) {
        d.mdiv[k] = (unsigned)((((unsigned long long)1 << 32) + (unsigned)lat->L[k] - 1) / (unsigned)lat->L[k]);
        lmax = lat->L[k] > lmax ? lat->L[k] : lmax;
    }
    d.fastdiv = (unsigned long long)lat->V * (unsigned long long)lmax <= ((unsigned long long)1 << 32);
    for (int k = 0; k < NLINKSET; k++) d.ls[k] = lat->ls[k];
    return d;
}

static hisq_status pack_set(hisq_lattice lat, int prec, int recon)
{
    const int slot = prec * 2 + (recon == 12);
    double a[2] = {1.0, 1.0};
    int s[2] = {0, 0};
    double *dtmp = nullptr;
    unsigned long long *dmax = nullptr;
    HIPCHK(lat, hipMalloc(&dtmp, 64));
    dmax = reinterpret_cast<unsigned long long *>(dtmp + 4);
    hisq_status st = HISQ_OK;
    if (recon == 12) {
        double det[4];
        HIPCHK(lat, launch_det_probe(lat->fat64, lat->lng64, dtmp, lat->s));
        HIPCHK(lat, hipMemcpyAsync(det, dtmp, sizeof det, hipMemcpyDeviceToHost, lat->s));
        HIPCHK(lat, hipStreamSynchronize(lat->s));
        for (int f = 0; f < 2; f++) {
            double re = det[2 * f], im = det[2 * f + 1];
            double mag = std::sqrt(re * re + im * im);
            if (!(mag > 0) || std::fabs(im) > 1e-8 * mag) {
                (void)hipFree(dtmp);
                return set_err(lat, HISQ_ERR_RECON, "recon-12: det of the first link is not real");
            }
            a[f] = std::cbrt(mag);
            s[f] = re > 0 ? 1 : -1;   // site 0 has eta = +1 in every direction
        }
    } else if (prec == 2) {
        // FP16 recon-18: normalise each field by its max |entry|
        for (int f = 0; f < 2; f++) {
            unsigned long long bits = 0;
            HIPCHK(lat, hipMemsetAsync(dmax, 0, 8, lat->s));
            HIPCHK(lat, launch_maxabs(f ? lat->lng64 : lat->fat64, lat->V * 4 * 18, dmax, lat->s));
            HIPCHK(lat, hipMemcpyAsync(&bits, dmax, 8, hipMemcpyDeviceToHost, lat->s));
            HIPCHK(lat, hipStreamSynchronize(lat->s));
            double m;
            memcpy(&m, &bits, 8);
            a[f] = m > 0 ? m : 1.0;
        }
    }
    const long long hs = link_plane_stride(lat->h);
    // the kernels address a direction block with 32-bit offsets
    if ((double)hs * (double)link_bytes(prec, recon) >= 2147483648.0) {
        (void)hipFree(dtmp);
        return set_err(lat, HISQ_ERR_ARG, "lattice too large for this link format (one direction block >= 2 GiB)");
    }
    const size_t per_par = (size_t)hs * NDIR * link_bytes(prec, recon);
    for (int par = 0; par < 2; par++) {
        if (!lat->lk[slot][par]) {
            hipError_t e = hipMalloc(&lat->lk[slot][par], per_par);
            if (e != hipSuccess) {
                (void)hipFree(dtmp);
                return hip_err(lat, e, "link allocation");
            }
        }
    }
    HIPCHK(lat, hipMemsetAsync(dmax, 0, 8, lat->s));
    for (int par = 0; par < 2; par++) {
        PackLaunch p;
        p.fat = lat->fat64;
        p.lng = lat->lng64;
        for (int k = 0; k < 4; k++) p.L[k] = lat->L[k];
        p.h = (int)lat->h;
        p.hs = (int)hs;
        p.out_par = par;
        p.dst = lat->lk[slot][par];
        p.a[0] = a[0];
        p.a[1] = a[1];
        p.s[0] = s[0];
        p.s[1] = s[1];
        p.maxerr = dmax;
        HIPCHK(lat, launch_pack(prec, recon, p, lat->s));
    }
    if (recon == 12) {
        unsigned long long bits = 0;
        HIPCHK(lat, hipMemcpyAsync(&bits, dmax, 8, hipMemcpyDeviceToHost, lat->s));
        HIPCHK(lat, hipStreamSynchronize(lat->s));
        double err;
        memcpy(&err, &bits, 8);
        if (!(err <= 1e-10)) {
            char b[160];
            snprintf(b, sizeof b, "recon-12: row 3 not recovered (max error %.3g of the link scale)", err);
            st = set_err(lat, HISQ_ERR_RECON, b);
        }
    }
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    (void)hipFree(dtmp);
    if (st != HISQ_OK) return st;
    LinkSet &ls = lat->ls[slot];
    ls.ptr[0] = lat->lk[slot][0];
    ls.ptr[1] = lat->lk[slot][1];
    ls.a[0] = a[0];
    ls.a[1] = a[1];
    ls.s[0] = s[0];
    ls.s[1] = s[1];
    ls.hs = (int)hs;
    ls.valid = 1;
    ProbDesc d = lattice_desc(lat);
    HIPCHK(lat, hipMemcpyAsync(lat->ddesc, &d, sizeof d, hipMemcpyHostToDevice, lat->s));
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    return HISQ_OK;
}

}  // namespace hisq

// The device FP64 copies lat->fat64 / lat->lng64 (written by the caller on
// lat->s) become the lattice's links: every packed set and solve workspace
// is discarded and the FP64 recon-18 operator is packed.
hisq_status adopt_device_links(hisq_lattice lat)
{
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    for (auto &ls : lat->ls) ls = LinkSet();
    lat->cg.release();
    lat->loaded = true;
    return pack_set(lat, 0, 18);
}

extern "C" {

hisq_status hisq_load_links(hisq_lattice lat, const double *fat, const double *lng, int flags)
{
    if (!lat || !fat || !lng) return set_err(lat, HISQ_ERR_ARG, "null argument");
    HIPCHK(lat, hipSetDevice(lat->device));
    const size_t bytes = (size_t)lat->V * 4 * 18 * sizeof(double);
    if (!lat->fat64) HIPCHK(lat, hipMalloc(&lat->fat64, bytes));
    if (!lat->lng64) HIPCHK(lat, hipMalloc(&lat->lng64, bytes));
    hipMemcpyKind k = (flags & HISQ_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(lat, hipMemcpyAsync(lat->fat64, fat, bytes, k, lat->s));
    HIPCHK(lat, hipMemcpyAsync(lat->lng64, lng, bytes, k, lat->s));
    return adopt_device_links(lat);
}

hisq_status hisq_prepare_links(hisq_lattice lat, hisq_prec prec, hisq_recon recon)
{
    if (!lat) return HISQ_ERR_ARG;
    if (!lat->loaded) return set_err(lat, HISQ_ERR_STATE, "no links loaded");
    if ((int)prec < 0 || (int)prec > 2 || (recon != 12 && recon != 18))
        return set_err(lat, HISQ_ERR_ARG, "bad precision or reconstruction");
    HIPCHK(lat, hipSetDevice(lat->device));
    const int slot = (int)prec * 2 + (recon == 12);
    if (lat->ls[slot].valid) return HISQ_OK;
    hisq_status st = pack_set(lat, (int)prec, (int)recon);
    if (st == HISQ_OK) lat->cg.release();   // descriptors changed
    return st;
}

}  // extern "C"

namespace hisq {

static std::string dslash_tune_key(const hipDeviceProp_t &prop, int prec, int recon, int ntile, int nprob,
                                   bool streamed = false)
{
    std::ostringstream ks;
    ks << (streamed ? "dslash3s:" : "dslash3:") << prop.gcnArchName << ":p" << prec << ":r" << recon << ":t" << ntile << ":n" << nprob;
    std::string key = ks.str();
    for (auto &ch : key)
        if (ch == ' ') ch = '_';
    return key;
}

// The launch shape pick_shape would return, without timing anything: the
// tuned choice if one is cached, else the default shape.
TuneChoice lookup_shape(hisq_lattice lat, int prec, int recon, int ntile, int nprob)
{
    TuneChoice def;
    def.W = prec == 0 ? 8 : 4;
    def.remap = 1;
    if (Tuner::get().disabled()) return def;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, lat->device) != hipSuccess) return def;
    TuneChoice c;
    return Tuner::get().lookup(dslash_tune_key(prop, prec, recon, ntile, nprob), c) ? c : def;
}

// Default and tuned launch shape of the Dslash for a geometry.  streamed:
// the best shape with every link streamed (cache policy 0), else the best
// shape and link-load policy together.  One timing run stores both.
TuneChoice pick_shape(hisq_lattice lat, int prec, int recon, const ProbDesc *ddesc, const int *dt2p,
                      int ntile, long long nsite, int nprob, bool no_tune, bool streamed)
{
    TuneChoice def;
    def.W = prec == 0 ? 8 : 4;
    def.remap = 1;
    if (no_tune || Tuner::get().disabled()) return def;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, lat->device) != hipSuccess) return def;
    std::string key = dslash_tune_key(prop, prec, recon, ntile, nprob);
    const std::string skey = dslash_tune_key(prop, prec, recon, ntile, nprob, true);
    TuneChoice c;
    if (Tuner::get().lookup(streamed ? skey : key, c)) return c;
    DVec in, out;
    if (dvec_alloc(in, prec, nsite) != hipSuccess || dvec_alloc(out, prec, nsite) != hipSuccess) {
        dvec_free(in);
        dvec_free(out);
        return def;
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    TuneChoice best = def;
    best.us = 1e30;
    // Overwrite twice the Infinity Cache's 256 MB, so that a measurement does
    // not start from links that the packing kernels or an earlier trial left
    // there.
    auto flush_cache = [&]() {
        void *junk = nullptr;
        const size_t jb = (size_t)512 << 20;
        if (hipMalloc(&junk, jb) == hipSuccess) {
            (void)hipMemsetAsync(junk, 0, jb, lat->s);
            (void)hipStreamSynchronize(lat->s);
            (void)hipFree(junk);
        }
        (void)hipGetLastError();
    };
    flush_cache();
    // every candidate shape, timed on both output parities in turn (the
    // solvers alternate them), best of three interleaved trials of 10 launches
    // waves per block, and the one- and two-wave blocks with the larger
    // register budget (W_LOWOCC)
    constexpr int NWS = 7;
    const int Ws[NWS] = {1, 2, 4, 8, 16, 1 | W_LOWOCC, 2 | W_LOWOCC};
    double tbest[NWS][2];
    bool okc[NWS][2];
    for (int wi = 0; wi < NWS; wi++)
        for (int remap = 0; remap < 2; remap++) {
            tbest[wi][remap] = 1e30;
            okc[wi][remap] = true;
        }
    auto make = [&](int remap, int par, int cpol = 0) {
        DslashLaunch a;
        memset(&a, 0, sizeof a);
        a.probs = ddesc;
        a.tile2prob = dt2p;
        a.remap = remap;
        a.cpol = cpol;
        a.out_par = par;
        a.lslot = prec * 2 + (recon == 12);
        a.in = in.p;
        a.in_nrm = in.n;
        a.out = out.p;
        a.out_nrm = out.n;
        return a;
    };
    for (int trial = 0; trial < 3; trial++)
        for (int wi = 0; wi < NWS; wi++)
            for (int remap = 0; remap < 2; remap++) {
                if (!okc[wi][remap]) continue;
                const int W = Ws[wi];
                const DslashLaunch a0 = make(remap, 0), a1 = make(remap, 1);
                if (trial == 0)
                    for (int r = 0; r < 2 && okc[wi][remap]; r++)
                        okc[wi][remap] = launch_dslash(prec, recon, prec, EPI_PLAIN, W, r & 1 ? a1 : a0, ntile,
                                                       lat->s) == hipSuccess;
                if (!okc[wi][remap]) continue;
                const int reps = 10;
                (void)hipEventRecord(e0, lat->s);
                for (int r = 0; r < reps; r++)
                    (void)launch_dslash(prec, recon, prec, EPI_PLAIN, W, r & 1 ? a1 : a0, ntile, lat->s);
                (void)hipEventRecord(e1, lat->s);
                (void)hipEventSynchronize(e1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const double us = 1000.0 * ms / reps;
                if (us < tbest[wi][remap]) tbest[wi][remap] = us;
            }
    for (int wi = 0; wi < NWS; wi++)
        for (int remap = 0; remap < 2; remap++)
            if (okc[wi][remap]) Tuner::get().note(skey, Ws[wi], remap, 0, tbest[wi][remap]);
    for (int wi = 0; wi < NWS; wi++)
        for (int remap = 0; remap < 2; remap++)
            if (okc[wi][remap] && tbest[wi][remap] < best.us) {
                best.us = tbest[wi][remap];
                best.W = Ws[wi];
                best.remap = remap;
            }
    if (best.us < 1e29) Tuner::get().store(skey, best);   // the streamed choice (cpol 0)
    const TuneChoice best_streamed = best;
    // The link-load policy for the chosen shape: all links cached when both
    // parities' links fit the Infinity Cache (they stay there between the
    // alternating launches); when they do not, a part of the direction blocks
    // cached (a stream larger than the cache would only evict itself) or none.
    // Each candidate is timed the same way from the same start: an emptied
    // cache, six warm-up applications, then the best of three trials of 10
    // (40 for an operator that fits the cache).  Cached loads change which block shape and tile order are best, so every
    // shape and order is tried with every cached candidate; streaming keeps
    // the shape found above.  An operator that fits is timed over longer
    // trials: the streamed policy loses rate over a long run of alternating
    // applications that a trial of ten does not show.
    if (best.us < 1e29) {
        const double op_bytes = 2.0 * (double)nsite * (double)link_site_bytes(prec, recon);
        const bool partial = op_bytes > 200e6;
        std::vector<int> cands{0, 16};
        if (partial)
            for (int c : {2, 4, 8, 12}) cands.push_back(c);
        TuneChoice bc = best;
        bc.us = 1e30;
        for (int wi = 0; wi < NWS; wi++)
        for (int rm = 0; rm < 2; rm++) {
            const int W = Ws[wi];
            if (!okc[wi][rm]) continue;
            for (size_t ci = 0; ci < cands.size(); ci++) {
                if (cands[ci] == 0 && (W != best.W || rm != best.remap)) continue;
                const DslashLaunch a0 = make(rm, 0, cands[ci]), a1 = make(rm, 1, cands[ci]);
                flush_cache();
                bool ok = true;
                for (int r = 0; r < 6 && ok; r++)
                    ok = launch_dslash(prec, recon, prec, EPI_PLAIN, W, r & 1 ? a1 : a0, ntile, lat->s) == hipSuccess;
                if (!ok) continue;
                double t = 1e30;
                for (int trial = 0; trial < 3; trial++) {
                    const int reps = partial ? 10 : 40;
                    (void)hipEventRecord(e0, lat->s);
                    for (int r = 0; r < reps; r++)
                        (void)launch_dslash(prec, recon, prec, EPI_PLAIN, W, r & 1 ? a1 : a0, ntile, lat->s);
                    (void)hipEventRecord(e1, lat->s);
                    (void)hipEventSynchronize(e1);
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    t = std::min(t, 1000.0 * ms / reps);
                }
                // an operator that fits the cache keeps it unless streaming is
                // clearly faster: the two time within a per cent or two here,
                // while over a long run of alternating applications the cached
                // one holds its rate and the streamed one does not
                Tuner::get().note(key, W, rm, cands[ci], t);
                const double bias = (!partial && cands[ci] == 16) ? 1.03 : 1.0;
                if (t < bias * bc.us) {
                    bc.us = t;
                    bc.W = W;
                    bc.remap = rm;
                    bc.cpol = cands[ci];
                }
            }
        }
        if (bc.us < 1e29) best = bc;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dvec_free(in);
    dvec_free(out);
    (void)hipGetLastError();
    if (best.us < 1e29) Tuner::get().store(key, best);
    else best = def;
    if (streamed) return best_streamed.us < 1e29 ? best_streamed : def;
    return best;
}

TuneChoice pick_shape_mrhs(hisq_lattice lat, int prec, int recon, int nr, bool no_tune)
{
    TuneChoice def;
    def.W = prec == 0 ? 8 : 4;
    def.remap = 1;
    if (no_tune || Tuner::get().disabled() || nr < 1 || nr > 4) return def;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, lat->device) != hipSuccess) return def;
    std::ostringstream ks;
    ks << "mrhs2:" << prop.gcnArchName << ":p" << prec << ":r" << recon << ":t" << lat->ntile << ":nr" << nr;
    std::string key = ks.str();
    for (auto &ch : key)
        if (ch == ' ') ch = '_';
    TuneChoice c;
    if (Tuner::get().lookup(key, c)) return c;
    DVec in, out;
    const int vprec = prec == 0 ? 0 : 1;   // FP64 vectors with FP64 links, FP32 otherwise
    if (dvec_alloc(in, vprec, lat->h * nr) != hipSuccess || dvec_alloc(out, vprec, lat->h * nr) != hipSuccess) {
        dvec_free(in);
        dvec_free(out);
        return def;
    }
    (void)hipMemsetAsync(in.p, 0, in.bytes, lat->s);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    TuneChoice best = def;
    best.us = 1e30;
    // the vector-ALU kernel with 2-16 waves per block, and for groups of four
    // FP32-vector right-hand sides the matrix-core kernel
    std::vector<int> shapes{2, 4, 8, 16};
    if (nr == 4 && prec != 0) shapes.push_back(MRHS_MFMA);
    for (int W : shapes) {
        for (int remap = 0; remap < 2; remap++) {
            MrhsLaunch a;
            memset(&a, 0, sizeof a);
            a.probs = lat->ddesc;
            a.desc_stride = 0;
            a.remap = remap;
            a.lslot = prec * 2 + (recon == 12);
            a.nrhs = nr;
            a.vstride = lat->h;
            a.in = in.p;
            a.out = out.p;
            a.epi = EPI_PLAIN;
            bool ok = true;
            for (int r = 0; r < 2 && ok; r++) ok = launch_dslash_mrhs(prec, recon, nr, W, a, lat->ntile, lat->s) == hipSuccess;
            if (!ok) continue;
            const int reps = 6;
            (void)hipEventRecord(e0, lat->s);
            for (int r = 0; r < reps; r++) (void)launch_dslash_mrhs(prec, recon, nr, W, a, lat->ntile, lat->s);
            (void)hipEventRecord(e1, lat->s);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double us = 1000.0 * ms / reps;
            Tuner::get().note(key, W, remap, 0, us);
            if (us < best.us) {
                best.us = us;
                best.W = W;
                best.remap = remap;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dvec_free(in);
    dvec_free(out);
    (void)hipGetLastError();
    if (best.us < 1e29) Tuner::get().store(key, best);
    else best = def;
    return best;
}

}  // namespace hisq

extern "C" {

hisq_status hisq_residual_history(hisq_lattice lat, int problem, double *out, int cap, int *count)
{
    if (!lat || !count || cap < 0 || (cap > 0 && !out)) return set_err(lat, HISQ_ERR_ARG, "bad history arguments");
    if (!lat->last_solve) return set_err(lat, HISQ_ERR_STATE, "no solve on this handle yet");
    const auto &H = lat->last_solve->hist;
    if (problem < 0 || problem >= (int)H.size()) return set_err(lat, HISQ_ERR_ARG, "problem index out of range");
    const std::vector<double> &h = H[problem];
    *count = (int)h.size();
    for (int i = 0; i < cap && i < (int)h.size(); i++) out[i] = h[i];
    return HISQ_OK;
}

hisq_status hisq_dslash_shape(hisq_lattice lat, hisq_prec prec, hisq_recon recon, int flags, int *waves, int *remap,
                              int *cache_blocks)
{
    if (!lat || !waves || !remap || !cache_blocks) return set_err(lat, HISQ_ERR_ARG, "null argument");
    if (!lat->loaded) return set_err(lat, HISQ_ERR_STATE, "no links loaded");
    if ((int)prec < 0 || (int)prec > 2 || (recon != 12 && recon != 18))
        return set_err(lat, HISQ_ERR_ARG, "bad precision or reconstruction");
    if (!lat->ls[(int)prec * 2 + (recon == 12)].valid)
        return set_err(lat, HISQ_ERR_STATE, "link set not prepared (hisq_prepare_links)");
    HIPCHK(lat, hipSetDevice(lat->device));
    const bool streamed = (flags & HISQ_STREAM_LINKS) != 0;
    TuneChoice tc = pick_shape(lat, (int)prec, recon, lat->ddesc, nullptr, lat->ntile, lat->h, 1,
                               (flags & HISQ_NO_TUNE) != 0, streamed);
    *waves = tc.W;
    *remap = tc.remap;
    *cache_blocks = streamed ? 0 : tc.cpol;
    return HISQ_OK;
}

hisq_status hisq_dslash(hisq_lattice lat, hisq_parity out_parity, hisq_prec prec, hisq_recon recon,
                        const void *in, void *out, int nrhs, int flags)
{
    if (!lat || !in || !out) return set_err(lat, HISQ_ERR_ARG, "null argument");
    if (!lat->loaded) return set_err(lat, HISQ_ERR_STATE, "no links loaded");
    if ((int)out_parity < 0 || (int)out_parity > 1 || (int)prec < 0 || (int)prec > 2 ||
        (recon != 12 && recon != 18) || nrhs < 1)
        return set_err(lat, HISQ_ERR_ARG, "bad parity, precision, reconstruction or nrhs");
    const int slot = (int)prec * 2 + (recon == 12);
    if (!lat->ls[slot].valid)
        return set_err(lat, HISQ_ERR_STATE, "link set not prepared (hisq_prepare_links)");
    HIPCHK(lat, hipSetDevice(lat->device));
    const int p = (int)prec;
    if (nrhs > 1) return hisq_dslash_mrhs_impl(lat, out_parity, p, recon, in, out, nrhs, flags);
    const bool streamed = (flags & HISQ_STREAM_LINKS) != 0;
    TuneChoice tc = pick_shape(lat, p, recon, lat->ddesc, nullptr, lat->ntile, lat->h, 1,
                               (flags & HISQ_NO_TUNE) != 0, streamed);
    DslashLaunch a;
    memset(&a, 0, sizeof a);
    a.probs = lat->ddesc;
    a.remap = tc.remap;
    a.cpol = streamed ? 0 : tc.cpol;
    a.out_par = (int)out_parity;
    a.lslot = slot;
    if (flags & HISQ_DEVICE_PTR) {
        a.in = in;
        a.in_nrm = p == 2 ? reinterpret_cast<const float *>((const char *)in + (size_t)lat->h * 12) : nullptr;
        a.out = out;
        a.out_nrm = p == 2 ? reinterpret_cast<float *>((char *)out + (size_t)lat->h * 12) : nullptr;
        HIPCHK(lat, launch_dslash(p, recon, p, EPI_PLAIN, tc.W, a, lat->ntile, lat->s));
        return HISQ_OK;
    }
    // host FP64 vectors: stage, convert, apply, convert back
    HIPCHK(lat, dvec_alloc(lat->tmp64a, 0, lat->h));
    HIPCHK(lat, dvec_alloc(lat->tmp_in, p, lat->h));
    HIPCHK(lat, dvec_alloc(lat->tmp_out, p, lat->h));
    HIPCHK(lat, hipMemcpyAsync(lat->tmp64a.p, in, vec_bytes(0, lat->h), hipMemcpyHostToDevice, lat->s));
    BlasLaunch b;
    memset(&b, 0, sizeof b);
    b.probs = lat->ddesc;
    b.v[0] = lat->tmp64a.p;
    b.v[1] = lat->tmp_in.p;
    b.n[1] = lat->tmp_in.n;
    HIPCHK(lat, launch_blas(BL_COPY_D2F, p, b, lat->ntile, 1, lat->s));
    a.in = lat->tmp_in.p;
    a.in_nrm = lat->tmp_in.n;
    a.out = lat->tmp_out.p;
    a.out_nrm = lat->tmp_out.n;
    HIPCHK(lat, launch_dslash(p, recon, p, EPI_PLAIN, tc.W, a, lat->ntile, lat->s));
    b.v[0] = lat->tmp_out.p;
    b.n[0] = lat->tmp_out.n;
    b.v[1] = lat->tmp64a.p;
    HIPCHK(lat, launch_blas(BL_COPY_F2D, p, b, lat->ntile, 1, lat->s));
    HIPCHK(lat, hipMemcpyAsync(out, lat->tmp64a.p, vec_bytes(0, lat->h), hipMemcpyDeviceToHost, lat->s));
    HIPCHK(lat, hipStreamSynchronize(lat->s));
    return HISQ_OK;
}

}  // extern "C"
