// CG solve that allocates nothing, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  Same iteration and kernels as hisq_cg (reading: plain
// FP64 or mixed precision with reliable updates); every work vector, the
// reduction partials, the solver state, the problem descriptor and the start
// stamp live in one static device array per GPU.
//
// The array's name is a host-side stand-in in host code: its device address
// is fetched once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to kernels and copies.  Every call
// on a device shares its array; calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "solver.h"

using namespace hisq;

#define HIPCHK(lat, x)                                     \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) return hip_err(lat, e_, #x); \
    } while (0)

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;

// the work memory of every hisq_cg_noalloc call on a device (one copy per GPU)
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

struct DeviceScratch {
    char *ptr = nullptr;    // device address of `scratch` on this device
    SolveState hst[1];      // host mirror of the solver state
    SolveSet set;           // borrowed work set carved out of ptr
};

DeviceScratch g_dev[MAX_DEVICES];
std::mutex g_mu;

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t vbytes(int prec, long long sites) { return prec == 0 ? sites * 48 : prec == 1 ? sites * 24 : sites * 16; }

// Bytes of scratch one solve of h sites per parity (ntile tiles) needs in
// sloppy precision `mode`: four FP64 vectors (b, x_hi, r_hi, t_hi), three
// accumulators in FP64 (plain) or FP32 (mixed), p and t in the sloppy
// precision, then state, descriptor, stamp and the per-tile partials.
size_t need_bytes(int mode, long long h, int ntile)
{
    const int rprec = mode == 0 ? 0 : 1;
    size_t n = align256(sizeof(SolveState)) + align256(sizeof(ProbDesc)) + align256(sizeof(long long)) +
               align256(sizeof(double) * NPART * (size_t)ntile) + align256(sizeof(double) * 2 * (size_t)ntile);
    n += 4 * align256(vbytes(0, h)) + 3 * align256(vbytes(rprec, h)) + 2 * align256(vbytes(mode, h));
    return n;
}

void carve_vec(DVec &v, char *&cur, int prec, long long sites)
{
    v.p = cur;
    v.prec = prec;
    v.sites = sites;
    v.bytes = vbytes(prec, sites);
    v.n = prec == 2 ? reinterpret_cast<float *>(cur + (size_t)sites * 12) : nullptr;
    cur += align256(v.bytes);
}

}  // namespace

extern "C" hisq_status hisq_cg_noalloc(hisq_lattice lat, double mass, const double *b, double *x,
                                       const hisq_solver_params *params, hisq_solver_info *info)
{
    if (!lat || !b || !x) return set_err(lat, HISQ_ERR_ARG, "null argument");
    if (!(mass > 0)) return set_err(lat, HISQ_ERR_ARG, "mass must be > 0");
    hisq_solver_params prm;
    if (params) prm = *params;
    else hisq_default_params(&prm);
    if (!(prm.flags & HISQ_DEVICE_PTR))
        return set_err(lat, HISQ_ERR_ARG, "hisq_cg_noalloc takes device vectors (HISQ_DEVICE_PTR)");
    if (prm.flags & HISQ_USE_GRAPH)
        return set_err(lat, HISQ_ERR_ARG, "hisq_cg_noalloc launches eagerly (instantiating a graph allocates)");
    const int mode = (int)prm.sloppy, recon = (int)prm.recon;
    if (mode < 0 || mode > 2 || (recon != 12 && recon != 18))
        return set_err(lat, HISQ_ERR_ARG, "bad sloppy precision or reconstruction");
    if (lat->device < 0 || lat->device >= MAX_DEVICES) return set_err(lat, HISQ_ERR_ARG, "device index");
    const size_t need = need_bytes(mode, lat->h, lat->ntile);
    if (need > SCRATCH_BYTES)
        return set_err(lat, HISQ_ERR_ARG,
                       "lattice too large for hisq_cg_noalloc: needs " + std::to_string(need) +
                           " bytes of scratch, the static buffer holds " + std::to_string(SCRATCH_BYTES));
    if (!lat->loaded) return set_err(lat, HISQ_ERR_STATE, "no links loaded");
    const int slot = mode * 2 + (recon == 12);
    if (!lat->ls[slot].valid || !lat->ls[0].valid)
        return set_err(lat, HISQ_ERR_STATE, "link set not prepared (hisq_prepare_links allocates: call it first)");
    HIPCHK(lat, hipSetDevice(lat->device));
    DeviceScratch &D = g_dev[lat->device];
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (!D.ptr) {
            void *p = nullptr;
            hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) return hip_err(lat, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                      "hipGetSymbolAddress(scratch)");
            D.ptr = (char *)p;
        }
    }
    // carve the work set out of this device's scratch
    SolveSet &S = D.set;
    S.borrowed = true;
    S.release();
    S.borrowed = true;
    char *cur = D.ptr;
    S.dst = reinterpret_cast<SolveState *>(cur);
    cur += align256(sizeof(SolveState));
    S.ddesc = reinterpret_cast<ProbDesc *>(cur);
    cur += align256(sizeof(ProbDesc));
    S.dclock = reinterpret_cast<long long *>(cur);
    cur += align256(sizeof(long long));
    S.dpart = reinterpret_cast<double *>(cur);
    cur += align256(sizeof(double) * NPART * (size_t)lat->ntile);
    S.dred = reinterpret_cast<double *>(cur);
    cur += align256(sizeof(double) * 2 * (size_t)lat->ntile);
    const int rprec = mode == 0 ? 0 : 1;
    for (DVec *v : {&S.b, &S.xhi, &S.rhi, &S.thi}) carve_vec(*v, cur, 0, lat->h);
    for (DVec *v : {&S.xlo, &S.rlo, &S.Ap}) carve_vec(*v, cur, rprec, lat->h);
    for (DVec *v : {&S.p, &S.t}) carve_vec(*v, cur, mode, lat->h);
    if ((size_t)(cur - D.ptr) != need) return set_err(lat, HISQ_ERR_STATE, "scratch layout");
    S.hst = D.hst;
    S.nprob = 1;
    S.ntile = lat->ntile;
    S.nsite = lat->h;
    S.one_lattice = false;
    S.max_ntile = lat->ntile;
    S.dt2p = nullptr;
    ProbDesc d = lattice_desc(lat);
    d.tile_begin = 0;
    d.voff = 0;
    d.mass = mass;
    d.diag = 4.0 * mass * mass;
    S.hdesc.assign(1, d);
    // the descriptor is copied from a host variable that outlives the copy
    HIPCHK(lat, hipMemcpyAsync(S.ddesc, &S.hdesc[0], sizeof(ProbDesc), hipMemcpyHostToDevice, lat->s));
    const double *bb[1] = {b};
    double *xx[1] = {x};
    return run_cg(lat, S, prm, bb, xx, info);
}
