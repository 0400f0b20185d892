// Host-side engine: lattice handles, device workspaces, launch-shape tuner and
// the solver drivers behind the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hisq.h"
#include "fcg_graph.h"
#include "launch.h"

namespace hisq {

struct DVec {
    void *p = nullptr;
    float *n = nullptr;     // FP16 per-site scales (inside the same allocation)
    size_t bytes = 0;
    int prec = -1;
    long long sites = 0;
};

size_t vec_bytes(int prec, long long sites);
hipError_t dvec_alloc(DVec &v, int prec, long long sites);
void dvec_free(DVec &v);

// Work set of one (possibly batched) solve: concatenated parity vectors of
// nprob problems, per-problem descriptors and FP64 states.
struct SolveSet {
    int nprob = 0;
    int ntile = 0;
    long long nsite = 0;
    int mode = -1;
    bool one_lattice = false;   // nprob > 1 problems on the same handle: vectors at q * h
    int max_ntile = 0;          // tiles of the largest problem
    std::vector<ProbDesc> hdesc;
    ProbDesc *ddesc = nullptr;
    int *dt2p = nullptr;        // nullptr when nprob == 1
    SolveState *dst = nullptr;
    SolveState *hst = nullptr;  // pinned host mirror
    double *dpart = nullptr;
    double *dred = nullptr;     // compact per-tile sums of the fused CG step: [2][ntile]
    DVec b, xhi, rhi, thi, xlo, rlo, Ap, p, t;
    ChunkGraphs chunks;   // captured iteration chunks (HISQ_USE_GRAPH)
    // flexible CG: z = M(r) and the compact tile sums of its fused iteration
    DVec fz;
    double *fred = nullptr;
    // FP64 true relative residual of every problem at each reliable update of
    // the last solve on this set
    std::vector<std::vector<double>> hist;
    // borrowed: every device pointer above points into memory the set does not
    // own (the static scratch of the no-allocation solver); the solver then
    // allocates nothing, never times launch shapes and release() frees nothing
    bool borrowed = false;
    long long *dclock = nullptr;   // device start stamp (borrowed sets; else allocated per solve)
    ~SolveSet();
    void release();
};

struct TuneChoice {
    int W = 4;
    int remap = 1;
    int cpol = 0;   // Dslash: link direction blocks (of 16) kept in the Infinity Cache (DslashLaunch::cpol)
    double us = 0;
};

// Launch-shape autotuner: times every candidate block shape of a kernel for a
// given problem geometry once, caches the fastest (in memory and, when
// HISQ_TUNE_CACHE names a file, on disk).
class Tuner {
  public:
    static Tuner &get();
    bool lookup(const std::string &key, TuneChoice &c);
    void store(const std::string &key, const TuneChoice &c);
    // HISQ_TUNE=0 in the environment: every launch takes its default shape
    bool disabled() const { return disabled_; }
    // HISQ_TUNE_VERBOSE=1: every timed candidate is printed to stderr
    void note(const std::string &key, int W, int remap, int cpol, double us);

  private:
    Tuner();
    std::mutex mu_;
    std::map<std::string, TuneChoice> cache_;
    std::string path_;
    bool disabled_ = false;
    bool verbose_ = false;
};

}  // namespace hisq

struct hisq_lattice_s {
    int L[4];
    long long V = 0, h = 0;
    int ntile = 0;
    int device = 0;
    hipStream_t s = nullptr;
    bool own_stream = false;
    double *fat64 = nullptr, *lng64 = nullptr;     // device FP64 copies [V][4][3][3]
    void *lk[hisq::NLINKSET][2] = {};
    hisq::LinkSet ls[hisq::NLINKSET] = {};
    bool loaded = false;
    std::string err;
    hisq::SolveSet cg;         // single-lattice solve workspace
    hisq::SolveSet batch;      // batched solves led by this handle
    hisq::SolveSet msref;      // multi-shift refinement (one problem per rhs x shift)
    hisq::SolveSet fcg;        // flexible CG with the learned preconditioner
    hisq::SolveSet *last_solve = nullptr;   // the set of the last solve led by this handle
    hisq::DVec tmp_in, tmp_out, tmp64a, tmp64b;  // host-pointer Dslash staging
    hisq::ProbDesc *ddesc = nullptr;             // this lattice alone
    double *dpart = nullptr;
    void *smear_ws = nullptr;                    // link-smearing workspace
    size_t smear_ws_bytes = 0;
};
