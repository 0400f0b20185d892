// Solver drivers shared by the C-ABI entry points.
#pragma once
#include <vector>

#include "engine.h"

hisq_status set_err(hisq_lattice lat, hisq_status st, const std::string &msg);
hisq_status hip_err(hisq_lattice lat, hipError_t e, const char *what);
// Make the device FP64 copies lat->fat64 / lat->lng64 the lattice's links
// (drops packed sets and solve workspaces, packs FP64 recon-18).
hisq_status adopt_device_links(hisq_lattice lat);

namespace hisq {

ProbDesc lattice_desc(hisq_lattice lat);
TuneChoice pick_shape(hisq_lattice lat, int prec, int recon, const ProbDesc *ddesc, const int *dt2p,
                      int ntile, long long nsite, int nprob, bool no_tune, bool streamed = false);
// pick_shape's answer without timing: the cached tuned choice or the default.
TuneChoice lookup_shape(hisq_lattice lat, int prec, int recon, int ntile, int nprob);
// Tuned launch shape of the multi-right-hand-side Dslash (nr right-hand
// sides per launch, FP32 vectors) on lattice lat.
TuneChoice pick_shape_mrhs(hisq_lattice lat, int prec, int recon, int nr, bool no_tune);

// Describe nprob problems (one per handle) in S: descriptors, tile map,
// states, partials.  sigma is added to every diagonal (4 m^2 + sigma).
hisq_status build_set(hisq_lattice lat0, SolveSet &S, const std::vector<hisq_lattice> &lats,
                      const std::vector<double> &masses, double sigma,
                      const std::vector<double> *sigmas = nullptr);

// Mixed / plain CG over every problem of S.  b[k], x[k]: FP64 vectors
// (host, or device with HISQ_DEVICE_PTR).  info: nprob entries or nullptr.
// hook: called after every chunk (after the status read, before any reliable
// update) with ctx; used to snapshot iterates.
typedef hipError_t (*ChunkHook)(SolveSet &S, void *ctx, hipStream_t s);
hisq_status run_cg(hisq_lattice lat0, SolveSet &S, const hisq_solver_params &prm,
                   const double *const *b, double *const *x, hisq_solver_info *info,
                   ChunkHook hook = nullptr, void *hook_ctx = nullptr);

size_t link_site_bytes(int prec, int recon);

}  // namespace hisq

hisq_status hisq_dslash_mrhs_impl(hisq_lattice lat, int out_parity, int prec, int recon,
                                  const void *in, void *out, int nrhs, int flags);
