// Kernel launch descriptors and launcher prototypes (host <-> kernel files).
#pragma once
#include "hisq_dev.h"

namespace hisq {

enum : int { EPI_PLAIN = 0, EPI_AX = 1, EPI_RES = 2 };

// Launch shape code of the single-RHS Dslash: the waves per block (1, 2, 4, 8
// or 16), or'ed with W_LOWOCC for the variant compiled for at most two waves
// per SIMD (1 and 2 waves per block only).
constexpr int W_LOWOCC = 0x100;
inline int shape_waves(int W) { return W & 0xff; }

struct DslashLaunch {
    const ProbDesc *probs;
    const int *tile2prob;   // nullptr: a single problem
    int remap;              // XCD-aware tile order
    int out_par;
    int lslot;              // link set slot (prec*2 + (recon==12))
    int want;               // status a problem must have to be processed
    SolveState *states;     // nullptr: no status gating, no reductions
    const void *in;
    const float *in_nrm;
    void *out;
    float *out_nrm;
    const void *aux;
    const float *aux_nrm;
    const double *bvec;
    double *partials;
    int fin;
    int cpol;               // link direction blocks (of 16) loaded to stay in the Infinity Cache between
                            // launches: 0 none (all streamed past the caches), 16 all, else a part
    double *red;            // non-null (AX/RES): block sum to red[tile] instead of partials
};

hipError_t launch_dslash(int prec, int recon, int out_prec, int epi, int W, const DslashLaunch &a,
                         int nblocks, hipStream_t s);

// Multi-RHS Dslash: nrhs vectors at stride vstride sites, links read once per
// group of NR right-hand sides.  One launch covers every group: block b works
// on group b / ntile, tile b % ntile.
struct MrhsLaunch {
    const ProbDesc *probs;  // descriptor of rhs r: probs[r * desc_stride], all on one lattice;
                            // EPI_AX: out_r = probs[r * desc_stride].diag aux_r - D in_r
    int desc_stride;        // 0: probs[0] for every rhs, 1: one descriptor per rhs
    int remap;
    int out_par;
    int lslot;
    int nrhs;               // right-hand sides in total
    long long vstride;      // sites between consecutive right-hand sides
    const void *in;
    void *out;
    const void *aux;        // EPI_AX: p vectors; EPI_RES: x vectors (same stride)
    const double *bvec;     // EPI_RES: FP64 right-hand sides b (same stride)
    double *partials;       // EPI_AX: Re(p.Ap), EPI_RES: |r|^2 of rhs r, tile t at [(r * ntile + t) * NPART]
    SolveState *states;     // per-rhs states (nrhs of them), nullptr: all active
    int epi;
    int want;
    double *red;            // non-null: EPI_AX/RES sums to red[r * ntile + t] instead of partials
};

// group: right-hand sides per link read (1..4); the grid is
// ceil(nrhs / group) * ntile blocks.  W: waves per block (2, 4, 8, 16) of the
// vector-ALU kernel, or MRHS_MFMA for the matrix-core kernel (group 4, FP32 or
// FP16 links, FP32 vectors, PLAIN and AX epilogues).
constexpr int MRHS_MFMA = 0x200;
hipError_t launch_dslash_mrhs(int prec, int recon, int group, int W, const MrhsLaunch &a, int ntile,
                              hipStream_t s);
hipError_t launch_dslash_mrhs_mfma(int prec, int recon, const MrhsLaunch &a, int nblocks, hipStream_t s);

// ---- packing
struct PackLaunch {
    const double *fat;   // device FP64 [V][4][3][3] complex
    const double *lng;
    int L[4];
    int h;
    int hs;              // plane stride of the destination, in sites (>= h)
    int out_par;
    void *dst;           // packed destination for this parity
    double a[2];
    int s[2];
    unsigned long long *maxerr;  // recon-12 check: max |U - c*recon(W)| / a as double bits
};
hipError_t launch_pack(int prec, int recon, const PackLaunch &p, hipStream_t s);
hipError_t launch_det_probe(const double *fat, const double *lng, double *out4, hipStream_t s);
hipError_t launch_maxabs(const double *links, long long n, unsigned long long *out, hipStream_t s);

// ---- CG vector kernels (blas.hip)
struct BlasLaunch {
    const ProbDesc *probs;
    const int *tile2prob;
    SolveState *states;
    ShiftState *ms;
    int want;
    int fin;
    double *partials;
    void *v[6];
    float *n[6];
    double coef;
    double *red;   // fused CG ops: compact per-tile sums, [2][ntot]: p.Ap, then |r|^2
    int ntot;      // tiles of the whole set
    int pad;
};
enum : int {
    BL_RUPDATE = 0,   // r -= alpha Ap; x += alpha p; partial |r|^2; FIN_BETA
    BL_PUPDATE = 1,   // p = r + beta p
    BL_XACCUM = 2,    // x_hi += x_lo; x_lo = 0
    BL_RESUME = 3,    // r_lo = r_hi; p = r_lo + beta p
    BL_NORM = 4,      // partial |v0|^2 (FP64 vector)
    BL_INIT = 5,      // r_lo = b; p = b; x_lo = 0 (cold start)
    BL_STATUS = 6,    // RESUME -> RUNNING (one thread per problem)
    BL_COPY_D2F = 7,  // v1 (prec) = v0 (FP64)
    BL_COPY_F2D = 8,  // v1 (FP64) = v0 (prec)
    BL_START = 9,     // r_lo = r_hi (v4); p = r_hi; x_lo = 0 (warm start)
    BL_MS_RUPDATE = 10,  // multi-shift: r -= alpha Ap; partial |r|^2 (FIN_MS)
    BL_MS_UPDATE = 11,   // multi-shift: x_k += a_k p_k; p_k = z_k r + b_k p_k; p = r + beta p
    BL_MS_INIT = 12,     // multi-shift: r = p = b (FP32); p_k = b; x_k = 0; partial |b|^2
    BL_STATUS_MS = 13,   // MS_LAST -> CONVERGED (one thread per problem)
    // The CG update with its finishers folded in: every block sums its
    // problem's compact tile sums itself (same order, same bits in every block).
    BL_RUPDATE_F = 14,   // snapshot the state; alpha = rr / sum(p.Ap); r -= alpha Ap; x += alpha p; |r|^2 to red
    BL_PUPDATE_F = 15,   // beta, convergence and reliable trigger from the snapshot; new state; p = r + beta p
};
// vector roles for the multi-shift ops: v0 = r, v1 = Ap, v3 = p, v5 = b (FP64),
// v2 = x_k base, v4 = p_k base ([rhs][shift][h][3] FP32); ms = per-rhs ShiftState
hipError_t launch_stamp(long long *out, hipStream_t s);
hipError_t launch_finish(const ProbDesc *probs, SolveState *states, const double *partials, int fin, int want,
                         int nv, int nprob, hipStream_t s, ShiftState *ms = nullptr);
// contiguous complex arrays: FP64 <-> FP32 (prec 0 / 1), n complex numbers
hipError_t launch_convert(const void *src, int sprec, void *dst, int dprec, long long n, hipStream_t s);
hipError_t launch_blas(int op, int prec, const BlasLaunch &a, int ntiles, int nprob, hipStream_t s);
hipError_t launch_ms(int op, const BlasLaunch &a, int ntiles, hipStream_t s);

}  // namespace hisq
