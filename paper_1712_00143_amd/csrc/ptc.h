// Launch descriptors of the PTC preconditioner and flexible-CG kernels.
#pragma once
#include "hisq_dev.h"

namespace hisq {

struct PtcLaunch {
    const ProbDesc *probs;   // the lattice (links, geometry)
    int lslot;               // link set for the transports
    int in_zero_par;         // parity whose input is known zero (-1: none)
    const void *w;           // weights [Cout][Cin][9] complex (float2 or half2)
    const float *in;         // input activations [B][Cin][2][h][3] complex
    long long in_bstride;    // floats between batch entries
    float *out;              // output [B][Cout][out_pstride][h][3]
    long long out_bstride;
    int out_pstride;         // parities stored per output channel (1 or 2)
    int out_par0;            // first stored output parity
    int par_lo;              // first output parity computed (grid: npar * ntile blocks)
    int pad;
    const float *g;          // weight gradient: output gradient [B][Cout][g_pstride][h][3]
    long long g_bstride;
    int g_pstride, g_par0;
    double *partials;
    const float *tgt;        // loss: targets [B][h][3]
    long long tgt_bstride;
    const double *ee;        // loss: normalisation per batch entry (|e|^2, or <e, r> for the energy norm)
    const float *wvec;       // energy-norm loss: D_eo D_oe z, so that A z = wdiag z - wvec (null: Euclidean)
    double wdiag;
    // flexible-CG fusion (all null / unused otherwise)
    const SolveState *gate;  // skip the launch unless gate->status == gate_want
    int gate_want;
    int dot_nt;              // tiles of the dot partials below
    const float *addin;      // out += addin (same layout as out, COUT = 1, one parity)
    long long addin_bstride;
    const float *dotq;       // with dotred: per-tile (dotq, out) into dotred[tile], dotred[dot_nt + tile]
    double *dotred;
};

// Fusion of the preconditioner into the flexible CG's iteration: launches are
// skipped unless gate->status == want, and the final layer also forms the
// per-tile partials of (q, z) (re in red[tile], im in red[nt + tile]).
struct PtcFuse {
    const SolveState *gate;
    int want;
    const float *q;
    double *red;
    int nt;
};

hipError_t launch_ptc_layer(int prec, int recon, bool w16, int cin, int cout, int W, const PtcLaunch &a, int nblk,
                            int batch, hipStream_t s);

// Inference layer with FP16 activation storage (ptc_infer.hip): activations
// [2 parities][h][C][3] half2 plus one FP32 scale per (parity, site).
struct PtcInferLaunch {
    const ProbDesc *probs;
    int lslot;
    int par_lo;              // first output parity (grid: npar * ntile blocks)
    const void *w;           // FP16 weights [Cout][Cin][9] complex
    const float *in32;       // input kind 0: even FP32 vector [h][3] complex (odd parity zero)
    const __half2 *in16;     // input kind 1: FP16 activation
    const float *in_scale;
    __half2 *out16;          // output kind 0: FP16 activation
    float *out_scale;
    float *out32;            // output kind 1: even FP32 vector z = addin + layer output
    const float *addin;
    const float *dotq;       // with dotred: per-tile (dotq, z) into dotred[tile], dotred[dot_nt + tile]
    double *dotred;
    int dot_nt;
    int gate_want;
    const SolveState *gate;  // skip the launch unless gate->status == gate_want
};
// W: 1, 3 or 9 waves per block, or'ed with PTC_MFMA (3 and 9, cout >= cin)
// for the matrix-core channel mixing
constexpr int PTC_MFMA = 0x100;
hipError_t launch_ptc_infer(int prec, int recon, int cin, int cout, int ik, int ok, int W, const PtcInferLaunch &a,
                            int nblk, hipStream_t s);
constexpr int WGRAD_ROWS = 1024;   // weight-gradient partial rows (blocks) at most

// Weight-gradient partials of npar output parities x batch entries, reduced
// into nrow rows (one per block) of [9][cout][cin] complex FP64.
hipError_t launch_ptc_wgrad(int prec, int recon, int cin, int cout, const PtcLaunch &a, int npar, int batch, int nrow,
                           hipStream_t s);
hipError_t launch_ptc_wsum(const double *partials, long long nrow, int cin, int cout, double *gw, int accumulate,
                           hipStream_t s);
hipError_t launch_ptc_loss(const PtcLaunch &a, int ntile, int batch, double *loss, hipStream_t s);
hipError_t launch_adam(float *w, float *m, float *v, const double *g, int n, int step, float lr, __half *w16,
                       hipStream_t s);
hipError_t launch_ptc_adjoint(const float *w, int cin, int cout, float *wadj, hipStream_t s);
hipError_t launch_to_half(const float *w, __half *w16, int n, hipStream_t s);
hipError_t launch_ptc_gadj(const double *gp, int cin_p, int cout_p, double *gw, hipStream_t s);
hipError_t launch_add_f32(float *z, const float *r, long long n, hipStream_t s);

// flexible CG vector kernels (FP32 vectors, complex FP64 scalars in SolveState::cplx)
struct FcgLaunch {
    const ProbDesc *probs;
    SolveState *states;
    int want;
    int op;
    double *partials;
    float *r, *x, *p, *q, *z;
    double *red;   // fused ops: compact tile sums [(p,q)][Re (p,r)][Im (p,r)][|r|^2][Re (q,z)][Im (q,z)], nt each
    int nt;
};
enum : int { FCG_DOTS_B = 2, FCG_P = 3, FCG_XR_F = 4, FCG_P_F = 5, FCG_DOT_PR = 6 };
// offsets of the compact sums in FcgLaunch::red, in units of nt
// (the three sums each fused op reads are adjacent)
enum : int { FRED_PQ = 0, FRED_PR = 1, FRED_RR = 3, FRED_QZ = 4, FRED_N = 6 };
hipError_t launch_fcg(const FcgLaunch &a, int ntile, hipStream_t s);

}  // namespace hisq
