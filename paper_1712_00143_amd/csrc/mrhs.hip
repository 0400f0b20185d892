// Multi-right-hand-side half-lattice Dslash: NR colour vectors share every
// link load, so the link stream (the dominant traffic of a single Dslash) is
// amortised NR ways.  Used by the multi-shift CG over several sources
// (Section 4.1) and by hisq_dslash with nrhs > 1.
//
// Per link the work is a complex 3x3 times 3xNR product, here on the vector
// ALUs; mrhs_mfma.hip holds the same operator for NR = 4 on the matrix cores
// (v_mfma_f32_4x4x1_16b_f32, one 4x4 block per site), and the autotuner times
// both and keeps the faster.
//
// Layout: right-hand side r of the vector arguments starts at r * vstride
// sites; each right-hand side may be a problem of a solve set (own FP64 state
// a.states[r], own descriptor with its diagonal term, all on the lattice of
// a.probs[0]), and its reduction partials go to tile r * ntile + tile.  The
// right-hand sides are processed NR at a time: with ng = ceil(nrhs / NR)
// groups, logical block b serves group b % ng (right-hand sides NR*g ..
// NR*g + NR - 1) on tile b / ng.
#include "fields.h"
#include "finish.h"
#include "launch.h"
#include "reduce.h"

namespace hisq {

// Vector element type of the multi-RHS kernel: FP64 vectors with FP64 links,
// FP32 vectors otherwise.
template <class LT> struct MrhsVec { using type = float; using pair = float2; };
template <> struct MrhsVec<double> { using type = double; using pair = double2; };

template <class LT, int R, int W, int NR, int EPI>
__global__ void __launch_bounds__(64 * W) k_dslash_mrhs(MrhsLaunch a)
{
    using A = typename AccOf<LT>::type;
    using V2 = typename MrhsVec<LT>::pair;
    constexpr int DPW = 16 / W;
    using F = LinkFmt<LT, R>;
    // the wave index is uniform: keep it (and the direction-block bases) scalar
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const ProbDesc &pd = a.probs[0];
    // groups innermost: the blocks of all groups on one tile run back to back
    // on the same XCD, so the tile's links come from that XCD's L2 after the
    // first group instead of being streamed from HBM once per group
    const int bt = xcd_tile(blockIdx.x, gridDim.x, a.remap);
    const int ng = gridDim.x / pd.ntile;
    const int tile = bt / ng;
    const int grp = bt - tile * ng;
    const int r0 = grp * NR;
    bool act[NR];
    bool any = false;
#pragma unroll
    for (int j = 0; j < NR; j++) {
        act[j] = r0 + j < a.nrhs && (a.states ? a.states[r0 + j].status == a.want : true);
        any |= act[j];
    }
    if (!any) return;
    const int h = pd.h;
    const int i = tile * TILE + lane;
    const bool valid = i < h;
    const int par = a.out_par;
    const LinkSet &ls = pd.ls[a.lslot];
    const char *lbase = (const char *)ls.ptr[par];
    const int L0 = pd.L[0], L1 = pd.L[1], L2 = pd.L[2], L3 = pd.L[3];
    const V2 *in = (const V2 *)a.in;

    Cx<A> acc[NR][3];
#pragma unroll
    for (int j = 0; j < NR; j++)
#pragma unroll
        for (int c = 0; c < 3; c++) acc[j][c] = {(A)0, (A)0};

    if (valid) {
        const Coord co = cb_to_coord_pd(i, par, pd);
        const int lex = 2 * i + (co.x[0] & 1);
        const int e1 = co.x[0] & 1, e2 = (co.x[0] + co.x[1]) & 1, e3 = (co.x[0] + co.x[1] + co.x[2]) & 1;
        // links in flight per thread: fewer when the gathered vectors are many or wide
        constexpr int GMAX = sizeof(LT) == 8 ? (NR >= 3 ? 1 : 2) : (NR >= 3 ? 2 : 4);
        constexpr int G = DPW < GMAX ? DPW : GMAX;
#pragma unroll
        for (int g0 = 0; g0 < DPW; g0 += G) {
            int nb[G];
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int d = wave * DPW + g0 + g;
                const int mu = d >> 2;
                const int k = dir_step(d);
                const int x = mu == 0 ? co.x[0] : mu == 1 ? co.x[1] : mu == 2 ? co.x[2] : co.x[3];
                const int Lm = mu == 0 ? L0 : mu == 1 ? L1 : mu == 2 ? L2 : L3;
                const int Sm = mu == 0 ? 1 : mu == 1 ? L0 : mu == 2 ? L0 * L1 : L0 * L1 * L2;
                int v = x + k;
                v -= v >= Lm ? Lm : 0;
                v -= v >= Lm ? Lm : 0;
                v += v < 0 ? Lm : 0;
                v += v < 0 ? Lm : 0;
                nb[g] = (lex + (v - x) * Sm) >> 1;
            }
            RawLink<LT, R> raw[G];
#pragma unroll
            for (int g = 0; g < G; g++)
                load_link_raw_wave<LT, R>(lbase + (size_t)(wave * DPW + g0 + g) * ls.hs * F::BYTES, i, ls.hs, raw[g]);
            Cx<A> v[G][NR][3];
#pragma unroll
            for (int g = 0; g < G; g++)
#pragma unroll
                for (int j = 0; j < NR; j++) {
                    const V2 *p = in + ((long long)(r0 + j) * a.vstride + nb[g]) * 3;
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        V2 t = act[j] ? p[c] : V2{(A)0, (A)0};
                        v[g][j][c] = {t.x, t.y};
                    }
                }
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int d = wave * DPW + g0 + g;
                const int mu = d >> 2;
                Cx<A> u[3][3];
                decode_link<LT, R, A>(raw[g], u);
                A coef = (A)1;
                if constexpr (R == 12 || sizeof(LT) == 2) {
                    const int fld = (d & 2) ? 1 : 0;
                    coef = (A)ls.a[fld];
                    if constexpr (R == 12) {
                        const int eb = mu == 0 ? 0 : mu == 1 ? e1 : mu == 2 ? e2 : e3;
                        const int neg = (ls.s[fld] < 0) ^ eb ^ (d & 1);
                        coef = neg ? -coef : coef;
                    }
                }
#pragma unroll
                for (int j = 0; j < NR; j++) {
                    if constexpr (R == 12 || sizeof(LT) == 2) matvec_acc_scaled(u, v[g][j], coef, acc[j]);
                    else matvec_acc(u, v[g][j], acc[j]);
                }
            }
        }
    }

    if constexpr (W > 1) {
        // pairwise tree over the waves (W is a power of two): the upper half
        // hands its partial vectors to the lower half through LDS, halving
        // each round, so LDS holds W/2 waves' worth (more blocks per CU than
        // a single round into wave 0) and the summation order is fixed
        __shared__ A red[(W / 2) * NR * 6 * 64];
#pragma unroll
        for (int half = W / 2; half >= 1; half >>= 1) {
            if (wave >= half && wave < 2 * half) {
#pragma unroll
                for (int j = 0; j < NR; j++)
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        red[(((wave - half) * NR + j) * 6 + 2 * c) * 64 + lane] = acc[j][c].re;
                        red[(((wave - half) * NR + j) * 6 + 2 * c + 1) * 64 + lane] = acc[j][c].im;
                    }
            }
            __syncthreads();
            if (wave < half) {
#pragma unroll
                for (int j = 0; j < NR; j++)
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        acc[j][c].re += red[((wave * NR + j) * 6 + 2 * c) * 64 + lane];
                        acc[j][c].im += red[((wave * NR + j) * 6 + 2 * c + 1) * 64 + lane];
                    }
            }
            if (half > 1) __syncthreads();
        }
    }

    double part[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) part[j] = 0.0;
    if (wave == 0 && valid) {
        V2 *out = (V2 *)a.out;
#pragma unroll
        for (int j = 0; j < NR; j++) {
            if (!act[j]) continue;
            const long long o = (long long)(r0 + j) * a.vstride + i;
            V2 *po = out + o * 3;
            if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
                for (int c = 0; c < 3; c++) po[c] = V2{acc[j][c].re, acc[j][c].im};
            } else if constexpr (EPI == EPI_AX) {
                const V2 *pp = (const V2 *)a.aux + o * 3;
                const A dg = (A)a.probs[(r0 + j) * a.desc_stride].diag;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    V2 p = pp[c];
                    A vr = dg * p.x - acc[j][c].re, vi = dg * p.y - acc[j][c].im;
                    po[c] = V2{vr, vi};
                    part[j] += (double)p.x * (double)vr + (double)p.y * (double)vi;
                }
            } else {  // EPI_RES: out = b - diag x + D in, |out|^2
                const V2 *px = (const V2 *)a.aux + o * 3;
                const double2 *pb = reinterpret_cast<const double2 *>(a.bvec) + o * 3;
                const A dg = (A)a.probs[(r0 + j) * a.desc_stride].diag;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    V2 x = px[c];
                    double2 bb = pb[c];
                    A vr = (A)bb.x - dg * x.x + acc[j][c].re, vi = (A)bb.y - dg * x.y + acc[j][c].im;
                    po[c] = V2{vr, vi};
                    part[j] += (double)vr * (double)vr + (double)vi * (double)vi;
                }
            }
        }
    }
    if constexpr (EPI != EPI_PLAIN) {
        __shared__ double lds[16 * NR];
        block_sum<NR>(part, lds);
        if (threadIdx.x == 0) {
            const int ntile = pd.ntile;
            for (int j = 0; j < NR; j++) {
                if (r0 + j >= a.nrhs) continue;
                if (a.red) a.red[(size_t)(r0 + j) * ntile + tile] = part[j];
                else a.partials[((size_t)(r0 + j) * ntile + tile) * NPART] = part[j];
            }
        }
    }
}

template <class LT, int R, int NR, int EPI>
static hipError_t mrhs_w(int W, const MrhsLaunch &a, int nb, hipStream_t s)
{
    switch (W) {
    case 2: hipLaunchKernelGGL((k_dslash_mrhs<LT, R, 2, NR, EPI>), dim3(nb), dim3(128), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_dslash_mrhs<LT, R, 4, NR, EPI>), dim3(nb), dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_dslash_mrhs<LT, R, 8, NR, EPI>), dim3(nb), dim3(512), 0, s, a); break;
    case 16:
        // the LDS reduction of 15 waves of FP64 partial vectors does not fit
        if constexpr (sizeof(LT) == 8) return hipErrorInvalidValue;
        else hipLaunchKernelGGL((k_dslash_mrhs<LT, R, 16, NR, EPI>), dim3(nb), dim3(1024), 0, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LT, int R, int EPI>
static hipError_t mrhs_n(int nr, int W, const MrhsLaunch &a, int nb, hipStream_t s)
{
    switch (nr) {
    case 1: return mrhs_w<LT, R, 1, EPI>(W, a, nb, s);
    case 2: return mrhs_w<LT, R, 2, EPI>(W, a, nb, s);
    case 3: return mrhs_w<LT, R, 3, EPI>(W, a, nb, s);
    case 4: return mrhs_w<LT, R, 4, EPI>(W, a, nb, s);
    }
    return hipErrorInvalidValue;
}

template <class LT, int R>
static hipError_t mrhs_e(int epi, int nr, int W, const MrhsLaunch &a, int nb, hipStream_t s)
{
    switch (epi) {
    case EPI_PLAIN: return mrhs_n<LT, R, EPI_PLAIN>(nr, W, a, nb, s);
    case EPI_AX: return mrhs_n<LT, R, EPI_AX>(nr, W, a, nb, s);
    }
    return hipErrorInvalidValue;
}

// Links FP64 (prec 0, FP64 vectors; recon-18, PLAIN and RES epilogues: the
// reliable updates), FP32 (prec 1) or FP16 (prec 2) with FP32 vectors (PLAIN
// and AX).  `nrhs` is the group size NR in 1..4; a.nrhs right-hand sides in
// total.
hipError_t launch_dslash_mrhs(int prec, int recon, int nrhs, int W, const MrhsLaunch &a, int ntile,
                              hipStream_t s)
{
    if (ntile <= 0 || a.nrhs <= 0) return hipSuccess;
    if (nrhs < 1 || nrhs > 4 || (nrhs < 4 && a.nrhs > nrhs)) return hipErrorInvalidValue;
    const long long nb = (long long)(a.nrhs + nrhs - 1) / nrhs * ntile;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    const int nblocks = (int)nb;
    if (nb > ntile && !a.remap) {
        // several groups: the XCD-contiguous order is what places the groups
        // of one tile on one XCD to share its links through the L2 (the
        // tuner times one group, where the order hardly matters)
        MrhsLaunch b = a;
        b.remap = 1;
        return launch_dslash_mrhs(prec, recon, nrhs, W, b, ntile, s);
    }
    if (W == MRHS_MFMA) {
        if (nrhs != 4 || prec == 0) return hipErrorInvalidValue;
        return launch_dslash_mrhs_mfma(prec, recon, a, nblocks, s);
    }
    if (prec == 0) {
        if (recon != 18) return hipErrorInvalidValue;
        switch (a.epi) {
        case EPI_PLAIN: return mrhs_n<double, 18, EPI_PLAIN>(nrhs, W, a, nblocks, s);
        case EPI_RES: return mrhs_n<double, 18, EPI_RES>(nrhs, W, a, nblocks, s);
        }
        return hipErrorInvalidValue;
    }
    if (prec == 1) return recon == 12 ? mrhs_e<float, 12>(a.epi, nrhs, W, a, nblocks, s)
                                      : mrhs_e<float, 18>(a.epi, nrhs, W, a, nblocks, s);
    if (prec == 2) return recon == 12 ? mrhs_e<__half, 12>(a.epi, nrhs, W, a, nblocks, s)
                                      : mrhs_e<__half, 18>(a.epi, nrhs, W, a, nblocks, s);
    return hipErrorInvalidValue;
}

}  // namespace hisq
