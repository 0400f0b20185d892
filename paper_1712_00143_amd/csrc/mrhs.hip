// Multi-right-hand-side half-lattice Dslash: NR colour vectors share every
// link load, so the link stream (the dominant traffic of a single Dslash) is
// amortised NR ways.  Used by the multi-shift CG over several sources
// (Section 4.1) and by hisq_dslash with nrhs > 1.
//
// Per link the work is a complex 3x3 times 3xNR product.  The kernel stays
// bandwidth-bound even at NR = 4 (about 3.4 flop/byte in FP32), far below
// the VALU ridge, so the contraction runs on the vector ALUs: staging it
// through MFMA tiles would add register shuffles without moving the bound.
//
// Layout: right-hand side j of the vector arguments starts at j * vstride
// sites; each right-hand side is a problem of the solve set (own FP64 state),
// and its reduction partials go to tile j * ntile + tile.
#include "fields.h"
#include "finish.h"
#include "launch.h"
#include "reduce.h"

namespace hisq {

template <class LT, int R, int W, int NR, int EPI>
__global__ void __launch_bounds__(64 * W) k_dslash_mrhs(MrhsLaunch a)
{
    using A = float;
    constexpr int DPW = 16 / W;
    using F = LinkFmt<LT, R>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, a.remap);
    const ProbDesc &pd = a.probs[0];
    bool act[NR];
    bool any = false;
#pragma unroll
    for (int j = 0; j < NR; j++) {
        act[j] = a.states ? a.states[j].status == a.want : true;
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
    const float *in = (const float *)a.in;

    Cx<A> acc[NR][3];
#pragma unroll
    for (int j = 0; j < NR; j++)
#pragma unroll
        for (int c = 0; c < 3; c++) acc[j][c] = {0.f, 0.f};

    if (valid) {
        const Coord co = cb_to_coord(i, par, pd.L);
        const int lex = 2 * i + (co.x[0] & 1);
        const int e1 = co.x[0] & 1, e2 = (co.x[0] + co.x[1]) & 1, e3 = (co.x[0] + co.x[1] + co.x[2]) & 1;
        constexpr int G = NR >= 3 ? (DPW < 2 ? DPW : 2) : (DPW < 4 ? DPW : 4);
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
                load_link_raw<LT, R>(lbase + (size_t)(wave * DPW + g0 + g) * h * F::BYTES, i, h, raw[g]);
            Cx<A> v[G][NR][3];
#pragma unroll
            for (int g = 0; g < G; g++)
#pragma unroll
                for (int j = 0; j < NR; j++) {
                    const float2 *p = reinterpret_cast<const float2 *>(in) + ((long long)j * a.vstride + nb[g]) * 3;
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        float2 t = act[j] ? p[c] : make_float2(0.f, 0.f);
                        v[g][j][c] = {t.x, t.y};
                    }
                }
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int d = wave * DPW + g0 + g;
                const int mu = d >> 2;
                Cx<A> u[3][3];
                decode_link<LT, R, A>(raw[g], u);
                A coef = 1.f;
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
                for (int j = 0; j < NR; j++)
#pragma unroll
                    for (int r = 0; r < 3; r++) {
                        Cx<A> s0 = cmul(u[r][0], v[g][j][0]);
                        Cx<A> t1 = cmul(u[r][1], v[g][j][1]);
                        Cx<A> t2 = cmul(u[r][2], v[g][j][2]);
                        acc[j][r].re += coef * (s0.re + t1.re + t2.re);
                        acc[j][r].im += coef * (s0.im + t1.im + t2.im);
                    }
            }
        }
    }

    if constexpr (W > 1) {
        __shared__ A red[(W - 1) * NR * 6 * 64];
        if (wave > 0) {
#pragma unroll
            for (int j = 0; j < NR; j++)
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    red[(((wave - 1) * NR + j) * 6 + 2 * c) * 64 + lane] = acc[j][c].re;
                    red[(((wave - 1) * NR + j) * 6 + 2 * c + 1) * 64 + lane] = acc[j][c].im;
                }
        }
        __syncthreads();
        if (wave == 0) {
            for (int w = 1; w < W; w++)
#pragma unroll
                for (int j = 0; j < NR; j++)
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        acc[j][c].re += red[(((w - 1) * NR + j) * 6 + 2 * c) * 64 + lane];
                        acc[j][c].im += red[(((w - 1) * NR + j) * 6 + 2 * c + 1) * 64 + lane];
                    }
        }
    }

    double part[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) part[j] = 0.0;
    if (wave == 0 && valid) {
        float *out = (float *)a.out;
#pragma unroll
        for (int j = 0; j < NR; j++) {
            if (!act[j]) continue;
            const long long o = (long long)j * a.vstride + i;
            float2 *po = reinterpret_cast<float2 *>(out) + o * 3;
            if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
                for (int c = 0; c < 3; c++) po[c] = make_float2(acc[j][c].re, acc[j][c].im);
            } else {
                const float2 *pp = reinterpret_cast<const float2 *>(a.aux) + o * 3;
                const float dg = (float)a.diag;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    float2 p = pp[c];
                    float vr = dg * p.x - acc[j][c].re, vi = dg * p.y - acc[j][c].im;
                    po[c] = make_float2(vr, vi);
                    part[j] += (double)p.x * (double)vr + (double)p.y * (double)vi;
                }
            }
        }
    }
    if constexpr (EPI == EPI_AX) {
        __shared__ double lds[16 * NR];
        block_sum<NR>(part, lds);
        if (threadIdx.x == 0) {
            const int ntile = pd.ntile;
            for (int j = 0; j < NR; j++) a.partials[((size_t)j * ntile + tile) * NPART] = part[j];
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
    case 16: hipLaunchKernelGGL((k_dslash_mrhs<LT, R, 16, NR, EPI>), dim3(nb), dim3(1024), 0, s, a); break;
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

// FP32 colour vectors; links FP32 (prec 1) or FP16 (prec 2); nrhs in 1..4
// per launch (callers split larger counts).
hipError_t launch_dslash_mrhs(int prec, int recon, int nrhs, int W, const MrhsLaunch &a, int nblocks,
                              hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    const bool ax = a.epi == EPI_AX;
    if (prec == 1) {
        if (recon == 12) return ax ? mrhs_n<float, 12, EPI_AX>(nrhs, W, a, nblocks, s)
                                   : mrhs_n<float, 12, EPI_PLAIN>(nrhs, W, a, nblocks, s);
        return ax ? mrhs_n<float, 18, EPI_AX>(nrhs, W, a, nblocks, s)
                  : mrhs_n<float, 18, EPI_PLAIN>(nrhs, W, a, nblocks, s);
    }
    if (prec == 2) {
        if (recon == 12) return ax ? mrhs_n<__half, 12, EPI_AX>(nrhs, W, a, nblocks, s)
                                   : mrhs_n<__half, 12, EPI_PLAIN>(nrhs, W, a, nblocks, s);
        return ax ? mrhs_n<__half, 18, EPI_AX>(nrhs, W, a, nblocks, s)
                  : mrhs_n<__half, 18, EPI_PLAIN>(nrhs, W, a, nblocks, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hisq
