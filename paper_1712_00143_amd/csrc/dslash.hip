// Half-lattice HISQ Dslash: for every site x of the output parity,
//   out(x) = sum_mu [ F_mu(x) in(x+mu) - F_mu(x-mu)^+ in(x-mu)
//                   + L_mu(x) in(x+3mu) - L_mu(x-3mu)^+ in(x-3mu) ]
// (fat one-hop plus Naik three-hop, staggered phases folded into the links).
// The paper describes this matrix-vector stencil as the inner work of the
// staggered CG (Section 4.2: matrix-vector multiplies, 0.26 flop/byte).
//
// Work decomposition: a block owns one 64-site tile; its W wavefronts split
// the 16 hop directions (16/W each), so every load instruction of a wave reads
// 64 consecutive link records of one direction block.  Partial colour vectors
// are summed through LDS in a fixed order, and wave 0 runs the epilogue:
//   PLAIN  out = D in
//   AX     out = diag*aux - D in,   partial Re(aux^+ out)      (CG: A p, p.Ap)
//   RES    out = b - diag*aux + D in, partial |out|^2           (FP64 true residual)
// Reductions leave per-tile FP64 partials for k_finish.
#include "finish.h"
#include "fields.h"
#include "launch.h"
#include "reduce.h"

namespace hisq {

template <class LT, int R, class ST, class OT, int W, int EPI, int CP>
__device__ __forceinline__ void dslash_body(const DslashLaunch &a)
{
    using A = typename AccOf<LT>::type;
    static_assert(16 % W == 0, "W must divide 16");
    constexpr int DPW = 16 / W;
    using F = LinkFmt<LT, R>;
    // the wave index is uniform: keep it (and the direction-block bases) scalar
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_tile(blockIdx.x, gridDim.x, a.remap);
    const int prob = a.tile2prob ? a.tile2prob[tile] : 0;
    const ProbDesc &pd = a.probs[prob];
    if (a.states && a.states[prob].status != a.want) return;
    const int i = (tile - pd.tile_begin) * TILE + lane;
    const int h = pd.h;
    const bool valid = i < h;
    const int par = a.out_par;
    const LinkSet &ls = pd.ls[a.lslot];
    const char *lbase = (const char *)ls.ptr[par];
    const int hs = ls.hs;   // link plane stride
    const long long voff = pd.voff;
    const int L0 = pd.L[0], L1 = pd.L[1], L2 = pd.L[2], L3 = pd.L[3];

    Cx<A> acc[3];
#pragma unroll
    for (int c = 0; c < 3; c++) acc[c] = {(A)0, (A)0};

    if (valid) {
        const Coord co = cb_to_coord_pd(i, par, pd);
        const int lex = 2 * i + (co.x[0] & 1);
        // prefix parities for eta_mu(x)
        const int e1 = co.x[0] & 1, e2 = (co.x[0] + co.x[1]) & 1, e3 = (co.x[0] + co.x[1] + co.x[2]) & 1;
        Spin<ST> in{(ST *)a.in, (float *)a.in_nrm};
        // Stage the work in groups of G directions: all index maths, then all
        // link loads, then all neighbour gathers, then the arithmetic, so that
        // G links are in flight per thread.
        constexpr int G = DPW < (sizeof(LT) == 8 ? 2 : 4) ? DPW : (sizeof(LT) == 8 ? 2 : 4);
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
            if constexpr (CP < 2) {
#pragma unroll
                for (int g = 0; g < G; g++)
                    load_link_raw_wave<LT, R, CP>(lbase + (size_t)(wave * DPW + g0 + g) * hs * F::BYTES, i, hs, raw[g]);
            } else {
                // part of the operator kept in the Infinity Cache: direction
                // blocks below a.cpol load cached, the rest stream.  The choice
                // is made once per group (uniform over the wave) so that the
                // group's loads still issue back to back.
                const int dg = wave * DPW + g0;
                if (dg + G <= a.cpol) {
#pragma unroll
                    for (int g = 0; g < G; g++)
                        load_link_raw_wave<LT, R, 1>(lbase + (size_t)(dg + g) * hs * F::BYTES, i, hs, raw[g]);
                } else if (dg >= a.cpol) {
#pragma unroll
                    for (int g = 0; g < G; g++)
                        load_link_raw_wave<LT, R, 0>(lbase + (size_t)(dg + g) * hs * F::BYTES, i, hs, raw[g]);
                } else {
#pragma unroll
                    for (int g = 0; g < G; g++) {
                        const char *db = lbase + (size_t)(dg + g) * hs * F::BYTES;
                        if (dg + g < a.cpol) load_link_raw_wave<LT, R, 1>(db, i, hs, raw[g]);
                        else load_link_raw_wave<LT, R, 0>(db, i, hs, raw[g]);
                    }
                }
            }
            Cx<A> v[G][3];
#pragma unroll
            for (int g = 0; g < G; g++) load_spinor<ST, A>(in, voff + nb[g], v[g]);
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int d = wave * DPW + g0 + g;
                const int mu = d >> 2;
                Cx<A> u[3][3];
                decode_link<LT, R, A>(raw[g], u);
                if constexpr (R == 12 || sizeof(LT) == 2) {
                    const int fld = (d & 2) ? 1 : 0;
                    A coef = (A)ls.a[fld];
                    if constexpr (R == 12) {
                        const int eb = mu == 0 ? 0 : mu == 1 ? e1 : mu == 2 ? e2 : e3;
                        const int neg = (ls.s[fld] < 0) ^ eb ^ (d & 1);
                        coef = neg ? -coef : coef;
                    }
                    matvec_acc_scaled(u, v[g], coef, acc);
                } else {
                    matvec_acc(u, v[g], acc);
                }
            }
        }
    }

    if constexpr (W > 1) {
        __shared__ A red[(W > 1 ? W - 1 : 1) * 6 * 64];
        if (wave > 0) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                red[((wave - 1) * 6 + 2 * c) * 64 + lane] = acc[c].re;
                red[((wave - 1) * 6 + 2 * c + 1) * 64 + lane] = acc[c].im;
            }
        }
        __syncthreads();
        if (wave == 0) {
            for (int w = 1; w < W; w++) {
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[c].re += red[((w - 1) * 6 + 2 * c) * 64 + lane];
                    acc[c].im += red[((w - 1) * 6 + 2 * c + 1) * 64 + lane];
                }
            }
        }
    }

    double part = 0.0;
    if (wave == 0 && valid) {
        const long long o = voff + i;
        Spin<OT> out{(OT *)a.out, a.out_nrm};
        if constexpr (EPI == EPI_PLAIN) {
            store_spinor<OT, A>(out, o, acc);
        } else if constexpr (EPI == EPI_AX) {
            Spin<ST> aux{(ST *)a.aux, (float *)a.aux_nrm};
            Cx<A> p[3], v[3];
            load_spinor<ST, A>(aux, o, p);
            const A dg = (A)pd.diag;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                v[c] = {dg * p[c].re - acc[c].re, dg * p[c].im - acc[c].im};
                part += (double)p[c].re * (double)v[c].re + (double)p[c].im * (double)v[c].im;
            }
            store_spinor<OT, A>(out, o, v);
        } else {  // EPI_RES
            Spin<ST> aux{(ST *)a.aux, (float *)a.aux_nrm};
            Cx<A> x[3], v[3];
            load_spinor<ST, A>(aux, o, x);
            const double2 *b = reinterpret_cast<const double2 *>(a.bvec) + o * 3;
            const A dg = (A)pd.diag;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                double2 bb = b[c];
                v[c] = {(A)bb.x - dg * x[c].re + acc[c].re, (A)bb.y - dg * x[c].im + acc[c].im};
                part += (double)v[c].re * (double)v[c].re + (double)v[c].im * (double)v[c].im;
            }
            store_spinor<OT, A>(out, o, v);
        }
    }
    if constexpr (EPI != EPI_PLAIN) {
        if (a.red) {
            publish_compact(part, a.red, tile);
        } else if (a.fin != FIN_NONE) {
            double mine[1] = {part};
            publish_partials<1>(mine, a.partials, tile);
        }
    }
}

template <class LT, int R, class ST, class OT, int W, int EPI, int CP>
__global__ void __launch_bounds__(64 * W) k_dslash(DslashLaunch a)
{
    dslash_body<LT, R, ST, OT, W, EPI, CP>(a);
}

// The same kernel compiled for at most two waves per SIMD: the register
// budget then lets a wave keep more of its link loads in flight before the
// first arithmetic (with the default budget the compiler interleaves them),
// which pays for the one- and two-wave blocks that walk many directions.
template <class LT, int R, class ST, class OT, int W, int EPI, int CP>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(1, 2))) k_dslash_lo(DslashLaunch a)
{
    dslash_body<LT, R, ST, OT, W, EPI, CP>(a);
}

// ------------------------------------------------------------- launchers

template <class LT, int R, class ST, class OT, int EPI, int CP>
static hipError_t launch_wc(int W, const DslashLaunch &a, int nblocks, hipStream_t s)
{
    switch (W) {
    case 1 | W_LOWOCC:
        hipLaunchKernelGGL((k_dslash_lo<LT, R, ST, OT, 1, EPI, CP>), dim3(nblocks), dim3(64), 0, s, a);
        break;
    case 2 | W_LOWOCC:
        hipLaunchKernelGGL((k_dslash_lo<LT, R, ST, OT, 2, EPI, CP>), dim3(nblocks), dim3(128), 0, s, a);
        break;
    case 1: hipLaunchKernelGGL((k_dslash<LT, R, ST, OT, 1, EPI, CP>), dim3(nblocks), dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_dslash<LT, R, ST, OT, 2, EPI, CP>), dim3(nblocks), dim3(128), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_dslash<LT, R, ST, OT, 4, EPI, CP>), dim3(nblocks), dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_dslash<LT, R, ST, OT, 8, EPI, CP>), dim3(nblocks), dim3(512), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_dslash<LT, R, ST, OT, 16, EPI, CP>), dim3(nblocks), dim3(1024), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LT, int R, class ST, class OT, int EPI>
static hipError_t launch_w(int W, const DslashLaunch &a, int nblocks, hipStream_t s)
{
    // a.cpol: 0 streams every link block, 16 keeps all in the Infinity Cache,
    // 1..15 keeps that many of the 16 direction blocks
    return a.cpol <= 0 ? launch_wc<LT, R, ST, OT, EPI, 0>(W, a, nblocks, s)
           : a.cpol >= 16 ? launch_wc<LT, R, ST, OT, EPI, 1>(W, a, nblocks, s)
                          : launch_wc<LT, R, ST, OT, EPI, 2>(W, a, nblocks, s);
}

template <class LT, class ST, class OT, int EPI>
static hipError_t launch_r(int recon, int W, const DslashLaunch &a, int nb, hipStream_t s)
{
    return recon == 12 ? launch_w<LT, 12, ST, OT, EPI>(W, a, nb, s)
                       : launch_w<LT, 18, ST, OT, EPI>(W, a, nb, s);
}

// prec: 0 = FP64, 1 = FP32, 2 = FP16 (links and input vectors); out_prec may
// differ from prec only for FP16 (out FP32).
hipError_t launch_dslash(int prec, int recon, int out_prec, int epi, int W, const DslashLaunch &a,
                         int nblocks, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    if (prec == 0) {
        if (out_prec != 0) return hipErrorInvalidValue;
        switch (epi) {
        case EPI_PLAIN: return launch_r<double, double, double, EPI_PLAIN>(recon, W, a, nblocks, s);
        case EPI_AX: return launch_r<double, double, double, EPI_AX>(recon, W, a, nblocks, s);
        case EPI_RES: return launch_r<double, double, double, EPI_RES>(recon, W, a, nblocks, s);
        }
    } else if (prec == 1) {
        if (out_prec != 1) return hipErrorInvalidValue;
        switch (epi) {
        case EPI_PLAIN: return launch_r<float, float, float, EPI_PLAIN>(recon, W, a, nblocks, s);
        case EPI_AX: return launch_r<float, float, float, EPI_AX>(recon, W, a, nblocks, s);
        }
    } else if (prec == 2) {
        if (epi == EPI_PLAIN && out_prec == 2)
            return launch_r<__half, __half, __half, EPI_PLAIN>(recon, W, a, nblocks, s);
        if (epi == EPI_AX && out_prec == 1)
            return launch_r<__half, __half, float, EPI_AX>(recon, W, a, nblocks, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hisq
