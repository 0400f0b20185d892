// Multi-right-hand-side half-lattice Dslash on the matrix cores: four right-
// hand sides per link read, the per-site product [3x3] x [3x4] complex done
// by v_mfma_f32_4x4x1_16b_f32.
//
// That instruction holds 16 independent 4x4 blocks, block b in lanes
// 4b .. 4b+3; lane 4b+t supplies row t of the block's A column and column t
// of its B row, and receives column t of the 4x4 result (one row per
// register).  Here block b is one output site and column t one right-hand
// side.  The complex product out[i][t] = sum_c U[i][c] V[c][t] in real form
// has six result rows (Re/Im of three colours): rows (Re 0, Im 0, Re 1,
// Im 1) in one accumulator and (Re 2, Im 2, 0, 0) in a second, and six rank-1
// steps per link (colour c, real or imaginary part of V):
//   Re_i += U_r[i][c] V_r[c] - U_i[i][c] V_i[c],
//   Im_i += U_i[i][c] V_r[c] + U_r[i][c] V_i[c],
// so 12 instructions per link for 16 sites x 4 right-hand sides.  Lane
// (b, t) loads the link of site b (the four lanes of a site read the same
// bytes, merged by the load unit) and the gathered colour vector of
// right-hand side t, so no lane exchanges are needed.
//
// A block is one 64-site tile: four waves of 16 sites each walk all 16
// directions.  Groups of four right-hand sides, descriptors, states and
// reduction layout are those of k_dslash_mrhs (FP32 vectors; FP32 or FP16
// links; PLAIN and AX epilogues).
#include "fields.h"
#include "finish.h"
#include "launch.h"
#include "reduce.h"

namespace hisq {

namespace {

typedef float mr_f4 __attribute__((ext_vector_type(4)));

}  // namespace

template <class LT, int R, int EPI>
__global__ void __launch_bounds__(256) k_dslash_mrhs_mfma(MrhsLaunch a)
{
    using F = LinkFmt<LT, R>;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const ProbDesc &pd = a.probs[0];
    const int bt = xcd_tile(blockIdx.x, gridDim.x, a.remap);
    const int ng = gridDim.x / pd.ntile;
    const int tile = bt / ng;
    const int grp = bt - tile * ng;
    const int r0 = grp * 4;
    bool any = false;
#pragma unroll
    for (int j = 0; j < 4; j++) any |= r0 + j < a.nrhs && (a.states ? a.states[r0 + j].status == a.want : true);
    if (!any) return;
    const int b = lane >> 2, t = lane & 3;
    const int rhs = r0 + t;
    const bool act = rhs < a.nrhs && (a.states ? a.states[rhs].status == a.want : true);
    const int h = pd.h;
    const int i = tile * TILE + 16 * wave + b;
    const bool valid = i < h;
    const int par = a.out_par;
    const LinkSet &ls = pd.ls[a.lslot];
    const char *lbase = (const char *)ls.ptr[par];
    const float2 *in = (const float2 *)a.in;
    // every lane runs the matrix instructions; lanes past the lattice or of
    // an inactive right-hand side feed zeros
    const int ic = valid ? i : 0;
    const Coord co = cb_to_coord_pd(ic, par, pd);
    const int lex = 2 * ic + (co.x[0] & 1);
    const int e1 = co.x[0] & 1, e2 = (co.x[0] + co.x[1]) & 1, e3 = (co.x[0] + co.x[1] + co.x[2]) & 1;
    const int L0 = pd.L[0], L1 = pd.L[1], L2 = pd.L[2], L3 = pd.L[3];
    const int ri = t >> 1, im = t & 1;   // the lane's rows: (Re|Im of colour ri) and (Re|Im of colour 2)
    mr_f4 C0 = {0.f, 0.f, 0.f, 0.f}, C1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int d = 0; d < 16; d++) {
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
        const int nb = (lex + (v - x) * Sm) >> 1;
        RawLink<LT, R> raw;
        load_link_raw_wave<LT, R, 0>(lbase + (size_t)d * ls.hs * F::BYTES, ic, ls.hs, raw);
        float2 vv[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
        if (valid && act) {
            const float2 *p = in + ((long long)rhs * a.vstride + nb) * 3;
#pragma unroll
            for (int c = 0; c < 3; c++) vv[c] = p[c];
        }
        Cx<float> u[3][3];
        decode_link<LT, R, float>(raw, u);
        float coef = 1.f;
        if constexpr (R == 12 || sizeof(LT) == 2) {
            const int fld = (d & 2) ? 1 : 0;
            coef = (float)ls.a[fld];
            if constexpr (R == 12) {
                const int eb = mu == 0 ? 0 : mu == 1 ? e1 : mu == 2 ? e2 : e3;
                const int neg = (ls.s[fld] < 0) ^ eb ^ (d & 1);
                coef = neg ? -coef : coef;
            }
        }
        if (!valid) coef = 0.f;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            // rows of this lane: colour ri (accumulator 0) and colour 2 (accumulator 1, lanes t < 2)
            const Cx<float> ua = ri == 0 ? u[0][c] : u[1][c];
            const Cx<float> ub = u[2][c];
            const float a0r = coef * (im ? ua.im : ua.re), a0i = coef * (im ? ua.re : -ua.im);
            const float a1r = t < 2 ? coef * (im ? ub.im : ub.re) : 0.f;
            const float a1i = t < 2 ? coef * (im ? ub.re : -ub.im) : 0.f;
            C0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a0r, vv[c].x, C0, 0, 0, 0);
            C0 = __builtin_amdgcn_mfma_f32_4x4x1f32(a0i, vv[c].y, C0, 0, 0, 0);
            C1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a1r, vv[c].x, C1, 0, 0, 0);
            C1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a1i, vv[c].y, C1, 0, 0, 0);
        }
    }
    // lane (b, t) now holds right-hand side t of site b: rows Re0 Im0 Re1 Im1
    // in C0 and Re2 Im2 in C1 (elements copied to scalars first)
    const float o0 = C0[0], o1 = C0[1], o2 = C0[2], o3 = C0[3], o4 = C1[0], o5 = C1[1];
    Cx<float> acc[3] = {{o0, o1}, {o2, o3}, {o4, o5}};
    double part = 0.0;
    if (valid && act) {
        const long long o = (long long)rhs * a.vstride + i;
        float2 *po = (float2 *)a.out + o * 3;
        if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
            for (int c = 0; c < 3; c++) po[c] = make_float2(acc[c].re, acc[c].im);
        } else {   // EPI_AX: out = diag p - D in, Re(p . out)
            const float2 *pp = (const float2 *)a.aux + o * 3;
            const float dg = (float)a.probs[rhs * a.desc_stride].diag;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const float2 pv = pp[c];
                const float vr = dg * pv.x - acc[c].re, vi = dg * pv.y - acc[c].im;
                po[c] = make_float2(vr, vi);
                part += (double)pv.x * (double)vr + (double)pv.y * (double)vi;
            }
        }
    }
    if constexpr (EPI != EPI_PLAIN) {
        // per right-hand side: sum over the wave's 16 sites (lanes t, t+4, ...),
        // then over the four waves in a fixed order
#pragma unroll
        for (int off = 4; off < 64; off <<= 1) part += __shfl_xor(part, off, 64);
        __shared__ double lds[4][4];
        if (lane < 4) lds[wave][lane] = part;
        __syncthreads();
        if (threadIdx.x < 4) {
            const int j = threadIdx.x;
            const double s = ((lds[0][j] + lds[1][j]) + lds[2][j]) + lds[3][j];
            if (r0 + j < a.nrhs) {
                const size_t idx = (size_t)(r0 + j) * pd.ntile + tile;
                if (a.red) a.red[idx] = s;
                else a.partials[idx * NPART] = s;
            }
        }
    }
}

// Four right-hand sides per link read on the matrix cores: FP32 (prec 1) or
// FP16 (prec 2) links, FP32 vectors, PLAIN and AX epilogues; nblocks = groups
// x tiles (the layout of launch_dslash_mrhs).
hipError_t launch_dslash_mrhs_mfma(int prec, int recon, const MrhsLaunch &a, int nblocks, hipStream_t s)
{
    const dim3 g(nblocks), blk(256);
#define MRM_LAUNCH(LT, R)                                                                       \
    do {                                                                                        \
        if (a.epi == EPI_PLAIN) hipLaunchKernelGGL((k_dslash_mrhs_mfma<LT, R, EPI_PLAIN>), g, blk, 0, s, a); \
        else if (a.epi == EPI_AX) hipLaunchKernelGGL((k_dslash_mrhs_mfma<LT, R, EPI_AX>), g, blk, 0, s, a); \
        else return hipErrorInvalidValue;                                                       \
        return hipGetLastError();                                                               \
    } while (0)
    if (prec == 1 && recon == 18) MRM_LAUNCH(float, 18);
    if (prec == 1 && recon == 12) MRM_LAUNCH(float, 12);
    if (prec == 2 && recon == 12) MRM_LAUNCH(__half, 12);
    if (prec == 2 && recon == 18) MRM_LAUNCH(__half, 18);
#undef MRM_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace hisq
