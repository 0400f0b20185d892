// Gauge-covariant parallel-transport convolution (PTC) layers of the learned
// preconditioner: forward / inference, input gradient, weight gradient, loss
// and Adam.  The network maps Cin to Cout channels of colour vectors:
//   out_c(x) = sum_{c'} [ w_{c c' 0} psi_{c'}(x)
//              + sum_mu ( w_{c c' 1+2mu} F_mu(x) psi_{c'}(x+mu)
//                       + w_{c c' 2+2mu} F_mu(x-mu)^+ psi_{c'}(x-mu) ) ]
// with the fat links F (no bias: a bias would break gauge covariance).
//
// Activations are parity-split: channel c of batch entry b is
// [2 parities][h sites][3 colours] complex FP32.  The hops reuse the packed
// fat-link directions of the Dslash operator (direction 4mu: F_mu(x);
// direction 4mu+1: -F_mu(x-mu)^+, hence the sign).  A parity known to be zero
// in the input (an even vector embedded on the full lattice) is skipped.
#include "fields.h"
#include "finish.h"
#include "launch.h"
#include "ptc.h"
#include "reduce.h"

namespace hisq {

template <class WT> __device__ __forceinline__ float2 ldw(const void *w, int idx)
{
    if constexpr (sizeof(WT) == 2) return __half22float2(reinterpret_cast<const __half2 *>(w)[idx]);
    else return reinterpret_cast<const float2 *>(w)[idx];
}

// neighbour cb index of (co, lex) along mu by +-1
__device__ __forceinline__ int nb1(const Coord &co, int lex, int mu, int k, int L0, int L1, int L2, int L3)
{
    const int x = mu == 0 ? co.x[0] : mu == 1 ? co.x[1] : mu == 2 ? co.x[2] : co.x[3];
    const int Lm = mu == 0 ? L0 : mu == 1 ? L1 : mu == 2 ? L2 : L3;
    const int Sm = mu == 0 ? 1 : mu == 1 ? L0 : mu == 2 ? L0 * L1 : L0 * L1 * L2;
    int v = x + k;
    v -= v >= Lm ? Lm : 0;
    v += v < 0 ? Lm : 0;
    return (lex + (v - x) * Sm) >> 1;
}

// Path k (0 identity, 1+2mu forward, 2+2mu backward) contributes unless the
// input parity it reads is known to be zero.  Uniform over the wavefront.
__device__ __forceinline__ bool path_live(const PtcLaunch &a, int par, int k)
{
    return k == 0 ? a.in_zero_par != par : a.in_zero_par != 1 - par;
}

// The loads of path k at output site (par, i): the input colour vectors of
// CIN channels at the site (identity) or at its neighbour, and the packed
// link.  k and par must be uniform over the wavefront (the link block is
// addressed through a wave-uniform buffer resource).
template <class LT, int R, int CIN>
__device__ __forceinline__ void path_load(const ProbDesc &pd, const LinkSet &ls, int par, int i, const Coord &co,
                                          int lex, int k, const float *in_b, RawLink<LT, R> &raw, float2 sv[CIN][3])
{
    const long long h = pd.h;
    int site = i, sp = par;
    if (k != 0) {
        const int mu = (k - 1) >> 1;
        const bool fwd = ((k - 1) & 1) == 0;
        site = nb1(co, lex, mu, fwd ? 1 : -1, pd.L[0], pd.L[1], pd.L[2], pd.L[3]);
        sp = 1 - par;
        using F = LinkFmt<LT, R>;
        const int d = 4 * mu + (fwd ? 0 : 1);
        // the fat links are re-read by every layer of every application: keep
        // them cached (temporal loads)
        load_link_raw_wave<LT, R, 1>((const char *)ls.ptr[par] + (size_t)d * ls.hs * F::BYTES, i, ls.hs, raw);
    }
#pragma unroll
    for (int c = 0; c < CIN; c++) {
        const float2 *p = reinterpret_cast<const float2 *>(in_b) + ((c * 2 + sp) * h + site) * 3;
#pragma unroll
        for (int q = 0; q < 3; q++) sv[c][q] = p[q];
    }
}

// The transported colour vectors v[c] of path k from what path_load fetched.
template <class LT, int R, int CIN>
__device__ __forceinline__ void path_apply(const LinkSet &ls, const Coord &co, int k, const RawLink<LT, R> &raw,
                                           const float2 sv[CIN][3], Cx<float> v[CIN][3])
{
    if (k == 0) {
#pragma unroll
        for (int c = 0; c < CIN; c++)
#pragma unroll
            for (int q = 0; q < 3; q++) v[c][q] = {sv[c][q].x, sv[c][q].y};
        return;
    }
    const int mu = (k - 1) >> 1;
    const bool fwd = ((k - 1) & 1) == 0;
    const int d = 4 * mu + (fwd ? 0 : 1);
    Cx<float> u[3][3];
    decode_link<LT, R, float>(raw, u);
    float coef = 1.f;
    if constexpr (R == 12 || sizeof(LT) == 2) {
        coef = (float)ls.a[0];
        if constexpr (R == 12) {
            const int eb = mu == 0 ? 0 : ((co.x[0] + (mu > 1 ? co.x[1] : 0) + (mu > 2 ? co.x[2] : 0)) & 1);
            const int neg = (ls.s[0] < 0) ^ eb ^ (d & 1);
            coef = neg ? -coef : coef;
        }
    }
    if (!fwd) coef = -coef;   // stored -F^+
#pragma unroll
    for (int c = 0; c < CIN; c++) {
        Cx<float> s3[3];
#pragma unroll
        for (int q = 0; q < 3; q++) s3[q] = {sv[c][q].x, sv[c][q].y};
#pragma unroll
        for (int r = 0; r < 3; r++) v[c][r] = {0.f, 0.f};
        matvec_acc_scaled(u, s3, coef, v[c]);
    }
}

// Forward layer (also the input-gradient layer, given the adjoint weights).
template <class LT, int R, class WT, int CIN, int COUT, int W>
__global__ void __launch_bounds__(64 * W) k_ptc_layer(PtcLaunch a)
{
    if (a.gate && a.gate->status != a.gate_want) return;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const ProbDesc &pd = a.probs[0];
    const int ntile = pd.ntile;
    const int par = a.par_lo + blockIdx.x / ntile;
    const int tile = blockIdx.x % ntile;
    const int b = blockIdx.y;
    const int i = tile * TILE + lane;
    const bool valid = i < pd.h;
    const LinkSet &ls = pd.ls[a.lslot];
    const float *in_b = a.in + (size_t)b * a.in_bstride;
    Cx<float> acc[COUT][3];
#pragma unroll
    for (int c = 0; c < COUT; c++)
#pragma unroll
        for (int q = 0; q < 3; q++) acc[c][q] = {0.f, 0.f};
    if (valid) {
        const Coord co = cb_to_coord_pd(i, par, pd);
        const int lex = 2 * i + (co.x[0] & 1);
        constexpr int PPW = (9 + W - 1) / W;   // paths of this wave
        constexpr int G = PPW < 3 ? PPW : 3;    // paths whose loads are in flight together
#pragma unroll
        for (int k0 = 0; k0 < PPW; k0 += G) {
            RawLink<LT, R> raw[G];
            float2 sv[G][CIN][3];
            bool live[G];
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int k = wave * PPW + k0 + g;
                live[g] = k0 + g < PPW && k < 9 && path_live(a, par, k);
                if (live[g]) path_load<LT, R, CIN>(pd, ls, par, i, co, lex, k, in_b, raw[g], sv[g]);
            }
#pragma unroll
            for (int g = 0; g < G; g++) {
                if (!live[g]) continue;
                const int k = wave * PPW + k0 + g;
                Cx<float> v[CIN][3];
                path_apply<LT, R, CIN>(ls, co, k, raw[g], sv[g], v);
#pragma unroll
                for (int c = 0; c < COUT; c++)
#pragma unroll
                    for (int cp = 0; cp < CIN; cp++) {
                        const float2 w = ldw<WT>(a.w, (c * CIN + cp) * 9 + k);
#pragma unroll
                        for (int q = 0; q < 3; q++) {
                            acc[c][q].re += w.x * v[cp][q].re - w.y * v[cp][q].im;
                            acc[c][q].im += w.x * v[cp][q].im + w.y * v[cp][q].re;
                        }
                    }
            }
        }
    }
    if constexpr (W > 1) {
        __shared__ float red[(W - 1) * COUT * 6 * 64];
        if (wave > 0)
#pragma unroll
            for (int c = 0; c < COUT; c++)
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    red[(((wave - 1) * COUT + c) * 6 + 2 * q) * 64 + lane] = acc[c][q].re;
                    red[(((wave - 1) * COUT + c) * 6 + 2 * q + 1) * 64 + lane] = acc[c][q].im;
                }
        __syncthreads();
        if (wave == 0)
            for (int w = 1; w < W; w++)
#pragma unroll
                for (int c = 0; c < COUT; c++)
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        acc[c][q].re += red[(((w - 1) * COUT + c) * 6 + 2 * q) * 64 + lane];
                        acc[c][q].im += red[(((w - 1) * COUT + c) * 6 + 2 * q + 1) * 64 + lane];
                    }
    }
    if (wave == 0) {
        double dr = 0.0, di = 0.0;
        if (valid) {
            float *out_b = a.out + (size_t)b * a.out_bstride;
            const long long h = pd.h;
#pragma unroll
            for (int c = 0; c < COUT; c++) {
                const long long o = ((c * a.out_pstride + (par - a.out_par0)) * h + i) * 3;
                float2 *p = reinterpret_cast<float2 *>(out_b) + o;
                if (a.addin) {   // the identity term of M, added in the same rounding as a separate pass
                    const float2 *ad = reinterpret_cast<const float2 *>(a.addin + (size_t)b * a.addin_bstride) + o;
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        const float2 t = ad[q];
                        acc[c][q].re += t.x;
                        acc[c][q].im += t.y;
                    }
                }
#pragma unroll
                for (int q = 0; q < 3; q++) p[q] = make_float2(acc[c][q].re, acc[c][q].im);
            }
            if (a.dotred) {   // (q, out) = sum conj(q) out over this tile (COUT = 1)
                const float2 *qv = reinterpret_cast<const float2 *>(a.dotq) + (size_t)i * 3;
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    const float2 t = qv[q];
                    dr += (double)t.x * acc[0][q].re + (double)t.y * acc[0][q].im;
                    di += (double)t.x * acc[0][q].im - (double)t.y * acc[0][q].re;
                }
            }
        }
        if (a.dotred) {   // wave 0 covers the whole 64-site tile
            dr = wave_sum(dr);
            di = wave_sum(di);
            if (lane == 0) {
                a.dotred[tile] = dr;
                a.dotred[a.dot_nt + tile] = di;
            }
        }
    }
}

// Weight gradient: sums of (T_k in_{c'})(x)^+ g_c(x) over sites and batch
// entries, one wavefront per path k.  Block j walks the work units (batch
// entry, output parity, tile) j, j + grid, j + 2 grid, ... accumulating in FP64
// per lane, and reduces once at the end: partials [block][9][COUT][CIN]
// complex FP64, in a fixed order for a given grid.
template <class LT, int R, int CIN, int COUT>
__global__ void __launch_bounds__(576) k_ptc_wgrad(PtcLaunch a, int npar, int batch)
{
    const int lane = threadIdx.x & 63, k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const ProbDesc &pd = a.probs[0];
    const int ntile = pd.ntile;
    const long long h = pd.h;
    const LinkSet &ls = pd.ls[a.lslot];
    const long long nunit = (long long)batch * npar * ntile;
    double acc[COUT][CIN][2];
#pragma unroll
    for (int c = 0; c < COUT; c++)
#pragma unroll
        for (int cp = 0; cp < CIN; cp++) acc[c][cp][0] = acc[c][cp][1] = 0.0;
    for (long long u = blockIdx.x; u < nunit; u += gridDim.x) {
        const int b = (int)(u / (npar * ntile));
        const int rem = (int)(u - (long long)b * npar * ntile);
        const int par = a.par_lo + rem / ntile;
        const int tile = rem % ntile;
        const int i = tile * TILE + lane;
        if (i >= pd.h) continue;
        const float *in_b = a.in + (size_t)b * a.in_bstride;
        const float *g_b = a.g + (size_t)b * a.g_bstride;
        const Coord co = cb_to_coord_pd(i, par, pd);
        const int lex = 2 * i + (co.x[0] & 1);
        if (!path_live(a, par, k)) continue;
        RawLink<LT, R> raw;
        float2 sv[CIN][3];
        path_load<LT, R, CIN>(pd, ls, par, i, co, lex, k, in_b, raw, sv);
        Cx<float> v[CIN][3];
        path_apply<LT, R, CIN>(ls, co, k, raw, sv, v);
#pragma unroll
        for (int c = 0; c < COUT; c++) {
            const float2 *gp = reinterpret_cast<const float2 *>(g_b) + ((c * a.g_pstride + (par - a.g_par0)) * h + i) * 3;
            const float2 g[3] = {gp[0], gp[1], gp[2]};
#pragma unroll
            for (int cp = 0; cp < CIN; cp++) {
                float re = 0.f, im = 0.f;
#pragma unroll
                for (int q = 0; q < 3; q++) {   // conj(v) g
                    re = fmaa(v[cp][q].re, g[q].x, re);
                    re = fmaa(v[cp][q].im, g[q].y, re);
                    im = fmaa(v[cp][q].re, g[q].y, im);
                    im = fmaa(-v[cp][q].im, g[q].x, im);
                }
                acc[c][cp][0] += re;
                acc[c][cp][1] += im;
            }
        }
    }
    double *out = a.partials + ((size_t)blockIdx.x * 9 + k) * (COUT * CIN * 2);
#pragma unroll
    for (int c = 0; c < COUT; c++)
#pragma unroll
        for (int cp = 0; cp < CIN; cp++) {
            const double re = wave_sum(acc[c][cp][0]), im = wave_sum(acc[c][cp][1]);
            if (lane == 0) {
                out[(c * CIN + cp) * 2] = re;
                out[(c * CIN + cp) * 2 + 1] = im;
            }
        }
}

// g_w[c][c'][k] = sum over the partial rows: one block per value, each thread
// summing rows t, t + 256, ... in order, then a fixed-order block sum, so the
// result does not depend on scheduling.
__global__ void __launch_bounds__(256) k_ptc_wsum(const double *partials, long long nrow, int cin, int cout,
                                                  double *gw, int accumulate)
{
    __shared__ double lds[16];
    const int v = blockIdx.x;   // value index in [9][cout][cin][2]
    const int nv = 9 * cout * cin * 2;
    double s[1] = {0.0};
    for (long long r = threadIdx.x; r < nrow; r += blockDim.x) s[0] += partials[r * nv + v];
    block_sum<1>(s, lds);
    if (threadIdx.x == 0) {
        const int ri = v & 1, q = v >> 1;
        const int k = q / (cout * cin), c = (q / cin) % cout, cp = q % cin;
        const int o = ((c * cin + cp) * 9 + k) * 2 + ri;
        gw[o] = accumulate ? gw[o] + s[0] : s[0];
    }
}

// Loss of a batch of B pairs (z_b = M r_b, e_b the target):
//   L = 1 - |S|^2 / (B Q),  S = sum_b <z_b, e_b> / |e_b|^2,  Q = sum_b |z_b|^2 / |e_b|^2,
// the normalised least-squares misfit of z_b ~ c e_b with one common c (M A
// close to a multiple of 1 on the error directions), invariant to the scale
// of M.  Passes: per-tile partials of (Re, Im <z, e>, |z|^2); per-pair totals;
// S, Q and L; the gradient g_b = -2 (conj(S) e_b Q - |S|^2 z_b) / (B Q^2 |e_b|^2)
// on even sites.
// The vector the loss measures z against: z itself (Euclidean), or A z =
// wdiag z - D_eo D_oe z (energy norm), element f of batch entry b.
__device__ __forceinline__ float2 weighted(const PtcLaunch &a, int b, long long f, float2 z)
{
    if (!a.wvec) return z;
    const float2 u = reinterpret_cast<const float2 *>(a.wvec + (size_t)b * a.in_bstride)[f];
    const float dg = (float)a.wdiag;
    return make_float2(dg * z.x - u.x, dg * z.y - u.y);
}

__global__ void __launch_bounds__(192) k_ptc_loss_dots(PtcLaunch a)
{
    const ProbDesc &pd = a.probs[0];
    const int tile = blockIdx.x, b = blockIdx.y;
    const long long f = (long long)tile * TILE * 3 + threadIdx.x;
    double part[3] = {0.0, 0.0, 0.0};
    if (f < (long long)pd.h * 3) {
        const float2 z = reinterpret_cast<const float2 *>(a.in + (size_t)b * a.in_bstride)[f];
        const float2 t = reinterpret_cast<const float2 *>(a.tgt + (size_t)b * a.tgt_bstride)[f];
        const float2 zw = weighted(a, b, f, z);
        part[0] = (double)z.x * t.x + (double)z.y * t.y;
        part[1] = (double)z.x * t.y - (double)z.y * t.x;
        part[2] = (double)z.x * zw.x + (double)z.y * zw.y;
    }
    publish_partials<3>(part, a.partials, b * gridDim.x + tile);
}

__global__ void __launch_bounds__(256) k_ptc_loss_fin(const double *partials, int ntile, double *pstat)
{
    __shared__ double lds[16 * 3];
    const int b = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < ntile; j += blockDim.x) {
        const double *p = partials + ((size_t)b * ntile + j) * NPART;
        acc[0] += p[0];
        acc[1] += p[1];
        acc[2] += p[2];
    }
    block_sum<3>(acc, lds);
    if (threadIdx.x == 0) {
        pstat[4 * b + 0] = acc[0];
        pstat[4 * b + 1] = acc[1];
        pstat[4 * b + 2] = acc[2];
    }
}

// one thread: S, Q, L over the batch (fixed order); S, Q, L kept after the pairs
__global__ void k_ptc_lsum(double *pstat, const double *ee, int npair, double *loss)
{
    if (threadIdx.x != 0) return;
    double sr = 0, si = 0, q = 0;
    for (int b = 0; b < npair; b++) {
        sr += pstat[4 * b] / ee[b];
        si += pstat[4 * b + 1] / ee[b];
        q += pstat[4 * b + 2] / ee[b];
    }
    const double l = 1.0 - (sr * sr + si * si) / (npair * q);
    pstat[4 * npair + 0] = sr;
    pstat[4 * npair + 1] = si;
    pstat[4 * npair + 2] = q;
    *loss = l;
}

__global__ void __launch_bounds__(192) k_ptc_loss_grad(PtcLaunch a, const double *pstat)
{
    const ProbDesc &pd = a.probs[0];
    const int tile = blockIdx.x, b = blockIdx.y, B = gridDim.y;
    const long long f = (long long)tile * TILE * 3 + threadIdx.x;
    if (f >= (long long)pd.h * 3) return;
    const double sr = pstat[4 * B], si = pstat[4 * B + 1], q = pstat[4 * B + 2];
    const double den = (double)B * q * q * a.ee[b];
    // g = Ac t + Bc z_w,  Ac = -2 conj(S) Q / den,  Bc = 2 |S|^2 / den (t the
    // target: e, or r for the energy norm; z_w = z, or A z)
    const float ar = (float)(-2.0 * sr * q / den), ai = (float)(2.0 * si * q / den);
    const float bc = (float)(2.0 * (sr * sr + si * si) / den);
    const float2 z = reinterpret_cast<const float2 *>(a.in + (size_t)b * a.in_bstride)[f];
    const float2 t = reinterpret_cast<const float2 *>(a.tgt + (size_t)b * a.tgt_bstride)[f];
    const float2 zw = weighted(a, b, f, z);
    reinterpret_cast<float2 *>(a.out + (size_t)b * a.out_bstride)[f] =
        make_float2(ar * t.x - ai * t.y + bc * zw.x, ar * t.y + ai * t.x + bc * zw.y);
}

// Adam on the FP32 master weights (complex weights as (re, im) pairs);
// refreshes the FP32 and FP16 working copies.
__global__ void k_adam(float *w, float *m, float *v, const double *g, int n, int step, float lr, float b1,
                       float b2, float eps, __half *w16)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = (float)g[j];
    const float mj = b1 * m[j] + (1.f - b1) * gj;
    const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    const float mh = mj / (1.f - powf(b1, (float)step));
    const float vh = vj / (1.f - powf(b2, (float)step));
    const float wj = w[j] - lr * mh / (sqrtf(vh) + eps);
    w[j] = wj;
    w16[j] = __float2half_rn(wj);
}

// ------------------------------------------------------------- launchers

template <class LT, int R, class WT, int CIN, int COUT>
static hipError_t layer_w(int W, const PtcLaunch &a, dim3 g, hipStream_t s)
{
    switch (W) {
    case 1: hipLaunchKernelGGL((k_ptc_layer<LT, R, WT, CIN, COUT, 1>), g, dim3(64), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_ptc_layer<LT, R, WT, CIN, COUT, 3>), g, dim3(192), 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_ptc_layer<LT, R, WT, CIN, COUT, 5>), g, dim3(320), 0, s, a); break;
    case 9: hipLaunchKernelGGL((k_ptc_layer<LT, R, WT, CIN, COUT, 9>), g, dim3(576), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LT, int R, class WT>
static hipError_t layer_c(int cin, int cout, int W, const PtcLaunch &a, dim3 g, hipStream_t s)
{
#define PTC_CASE(I, O) \
    if (cin == I && cout == O) return layer_w<LT, R, WT, I, O>(W, a, g, s);
    PTC_CASE(1, 1) PTC_CASE(1, 4) PTC_CASE(4, 4) PTC_CASE(4, 1) PTC_CASE(1, 2) PTC_CASE(2, 2) PTC_CASE(2, 1)
    PTC_CASE(2, 4) PTC_CASE(4, 2) PTC_CASE(1, 8) PTC_CASE(8, 8) PTC_CASE(8, 1)
#undef PTC_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_ptc_layer(int prec, int recon, bool w16, int cin, int cout, int W, const PtcLaunch &a, int nblk,
                            int batch, hipStream_t s)
{
    dim3 g(nblk, batch);
    if (prec == 1 && recon == 18)
        return w16 ? layer_c<float, 18, __half>(cin, cout, W, a, g, s) : layer_c<float, 18, float>(cin, cout, W, a, g, s);
    if (prec == 2 && recon == 12)
        return w16 ? layer_c<__half, 12, __half>(cin, cout, W, a, g, s) : layer_c<__half, 12, float>(cin, cout, W, a, g, s);
    return hipErrorInvalidValue;
}

template <class LT, int R>
static hipError_t wgrad_c(int cin, int cout, const PtcLaunch &a, int npar, int batch, dim3 g, hipStream_t s)
{
    const dim3 b(576);
#define WG_CASE(I, O) \
    if (cin == I && cout == O) { hipLaunchKernelGGL((k_ptc_wgrad<LT, R, I, O>), g, b, 0, s, a, npar, batch); return hipGetLastError(); }
    WG_CASE(1, 1) WG_CASE(1, 4) WG_CASE(4, 4) WG_CASE(4, 1) WG_CASE(1, 2) WG_CASE(2, 2) WG_CASE(2, 1)
    WG_CASE(2, 4) WG_CASE(4, 2) WG_CASE(1, 8) WG_CASE(8, 8) WG_CASE(8, 1)
#undef WG_CASE
    return hipErrorInvalidValue;
}

// transports on FP32 recon-18 (prec 1) or FP16 recon-12 (prec 2) fat links
hipError_t launch_ptc_wgrad(int prec, int recon, int cin, int cout, const PtcLaunch &a, int npar, int batch, int nrow,
                            hipStream_t s)
{
    const dim3 g(nrow);
    if (prec == 1 && recon == 18) return wgrad_c<float, 18>(cin, cout, a, npar, batch, g, s);
    if (prec == 2 && recon == 12) return wgrad_c<__half, 12>(cin, cout, a, npar, batch, g, s);
    return hipErrorInvalidValue;
}

hipError_t launch_ptc_wsum(const double *partials, long long nrow, int cin, int cout, double *gw, int accumulate,
                           hipStream_t s)
{
    const int nv = 9 * cout * cin * 2;
    hipLaunchKernelGGL(k_ptc_wsum, dim3(nv), dim3(256), 0, s, partials, nrow, cin, cout, gw, accumulate);
    return hipGetLastError();
}

hipError_t launch_ptc_loss(const PtcLaunch &a, int ntile, int batch, double *loss, hipStream_t s)
{
    double *pstat = a.partials + (size_t)batch * ntile * NPART;
    hipLaunchKernelGGL(k_ptc_loss_dots, dim3(ntile, batch), dim3(192), 0, s, a);
    hipLaunchKernelGGL(k_ptc_loss_fin, dim3(batch), dim3(256), 0, s, a.partials, ntile, pstat);
    hipLaunchKernelGGL(k_ptc_lsum, dim3(1), dim3(64), 0, s, pstat, a.ee, batch, loss);
    hipLaunchKernelGGL(k_ptc_loss_grad, dim3(ntile, batch), dim3(192), 0, s, a, (const double *)pstat);
    return hipGetLastError();
}

hipError_t launch_adam(float *w, float *m, float *v, const double *g, int n, int step, float lr, __half *w16,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, m, v, g, n, step, lr, 0.9f, 0.999f,
                       1e-8f, w16);
    return hipGetLastError();
}

}  // namespace hisq
