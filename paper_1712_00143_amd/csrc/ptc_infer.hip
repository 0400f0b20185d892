// Inference layers of the PTC preconditioner with FP16 activation storage.
//
// The same layer as k_ptc_layer (out_c(x) = sum_{c'} [w0 psi_c'(x) + sum_mu
// (w_{+mu} F_mu(x) psi_c'(x+mu) + w_{-mu} F_mu(x-mu)^+ psi_c'(x-mu))], FP16
// weights, FP32 arithmetic), for z = M(r) inside the flexible CG only, with
// the intermediate activations stored site-major and channel-interleaved in
// FP16: activation parity p, site s holds [C][3] half2 (value / scale) at
// ((p * h + s) * C) * 3, and one FP32 scale (the largest |component| of the
// site's C colour vectors) at p * h + s.  One gathered neighbour is then C*12
// contiguous bytes instead of C separate colour vectors, and the activation
// bytes of a 4-channel layer drop from 192 to 100 per site.
//
// Input kinds:  IK 0 -- the even FP32 vector r ([h][3] complex; the odd
//               parity is zero), IK 1 -- an FP16 activation.
// Output kinds: OK 0 -- an FP16 activation (parities par_lo ..),
//               OK 1 -- the even FP32 vector z = r + (layer output), with the
//               flexible CG's per-tile (q, z) sums (COUT = 1, even parity).
#include "fields.h"
#include "finish.h"
#include "launch.h"
#include "ptc.h"

namespace hisq {

namespace {

// neighbour cb index of (co, lex) along mu by +-1 (selects, not indexing, so
// that the coordinates stay in registers)
__device__ __forceinline__ int nbr1(const Coord &co, int lex, int mu, int k, const int L[4])
{
    const int x = mu == 0 ? co.x[0] : mu == 1 ? co.x[1] : mu == 2 ? co.x[2] : co.x[3];
    const int Lm = mu == 0 ? L[0] : mu == 1 ? L[1] : mu == 2 ? L[2] : L[3];
    const int Sm = mu == 0 ? 1 : mu == 1 ? L[0] : mu == 2 ? L[0] * L[1] : L[0] * L[1] * L[2];
    int v = x + k;
    v -= v >= Lm ? Lm : 0;
    v += v < 0 ? Lm : 0;
    return (lex + (v - x) * Sm) >> 1;
}

// C*3 half2 of one site (C*12 bytes, 4-byte aligned; 16-byte aligned when
// C*12 is a multiple of 16) into floats scaled by sc.
template <int C>
__device__ __forceinline__ void load_act16(const __half2 *p, float sc, float2 v[C][3])
{
    constexpr int NW = C * 3;   // 32-bit words
    uint32_t w[NW];
    if constexpr ((NW % 4) == 0) {
#pragma unroll
        for (int q = 0; q < NW / 4; q++) {
            const uint4 t = reinterpret_cast<const uint4 *>(p)[q];
            w[4 * q] = t.x;
            w[4 * q + 1] = t.y;
            w[4 * q + 2] = t.z;
            w[4 * q + 3] = t.w;
        }
    } else if constexpr ((NW % 2) == 0) {
#pragma unroll
        for (int q = 0; q < NW / 2; q++) {
            const uint2 t = reinterpret_cast<const uint2 *>(p)[q];
            w[2 * q] = t.x;
            w[2 * q + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < NW; q++) w[q] = reinterpret_cast<const uint32_t *>(p)[q];
    }
#pragma unroll
    for (int c = 0; c < C; c++)
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const float2 f = __half22float2(__builtin_bit_cast(__half2, w[c * 3 + q]));
            v[c][q] = make_float2(f.x * sc, f.y * sc);
        }
}

// The same site read without its scale (values / scale, in [-1, 1]).
template <int C>
__device__ __forceinline__ void load_act16_raw(const __half2 *p, float2 v[C][3])
{
    load_act16<C>(p, 1.f, v);
}

typedef _Float16 mf_h4 __attribute__((ext_vector_type(4)));
typedef float mf_f16 __attribute__((ext_vector_type(16)));

template <int C>
__device__ __forceinline__ void store_act16(__half2 *p, float *scale, const Cx<float> v[C][3])
{
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < C; c++)
#pragma unroll
        for (int q = 0; q < 3; q++) m = fmaxf(m, fmaxf(fabsf(v[c][q].re), fabsf(v[c][q].im)));
    const float inv = m > 0.f ? 1.f / m : 0.f;
    constexpr int NW = C * 3;
    uint32_t w[NW];
#pragma unroll
    for (int c = 0; c < C; c++)
#pragma unroll
        for (int q = 0; q < 3; q++)
            w[c * 3 + q] = __builtin_bit_cast(uint32_t, __floats2half2_rn(v[c][q].re * inv, v[c][q].im * inv));
    if constexpr ((NW % 4) == 0) {
#pragma unroll
        for (int q = 0; q < NW / 4; q++)
            reinterpret_cast<uint4 *>(p)[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    } else if constexpr ((NW % 2) == 0) {
#pragma unroll
        for (int q = 0; q < NW / 2; q++) reinterpret_cast<uint2 *>(p)[q] = make_uint2(w[2 * q], w[2 * q + 1]);
    } else {
#pragma unroll
        for (int q = 0; q < NW; q++) reinterpret_cast<uint32_t *>(p)[q] = w[q];
    }
    *scale = m;
}

}  // namespace

// Channel mixing on the matrix cores (MM): after the transports, the wave's
// contribution to its 64 sites is, per colour q, the real matrix product
//   out[(c, re|im)][site] = sum_e A[(c, re|im)][(e, re|im)] v[(e, re|im)][site]
// over the entries e = (path of this wave, input channel), A the complex
// weights in 2x2 real blocks [[w_r, -w_i], [w_i, w_r]]: a dense contraction
// whose left operand all sites share.  It runs as v_mfma_f32_32x32x8_f16 on
// two 32-site column tiles, FP16 operands, FP32 accumulation.  The B operand
// of a tile wants the first four reals of a K step from lanes 0-31 and the
// next four from lanes 32-63 of the same 32 sites; v_permlane32_swap builds
// both tiles' operands from every lane's own values, and swaps the result
// rows back to their sites.  The transported vectors of one site are
// normalised together (by the largest gathered scale, which then multiplies
// the result) so that FP16 holds them whatever the residual's magnitude.
template <class LT, int R, int CIN, int COUT, int W, int IK>
__device__ __forceinline__ void ptc_mix_mfma(const PtcInferLaunch &a, const ProbDesc &pd, const LinkSet &ls, int par,
                                             int i, bool valid, int lane, int wave, Cx<float> acc[COUT][3])
{
    using F = LinkFmt<LT, R>;
    constexpr int PPW = (9 + W - 1) / W;
    constexpr int NE = PPW * CIN, NK = (NE + 3) / 4;
    static_assert(2 * COUT <= 16, "at most 16 result rows (8 output channels)");
    const int h = pd.h;
    uint32_t vh[NK * 4][3];
#pragma unroll
    for (int e = 0; e < NK * 4; e++)
#pragma unroll
        for (int q = 0; q < 3; q++) vh[e][q] = 0u;
    float S = 0.f;
    if (valid) {
        const Coord co = cb_to_coord_pd(i, par, pd);
        const int lex = 2 * i + (co.x[0] & 1);
        RawLink<LT, R> raw[PPW];
        float2 sv[PPW][CIN][3];
        float sc[PPW];
        bool live[PPW];
#pragma unroll
        for (int g = 0; g < PPW; g++) {
            const int k = wave * PPW + g;
            live[g] = k < 9 && (IK != 0 || (k == 0 ? par == 0 : par == 1));
            sc[g] = 0.f;
            if (!live[g]) continue;
            int site = i, sp = par;
            if (k != 0) {
                const int mu = (k - 1) >> 1;
                const bool fwd = ((k - 1) & 1) == 0;
                site = nbr1(co, lex, mu, fwd ? 1 : -1, pd.L);
                sp = 1 - par;
                const int d = 4 * mu + (fwd ? 0 : 1);
                load_link_raw_wave<LT, R, 1>((const char *)ls.ptr[par] + (size_t)d * ls.hs * F::BYTES, i, ls.hs, raw[g]);
            }
            if constexpr (IK == 0) {
                const float2 *p = reinterpret_cast<const float2 *>(a.in32) + (size_t)site * 3;
                float m = 0.f;
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    sv[g][0][q] = p[q];
                    m = fmaxf(m, fmaxf(fabsf(sv[g][0][q].x), fabsf(sv[g][0][q].y)));
                }
                const float inv = m > 0.f ? 1.f / m : 0.f;
#pragma unroll
                for (int q = 0; q < 3; q++) sv[g][0][q] = make_float2(sv[g][0][q].x * inv, sv[g][0][q].y * inv);
                sc[g] = m;
            } else {
                const size_t st = (size_t)sp * h + site;
                load_act16_raw<CIN>(a.in16 + st * CIN * 3, sv[g]);
                sc[g] = a.in_scale[st];
            }
        }
#pragma unroll
        for (int g = 0; g < PPW; g++) S = fmaxf(S, sc[g]);
        const float invS = S > 0.f ? 1.f / S : 0.f;
#pragma unroll
        for (int g = 0; g < PPW; g++) {
            if (!live[g]) continue;
            const int k = wave * PPW + g;
            float f = sc[g] * invS;
            Cx<float> v[CIN][3];
            if (k == 0) {
#pragma unroll
                for (int c = 0; c < CIN; c++)
#pragma unroll
                    for (int q = 0; q < 3; q++) v[c][q] = {sv[g][c][q].x, sv[g][c][q].y};
            } else {
                const int mu = (k - 1) >> 1;
                const bool fwd = ((k - 1) & 1) == 0;
                const int d = 4 * mu + (fwd ? 0 : 1);
                Cx<float> u[3][3];
                decode_link<LT, R, float>(raw[g], u);
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
                    for (int q = 0; q < 3; q++) s3[q] = {sv[g][c][q].x, sv[g][c][q].y};
#pragma unroll
                    for (int r = 0; r < 3; r++) v[c][r] = {0.f, 0.f};
                    matvec_acc_scaled(u, s3, coef, v[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < CIN; c++)
#pragma unroll
                for (int q = 0; q < 3; q++)
                    vh[g * CIN + c][q] = __builtin_bit_cast(uint32_t, __floats2half2_rn(v[c][q].re * f, v[c][q].im * f));
        }
    }
    // A operand of each K step (the lane's row m = lane % 32, columns
    // 4 (lane / 32) .. + 3 of the step's eight reals)
    const __half2 *wt = reinterpret_cast<const __half2 *>(a.w);
    const int m = lane & 31, c_out = m >> 1, rim = m & 1;
    mf_h4 A[NK];
#pragma unroll
    for (int st = 0; st < NK; st++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int kk = 4 * (lane >> 5) + t;        // real column of the step
            const int e = 4 * st + (kk >> 1), cim = kk & 1;
            const int g = e / CIN, cp = e % CIN, path = wave * PPW + g;
            float val = 0.f;
            if (c_out < COUT && e < NE && path < 9) {
                const float2 w = __half22float2(wt[(c_out * CIN + cp) * 9 + path]);
                // [[w_r, -w_i], [w_i, w_r]]
                val = rim == 0 ? (cim == 0 ? w.x : -w.y) : (cim == 0 ? w.y : w.x);
            }
            A[st][t] = (_Float16)val;
        }
#pragma unroll
    for (int q = 0; q < 3; q++) {
        mf_f16 C0 = {}, C1 = {};
#pragma unroll
        for (int st = 0; st < NK; st++) {
            // lanes' own entries 4st, 4st+1 (X) and 4st+2, 4st+3 (Y); the swap
            // gives tile 0 (sites 0-31) and tile 1 (sites 32-63) operands
            const auto s0 = __builtin_amdgcn_permlane32_swap(vh[4 * st][q], vh[4 * st + 2][q], false, false);
            const auto s1 = __builtin_amdgcn_permlane32_swap(vh[4 * st + 1][q], vh[4 * st + 3][q], false, false);
            const uint32_t s00 = s0[0], s01 = s0[1], s10 = s1[0], s11 = s1[1];
            const uint32_t t0[2] = {s00, s10}, t1[2] = {s01, s11};
            const mf_h4 B0 = __builtin_bit_cast(mf_h4, t0), B1 = __builtin_bit_cast(mf_h4, t1);
            C0 = __builtin_amdgcn_mfma_f32_32x32x8f16(A[st], B0, C0, 0, 0, 0);
            C1 = __builtin_amdgcn_mfma_f32_32x32x8f16(A[st], B1, C1, 0, 0, 0);
        }
        // rows back to their sites: register j of the tiles holds rows
        // 8 (j / 4) + 4 (lane / 32) + j % 4
#pragma unroll
        for (int j = 0; j < (COUT > 4 ? 8 : 4); j++) {
            // (elements are copied out before any bit cast: a bit cast of a
            // vector element expression reads element 0 with this compiler)
            const float c0 = C0[j], c1 = C1[j];
            const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(c0), __float_as_uint(c1), false, false);
            const unsigned r0 = r[0], r1 = r[1];
            const int row0 = 8 * (j / 4) + (j % 4), row1 = row0 + 4;   // rows now held for the lane's own site
            const float v0 = __uint_as_float(r0) * S, v1 = __uint_as_float(r1) * S;
            if (row0 / 2 < COUT) {
                if (row0 & 1) acc[row0 / 2][q].im += v0;
                else acc[row0 / 2][q].re += v0;
            }
            if (row1 / 2 < COUT) {
                if (row1 & 1) acc[row1 / 2][q].im += v1;
                else acc[row1 / 2][q].re += v1;
            }
        }
    }
}

template <class LT, int R, int CIN, int COUT, int W, int IK, int OK, int MIX>
__global__ void __launch_bounds__(64 * W) k_ptc_infer(PtcInferLaunch a)
{
    if (a.gate && a.gate->status != a.gate_want) return;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const ProbDesc &pd = a.probs[0];
    const int ntile = pd.ntile;
    const int par = a.par_lo + blockIdx.x / ntile;
    const int tile = blockIdx.x % ntile;
    const int i = tile * TILE + lane;
    const int h = pd.h;
    const bool valid = i < h;
    const LinkSet &ls = pd.ls[a.lslot];
    using F = LinkFmt<LT, R>;
    Cx<float> acc[COUT][3];
#pragma unroll
    for (int c = 0; c < COUT; c++)
#pragma unroll
        for (int q = 0; q < 3; q++) acc[c][q] = {0.f, 0.f};
    // MIX 1: matrix-core channel mixing (a wave holds a single group of paths,
    // at least as many outputs as inputs); MIX 0: vector-ALU mixing
    constexpr bool MM = MIX == 1;
    static_assert(!MM || (W >= 3 && COUT >= CIN), "matrix-core mixing needs W >= 3 and COUT >= CIN");
    if constexpr (MM) {
        ptc_mix_mfma<LT, R, CIN, COUT, W, IK>(a, pd, ls, par, i, valid, lane, wave, acc);
    } else if (valid) {
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
                // the even input vector is zero on the odd parity: the identity
                // path reads the output parity, the hops the other one
                live[g] = k0 + g < PPW && k < 9 && (IK != 0 || (k == 0 ? par == 0 : par == 1));
                if (!live[g]) continue;
                int site = i, sp = par;
                if (k != 0) {
                    const int mu = (k - 1) >> 1;
                    const bool fwd = ((k - 1) & 1) == 0;
                    site = nbr1(co, lex, mu, fwd ? 1 : -1, pd.L);
                    sp = 1 - par;
                    const int d = 4 * mu + (fwd ? 0 : 1);
                    // the fat links are read by every layer: cached loads
                    load_link_raw_wave<LT, R, 1>((const char *)ls.ptr[par] + (size_t)d * ls.hs * F::BYTES, i, ls.hs, raw[g]);
                }
                if constexpr (IK == 0) {
                    const float2 *p = reinterpret_cast<const float2 *>(a.in32) + (size_t)site * 3;
#pragma unroll
                    for (int q = 0; q < 3; q++) sv[g][0][q] = p[q];
                } else {
                    const size_t s = (size_t)sp * h + site;
                    load_act16<CIN>(a.in16 + s * CIN * 3, a.in_scale[s], sv[g]);
                }
            }
#pragma unroll
            for (int g = 0; g < G; g++) {
                if (!live[g]) continue;
                const int k = wave * PPW + k0 + g;
                if constexpr (COUT < CIN) {
                    // fewer outputs than inputs: mix the channels first and
                    // transport COUT vectors (the transport is linear)
                    Cx<float> ph[COUT][3];
#pragma unroll
                    for (int c = 0; c < COUT; c++) {
#pragma unroll
                        for (int q = 0; q < 3; q++) ph[c][q] = {0.f, 0.f};
#pragma unroll
                        for (int cp = 0; cp < CIN; cp++) {
                            const float2 w =
                                __half22float2(reinterpret_cast<const __half2 *>(a.w)[(c * CIN + cp) * 9 + k]);
#pragma unroll
                            for (int q = 0; q < 3; q++) {
                                ph[c][q].re += w.x * sv[g][cp][q].x - w.y * sv[g][cp][q].y;
                                ph[c][q].im += w.x * sv[g][cp][q].y + w.y * sv[g][cp][q].x;
                            }
                        }
                    }
                    if (k == 0) {
#pragma unroll
                        for (int c = 0; c < COUT; c++)
#pragma unroll
                            for (int q = 0; q < 3; q++) {
                                acc[c][q].re += ph[c][q].re;
                                acc[c][q].im += ph[c][q].im;
                            }
                    } else {
                        const int mu = (k - 1) >> 1;
                        const bool fwd = ((k - 1) & 1) == 0;
                        const int d = 4 * mu + (fwd ? 0 : 1);
                        Cx<float> u[3][3];
                        decode_link<LT, R, float>(raw[g], u);
                        float coef = 1.f;
                        if constexpr (R == 12 || sizeof(LT) == 2) {
                            coef = (float)ls.a[0];
                            if constexpr (R == 12) {
                                const int eb =
                                    mu == 0 ? 0 : ((co.x[0] + (mu > 1 ? co.x[1] : 0) + (mu > 2 ? co.x[2] : 0)) & 1);
                                const int neg = (ls.s[0] < 0) ^ eb ^ (d & 1);
                                coef = neg ? -coef : coef;
                            }
                        }
                        if (!fwd) coef = -coef;   // stored -F^+
#pragma unroll
                        for (int c = 0; c < COUT; c++) matvec_acc_scaled(u, ph[c], coef, acc[c]);
                    }
                    continue;
                }
                Cx<float> v[CIN][3];
                if (k == 0) {
#pragma unroll
                    for (int c = 0; c < CIN; c++)
#pragma unroll
                        for (int q = 0; q < 3; q++) v[c][q] = {sv[g][c][q].x, sv[g][c][q].y};
                } else {
                    const int mu = (k - 1) >> 1;
                    const bool fwd = ((k - 1) & 1) == 0;
                    const int d = 4 * mu + (fwd ? 0 : 1);
                    Cx<float> u[3][3];
                    decode_link<LT, R, float>(raw[g], u);
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
                        for (int q = 0; q < 3; q++) s3[q] = {sv[g][c][q].x, sv[g][c][q].y};
#pragma unroll
                        for (int r = 0; r < 3; r++) v[c][r] = {0.f, 0.f};
                        matvec_acc_scaled(u, s3, coef, v[c]);
                    }
                }
#pragma unroll
                for (int c = 0; c < COUT; c++)
#pragma unroll
                    for (int cp = 0; cp < CIN; cp++) {
                        const float2 w = __half22float2(reinterpret_cast<const __half2 *>(a.w)[(c * CIN + cp) * 9 + k]);
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
    if (wave != 0) return;
    if constexpr (OK == 0) {
        if (valid) {
            const size_t s = (size_t)par * h + i;
            store_act16<COUT>(a.out16 + s * COUT * 3, a.out_scale + s, acc);
        }
    } else {
        // z = r + (layer output) on even sites, and the (q, z) tile sums
        double dr = 0.0, di = 0.0;
        if (valid) {
            float2 *p = reinterpret_cast<float2 *>(a.out32) + (size_t)i * 3;
            const float2 *ad = reinterpret_cast<const float2 *>(a.addin) + (size_t)i * 3;
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const float2 t = ad[q];
                acc[0][q].re += t.x;
                acc[0][q].im += t.y;
                p[q] = make_float2(acc[0][q].re, acc[0][q].im);
            }
            if (a.dotred) {
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

// ------------------------------------------------------------- launchers

namespace {

// W: waves per block (1, 3 or 9), or'ed with PTC_MFMA for the matrix-core
// channel mixing (W 3 and 9, COUT >= CIN)
template <class LT, int R, int CIN, int COUT, int IK, int OK>
hipError_t infer_w(int W, const PtcInferLaunch &a, int nblk, hipStream_t s)
{
    switch (W) {
    case 1: hipLaunchKernelGGL((k_ptc_infer<LT, R, CIN, COUT, 1, IK, OK, 0>), dim3(nblk), dim3(64), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_ptc_infer<LT, R, CIN, COUT, 3, IK, OK, 0>), dim3(nblk), dim3(192), 0, s, a); break;
    case 9: hipLaunchKernelGGL((k_ptc_infer<LT, R, CIN, COUT, 9, IK, OK, 0>), dim3(nblk), dim3(576), 0, s, a); break;
    case 3 | PTC_MFMA:
    case 9 | PTC_MFMA:
        if constexpr (COUT >= CIN) {
            if (W == (3 | PTC_MFMA))
                hipLaunchKernelGGL((k_ptc_infer<LT, R, CIN, COUT, 3, IK, OK, 1>), dim3(nblk), dim3(192), 0, s, a);
            else
                hipLaunchKernelGGL((k_ptc_infer<LT, R, CIN, COUT, 9, IK, OK, 1>), dim3(nblk), dim3(576), 0, s, a);
            break;
        } else {
            return hipErrorInvalidValue;
        }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class LT, int R>
hipError_t infer_c(int cin, int cout, int ik, int ok, int W, const PtcInferLaunch &a, int nblk, hipStream_t s)
{
    // first layer (even FP32 input, one channel), hidden layers, last adjoint
    // layer (one output channel written as the even FP32 z)
    if (ik == 0 && ok == 0) {
        if (cin != 1) return hipErrorInvalidValue;
        switch (cout) {
        case 1: return infer_w<LT, R, 1, 1, 0, 0>(W, a, nblk, s);
        case 2: return infer_w<LT, R, 1, 2, 0, 0>(W, a, nblk, s);
        case 4: return infer_w<LT, R, 1, 4, 0, 0>(W, a, nblk, s);
        case 8: return infer_w<LT, R, 1, 8, 0, 0>(W, a, nblk, s);
        }
        return hipErrorInvalidValue;
    }
    if (ik == 1 && ok == 1) {
        if (cout != 1) return hipErrorInvalidValue;
        switch (cin) {
        case 1: return infer_w<LT, R, 1, 1, 1, 1>(W, a, nblk, s);
        case 2: return infer_w<LT, R, 2, 1, 1, 1>(W, a, nblk, s);
        case 4: return infer_w<LT, R, 4, 1, 1, 1>(W, a, nblk, s);
        case 8: return infer_w<LT, R, 8, 1, 1, 1>(W, a, nblk, s);
        }
        return hipErrorInvalidValue;
    }
    if (ik == 1 && ok == 0) {
#define INF_CASE(I, O) \
    if (cin == I && cout == O) return infer_w<LT, R, I, O, 1, 0>(W, a, nblk, s);
        INF_CASE(1, 1) INF_CASE(1, 2) INF_CASE(1, 4) INF_CASE(1, 8) INF_CASE(2, 1) INF_CASE(2, 2) INF_CASE(2, 4)
        INF_CASE(4, 1) INF_CASE(4, 2) INF_CASE(4, 4) INF_CASE(8, 1) INF_CASE(8, 8)
#undef INF_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_ptc_infer(int prec, int recon, int cin, int cout, int ik, int ok, int W, const PtcInferLaunch &a,
                            int nblk, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    if (prec == 1 && recon == 18) return infer_c<float, 18>(cin, cout, ik, ok, W, a, nblk, s);
    if (prec == 2 && recon == 12) return infer_c<__half, 12>(cin, cout, ik, ok, W, a, nblk, s);
    return hipErrorInvalidValue;
}

}  // namespace hisq
