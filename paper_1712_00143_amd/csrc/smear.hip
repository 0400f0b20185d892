// HISQ link smearing kernels (FP64): staple passes, the U(3) projection and
// the final fat / Naik links with the staggered phases.
//
// The smearing (the link construction of the HISQ action, Follana et al.,
// hep-lat/0610092; the paper's run-time breakdown in Section 2 lists it
// beside the two forces) is a sum of path products of 3x3 matrices.  The
// 5- and 7-link staples are staples of staples, so one kernel, the staple of
// a field M through one direction, builds all of them: the host walks
// nu -> rho -> sigma and every pass reads the previous pass's output (see
// smear.cpp).  Each pass touches a handful of planar fields once, so it is
// bound by HBM traffic (about 1.1 flop per byte), not by the FP64 units.
#include "hisq_dev.h"
#include "smear.h"

namespace hisq {

namespace {

struct M3 {
    double2 e[9];
};

__device__ __forceinline__ M3 ld(const double2 *__restrict__ f, size_t V, long long s)
{
    M3 m;
#pragma unroll
    for (int i = 0; i < 9; i++) m.e[i] = f[i * V + s];
    return m;
}

__device__ __forceinline__ void st(double2 *__restrict__ f, size_t V, long long s, const M3 &m)
{
#pragma unroll
    for (int i = 0; i < 9; i++) f[i * V + s] = m.e[i];
}

// c = a b
__device__ __forceinline__ M3 mul_nn(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double2 x = a.e[3 * i + k], y = b.e[3 * k + j];
                re = __builtin_fma(x.x, y.x, re);
                re = __builtin_fma(-x.y, y.y, re);
                im = __builtin_fma(x.x, y.y, im);
                im = __builtin_fma(x.y, y.x, im);
            }
            c.e[3 * i + j] = make_double2(re, im);
        }
    return c;
}

// c = a b^+
__device__ __forceinline__ M3 mul_na(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double2 x = a.e[3 * i + k], y = b.e[3 * j + k];
                re = __builtin_fma(x.x, y.x, re);
                re = __builtin_fma(x.y, y.y, re);
                im = __builtin_fma(x.y, y.x, im);
                im = __builtin_fma(-x.x, y.y, im);
            }
            c.e[3 * i + j] = make_double2(re, im);
        }
    return c;
}

// c = a^+ b
__device__ __forceinline__ M3 mul_an(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double2 x = a.e[3 * k + i], y = b.e[3 * k + j];
                re = __builtin_fma(x.x, y.x, re);
                re = __builtin_fma(x.y, y.y, re);
                im = __builtin_fma(x.x, y.y, im);
                im = __builtin_fma(-x.y, y.x, im);
            }
            c.e[3 * i + j] = make_double2(re, im);
        }
    return c;
}

// acc += c m
__device__ __forceinline__ void axpy(M3 &acc, double c, const M3 &m)
{
#pragma unroll
    for (int i = 0; i < 9; i++)
        acc.e[i] = make_double2(__builtin_fma(c, m.e[i].x, acc.e[i].x), __builtin_fma(c, m.e[i].y, acc.e[i].y));
}

__device__ __forceinline__ int wrap(int v, int L)
{
    v -= v >= L ? L : 0;
    v -= v >= L ? L : 0;
    v += v < 0 ? L : 0;
    v += v < 0 ? L : 0;
    return v;
}

// site x + k * dir, for x's coordinate xd along dir (|k| <= 2 L)
__device__ __forceinline__ long long shift(long long s, int xd, int S, int L, int k)
{
    return s + (long long)(wrap(xd + k, L) - xd) * S;
}

__device__ __forceinline__ int pick(const int v[4], int d)
{
    return d == 0 ? v[0] : d == 1 ? v[1] : d == 2 ? v[2] : v[3];
}

template <bool LEP, bool WT>
__global__ void __launch_bounds__(256) k_smear_staple(SmearGeom g, StapleArgs a)
{
    const long long s = (long long)xcd_tile(blockIdx.x, gridDim.x, 1) * 256 + threadIdx.x;
    if (s >= g.V) return;
    const size_t V = (size_t)g.V;
    const int Sm = pick(g.S, a.mu), Lm = pick(g.L, a.mu), Sn = pick(g.S, a.nu), Ln = pick(g.L, a.nu);
    const unsigned su = (unsigned)s;   // V <= 2^31
    const int xm = (int)((su / (unsigned)Sm) % (unsigned)Lm), xn = (int)((su / (unsigned)Sn) % (unsigned)Ln);
    const long long pn = shift(s, xn, Sn, Ln, 1), mn = shift(s, xn, Sn, Ln, -1);
    const long long pm = shift(s, xm, Sm, Lm, 1), mn_pm = shift(mn, xm, Sm, Lm, 1);
    M3 T;
    {
        const M3 P = mul_nn(ld(a.Un, V, s), ld(a.M, V, pn));
        T = mul_na(P, ld(a.Un, V, pm));
    }
    {
        const M3 P = mul_an(ld(a.Un, V, mn), ld(a.M, V, mn));
        const M3 Q = mul_nn(P, ld(a.Un, V, mn_pm));
#pragma unroll
        for (int i = 0; i < 9; i++) T.e[i] = make_double2(T.e[i].x + Q.e[i].x, T.e[i].y + Q.e[i].y);
    }
    M3 F;
    if (a.init) {
        F = ld(a.M, V, s);
#pragma unroll
        for (int i = 0; i < 9; i++) F.e[i] = make_double2(a.cM * F.e[i].x, a.cM * F.e[i].y);
    } else {
        F = ld(a.F, V, s);
    }
    axpy(F, a.cT, T);
    if constexpr (LEP) {
        // two steps out along nu, across mu, two steps back
        const long long p2n = shift(s, xn, Sn, Ln, 2), m2n = shift(s, xn, Sn, Ln, -2);
        const long long pn_pm = shift(pn, xm, Sm, Lm, 1), m2n_pm = shift(m2n, xm, Sm, Lm, 1);
        {
            M3 P = mul_nn(ld(a.Un, V, s), ld(a.Un, V, pn));
            P = mul_nn(P, ld(a.M, V, p2n));
            P = mul_na(P, ld(a.Un, V, pn_pm));
            P = mul_na(P, ld(a.Un, V, pm));
            axpy(F, a.cL, P);
        }
        {
            M3 P = mul_nn(ld(a.Un, V, m2n), ld(a.Un, V, mn));
            P = mul_an(P, ld(a.M, V, m2n));
            P = mul_nn(P, ld(a.Un, V, m2n_pm));
            P = mul_nn(P, ld(a.Un, V, mn_pm));
            axpy(F, a.cL, P);
        }
    }
    st(a.F, V, s, F);
    if constexpr (WT) st(a.T_out, V, s, T);
}

// Blocks of 64 sites x 4 directions; the [64][4][9] slab of the site-major
// array is staged in LDS so that both sides move contiguous segments.
constexpr int SB = 64;

__global__ void __launch_bounds__(256) k_smear_to_planar(SmearGeom g, const double2 *__restrict__ aos,
                                                         double2 *__restrict__ pl)
{
    __shared__ double2 buf[SB * 36];
    const long long s0 = (long long)blockIdx.x * SB;
    const int n = (int)((g.V - s0 < SB ? g.V - s0 : SB) * 36);
    for (int i = threadIdx.x; i < n; i += 256) buf[i] = aos[s0 * 36 + i];
    __syncthreads();
    const int sl = threadIdx.x & (SB - 1), d = threadIdx.x >> 6;
    const long long s = s0 + sl;
    if (s >= g.V) return;
    const size_t V = (size_t)g.V;
    double2 *f = pl + (size_t)d * 9 * V;
#pragma unroll
    for (int e = 0; e < 9; e++) f[e * V + s] = buf[(sl * 4 + d) * 9 + e];
}

template <int MODE>   // 0: plain conversion of X; 1: fat and Naik links with phases
__global__ void __launch_bounds__(256) k_smear_out(SmearGeom g, const double2 *__restrict__ X,
                                                   const double2 *__restrict__ W, double cN,
                                                   double2 *__restrict__ out0, double2 *__restrict__ out1)
{
    __shared__ double2 buf[SB * 36];
    const long long s0 = (long long)blockIdx.x * SB;
    const int n = (int)((g.V - s0 < SB ? g.V - s0 : SB) * 36);
    const int sl = threadIdx.x & (SB - 1), d = threadIdx.x >> 6;
    const long long s = s0 + sl;
    const bool valid = s < g.V;
    const size_t V = (size_t)g.V;
    const unsigned sc = valid ? (unsigned)s : 0u;
    const int x0 = (int)(sc % (unsigned)g.L[0]), x1 = (int)((sc / (unsigned)g.S[1]) % (unsigned)g.L[1]);
    const int x2 = (int)((sc / (unsigned)g.S[2]) % (unsigned)g.L[2]), x3 = (int)(sc / (unsigned)g.S[3]);
    const int ph = d == 0 ? 0 : d == 1 ? x0 : d == 2 ? x0 + x1 : x0 + x1 + x2;
    const double eta = (MODE == 1 && (ph & 1)) ? -1.0 : 1.0;
    if (valid) {
        const M3 m = ld(X + (size_t)d * 9 * V, V, s);
#pragma unroll
        for (int e = 0; e < 9; e++) buf[(sl * 4 + d) * 9 + e] = make_double2(eta * m.e[e].x, eta * m.e[e].y);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) out0[s0 * 36 + i] = buf[i];
    if constexpr (MODE == 1) {
        __syncthreads();
        if (valid) {
            const int xd = d == 0 ? x0 : d == 1 ? x1 : d == 2 ? x2 : x3;
            const int Sd = pick(g.S, d), Ld = pick(g.L, d);
            const double2 *w = W + (size_t)d * 9 * V;
            M3 P = mul_nn(ld(w, V, s), ld(w, V, shift(s, xd, Sd, Ld, 1)));
            P = mul_nn(P, ld(w, V, shift(s, xd, Sd, Ld, 2)));
            const double k = cN * eta;
#pragma unroll
            for (int e = 0; e < 9; e++) buf[(sl * 4 + d) * 9 + e] = make_double2(k * P.e[e].x, k * P.e[e].y);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += 256) out1[s0 * 36 + i] = buf[i];
    }
}

// W = V (V^+ V)^{-1/2}.  Q = V^+ V is Hermitian positive definite; its
// eigenvalues g_k come from the trigonometric solution of the characteristic
// cubic, and Q^{-1/2} = f0 + f1 Q + f2 Q^2 (Cayley-Hamilton) with the f's
// symmetric functions of sqrt(g_k) (u = sum, v = sum of pairwise products,
// w = product), which stay finite when eigenvalues coincide.
__global__ void __launch_bounds__(256) k_smear_unitarize(SmearGeom g, double2 *__restrict__ pl, int *bad)
{
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= g.V) return;
    const size_t V = (size_t)g.V;
    const int d = blockIdx.y;
    double2 *f = pl + (size_t)d * 9 * V;
    const M3 Vm = ld(f, V, s);
    const M3 Q = mul_an(Vm, Vm);
    const double c0 = (Q.e[0].x + Q.e[4].x + Q.e[8].x) * (1.0 / 3.0);
    const double a0 = Q.e[0].x - c0, a1 = Q.e[4].x - c0, a2 = Q.e[8].x - c0;
    const double2 q01 = Q.e[1], q02 = Q.e[2], q12 = Q.e[5];
    const double n01 = q01.x * q01.x + q01.y * q01.y, n02 = q02.x * q02.x + q02.y * q02.y;
    const double n12 = q12.x * q12.x + q12.y * q12.y;
    const double p = (a0 * a0 + a1 * a1 + a2 * a2 + 2.0 * (n01 + n02 + n12)) * (1.0 / 6.0);
    // det of the traceless Hermitian part: real, 2 Re(q01 q12 conj(q02)) enters once
    const double re3 = (q01.x * q12.x - q01.y * q12.y) * q02.x + (q01.x * q12.y + q01.y * q12.x) * q02.y;
    const double det = a0 * a1 * a2 + 2.0 * re3 - a0 * n12 - a1 * n02 - a2 * n01;
    double g0 = c0, g1 = c0, g2 = c0;
    if (p > 1e-28 * c0 * c0) {
        const double sp = sqrt(p);
        double r = 0.5 * det / (p * sp);
        r = r > 1.0 ? 1.0 : (r < -1.0 ? -1.0 : r);
        const double th = acos(r) * (1.0 / 3.0);
        const double tp = 2.0943951023931954923;   // 2 pi / 3
        g0 = c0 + 2.0 * sp * cos(th);
        g1 = c0 + 2.0 * sp * cos(th + tp);
        g2 = c0 + 2.0 * sp * cos(th - tp);
    }
    bool ok = g0 > 0.0 && g1 > 0.0 && g2 > 0.0;
    const double r0 = sqrt(ok ? g0 : 1.0), r1 = sqrt(ok ? g1 : 1.0), r2 = sqrt(ok ? g2 : 1.0);
    const double u = r0 + r1 + r2, v = r0 * r1 + r0 * r2 + r1 * r2, w = r0 * r1 * r2;
    const double den = 1.0 / (w * (u * v - w));
    const double f0 = (u * v * v - w * (u * u + v)) * den;
    const double f1 = (2.0 * u * v - w - u * u * u) * den;
    const double f2 = u * den;
    const M3 Q2 = mul_nn(Q, Q);
    M3 Mx;
#pragma unroll
    for (int i = 0; i < 9; i++)
        Mx.e[i] = make_double2(__builtin_fma(f1, Q.e[i].x, f2 * Q2.e[i].x), __builtin_fma(f1, Q.e[i].y, f2 * Q2.e[i].y));
    Mx.e[0].x += f0;
    Mx.e[4].x += f0;
    Mx.e[8].x += f0;
    const M3 Wm = mul_nn(Vm, Mx);
#pragma unroll
    for (int i = 0; i < 9; i++) ok = ok && __builtin_isfinite(Wm.e[i].x) && __builtin_isfinite(Wm.e[i].y);
    st(f, V, s, Wm);
    if (!ok) atomicAdd(bad, 1);
}

}  // namespace

hipError_t launch_smear_staple(const SmearGeom &g, const StapleArgs &a, hipStream_t s)
{
    const dim3 grid((unsigned)((g.V + 255) / 256)), blk(256);
    const bool lep = a.cL != 0.0, wt = a.T_out != nullptr;
    if (lep && wt) hipLaunchKernelGGL((k_smear_staple<true, true>), grid, blk, 0, s, g, a);
    else if (lep) hipLaunchKernelGGL((k_smear_staple<true, false>), grid, blk, 0, s, g, a);
    else if (wt) hipLaunchKernelGGL((k_smear_staple<false, true>), grid, blk, 0, s, g, a);
    else hipLaunchKernelGGL((k_smear_staple<false, false>), grid, blk, 0, s, g, a);
    return hipGetLastError();
}

hipError_t launch_smear_to_planar(const SmearGeom &g, const double2 *aos, double2 *pl, hipStream_t s)
{
    hipLaunchKernelGGL(k_smear_to_planar, dim3((unsigned)((g.V + SB - 1) / SB)), dim3(256), 0, s, g, aos, pl);
    return hipGetLastError();
}

hipError_t launch_smear_from_planar(const SmearGeom &g, const double2 *pl, double2 *aos, hipStream_t s)
{
    hipLaunchKernelGGL((k_smear_out<0>), dim3((unsigned)((g.V + SB - 1) / SB)), dim3(256), 0, s, g, pl,
                       (const double2 *)nullptr, 0.0, aos, (double2 *)nullptr);
    return hipGetLastError();
}

hipError_t launch_smear_unitarize(const SmearGeom &g, double2 *pl, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_smear_unitarize, dim3((unsigned)((g.V + 255) / 256), 4), dim3(256), 0, s, g, pl, bad);
    return hipGetLastError();
}

hipError_t launch_smear_output(const SmearGeom &g, const double2 *X, const double2 *W, double cN,
                               double2 *fat, double2 *lng, hipStream_t s)
{
    hipLaunchKernelGGL((k_smear_out<1>), dim3((unsigned)((g.V + SB - 1) / SB)), dim3(256), 0, s, g, X, W, cN,
                       fat, lng);
    return hipGetLastError();
}

}  // namespace hisq
