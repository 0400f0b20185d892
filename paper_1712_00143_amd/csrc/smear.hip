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
#include "gforce.h"
#include "hisq_dev.h"
#include "smear.h"
#include "su3.h"

namespace hisq {

using namespace su3;

namespace {

// The two single-sign staples of field M through direction (S, L) at site
// y, whose coordinates along that direction and along mu are yd and ym:
// P = U(y) M(y+d) U(y+mu)^+, Q = U(y-d)^+ M(y-d) U(y-d+mu).
__device__ __forceinline__ void staple_halves(const double2 *__restrict__ U, const double2 *__restrict__ M, size_t V,
                                              long long y, int yd, int S, int L, int ym, int Sm, int Lm, M3 &P, M3 &Q)
{
    const long long pd = shift(y, yd, S, L, 1), md = shift(y, yd, S, L, -1);
    const long long pm = shift(y, ym, Sm, Lm, 1), md_pm = shift(md, ym, Sm, Lm, 1);
    P = mul_na(mul_nn(ld(U, V, y), ld(M, V, pd)), ld(U, V, pm));
    Q = mul_nn(mul_an(ld(U, V, md), ld(M, V, md)), ld(U, V, md_pm));
}

// The one-step staple P + Q of M through (S, L).
__device__ __forceinline__ M3 staple_at(const double2 *__restrict__ U, const double2 *__restrict__ M, size_t V,
                                        long long y, int yd, int S, int L, int ym, int Sm, int Lm)
{
    M3 T, Q;
    staple_halves(U, M, V, y, yd, S, L, ym, Sm, Lm, T, Q);
#pragma unroll
    for (int i = 0; i < 9; i++) T.e[i] = make_double2(T.e[i].x + Q.e[i].x, T.e[i].y + Q.e[i].y);
    return T;
}

// A staple through (S, L) whose two signs transport different fields:
// U(y) Mp(y+d) U(y+mu)^+ + U(y-d)^+ Mm(y-d) U(y-d+mu).  With Mp, Mm the
// single-sign 3-staples of U_mu through d this is the two-step (Lepage)
// staple U(y) U(y+d) U_mu(y+2d) U(y+d+mu)^+ U(y+mu)^+ + (its -d image).
// Every element of Mp and Mm is read by one site only: non-temporal loads.
__device__ __forceinline__ M3 staple_pm(const double2 *__restrict__ U, const double2 *__restrict__ Mp,
                                        const double2 *__restrict__ Mm, size_t V, long long y, int yd, int S, int L,
                                        int ym, int Sm, int Lm)
{
    const long long pd = shift(y, yd, S, L, 1), md = shift(y, yd, S, L, -1);
    const long long pm = shift(y, ym, Sm, Lm, 1), md_pm = shift(md, ym, Sm, Lm, 1);
    M3 T = mul_na(mul_nn(ld(U, V, y), ld_nt(Mp, V, pd)), ld(U, V, pm));
    const M3 Q = mul_nn(mul_an(ld(U, V, md), ld_nt(Mm, V, md)), ld(U, V, md_pm));
#pragma unroll
    for (int i = 0; i < 9; i++) T.e[i] = make_double2(T.e[i].x + Q.e[i].x, T.e[i].y + Q.e[i].y);
    return T;
}

// Pass 1 of every output direction at once: a block holds 64 sites of one
// x-y-z slab, one wave per direction mu, and walks a run of tch time slices
// (the block grid of gauge_force_grid), so that the neighbour links one
// direction's staples fetch serve the other directions from L1 / L2 and the
// t neighbours are the block's own recent loads.  For each mu, the 3-link
// staples through the three nu != mu, stored as T1[3 mu + k] when WT (and
// their single-sign halves as H[6 mu + 2 k], H[6 mu + 2 k + 1] when WH), and
//   F_mu = c1 U_mu + c3 sum_nu T1_nu.
template <bool WT, bool WH>
__global__ void __launch_bounds__(256) k_smear_pass1(SmearGeom g, Pass1Args a, int ntile, int tch)
{
    const int lb = xcd_tile(blockIdx.x, gridDim.x, 1);
    const int chunk = lb / ntile, tile = lb - chunk * ntile;
    const long long i = (long long)tile * 64 + (threadIdx.x & 63);
    if (i >= (long long)g.S[3]) return;   // no barriers below
    const size_t V = (size_t)g.P;   // plane stride
    const int mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int x[4];
    {
        unsigned r = (unsigned)i;
        x[0] = (int)(r % (unsigned)g.L[0]);
        r /= (unsigned)g.L[0];
        x[1] = (int)(r % (unsigned)g.L[1]);
        x[2] = (int)(r / (unsigned)g.L[1]);
    }
    const int t0 = chunk * tch, t1 = t0 + tch < g.L[3] ? t0 + tch : g.L[3];
    const int Sm = pick(g.S, mu), Lm = pick(g.L, mu);
    const double2 *Umu = a.U + (size_t)mu * 9 * V;
#pragma unroll 1
    for (int t = t0; t < t1; t++) {
        x[3] = t;
        const long long s = i + (long long)t * g.S[3];
        const int xm = pick(x, mu);
        M3 F = ld(Umu, V, s);
#pragma unroll
        for (int e = 0; e < 9; e++) F.e[e] = make_double2(a.c1 * F.e[e].x, a.c1 * F.e[e].y);
        // one direction at a time: unrolled, the three staples' loads are all
        // hoisted and spill
#pragma unroll 1
        for (int k = 0; k < 3; k++) {
            const int nu = k + (k >= mu ? 1 : 0);
            const int Sn = pick(g.S, nu), Ln = pick(g.L, nu), xn = pick(x, nu);
            const double2 *Un = a.U + (size_t)nu * 9 * V;
            M3 T;
            if constexpr (WH) {
                M3 Q;
                staple_halves(Un, Umu, V, s, xn, Sn, Ln, xm, Sm, Lm, T, Q);
                st(a.H + (size_t)(6 * mu + 2 * k) * 9 * V, V, s, T);
                st(a.H + (size_t)(6 * mu + 2 * k + 1) * 9 * V, V, s, Q);
#pragma unroll
                for (int e = 0; e < 9; e++) T.e[e] = make_double2(T.e[e].x + Q.e[e].x, T.e[e].y + Q.e[e].y);
            } else {
                T = staple_at(Un, Umu, V, s, xn, Sn, Ln, xm, Sm, Lm);
            }
            axpy(F, a.c3, T);
            if constexpr (WT) st(a.T1 + (size_t)(3 * mu + k) * 9 * V, V, s, T);
        }
        st(a.F + (size_t)mu * 9 * V, V, s, F);
    }
}

// The Lepage term of every output direction, with the block grid of pass 1
// (its tiles in the brick order of brick_tile, as in passes 2 and 3; pass 1
// itself is 4 % faster in the plain order):
//   F_mu += cL sum over nu != mu of staple_pm(U_nu; H+, H-),
// H+- the single-sign 3-staples of U_mu through nu that pass 1 stored.
__global__ void __launch_bounds__(256) k_smear_lepage(SmearGeom g, LepageArgs a, int ntile, int tch)
{
    const int lb = xcd_tile(blockIdx.x, gridDim.x, 1);
    const int chunk = lb / ntile, tile = brick_tile(lb - chunk * ntile, g);
    const long long i = (long long)tile * 64 + (threadIdx.x & 63);
    if (i >= (long long)g.S[3]) return;   // no barriers below
    const size_t V = (size_t)g.P;   // plane stride
    const int mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int x[4];
    {
        unsigned r = (unsigned)i;
        x[0] = (int)(r % (unsigned)g.L[0]);
        r /= (unsigned)g.L[0];
        x[1] = (int)(r % (unsigned)g.L[1]);
        x[2] = (int)(r / (unsigned)g.L[1]);
    }
    const int t0 = chunk * tch, t1 = t0 + tch < g.L[3] ? t0 + tch : g.L[3];
    const int Sm = pick(g.S, mu), Lm = pick(g.L, mu);
    double2 *Fmu = a.F + (size_t)mu * 9 * V;
#pragma unroll 1
    for (int t = t0; t < t1; t++) {
        x[3] = t;
        const long long s = i + (long long)t * g.S[3];
        const int xm = pick(x, mu);
        M3 F = ld(Fmu, V, s);
#pragma unroll 1
        for (int k = 0; k < 3; k++) {
            const int nu = k + (k >= mu ? 1 : 0);
            const double2 *Hp = a.H + (size_t)(6 * mu + 2 * k) * 9 * V;
            axpy(F, a.cL,
                 staple_pm(a.U + (size_t)nu * 9 * V, Hp, Hp + 9 * V, V, s, pick(x, nu), pick(g.S, nu), pick(g.L, nu),
                           xm, Sm, Lm));
        }
        st(Fmu, V, s, F);
    }
}

// Passes 2 and 3 of output direction mu take its three sig at once, one
// wave per sig on the same 64 sites (they share the fields they read), with
// the block grid and time-slice walk of pass 1; k is the index of sig among
// the directions other than mu, {nu, rho} the other two.
__device__ __forceinline__ int other_dir(int k, int mu) { return k + (k >= mu ? 1 : 0); }

// Pass 2: T2_k = staple(T1_nu through rho) + staple(T1_rho through nu), the
// 5-link staples whose transverse steps avoid sig, in both orders.  Two
// waves per sig (wave 2k the first staple, 2k + 1 the second, summed through
// LDS) and one block per CU: a CU then holds 64 sites at a time instead of
// 128, so a time slice's fields and their neighbours stay in L2 until the
// next slice reuses them (1.6 KB fetched per site instead of 2.8 KB), with
// six short chains of loads per CU to hide the latency.
__global__ void __launch_bounds__(384) __attribute__((amdgpu_waves_per_eu(1, 2))) k_smear_pass2(SmearGeom g,
                                                                                               Pass2Args a, int ntile,
                                                                                               int tch)
{
    const int lb = xcd_tile(blockIdx.x, gridDim.x, 1);
    const int chunk = lb / ntile, tile = brick_tile(lb - chunk * ntile, g);
    const int lane = threadIdx.x & 63;
    const long long i0 = (long long)tile * 64 + lane;
    const bool valid = i0 < (long long)g.S[3];
    const long long i = valid ? i0 : 0;
    const size_t V = (size_t)g.P;   // plane stride
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), mu = a.mu;
    const int k = w >> 1, second = w & 1;
    const int inu = k == 2 ? 0 : k + 1, irho = k == 0 ? 2 : k - 1;
    // the first staple transports T1_nu through rho, the second T1_rho through nu
    const int dir = other_dir(second ? inu : irho, mu), jt = second ? irho : inu;
    int x[4];
    {
        unsigned r = (unsigned)i;
        x[0] = (int)(r % (unsigned)g.L[0]);
        r /= (unsigned)g.L[0];
        x[1] = (int)(r % (unsigned)g.L[1]);
        x[2] = (int)(r / (unsigned)g.L[1]);
    }
    const int Sm = pick(g.S, mu), Lm = pick(g.L, mu), Sd = pick(g.S, dir), Ld = pick(g.L, dir);
    const double2 *Ud = a.U + (size_t)dir * 9 * V, *T1j = a.T1 + (size_t)jt * 9 * V;
    double2 *T2 = a.T2 + (size_t)k * 9 * V;
    __shared__ double2 red[3][9][64];
    const int t0 = chunk * tch, t1 = t0 + tch < g.L[3] ? t0 + tch : g.L[3];
#pragma unroll 1
    for (int t = t0; t < t1; t++) {
        x[3] = t;
        const long long s = i + (long long)t * g.S[3];
        M3 T = staple_at(Ud, T1j, V, s, pick(x, dir), Sd, Ld, pick(x, mu), Sm, Lm);
        if (second)
#pragma unroll
            for (int e = 0; e < 9; e++) red[k][e][lane] = T.e[e];
        __syncthreads();
        if (!second && valid) {
#pragma unroll
            for (int e = 0; e < 9; e++)
                T.e[e] = make_double2(T.e[e].x + red[k][e][lane].x, T.e[e].y + red[k][e][lane].y);
            st(T2, V, s, T);
        }
        __syncthreads();
    }
}

// Pass 3: F_mu += sum over sig of (c5 T2_k + c7 staple(T2_k through sig)),
// the 7-link staples being the staples of the 5-link ones; the three waves'
// terms meet in LDS and wave 0 updates F once, adding them in the order of k.
__global__ void __launch_bounds__(192) k_smear_pass3(SmearGeom g, Pass3Args a, int ntile, int tch)
{
    const int lb = xcd_tile(blockIdx.x, gridDim.x, 1);
    const int chunk = lb / ntile, tile = brick_tile(lb - chunk * ntile, g);
    const int lane = threadIdx.x & 63;
    const long long i0 = (long long)tile * 64 + lane;
    const bool valid = i0 < (long long)g.S[3];
    const long long i = valid ? i0 : 0;
    const size_t V = (size_t)g.P;   // plane stride
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), mu = a.mu;
    const int sig = other_dir(k, mu);
    int x[4];
    {
        unsigned r = (unsigned)i;
        x[0] = (int)(r % (unsigned)g.L[0]);
        r /= (unsigned)g.L[0];
        x[1] = (int)(r % (unsigned)g.L[1]);
        x[2] = (int)(r / (unsigned)g.L[1]);
    }
    const int Sm = pick(g.S, mu), Lm = pick(g.L, mu), Ss = pick(g.S, sig), Ls = pick(g.L, sig);
    const double2 *Us = a.U + (size_t)sig * 9 * V, *T2 = a.T2 + (size_t)k * 9 * V;
    double2 *F = a.F;
    __shared__ double2 red[2][9][64];
    const int t0 = chunk * tch, t1 = t0 + tch < g.L[3] ? t0 + tch : g.L[3];
#pragma unroll 1
    for (int t = t0; t < t1; t++) {
        x[3] = t;
        const long long s = i + (long long)t * g.S[3];
        M3 T = zero3();
        if (valid) {
            axpy(T, a.c5, ld(T2, V, s));
            axpy(T, a.c7, staple_at(Us, T2, V, s, pick(x, sig), Ss, Ls, pick(x, mu), Sm, Lm));
        }
        if (k > 0)
#pragma unroll
            for (int e = 0; e < 9; e++) red[k - 1][e][lane] = T.e[e];
        __syncthreads();
        if (k == 0 && valid) {
            M3 f = ld(F, V, s);
#pragma unroll
            for (int e = 0; e < 9; e++) {
                f.e[e] = make_double2(f.e[e].x + T.e[e].x, f.e[e].y + T.e[e].y);
                f.e[e] = make_double2(f.e[e].x + red[0][e][lane].x, f.e[e].y + red[0][e][lane].y);
                f.e[e] = make_double2(f.e[e].x + red[1][e][lane].x, f.e[e].y + red[1][e][lane].y);
            }
            st(F, V, s, f);
        }
        __syncthreads();
    }
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
    const size_t V = (size_t)g.P;   // plane stride
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
    const size_t V = (size_t)g.P;   // plane stride
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
    const size_t V = (size_t)g.P;   // plane stride
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

void smear_order(const int *first, int n, int ord[4])
{
    bool used[4] = {true, false, false, false};
    int k = 0;
    ord[k++] = 0;
    for (int i = 0; i < n; i++)
        if (first[i] > 0 && first[i] < 4 && !used[first[i]]) {
            used[first[i]] = true;
            ord[k++] = first[i];
        }
    for (int d = 1; d < 4; d++)
        if (!used[d]) ord[k++] = d;
}

hipError_t launch_smear_pass1(const SmearGeom &g, const Pass1Args &a, hipStream_t s)
{
    int ntile, tch, nb;
    gauge_force_grid(g, &ntile, &tch, &nb);
    const dim3 grid((unsigned)nb), blk(256);
    const bool wt = a.T1 != nullptr, wh = a.H != nullptr;
    if (wt && wh) hipLaunchKernelGGL((k_smear_pass1<true, true>), grid, blk, 0, s, g, a, ntile, tch);
    else if (wt) hipLaunchKernelGGL((k_smear_pass1<true, false>), grid, blk, 0, s, g, a, ntile, tch);
    else if (wh) hipLaunchKernelGGL((k_smear_pass1<false, true>), grid, blk, 0, s, g, a, ntile, tch);
    else hipLaunchKernelGGL((k_smear_pass1<false, false>), grid, blk, 0, s, g, a, ntile, tch);
    return hipGetLastError();
}

hipError_t launch_smear_lepage(const SmearGeom &g, const LepageArgs &a, hipStream_t s)
{
    int ntile, tch, nb;
    gauge_force_grid(g, &ntile, &tch, &nb);
    hipLaunchKernelGGL(k_smear_lepage, dim3((unsigned)nb), dim3(256), 0, s, g, a, ntile, tch);
    return hipGetLastError();
}

// The tile grid of gauge_force_grid aimed at `target` blocks: fewer blocks
// walk longer runs of time slices.  Passes 2 and 3 take 512 (at 32^4 every
// block walks the whole time extent: pass 3 310 us against 322 with 2048
// blocks, pass 2 unchanged).
static void tile_grid(const SmearGeom &g, int target, int *ntile, int *tch, int *nblocks)
{
    const long long nxyz = (long long)g.L[0] * g.L[1] * g.L[2];
    *ntile = (int)((nxyz + 63) / 64);
    int nchunk = (int)((target + *ntile - 1) / *ntile);
    nchunk = nchunk < 1 ? 1 : (nchunk > g.L[3] ? g.L[3] : nchunk);
    *tch = (g.L[3] + nchunk - 1) / nchunk;
    nchunk = (g.L[3] + *tch - 1) / *tch;
    *nblocks = *ntile * nchunk;
}

hipError_t launch_smear_pass2(const SmearGeom &g, const Pass2Args &a, hipStream_t s)
{
    int ntile, tch, nb;
    tile_grid(g, 512, &ntile, &tch, &nb);
    hipLaunchKernelGGL(k_smear_pass2, dim3((unsigned)nb), dim3(384), 0, s, g, a, ntile, tch);
    return hipGetLastError();
}

hipError_t launch_smear_pass3(const SmearGeom &g, const Pass3Args &a, hipStream_t s)
{
    int ntile, tch, nb;
    tile_grid(g, 512, &ntile, &tch, &nb);
    hipLaunchKernelGGL(k_smear_pass3, dim3((unsigned)nb), dim3(192), 0, s, g, a, ntile, tch);
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
