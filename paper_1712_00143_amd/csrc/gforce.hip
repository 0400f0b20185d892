// Symanzik-improved gauge force and action (FP64), the gauge-field half of
// the RHMC step the paper benchmarks beside the fermion force (Section 4.2).
//
// S = beta sum over loops of c (1 - Re Tr U_loop / 3) over the 1x1
// plaquettes, the 1x2 / 2x1 rectangles and the six-link parallelograms;
// the force on U_mu(x) is (beta/3) TA[U_mu(x) B^+], B the weighted sum of
// the paths from x to x+mu that close each loop through the link.
//
// One thread per link, the whole staple sum in registers:
// 6 signed transverse steps n, each giving the plaquette and the three
// rectangles (11 products with the shared prefix and suffix factored out),
// and 24 parallelograms (b, a, mu, -b, -a), summed over b before the common
// last step along -a (13 products per signed a).  145 3x3 products per link:
// about 29 kflop against 288 B of link reads and writes, so the kernel is
// bound by the FP64 units and load latency, not by HBM bandwidth; the
// neighbour links come from L1 / L2.
#include "gforce.h"
#include "hisq_dev.h"
#include "su3.h"

namespace hisq {

using namespace su3;

namespace {

// Link of the step from site `from` to `to` = from + SG * axis.
template <int SG>
__device__ __forceinline__ M3 stp(const double2 *__restrict__ Ua, size_t V, long long from, long long to)
{
    if constexpr (SG > 0) return ld(Ua, V, from);
    else return dag(ld(Ua, V, to));
}

struct Geo {
    long long s;
    int x[4];
};

// x + ka * a + kb * b (distinct axes a, b)
__device__ __forceinline__ long long at2(const SmearGeom &g, const Geo &q, int a, int ka, int b, int kb)
{
    long long y = q.s;
    if (ka) y = shift(y, pick(q.x, a), pick(g.S, a), pick(g.L, a), ka);
    if (kb) y = shift(y, pick(q.x, b), pick(g.S, b), pick(g.L, b), kb);
    return y;
}

__device__ __forceinline__ long long at3(const SmearGeom &g, const Geo &q, int a, int ka, int b, int kb, int c, int kc)
{
    long long y = at2(g, q, a, ka, b, kb);
    if (kc) y = shift(y, pick(q.x, c), pick(g.S, c), pick(g.L, c), kc);
    return y;
}

// Plaquette and rectangle paths for the signed transverse step n = SN nu:
//   plaquette      L(x->x+n) U_mu(x+n) L(x+n+mu->x+mu)
//   nu-long        L(x->x+n) L(x+n->x+2n) U_mu(x+2n) L(x+2n+mu->x+n+mu) L(x+n+mu->x+mu)
//   mu-long, link first   L(x->x+n) U_mu(x+n) U_mu(x+n+mu) L(x+n+2mu->x+2mu) U_mu(x+mu)^+
//   mu-long, link second  U_mu(x-mu)^+ L(x-mu->x-mu+n) U_mu(x-mu+n) U_mu(x+n) L(x+n+mu->x+mu)
template <int SN>
__device__ __forceinline__ void plaq_rect(const SmearGeom &g, const Geo &q, const double2 *__restrict__ U, size_t V,
                                          int mu, int nu, double cp, double cr, M3 &B)
{
    const double2 *Un = U + (size_t)nu * 9 * V, *Um = U + (size_t)mu * 9 * V;
    const long long xn1 = at2(g, q, nu, SN, mu, 0), xn2 = at2(g, q, nu, 2 * SN, mu, 0);
    const long long xm1 = at2(g, q, nu, 0, mu, 1), xn1m1 = at2(g, q, nu, SN, mu, 1), xn2m1 = at2(g, q, nu, 2 * SN, mu, 1);
    const long long xm2 = at2(g, q, nu, 0, mu, 2), xn1m2 = at2(g, q, nu, SN, mu, 2);
    const long long xmm = at2(g, q, nu, 0, mu, -1), xn1mm = at2(g, q, nu, SN, mu, -1);
    const M3 Ln0 = stp<SN>(Un, V, q.s, xn1);
    const M3 H = mul_nn(Ln0, ld(Um, V, xn1));
    M3 X = H;
#pragma unroll
    for (int i = 0; i < 9; i++) X.e[i] = make_double2(cp * X.e[i].x, cp * X.e[i].y);
    {
        M3 P = mul_an(ld(Um, V, xmm), stp<SN>(Un, V, xmm, xn1mm));
        P = mul_nn(P, ld(Um, V, xn1mm));
        P = mul_nn(P, ld(Um, V, xn1));
        axpy(X, cr, P);
    }
    {
        M3 P = mul_nn(Ln0, stp<SN>(Un, V, xn1, xn2));
        P = mul_nn(P, ld(Um, V, xn2));
        P = mul_nn(P, stp<-SN>(Un, V, xn2m1, xn1m1));
        axpy(X, cr, P);
    }
    B = add(B, mul_nn(X, stp<-SN>(Un, V, xn1m1, xm1)));
    {
        M3 P = mul_nn(H, ld(Um, V, xn1m1));
        P = mul_nn(P, stp<-SN>(Un, V, xn1m2, xm2));
        P = mul_na(P, ld(Um, V, xm1));
        axpy(B, cr, P);
    }
}

// Parallelograms with first step a = SA * ax_a: sum over the four signed b
// on the two remaining axes of L(x->x+b) L(x+b->x+a+b) U_mu(x+a+b)
// L(x+a+b+mu->x+a+mu), then the common last step L(x+a+mu->x+mu).
template <int SA>
__device__ __forceinline__ void parallelograms(const SmearGeom &g, const Geo &q, const double2 *__restrict__ U,
                                               size_t V, int mu, int a, int b0, int b1, double cg, M3 &B)
{
    const double2 *Ua = U + (size_t)a * 9 * V, *Um = U + (size_t)mu * 9 * V;
    M3 S = zero3();
#pragma unroll 1
    for (int k = 0; k < 2; k++) {
        const int b = k == 0 ? b0 : b1;
        const double2 *Ub = U + (size_t)b * 9 * V;
#pragma unroll
        for (int sb = 0; sb < 2; sb++) {
            const int SB = sb == 0 ? 1 : -1;
            const long long xb = at3(g, q, b, SB, a, 0, mu, 0), xab = at3(g, q, b, SB, a, SA, mu, 0);
            const long long xabm = at3(g, q, b, SB, a, SA, mu, 1), xam = at3(g, q, b, 0, a, SA, mu, 1);
            M3 P = sb == 0 ? stp<1>(Ub, V, q.s, xb) : stp<-1>(Ub, V, q.s, xb);
            P = mul_nn(P, stp<SA>(Ua, V, xb, xab));
            P = mul_nn(P, ld(Um, V, xab));
            P = mul_nn(P, sb == 0 ? stp<-1>(Ub, V, xabm, xam) : stp<1>(Ub, V, xabm, xam));
            S = add(S, P);
        }
    }
    const long long xam = at2(g, q, a, SA, mu, 1), xm1 = at2(g, q, a, 0, mu, 1);
    axpy(B, cg, mul_nn(S, stp<-SA>(Ua, V, xam, xm1)));
}

template <int MODE>   // 0: force, 1: action partials
__global__ void __launch_bounds__(256) k_gauge_force(SmearGeom g, GForceArgs a)
{
    // A block holds the four links (one wave per direction) of 64 sites of
    // one x-y-z slab and walks a run of tch time slices: the links one
    // direction's staples fetch serve the other directions, and those of the
    // next slices, from L1 / L2 (the t neighbours are the block's own recent
    // loads instead of a lattice-volume stride away).
    const int lb = xcd_tile(blockIdx.x, gridDim.x, 1);
    const int chunk = lb / a.ntile, tile = brick_tile(lb - chunk * a.ntile, g);
    const long long nxyz = (long long)g.L[0] * g.L[1] * g.L[2];
    const long long i = (long long)tile * 64 + (threadIdx.x & 63);
    const bool valid = i < nxyz;
    const size_t V = (size_t)g.P;   // plane stride
    const int mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Geo q;
    {
        unsigned r = valid ? (unsigned)i : 0u;
        q.x[0] = (int)(r % (unsigned)g.L[0]);
        r /= (unsigned)g.L[0];
        q.x[1] = (int)(r % (unsigned)g.L[1]);
        q.x[2] = (int)(r / (unsigned)g.L[1]);
    }
    const long long ixyz = valid ? i : 0;
    const int t0 = chunk * a.tch, t1 = t0 + a.tch < g.L[3] ? t0 + a.tch : g.L[3];
    const int perp[3] = {mu == 0 ? 1 : 0, mu <= 1 ? 2 : 1, mu <= 2 ? 3 : 2};
    double v = 0.0;
#pragma unroll 1
    for (int t = t0; t < t1; t++) {
        q.x[3] = t;
        q.s = ixyz + (long long)t * g.S[3];
    M3 B = zero3();
#pragma unroll 1
    for (int k = 0; k < 3; k++) {
        const int nu = k == 0 ? perp[0] : k == 1 ? perp[1] : perp[2];
        plaq_rect<1>(g, q, a.U, V, mu, nu, a.cp, a.cr, B);
        plaq_rect<-1>(g, q, a.U, V, mu, nu, a.cp, a.cr, B);
    }
    if (a.cg != 0.0) {
#pragma unroll 1
        for (int k = 0; k < 3; k++) {
            const int ax = k == 0 ? perp[0] : k == 1 ? perp[1] : perp[2];
            const int b0 = k == 0 ? perp[1] : perp[0], b1 = k == 2 ? perp[1] : perp[2];
            parallelograms<1>(g, q, a.U, V, mu, ax, b0, b1, a.cg, B);
            parallelograms<-1>(g, q, a.U, V, mu, ax, b0, b1, a.cg, B);
        }
    }
    const M3 M = mul_na(ld(a.U + (size_t)mu * 9 * V, V, q.s), B);
    if constexpr (MODE == 0) {
        if (valid) {
            const double im3 = (M.e[0].y + M.e[4].y + M.e[8].y) * (1.0 / 3.0);
            M3 F;
#pragma unroll
            for (int i2 = 0; i2 < 3; i2++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    const double2 p = M.e[3 * i2 + j], r = M.e[3 * j + i2];
                    F.e[3 * i2 + j] = make_double2(a.scale * 0.5 * (p.x - r.x),
                                                   a.scale * (0.5 * (p.y + r.y) - (i2 == j ? im3 : 0.0)));
                }
            st(a.F + (size_t)mu * 9 * V, V, q.s, F);
        }
    } else {
        if (valid) v += M.e[0].x + M.e[4].x + M.e[8].x;
    }
    }
    if constexpr (MODE == 1) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        __shared__ double red[4];
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) a.part[lb] = ((red[0] + red[1]) + red[2]) + red[3];
    }
}

}  // namespace

void gauge_force_grid(const SmearGeom &g, int *ntile, int *tch, int *nblocks)
{
    const long long nxyz = (long long)g.L[0] * g.L[1] * g.L[2];
    *ntile = (int)((nxyz + 63) / 64);
    // enough blocks to fill the chip (about 2048), each with a run of slices
    int nchunk = (int)((2048 + *ntile - 1) / *ntile);
    nchunk = nchunk < 1 ? 1 : (nchunk > g.L[3] ? g.L[3] : nchunk);
    *tch = (g.L[3] + nchunk - 1) / nchunk;
    nchunk = (g.L[3] + *tch - 1) / *tch;
    *nblocks = *ntile * nchunk;
}

hipError_t launch_gauge_force(const SmearGeom &g, const GForceArgs &a0, int mode, hipStream_t s)
{
    GForceArgs a = a0;
    int nb;
    gauge_force_grid(g, &a.ntile, &a.tch, &nb);
    const dim3 grid((unsigned)nb), blk(256);
    if (mode == 0) hipLaunchKernelGGL((k_gauge_force<0>), grid, blk, 0, s, g, a);
    else hipLaunchKernelGGL((k_gauge_force<1>), grid, blk, 0, s, g, a);
    return hipGetLastError();
}

}  // namespace hisq
