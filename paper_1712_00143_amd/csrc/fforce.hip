// HISQ fermion-force kernels (FP64): the chain rule of the force from the
// multi-shift solutions back to the thin links (Section 4.2's fermion
// force; the smearing it differentiates is the HISQ construction of
// smear.hip).
//
// The gradient flows backwards through the forward passes: outer products
// of the solution vectors give the gradients with respect to the fat and
// long links; the Naik product and every staple pass of the two fat7 levels
// have a gather-form adjoint (each thread owns the gradient of its own
// site's links, so there are no scattered updates); the U(3) projection has
// a closed-form adjoint from the Cayley-Hamilton form of (V^+ V)^{-1/2},
// whose coefficients are symmetric functions of the singular values and
// stay finite when they coincide.  Every kernel is an FP64 pass over planar
// fields (one thread per site, except the staple adjoint's four waves per
// 64 sites), bound by memory traffic and latency.
#include "fforce.h"
#include "hisq_dev.h"
#include "su3.h"

namespace hisq {

using namespace su3;

namespace {

__device__ __forceinline__ void coords4(const SmearGeom &g, long long s, int x[4])
{
    unsigned r = (unsigned)s;   // V <= 2^31
    x[0] = (int)(r % (unsigned)g.L[0]);
    r /= (unsigned)g.L[0];
    x[1] = (int)(r % (unsigned)g.L[1]);
    r /= (unsigned)g.L[1];
    x[2] = (int)(r % (unsigned)g.L[2]);
    x[3] = (int)(r / (unsigned)g.L[2]);
}

__device__ __forceinline__ void scale3(M3 &m, double k)
{
#pragma unroll
    for (int i = 0; i < 9; i++) m.e[i] = make_double2(k * m.e[i].x, k * m.e[i].y);
}

__global__ void __launch_bounds__(256) k_ff_outer(SmearGeom g, OuterArgs a)
{
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= g.V) return;
    const size_t V = (size_t)g.P;   // plane stride
    int x[4];
    coords4(g, s, x);
    const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
    const double eps2 = par ? 2.0 : -2.0;   // -2 eps(x)
    const double2 *vs = par ? a.Y : a.X, *vo = par ? a.X : a.Y;
    const long long cb = s >> 1;
#pragma unroll 1
    for (int mu = 0; mu < 4; mu++) {
        const int xm = pick(x, mu), Sm = pick(g.S, mu), Lm = pick(g.L, mu);
        const long long cb1 = shift(s, xm, Sm, Lm, 1) >> 1, cb3 = shift(s, xm, Sm, Lm, 3) >> 1;
        M3 F = zero3(), L = zero3();
#pragma unroll 1
        for (int k = 0; k < a.n; k++) {
            const double al = a.alpha[k];
            const double2 *p0 = vs + ((long long)k * a.h + cb) * 3;
            const double2 *p1 = vo + ((long long)k * a.h + cb1) * 3;
            const double2 *p3 = vo + ((long long)k * a.h + cb3) * 3;
            double2 c0[3], c1[3], c3[3];
#pragma unroll
            for (int i = 0; i < 3; i++) {
                c0[i] = p0[i];
                c1[i] = make_double2(al * p1[i].x, al * p1[i].y);
                c3[i] = make_double2(al * p3[i].x, al * p3[i].y);
            }
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    // alpha psi(x+mu)_i conj(psi(x)_j)
                    F.e[3 * i + j].x = __builtin_fma(c1[i].x, c0[j].x, __builtin_fma(c1[i].y, c0[j].y, F.e[3 * i + j].x));
                    F.e[3 * i + j].y = __builtin_fma(c1[i].y, c0[j].x, __builtin_fma(-c1[i].x, c0[j].y, F.e[3 * i + j].y));
                    L.e[3 * i + j].x = __builtin_fma(c3[i].x, c0[j].x, __builtin_fma(c3[i].y, c0[j].y, L.e[3 * i + j].x));
                    L.e[3 * i + j].y = __builtin_fma(c3[i].y, c0[j].x, __builtin_fma(-c3[i].x, c0[j].y, L.e[3 * i + j].y));
                }
        }
        double kf = eps2, kl = eps2;
        if (a.fold) {
            const int ph = mu == 0 ? 0 : mu == 1 ? x[0] : mu == 2 ? x[0] + x[1] : x[0] + x[1] + x[2];
            const double eta = (ph & 1) ? -1.0 : 1.0;
            kf *= eta;
            kl *= eta * a.cN;
        }
        scale3(F, kf);
        scale3(L, kl);
        st(a.OF + (size_t)mu * 9 * V, V, s, F);
        st(a.OL + (size_t)mu * 9 * V, V, s, L);
    }
}

__device__ __forceinline__ M3 ld_grad(const double2 *const G[2], size_t V, long long s)
{
    M3 m = ld(G[0], V, s);
    if (G[1]) m = add(m, ld(G[1], V, s));
    return m;
}

// A block holds 64 sites and four waves with one share of the work each, so
// that each carries a short chain of loads and products (one thread doing all
// of it needs over 200 registers and leaves two waves per SIMD): waves 0 and
// 1 the + and - staples' gradients with respect to M, waves 2 and 3 their
// shares of the gradient with respect to U_d, each pair summed through LDS.
__global__ void __launch_bounds__(256) k_staple_adjoint(SmearGeom g, StapleAdjArgs a)
{
    const int lane = threadIdx.x & 63, role = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long vi = (long long)xcd_tile(blockIdx.x, gridDim.x, 1) * 64 + lane;
    const bool valid = vi < g.V;
    const size_t V = (size_t)g.P;   // plane stride
    const bool plus = a.M[0] != nullptr, minus = a.M[1] != nullptr;
    const bool gm = a.GM[0] || a.GM[1], gm_one = a.GM[0] == a.GM[1];
    long long s = 0, pd = 0, md = 0, pm = 0, mm = 0, md_pm = 0, mm_pd = 0;
    if (valid) {
        int c[4];
        s = walk((unsigned)vi, g, a.ord, c);
        const int Sm = pick(g.S, a.mu), Lm = pick(g.L, a.mu), xm = coord(c, a.ord, a.mu);
        const int Sd = pick(g.S, a.d), Ld = pick(g.L, a.d), xd = coord(c, a.ord, a.d);
        pd = shift(s, xd, Sd, Ld, 1);
        md = shift(s, xd, Sd, Ld, -1);
        pm = shift(s, xm, Sm, Lm, 1);
        mm = shift(s, xm, Sm, Lm, -1);
        md_pm = shift(md, xm, Sm, Lm, 1);
        mm_pd = shift(mm, xd, Sd, Ld, 1);
    }
    // gradient with respect to M_s(y): the + staple at x = y - d and the -
    // staple at x = y + d read it.  U_d(z) is the first link of the + staple
    // at z and of the - staple at z + d, the last link of the + staple at
    // z - mu and of the - staple at z - mu + d.
    M3 t = zero3();
    if (valid) {
        if (role == 0) {
            if (plus && a.GM[0]) t = mul_nn(mul_an(ld(a.Ud, V, md_pm), ld_grad(a.G[0], V, md)), ld(a.Ud, V, md));
        } else if (role == 1) {
            if (minus && a.GM[1]) t = mul_na(mul_nn(ld(a.Ud, V, pm), ld_grad(a.G[1], V, pd)), ld(a.Ud, V, s));
        } else if (role == 2) {
            if (plus && a.GUd) {
                t = mul_nn(mul_na(ld(a.M[0], V, pd), ld(a.Ud, V, pm)), ld_grad(a.G[0], V, s));
                t = add(t, dag(mul_nn(mul_nn(ld_grad(a.G[0], V, mm), ld(a.Ud, V, mm)), ld(a.M[0], V, mm_pd))));
            }
        } else {
            if (minus && a.GUd) {
                t = dag(mul_nn(mul_nn(ld(a.M[1], V, s), ld(a.Ud, V, pm)), ld_grad(a.G[1], V, pd)));
                t = add(t, mul_nn(mul_na(ld_grad(a.G[1], V, mm_pd), ld(a.Ud, V, mm)), ld(a.M[1], V, mm)));
            }
        }
    }
    // separate gradient fields per sign: each of waves 0 and 1 writes its own
    if (valid && gm && !gm_one && role < 2) {
        double2 *f = a.GM[role];
        if (f && (role == 0 ? plus : minus)) {
            M3 out = a.gm_init ? zero3() : ld(f, V, s);
            axpy(out, a.c, t);
            st(f, V, s, out);
        }
    }
    __shared__ double2 red[2][9][64];   // the partials of waves 1 and 3
    if (role & 1)
#pragma unroll
        for (int i = 0; i < 9; i++) red[role >> 1][i][lane] = t.e[i];
    __syncthreads();
    if (!valid) return;
    if (role == 0 && gm && gm_one) {
        M3 out = a.gm_init ? zero3() : ld(a.GM[0], V, s);
        if (a.Gb) axpy(out, a.gb, ld(a.Gb, V, s));
#pragma unroll
        for (int i = 0; i < 9; i++) t.e[i] = make_double2(t.e[i].x + red[0][i][lane].x, t.e[i].y + red[0][i][lane].y);
        axpy(out, a.c, t);
        st(a.GM[0], V, s, out);
    }
    if (role == 2 && a.GUd) {
#pragma unroll
        for (int i = 0; i < 9; i++) t.e[i] = make_double2(t.e[i].x + red[1][i][lane].x, t.e[i].y + red[1][i][lane].y);
        M3 out = ld(a.GUd, V, s);
        axpy(out, a.c, t);
        st(a.GUd, V, s, out);
    }
}

__global__ void __launch_bounds__(256) k_ff_naik_adjoint(SmearGeom g, const double2 *W, const double2 *GN,
                                                         double2 *GW)
{
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= g.V) return;
    const size_t V = (size_t)g.P;   // plane stride
    const int mu = blockIdx.y;
    int x[4];
    coords4(g, s, x);
    const int Sm = pick(g.S, mu), Lm = pick(g.L, mu), xm = pick(x, mu);
    const double2 *w = W + (size_t)mu * 9 * V, *gn = GN + (size_t)mu * 9 * V;
    double2 *gw = GW + (size_t)mu * 9 * V;
    const long long p1 = shift(s, xm, Sm, Lm, 1), p2 = shift(s, xm, Sm, Lm, 2);
    const long long m1 = shift(s, xm, Sm, Lm, -1), m2 = shift(s, xm, Sm, Lm, -2);
    // W(z) is the first, second and third factor of N at z, z - mu, z - 2 mu
    M3 acc = mul_nn(mul_nn(ld(w, V, p1), ld(w, V, p2)), ld(gn, V, s));
    acc = add(acc, mul_nn(mul_nn(ld(w, V, p1), ld(gn, V, m1)), ld(w, V, m1)));
    acc = add(acc, mul_nn(mul_nn(ld(gn, V, m2), ld(w, V, m2)), ld(w, V, m1)));
    st(gw, V, s, add(ld(gw, V, s), acc));
}

// G <- M G + 2 Kh V^+: the gradient of Re Tr(W G) with respect to V for
// W = V M, M = (V^+ V)^{-1/2} = f0 + f1 Q + f2 Q^2, Q = V^+ V.  The f's are
// rational in u, v, w (sum, pairwise products and product of the square
// roots of Q's eigenvalues), which are functions of the invariants
// I = (Tr Q, Tr Q^2, det Q) with an invertible Jacobian (det = -16 w (uv - w));
// dM = sum_a (df/dI_a) dI_a + f1 dQ + f2 (dQ Q + Q dQ), dI = (Tr dQ,
// 2 Tr Q dQ, Tr adj(Q) dQ), and dQ = dV^+ V + V^+ dV gives the V^+ factor.
__global__ void __launch_bounds__(256) k_ff_unitarize_adjoint(SmearGeom g, const double2 *Vf, double2 *Gf)
{
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= g.V) return;
    const size_t V = (size_t)g.P;   // plane stride
    const double2 *vf = Vf + (size_t)blockIdx.y * 9 * V;
    double2 *gf = Gf + (size_t)blockIdx.y * 9 * V;
    const M3 Vm = ld(vf, V, s), G = ld(gf, V, s);
    const M3 Q = mul_an(Vm, Vm);
    const double c0 = (Q.e[0].x + Q.e[4].x + Q.e[8].x) * (1.0 / 3.0);
    const double a0 = Q.e[0].x - c0, a1 = Q.e[4].x - c0, a2 = Q.e[8].x - c0;
    const double2 q01 = Q.e[1], q02 = Q.e[2], q12 = Q.e[5];
    const double n01 = q01.x * q01.x + q01.y * q01.y, n02 = q02.x * q02.x + q02.y * q02.y;
    const double n12 = q12.x * q12.x + q12.y * q12.y;
    const double p = (a0 * a0 + a1 * a1 + a2 * a2 + 2.0 * (n01 + n02 + n12)) * (1.0 / 6.0);
    const double re3 = (q01.x * q12.x - q01.y * q12.y) * q02.x + (q01.x * q12.y + q01.y * q12.x) * q02.y;
    const double detd = a0 * a1 * a2 + 2.0 * re3 - a0 * n12 - a1 * n02 - a2 * n01;
    double g0 = c0, g1 = c0, g2 = c0;
    if (p > 1e-28 * c0 * c0) {
        const double sp = sqrt(p);
        double r = 0.5 * detd / (p * sp);
        r = r > 1.0 ? 1.0 : (r < -1.0 ? -1.0 : r);
        const double th = acos(r) * (1.0 / 3.0);
        const double tp = 2.0943951023931954923;   // 2 pi / 3
        g0 = c0 + 2.0 * sp * cos(th);
        g1 = c0 + 2.0 * sp * cos(th + tp);
        g2 = c0 + 2.0 * sp * cos(th - tp);
    }
    const double r0 = sqrt(fmax(g0, 0.0)), r1 = sqrt(fmax(g1, 0.0)), r2 = sqrt(fmax(g2, 0.0));
    const double u = r0 + r1 + r2, v = r0 * r1 + r0 * r2 + r1 * r2, w = r0 * r1 * r2;
    const double D = w * (u * v - w), iD = 1.0 / D;
    const double f[3] = {(u * v * v - w * (u * u + v)) * iD, (2.0 * u * v - w - u * u * u) * iD, u * iD};
    const double dN[3][3] = {{v * v - 2.0 * u * w, 2.0 * u * v - w, -u * u - v}, {2.0 * v - 3.0 * u * u, 2.0 * u, -1.0},
                             {1.0, 0.0, 0.0}};
    const double dD[3] = {v * w, u * w, u * v - 2.0 * w};
    // J = d(I1, I2, I3)/d(u, v, w) and its inverse
    const double J[3][3] = {{2.0 * u, -2.0, 0.0},
                            {4.0 * u * (u * u - 2.0 * v) + 4.0 * w, -4.0 * (u * u - 2.0 * v) - 4.0 * v, 4.0 * u},
                            {0.0, 0.0, 2.0 * w}};
    double Ji[3][3];
    {
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        const double id = 1.0 / det;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
                Ji[i][j] = (J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1]) * id;
            }
    }
    const M3 Q2 = mul_nn(Q, Q);
    const M3 R = mul_nn(G, Vm);
    const M3 QR = mul_nn(Q, R), RQ = mul_nn(R, Q);
    double rho[3] = {R.e[0].x + R.e[4].x + R.e[8].x, QR.e[0].x + QR.e[4].x + QR.e[8].x, 0.0};
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++)   // Re Tr(Q QR)
            rho[2] += Q.e[3 * i + k].x * QR.e[3 * k + i].x - Q.e[3 * i + k].y * QR.e[3 * k + i].y;
    double beta[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 3; i++) {
        double df[3];
#pragma unroll
        for (int j = 0; j < 3; j++) df[j] = (dN[i][j] - f[i] * dD[j]) * iD;
#pragma unroll
        for (int a = 0; a < 3; a++) beta[a] += (df[0] * Ji[0][a] + df[1] * Ji[1][a] + df[2] * Ji[2][a]) * rho[i];
    }
    // adj(Q)_ij = cofactor C_ji
    M3 K;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
            const double2 a11 = Q.e[3 * i1 + j1], a22 = Q.e[3 * i2 + j2], a12 = Q.e[3 * i1 + j2], a21 = Q.e[3 * i2 + j1];
            const double2 adj = make_double2(a11.x * a22.x - a11.y * a22.y - (a12.x * a21.x - a12.y * a21.y),
                                             a11.x * a22.y + a11.y * a22.x - (a12.x * a21.y + a12.y * a21.x));
            const double2 q = Q.e[3 * i + j], r = R.e[3 * i + j], qr = QR.e[3 * i + j], rq = RQ.e[3 * i + j];
            K.e[3 * i + j] = make_double2(2.0 * beta[1] * q.x + beta[2] * adj.x + f[1] * r.x + f[2] * (qr.x + rq.x),
                                          2.0 * beta[1] * q.y + beta[2] * adj.y + f[1] * r.y + f[2] * (qr.y + rq.y));
        }
    K.e[0].x += beta[0];
    K.e[4].x += beta[0];
    K.e[8].x += beta[0];
    M3 Kh;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            Kh.e[3 * i + j] = make_double2(K.e[3 * i + j].x + K.e[3 * j + i].x, K.e[3 * i + j].y - K.e[3 * j + i].y);   // 2 Kh
    M3 Mx;
#pragma unroll
    for (int i = 0; i < 9; i++)
        Mx.e[i] = make_double2(__builtin_fma(f[1], Q.e[i].x, f[2] * Q2.e[i].x), __builtin_fma(f[1], Q.e[i].y, f[2] * Q2.e[i].y));
    Mx.e[0].x += f[0];
    Mx.e[4].x += f[0];
    Mx.e[8].x += f[0];
    st(gf, V, s, add(mul_nn(Mx, G), mul_na(Kh, Vm)));
}

__global__ void k_field_axpby(double2 *out, double a, const double2 *in, double b, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double2 v = in[i];
        if (a == 0.0) {   // out may hold anything (never read)
            out[i] = make_double2(b * v.x, b * v.y);
        } else {
            const double2 o = out[i];
            out[i] = make_double2(a * o.x + b * v.x, a * o.y + b * v.y);
        }
    }
}

__global__ void __launch_bounds__(256) k_ff_project(SmearGeom g, const double2 *U, const double2 *G, double2 *F)
{
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= g.V) return;
    const size_t V = (size_t)g.P;   // plane stride
    const size_t off = (size_t)blockIdx.y * 9 * V;
    const M3 M = mul_nn(ld(U + off, V, s), ld(G + off, V, s));
    const double im3 = (M.e[0].y + M.e[4].y + M.e[8].y) * (1.0 / 3.0);
    M3 T;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const double2 p = M.e[3 * i + j], r = M.e[3 * j + i];
            T.e[3 * i + j] = make_double2(0.5 * (p.x - r.x), 0.5 * (p.y + r.y) - (i == j ? im3 : 0.0));
        }
    st(F + off, V, s, T);
}

}  // namespace

hipError_t launch_ff_outer(const SmearGeom &g, const OuterArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_ff_outer, dim3((unsigned)((g.V + 255) / 256)), dim3(256), 0, s, g, a);
    return hipGetLastError();
}

hipError_t launch_staple_adjoint(const SmearGeom &g, const StapleAdjArgs &a, hipStream_t s)
{
    if (!a.Ud || (!a.M[0] && !a.M[1]) || (a.M[0] && !a.G[0][0]) || (a.M[1] && !a.G[1][0])) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_staple_adjoint, dim3((unsigned)((g.V + 63) / 64)), dim3(256), 0, s, g, a);
    return hipGetLastError();
}

hipError_t launch_ff_naik_adjoint(const SmearGeom &g, const double2 *W, const double2 *GN, double2 *GW,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(k_ff_naik_adjoint, dim3((unsigned)((g.V + 255) / 256), 4), dim3(256), 0, s, g, W, GN, GW);
    return hipGetLastError();
}

hipError_t launch_ff_unitarize_adjoint(const SmearGeom &g, const double2 *V, double2 *G, hipStream_t s)
{
    hipLaunchKernelGGL(k_ff_unitarize_adjoint, dim3((unsigned)((g.V + 255) / 256), 4), dim3(256), 0, s, g, V, G);
    return hipGetLastError();
}

hipError_t launch_field_axpby(double2 *out, double a, const double2 *in, double b, size_t n, hipStream_t s)
{
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_field_axpby, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, out, a, in, b,
                       n);
    return hipGetLastError();
}

hipError_t launch_ff_project(const SmearGeom &g, const double2 *U, const double2 *G, double2 *F, hipStream_t s)
{
    hipLaunchKernelGGL(k_ff_project, dim3((unsigned)((g.V + 255) / 256), 4), dim3(256), 0, s, g, U, G, F);
    return hipGetLastError();
}

}  // namespace hisq
