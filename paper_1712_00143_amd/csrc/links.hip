// Link packing: FP64 site-major links [V][4][3][3] (phases folded) ->
// per-output-parity, per-direction, chunk-planar storage in FP64/FP32/FP16
// with 18 or 12 reals per link.  This is the library-side remap that the
// paper times separately from the solver (Section 4.2: data remapping).
//
// For output site x and direction d the stored matrix M_d is the whole hop
// term: F_mu(x), -F_mu(x-mu)^+, L_mu(x), -L_mu(x-3mu)^+ (backward links are
// stored daggered and negated at the output site, so all 16 loads of a site
// are coalesced).  Recon-18 stores M_d / a.  Recon-12 requires every link to
// be c * SU(3) with c = s * eta_mu(x) * a (a per field, s = +-1 per field);
// it stores the first two rows of M_d / c_d, c_d = c (forward) or -c
// (backward), and the kernels rebuild row 2 as conj(row0 x row1).
#include "fields.h"
#include "launch.h"

namespace hisq {

using cd = Cx<double>;

__device__ __forceinline__ void load_u(const double *f, long long site, int mu, cd u[3][3])
{
    const double2 *p = reinterpret_cast<const double2 *>(f) + (site * 4 + mu) * 9;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            double2 v = p[3 * r + c];
            u[r][c] = {v.x, v.y};
        }
}

template <class LT, int R>
__global__ void k_pack(PackLaunch p)
{
    using F = LinkFmt<LT, R>;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)p.h * NDIR) return;
    const int d = (int)(t / p.h);
    const int i = (int)(t - (long long)d * p.h);
    const int mu = d >> 2, kind = d & 3;
    Coord co = cb_to_coord(i, p.out_par, p.L);
    const int fld = kind >> 1;
    const double *src = fld ? p.lng : p.fat;
    const bool bwd = kind & 1;
    const int step = kind == 0 ? 0 : kind == 1 ? -1 : kind == 2 ? 0 : -3;
    Coord cs = co;
    cs.x[mu] = ((cs.x[mu] + step) % p.L[mu] + p.L[mu]) % p.L[mu];
    long long site = cs.x[0] + (long long)p.L[0] * (cs.x[1] + (long long)p.L[1] * (cs.x[2] + (long long)p.L[2] * cs.x[3]));
    cd u[3][3], m[3][3];
    load_u(src, site, mu, u);
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++)
            m[r][c] = bwd ? cd{-u[c][r].re, u[c][r].im} : u[r][c];   // -(U^+)

    double scale;
    if constexpr (R == 12) {
        int sg = p.s[fld] * eta_sign(co, mu) * (bwd ? -1 : 1);
        scale = sg * p.a[fld];
        // check that row 2 is recoverable
        cd w0[3], w1[3];
        for (int c = 0; c < 3; c++) {
            w0[c] = {m[0][c].re / scale, m[0][c].im / scale};
            w1[c] = {m[1][c].re / scale, m[1][c].im / scale};
        }
        cd x0 = cmul(w0[1], w1[2]), y0 = cmul(w0[2], w1[1]);
        cd x1 = cmul(w0[2], w1[0]), y1 = cmul(w0[0], w1[2]);
        cd x2 = cmul(w0[0], w1[1]), y2 = cmul(w0[1], w1[0]);
        cd w2[3] = {{x0.re - y0.re, -(x0.im - y0.im)},
                    {x1.re - y1.re, -(x1.im - y1.im)},
                    {x2.re - y2.re, -(x2.im - y2.im)}};
        double err = 0;
        for (int c = 0; c < 3; c++) {
            double dr = w2[c].re * scale - m[2][c].re, di = w2[c].im * scale - m[2][c].im;
            err = fmax(err, sqrt(dr * dr + di * di) / p.a[fld]);
        }
        if (!(err <= 1e300)) err = 1e300;  // NaN -> huge
        atomicMax(p.maxerr, (unsigned long long)__double_as_longlong(err));
    } else {
        scale = p.a[fld];
    }
    const double inv = 1.0 / scale;
    LT e[R];
#pragma unroll
    for (int k = 0; k < R / 2; k++) {
        int r = k / 3, c = k % 3;
        e[2 * k] = (LT)(m[r][c].re * inv);
        e[2 * k + 1] = (LT)(m[r][c].im * inv);
    }
    const uint32_t *raw = reinterpret_cast<const uint32_t *>(e);
    char *dirbase = (char *)p.dst + (size_t)d * p.hs * F::BYTES;
#pragma unroll
    for (int q = 0; q < F::NQ; q++)
        *reinterpret_cast<uint4 *>(dirbase + ((size_t)q * p.hs + i) * 16) =
            make_uint4(raw[4 * q], raw[4 * q + 1], raw[4 * q + 2], raw[4 * q + 3]);
    if constexpr (F::REM == 8)
        *reinterpret_cast<uint2 *>(dirbase + (size_t)F::NQ * p.hs * 16 + (size_t)i * 8) =
            make_uint2(raw[4 * F::NQ], raw[4 * F::NQ + 1]);
    else if constexpr (F::REM == 4)
        *reinterpret_cast<uint32_t *>(dirbase + (size_t)F::NQ * p.hs * 16 + (size_t)i * 4) = raw[4 * F::NQ];
}

template <class LT, int R>
static hipError_t pack_t(const PackLaunch &p, hipStream_t s)
{
    long long n = (long long)p.h * NDIR;
    int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL((k_pack<LT, R>), dim3(nb), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_pack(int prec, int recon, const PackLaunch &p, hipStream_t s)
{
    if (prec == 0) return recon == 12 ? pack_t<double, 12>(p, s) : pack_t<double, 18>(p, s);
    if (prec == 1) return recon == 12 ? pack_t<float, 12>(p, s) : pack_t<float, 18>(p, s);
    if (prec == 2) return recon == 12 ? pack_t<__half, 12>(p, s) : pack_t<__half, 18>(p, s);
    return hipErrorInvalidValue;
}

// determinant of the mu=0 link at site 0 of both fields: out = {Re, Im} x 2
__global__ void k_det_probe(const double *fat, const double *lng, double *out)
{
    if (threadIdx.x >= 2) return;
    const double *f = threadIdx.x ? lng : fat;
    cd u[3][3];
    load_u(f, 0, 0, u);
    cd a = cmul(u[1][1], u[2][2]), b = cmul(u[1][2], u[2][1]);
    cd c = cmul(u[1][0], u[2][2]), d = cmul(u[1][2], u[2][0]);
    cd e = cmul(u[1][0], u[2][1]), g = cmul(u[1][1], u[2][0]);
    cd m0 = {a.re - b.re, a.im - b.im}, m1 = {c.re - d.re, c.im - d.im}, m2 = {e.re - g.re, e.im - g.im};
    cd t0 = cmul(u[0][0], m0), t1 = cmul(u[0][1], m1), t2 = cmul(u[0][2], m2);
    out[2 * threadIdx.x] = t0.re - t1.re + t2.re;
    out[2 * threadIdx.x + 1] = t0.im - t1.im + t2.im;
}

hipError_t launch_det_probe(const double *fat, const double *lng, double *out4, hipStream_t s)
{
    hipLaunchKernelGGL(k_det_probe, dim3(1), dim3(64), 0, s, fat, lng, out4);
    return hipGetLastError();
}

__global__ void k_maxabs(const double *v, long long n, unsigned long long *out)
{
    double m = 0;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        m = fmax(m, fabs(v[k]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

hipError_t launch_maxabs(const double *links, long long n, unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_maxabs, dim3(1024), dim3(256), 0, s, links, n, out);
    return hipGetLastError();
}

}  // namespace hisq
