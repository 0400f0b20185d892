// Storage formats of links and colour vectors, and the small complex 3x3
// algebra the stencil kernels use.
//
// Links: per output parity, 16 direction blocks of h links; a link of R reals
// (R = 18: full 3x3 complex, row-major; R = 12: the first two rows) is split
// into 16-byte chunks stored plane by plane ([dir][chunk][h]) followed by one
// remainder plane of 4 or 8 bytes, so that each load instruction of a
// wavefront reads one contiguous 1 KiB (or 256/512 B) segment.
//
// Colour vectors: [site][3] complex of double, float or half; half vectors
// carry a per-site float scale (the max |component|), stored separately.
#pragma once
#include "hisq_dev.h"

namespace hisq {

template <class T> struct AccOf { using type = float; };
template <> struct AccOf<double> { using type = double; };

template <class T, int R> struct LinkFmt {
    static constexpr int BYTES = R * (int)sizeof(T);
    static constexpr int NQ = BYTES / 16;
    static constexpr int REM = BYTES % 16;
};

template <class A> struct Cx {
    A re, im;
};

template <class A> __device__ __forceinline__ A fmaa(A a, A b, A c)
{
    if constexpr (sizeof(A) == 8) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

// Complex products with every fused multiply-add written out, so that the
// compiler's contraction of a*b - c*d cannot differ between kernel variants
// that share this arithmetic (they must give identical bits).
template <class A> __device__ __forceinline__ Cx<A> cmul(Cx<A> a, Cx<A> b)
{
    return {fmaa(a.re, b.re, -(a.im * b.im)), fmaa(a.re, b.im, a.im * b.re)};
}

template <class A> __device__ __forceinline__ Cx<A> cconjmul(Cx<A> a, Cx<A> b)  // conj(a) b
{
    return {fmaa(a.re, b.re, a.im * b.im), fmaa(a.re, b.im, -(a.im * b.re))};
}

// acc[r] += sum_c u[r][c] v[c]: 36 fused multiply-adds, no temporaries.
template <class A> __device__ __forceinline__ void matvec_acc(const Cx<A> u[3][3], const Cx<A> v[3], Cx<A> acc[3])
{
#pragma unroll
    for (int r = 0; r < 3; r++) {
        A re = acc[r].re, im = acc[r].im;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            re = fmaa(u[r][c].re, v[c].re, re);
            re = fmaa(-u[r][c].im, v[c].im, re);
            im = fmaa(u[r][c].re, v[c].im, im);
            im = fmaa(u[r][c].im, v[c].re, im);
        }
        acc[r] = {re, im};
    }
}

// acc[r] += k * sum_c u[r][c] v[c] (a scaled link: recon-12 sign, FP16 scale).
template <class A>
__device__ __forceinline__ void matvec_acc_scaled(const Cx<A> u[3][3], const Cx<A> v[3], A k, Cx<A> acc[3])
{
    Cx<A> y[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        A re = u[r][0].re * v[0].re, im = u[r][0].re * v[0].im;
        re = fmaa(-u[r][0].im, v[0].im, re);
        im = fmaa(u[r][0].im, v[0].re, im);
#pragma unroll
        for (int c = 1; c < 3; c++) {
            re = fmaa(u[r][c].re, v[c].re, re);
            re = fmaa(-u[r][c].im, v[c].im, re);
            im = fmaa(u[r][c].re, v[c].im, im);
            im = fmaa(u[r][c].im, v[c].re, im);
        }
        y[r] = {re, im};
    }
#pragma unroll
    for (int r = 0; r < 3; r++) {
        acc[r].re = fmaa(k, y[r].re, acc[r].re);
        acc[r].im = fmaa(k, y[r].im, acc[r].im);
    }
}

template <class T> __device__ __forceinline__ float to_f(T v) { return (float)v; }
template <> __device__ __forceinline__ float to_f<__half>(__half v) { return __half2float(v); }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Raw bytes of one packed link (R reals of LT).
template <class LT, int R> struct RawLink {
    uint32_t w[LinkFmt<LT, R>::BYTES / 4];
};

// Issue the loads of one packed link of direction block `dirbase` at site i;
// hs is the link set's plane stride in sites (LinkSet::hs).  Links are
// streamed exactly once per Dslash, so they are loaded non-temporally to
// leave the caches to the gathered colour vectors.
template <class LT, int R>
__device__ __forceinline__ void load_link_raw(const char *__restrict__ dirbase, int i, int hs,
                                              RawLink<LT, R> &raw)
{
    using F = LinkFmt<LT, R>;
#pragma unroll
    for (int q = 0; q < F::NQ; q++) {
        u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(dirbase + ((size_t)q * hs + i) * 16));
        raw.w[4 * q + 0] = v.x;
        raw.w[4 * q + 1] = v.y;
        raw.w[4 * q + 2] = v.z;
        raw.w[4 * q + 3] = v.w;
    }
    if constexpr (F::REM == 8) {
        u32x2 v = __builtin_nontemporal_load(
            reinterpret_cast<const u32x2 *>(dirbase + (size_t)F::NQ * hs * 16 + (size_t)i * 8));
        raw.w[4 * F::NQ + 0] = v.x;
        raw.w[4 * F::NQ + 1] = v.y;
    } else if constexpr (F::REM == 4) {
        raw.w[4 * F::NQ] = __builtin_nontemporal_load(
            reinterpret_cast<const uint32_t *>(dirbase + (size_t)F::NQ * hs * 16 + (size_t)i * 4));
    }
}

// The same loads through a buffer resource: `dirbase` must be the same for the
// whole wavefront (one direction block), so the base and the chunk-plane
// offsets live in scalar registers and each lane supplies only i * 16.  The
// offsets are 32-bit: one direction block must stay below 4 GiB.  CP = 0:
// non-temporal loads (an operator larger than the Infinity Cache is streamed
// once per application and should not evict the gathered vectors); CP = 1:
// ordinary loads, so that an operator that fits the Infinity Cache stays
// there from one application to the next.
template <class LT, int R, int CP = 0>
__device__ __forceinline__ void load_link_raw_wave(const char *dirbase, int i, int hs, RawLink<LT, R> &raw)
{
    using F = LinkFmt<LT, R>;
    constexpr int NT = CP ? 0 : 2;   // cache-policy bits of the load
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)dirbase, (short)0, hs * F::BYTES, 0x00020000);
#pragma unroll
    for (int q = 0; q < F::NQ; q++) {
        u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, i * 16, q * hs * 16, NT));
        raw.w[4 * q + 0] = v.x;
        raw.w[4 * q + 1] = v.y;
        raw.w[4 * q + 2] = v.z;
        raw.w[4 * q + 3] = v.w;
    }
    if constexpr (F::REM == 8) {
        u32x2 v = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, i * 8, F::NQ * hs * 16, NT));
        raw.w[4 * F::NQ + 0] = v.x;
        raw.w[4 * F::NQ + 1] = v.y;
    } else if constexpr (F::REM == 4) {
        raw.w[4 * F::NQ] = __builtin_amdgcn_raw_buffer_load_b32(rs, i * 4, F::NQ * hs * 16, NT);
    }
}

// Unpack a raw link into a 3x3 complex matrix; recon-12 rebuilds row 2 as
// conj(row0 x row1).
template <class LT, int R, class A>
__device__ __forceinline__ void decode_link(const RawLink<LT, R> &raw, Cx<A> u[3][3])
{
    const LT *e = reinterpret_cast<const LT *>(raw.w);
    constexpr int ROWS = R == 18 ? 3 : 2;
#pragma unroll
    for (int r = 0; r < ROWS; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            if constexpr (sizeof(LT) == 2) {
                u[r][c].re = (A)to_f(e[6 * r + 2 * c]);
                u[r][c].im = (A)to_f(e[6 * r + 2 * c + 1]);
            } else {
                u[r][c].re = (A)e[6 * r + 2 * c];
                u[r][c].im = (A)e[6 * r + 2 * c + 1];
            }
        }
    if constexpr (R == 12) {
        Cx<A> a0 = u[0][0], a1 = u[0][1], a2 = u[0][2];
        Cx<A> b0 = u[1][0], b1 = u[1][1], b2 = u[1][2];
        Cx<A> c0 = cmul(a1, b2), c1 = cmul(a2, b0), c2 = cmul(a0, b1);
        Cx<A> d0 = cmul(a2, b1), d1 = cmul(a0, b2), d2 = cmul(a1, b0);
        u[2][0] = {c0.re - d0.re, -(c0.im - d0.im)};
        u[2][1] = {c1.re - d1.re, -(c1.im - d1.im)};
        u[2][2] = {c2.re - d2.re, -(c2.im - d2.im)};
    }
}

template <class LT, int R, class A>
__device__ __forceinline__ void load_link(const char *__restrict__ dirbase, int i, int hs, Cx<A> u[3][3])
{
    RawLink<LT, R> raw;
    load_link_raw<LT, R>(dirbase, i, hs, raw);
    decode_link<LT, R, A>(raw, u);
}

// Colour-vector access --------------------------------------------------

template <class ST> struct Spin {
    ST *v;        // [sites][3] complex
    float *nrm;   // per-site scale (half only)
};

template <class ST, class A>
__device__ __forceinline__ void load_spinor(const Spin<ST> &s, long long i, Cx<A> out[3])
{
    if constexpr (sizeof(ST) == 8) {
        const double2 *p = reinterpret_cast<const double2 *>(s.v) + i * 3;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            double2 v = p[c];
            out[c] = {(A)v.x, (A)v.y};
        }
    } else if constexpr (sizeof(ST) == 4) {
        const float2 *p = reinterpret_cast<const float2 *>(s.v) + i * 3;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            float2 v = p[c];
            out[c] = {(A)v.x, (A)v.y};
        }
    } else {
        const __half2 *p = reinterpret_cast<const __half2 *>(s.v) + i * 3;
        float n = s.nrm[i];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            float2 v = __half22float2(p[c]);
            out[c] = {(A)(v.x * n), (A)(v.y * n)};
        }
    }
}

template <class ST, class A>
__device__ __forceinline__ void store_spinor(const Spin<ST> &s, long long i, const Cx<A> in[3])
{
    if constexpr (sizeof(ST) == 8) {
        double2 *p = reinterpret_cast<double2 *>(s.v) + i * 3;
#pragma unroll
        for (int c = 0; c < 3; c++) p[c] = make_double2((double)in[c].re, (double)in[c].im);
    } else if constexpr (sizeof(ST) == 4) {
        float2 *p = reinterpret_cast<float2 *>(s.v) + i * 3;
#pragma unroll
        for (int c = 0; c < 3; c++) p[c] = make_float2((float)in[c].re, (float)in[c].im);
    } else {
        float m = 0.f;
#pragma unroll
        for (int c = 0; c < 3; c++) m = fmaxf(m, fmaxf(fabsf((float)in[c].re), fabsf((float)in[c].im)));
        float inv = m > 0.f ? 1.f / m : 0.f;
        __half2 *p = reinterpret_cast<__half2 *>(s.v) + i * 3;
#pragma unroll
        for (int c = 0; c < 3; c++)
            p[c] = __floats2half2_rn((float)in[c].re * inv, (float)in[c].im * inv);
        s.nrm[i] = m;
    }
}

}  // namespace hisq
