// FP64 3x3 complex matrices in registers, loaded from and stored to
// site-planar fields (nine planes, element (i, j) in plane 3i + j; the
// argument V of ld / st is the plane stride, SmearGeom::P), and the lattice
// shifts the link kernels use.
#pragma once
#include <hip/hip_runtime.h>

#include "smear.h"

namespace hisq {
namespace su3 {

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

// Stores are non-temporal: the passes write as many bytes as they read or
// more (pass 1 four times as many), and write-allocated lines would push the
// neighbour links the next sites reuse out of L2.  Every stored field is read
// again only by a later launch.
typedef double nt_double2 __attribute__((ext_vector_type(2)));

// A load of a field element that no other site reads again (non-temporal, so
// that it does not push reusable lines out of L2).
__device__ __forceinline__ M3 ld_nt(const double2 *__restrict__ f, size_t V, long long s)
{
    M3 m;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const nt_double2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_double2 *>(f + i * V + s));
        m.e[i] = make_double2(v.x, v.y);
    }
    return m;
}

__device__ __forceinline__ void st(double2 *__restrict__ f, size_t V, long long s, const M3 &m)
{
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const nt_double2 v = {m.e[i].x, m.e[i].y};
        __builtin_nontemporal_store(v, reinterpret_cast<nt_double2 *>(f + i * V + s));
    }
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

// a^+
__device__ __forceinline__ M3 dag(const M3 &a)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) c.e[3 * i + j] = make_double2(a.e[3 * j + i].x, -a.e[3 * j + i].y);
    return c;
}

// a + b
__device__ __forceinline__ M3 add(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 9; i++) c.e[i] = make_double2(a.e[i].x + b.e[i].x, a.e[i].y + b.e[i].y);
    return c;
}

__device__ __forceinline__ M3 zero3()
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 9; i++) c.e[i] = make_double2(0.0, 0.0);
    return c;
}

// Sites are visited in the order of the axis permutation o (o[0] = 0, x
// fastest, so that a wavefront's loads stay contiguous): the host puts the
// directions a pass steps along right after x, so that a site's neighbours
// along them are visited, and held in L2 / the Infinity Cache, soon after it.
// Returns lex(x) for visit index i and the coordinates c[k] along o[k].
__device__ __forceinline__ long long walk(unsigned i, const SmearGeom &g, const int o[4], int c[4])
{
    const unsigned L0 = (unsigned)pick(g.L, o[0]), L1 = (unsigned)pick(g.L, o[1]), L2 = (unsigned)pick(g.L, o[2]);
    c[0] = (int)(i % L0);
    i /= L0;
    c[1] = (int)(i % L1);
    i /= L1;
    c[2] = (int)(i % L2);
    c[3] = (int)(i / L2);
    return (long long)c[0] * pick(g.S, o[0]) + (long long)c[1] * pick(g.S, o[1]) + (long long)c[2] * pick(g.S, o[2]) +
           (long long)c[3] * pick(g.S, o[3]);
}

__device__ __forceinline__ int coord(const int c[4], const int o[4], int d)
{
    return o[0] == d ? c[0] : o[1] == d ? c[1] : o[2] == d ? c[2] : c[3];
}

}  // namespace su3
}  // namespace hisq
