// Device-side types and helpers shared by the HIP kernels of the library.
//
// Lattice geometry: extents L0..L3 (all even), lex(x) = x0 + L0(x1 + L1(x2 + L2 x3)),
// parity (x0+x1+x2+x3) mod 2, a parity-p vector is indexed by cb = lex/2.
// Because L0 is even, cb determines x1..x3 and x0 up to its lowest bit, which
// the parity fixes.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hisq {

constexpr int TILE = 64;        // sites per logical tile (one wavefront)
constexpr int NPART = 8;        // doubles of reduction partials per tile
constexpr int MAXSHIFT = 64;
constexpr int NDIR = 16;        // 4 mu x {+1 fat, -1 fat, +3 long, -3 long}

// Solver status codes kept per problem in device memory.
enum : int {
    ST_RUNNING = 0,
    ST_RELIABLE = 1,   // sloppy loop paused: needs an FP64 reliable update
    ST_RESUME = 2,     // reliable update done, continue iterating
    ST_CONVERGED = 3,
    ST_BREAKDOWN = 4,
    ST_IDLE = 5,       // not part of the current solve
    ST_MS_LAST = 6,    // multi-shift: apply this iteration's shift updates, then stop
};

// One packed link set (precision x reconstruction) of one lattice.
struct LinkSet {
    const void *ptr[2];   // per output parity: [16 dirs][planes][h] chunks
    double a[2];          // per-field scale (fat, long): stored value = link / (a * sign)
    int s[2];             // recon-12 sign of the field (+1 / -1), 0 for recon-18
    int valid;
    int hs;               // plane stride of the packed links, in sites (link_plane_stride(h))
};

// Plane stride (in sites) of a packed link set: h rounded up to 8 sites plus
// 296, i.e. 37 lines of 128 bytes for the 16-byte chunks.  With a stride of
// exactly h the 16 x NQ chunk planes of a parity start at multiples of a
// large power of two whenever the half volume is one (8 MiB at 32^4), so one
// wavefront's loads of a link all fall on the same memory channel and cache
// set; the odd line offset spreads them.
inline long long link_plane_stride(long long h)
{
    return (h + 7) / 8 * 8 + 296;
}

// Precision slots: index = prec * 2 + (recon == 12)
constexpr int NLINKSET = 6;

struct ProbDesc {
    int L[4];
    int h;            // sites per parity
    int tile_begin;   // first logical tile of this problem
    int ntile;        // tiles of this problem
    int fastdiv;      // 1: mdiv[] divides every site index of this lattice exactly
    unsigned mdiv[3]; // ceil(2^32 / L[k]): n / L[k] = umulhi(n, mdiv[k]) when n * L[k] <= 2^32
    int pad;
    long long voff;   // offset (in sites) of this problem's parity vectors
    double diag;      // 4 m^2 (+ base shift)
    double mass;
    LinkSet ls[NLINKSET];
};

// Per-problem solver state (device memory, FP64 scalars).
struct SolveState {
    double rr;        // current (recursive) |r|^2
    double rr_old;    // |r|^2 before the last update (beta denominator)
    double pAp;
    double alpha;
    double beta;
    double bb;        // |b|^2
    double tol2;      // tol^2
    double maxrr;     // max |r|^2 since the last reliable update
    double delta2;    // reliable-update threshold squared
    double rr_true;   // last FP64 true residual^2
    double cplx[8];   // complex scalars (FCG): alpha, beta, (p,q), ...
    int status;
    int iter;
    int reliable;     // reliable updates done
    int maxiter;
    unsigned int counter;  // last-tile ticket for the in-kernel reductions
    int nshift_active;
    long long t_done;      // device clock when it converged
    int restarts;          // reliable updates that restarted p = r
    int pad;
    // state at the start of the current CG iteration, copied by the fused
    // r/x update so that the fused p update can read it while the leading
    // block of each problem writes the new state
    double snap_rr, snap_maxrr;
    int snap_iter, snap_status;
};

// Multi-shift per (problem, rhs) recurrence state
struct ShiftState {
    double zeta[MAXSHIFT];
    double zeta_old[MAXSHIFT];
    double ak[MAXSHIFT];
    double bk[MAXSHIFT];
    double shift[MAXSHIFT];   // sigma_k - sigma_base
    int active[MAXSHIFT];
    int upd[MAXSHIFT];     // shift updated by the current iteration
    int iters[MAXSHIFT];
    double alpha_old, beta_old;
    int nshift;
    int pad;
};

// ---------------------------------------------------------------- geometry

struct Coord {
    int x[4];
};

__device__ __forceinline__ Coord cb_to_coord(int cb, int par, const int L[4])
{
    Coord c;
    int y = 2 * cb;
    int L0 = L[0];
    int r = y / L0;
    int x0e = y - r * L0;
    c.x[1] = r % L[1];
    r /= L[1];
    c.x[2] = r % L[2];
    c.x[3] = r / L[2];
    c.x[0] = x0e + ((par + c.x[1] + c.x[2] + c.x[3]) & 1);
    return c;
}

// cb_to_coord with the three divisions done as multiply-high by the
// descriptor's reciprocals.  With m = ceil(2^32/d) = (2^32 + e)/d, 0 <= e < d,
// n m / 2^32 = n/d + n e / (d 2^32), and the floor is exact when n e < 2^32,
// which n d <= 2^32 guarantees; every numerator here is below V, so the host
// sets fastdiv when V * max(L0, L1, L2) <= 2^32.
__device__ __forceinline__ Coord cb_to_coord_pd(int cb, int par, const ProbDesc &pd)
{
    if (!pd.fastdiv) return cb_to_coord(cb, par, pd.L);
    Coord c;
    const unsigned y = 2u * (unsigned)cb;
    const unsigned r0 = __umulhi(y, pd.mdiv[0]);
    const int x0e = (int)(y - r0 * (unsigned)pd.L[0]);
    const unsigned r1 = __umulhi(r0, pd.mdiv[1]);
    c.x[1] = (int)(r0 - r1 * (unsigned)pd.L[1]);
    const unsigned r2 = __umulhi(r1, pd.mdiv[2]);
    c.x[2] = (int)(r1 - r2 * (unsigned)pd.L[2]);
    c.x[3] = (int)r2;
    c.x[0] = x0e + ((par + c.x[1] + c.x[2] + c.x[3]) & 1);
    return c;
}

__device__ __forceinline__ int coord_to_cb(const int x[4], const int L[4])
{
    return (x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]))) >> 1;
}

__device__ __forceinline__ int wrap(int v, int L)
{
    v = v < 0 ? v + L : v;
    return v >= L ? v - L : v;
}

// cb index of x + k*mu (|k| <= 3 <= L is not required: wraps twice if needed)
__device__ __forceinline__ int hop_cb(Coord c, int mu, int k, const int L[4])
{
    int v = c.x[mu] + k;
    int Lm = L[mu];
    v = ((v % Lm) + Lm) % Lm;
    c.x[mu] = v;
    return coord_to_cb(c.x, L);
}

// staggered phase eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1})
__device__ __forceinline__ int eta_sign(const Coord &c, int mu)
{
    int s = 0;
    for (int nu = 0; nu < mu; nu++) s += c.x[nu];
    return (s & 1) ? -1 : 1;
}

// direction d in [0,16): mu = d >> 2, kind = d & 3: 0 = +1 fat, 1 = -1 fat, 2 = +3 long, 3 = -3 long
__device__ __forceinline__ int dir_step(int d)
{
    int k = d & 3;
    return k == 0 ? 1 : k == 1 ? -1 : k == 2 ? 3 : -3;
}

// ------------------------------------------------------- wave reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// Map a hardware block index to a logical tile so that each XCD (blocks are
// dispatched round-robin over the 8 XCDs) works on a contiguous range of
// tiles, keeping neighbouring spinors in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb, int remap)
{
    if (!remap) return b;
    const int nx = 8;
    int per = nb / nx, rem = nb % nx;
    int x = b % nx, k = b / nx;
    // XCD x owns tiles [x*per + min(x,rem), ...) of length per + (x < rem)
    int start = x * per + (x < rem ? x : rem);
    int len = per + (x < rem ? 1 : 0);
    return k < len ? start + k : b;  // b beyond the even split: identity (never happens when nb % 8 == 0)
}

}  // namespace hisq
