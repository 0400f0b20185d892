// Launchers of the HISQ link-smearing kernels (FP64).
//
// Working fields are site-planar: a field of nd directions is nd blocks of
// nine planes (the 3x3 elements, row-major), each plane P double2 slots of
// which the first V hold the sites in lex(x) order, so that a wavefront's
// load of one element is one contiguous 1 KiB segment.  P pads V so that
// the planes of a field and successive fields start at different cache
// sets: with P = V a power of two every plane of every field would map the
// same site to the same L2 set, and a pass reading some fifty planes would
// evict its neighbours' lines before they are used again.  The library's
// link arrays ([V][4][3][3] complex, site-major) are converted on the way in
// and out.
#pragma once
#include <hip/hip_runtime.h>

namespace hisq {

struct SmearGeom {
    long long V;
    long long P;   // plane stride (plane_stride(V))
    int L[4];
    int S[4];   // lex strides 1, L0, L0 L1, L0 L1 L2
};

// V rounded up to 128-byte lines plus 37 lines: successive planes start 37
// lines apart, which cycles through every L2 channel and set.
inline long long plane_stride(long long V)
{
    return (V + 7) / 8 * 8 + 296;
}

// fat7(U; c1, c3, c5, c7; cL) in three kinds of pass over planar fields
// (U: the four-direction input); for output direction mu, nu_k denotes the
// k-th direction other than mu (k = 0, 1, 2):
//   pass 1       (every mu in one launch) F_mu = c1 U_mu + c3 sum over k of
//                T1_k, T1_k = H+_k + H-_k, H+_k = U_nu(x) U_mu(x+nu)
//                U_nu(x+mu)^+ and H-_k the -nu staple (nu = nu_k), stored for
//                pass 2 as T1 field 3 mu + k, and with a Lepage term its
//                halves as H fields 6 mu + 2 k (H+) and 6 mu + 2 k + 1 (H-);
//   Lepage       (every mu in one launch) F_mu += cL sum over k of the
//                staple through nu_k of H+_k (+ sign) and H-_k (- sign): the
//                two-step staples;
//   pass 2 (mu)  for each k, sig = nu_k and {nu, rho} the other two:
//                T2_k = staple of T1_nu through rho + staple of T1_rho
//                through nu (all 5-link staples whose steps avoid sig);
//   pass 3 (mu)  F_mu += sum over k of c5 T2_k + c7 (staple of T2_k through
//                sig) (the 7-link staples through sig).
struct Pass1Args {
    const double2 *U;
    double2 *F;    // four fields
    double2 *T1;   // twelve fields, or null: not stored
    double2 *H;    // twenty-four fields, or null: not stored
    double c1, c3;
};
struct LepageArgs {
    const double2 *U;
    const double2 *H;   // the twenty-four H fields of pass 1
    double2 *F;         // four fields, updated
    double cL;
};
struct Pass2Args {
    const double2 *U;
    const double2 *T1;   // the three T1 fields of mu
    double2 *T2;         // three fields
    int mu;
};
struct Pass3Args {
    const double2 *U;
    const double2 *T2;   // three fields
    double2 *F;          // the field of mu
    double c5, c7;
    int mu;
};

hipError_t launch_smear_pass1(const SmearGeom &g, const Pass1Args &a, hipStream_t s);
hipError_t launch_smear_lepage(const SmearGeom &g, const LepageArgs &a, hipStream_t s);
hipError_t launch_smear_pass2(const SmearGeom &g, const Pass2Args &a, hipStream_t s);
hipError_t launch_smear_pass3(const SmearGeom &g, const Pass3Args &a, hipStream_t s);

// Visiting order x, then the directions of `first` (in that order, skipping
// x and repeats), then the rest: the order in which the fermion force's
// staple adjoints visit the sites (the smearing passes instead walk runs of
// time slices per x-y-z tile).
void smear_order(const int *first, int n, int ord[4]);

// [V][4][3][3] complex (site-major) -> four-direction planar field.
hipError_t launch_smear_to_planar(const SmearGeom &g, const double2 *aos, double2 *pl, hipStream_t s);

// Planar four-direction field -> [V][4][3][3].
hipError_t launch_smear_from_planar(const SmearGeom &g, const double2 *pl, double2 *aos, hipStream_t s);

// Unitary polar factor W = V (V^+ V)^{-1/2} of every link of a four-direction
// planar field, in place; *bad (device int) counts links whose V^+ V is not
// positive definite or whose result is not finite.
hipError_t launch_smear_unitarize(const SmearGeom &g, double2 *pl, int *bad, hipStream_t s);

// Final HISQ links with the staggered phases eta_mu(x) folded in:
//   fat_mu(x) = eta_mu(x) X_mu(x),  lng_mu(x) = cN eta_mu(x) W_mu(x) W_mu(x+mu) W_mu(x+2mu)
// X, W planar four-direction fields; fat, lng: [V][4][3][3].
hipError_t launch_smear_output(const SmearGeom &g, const double2 *X, const double2 *W, double cN,
                               double2 *fat, double2 *lng, hipStream_t s);

}  // namespace hisq
