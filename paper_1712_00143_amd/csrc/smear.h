// Launchers of the HISQ link-smearing kernels (FP64).
//
// Working fields are site-planar: a field of nd directions is nd blocks of
// nine planes (the 3x3 elements, row-major), each plane V double2 values
// indexed by lex(x), so that a wavefront's load of one element is one
// contiguous 1 KiB segment.  The library's link arrays ([V][4][3][3]
// complex, site-major) are converted on the way in and out.
#pragma once
#include <hip/hip_runtime.h>

namespace hisq {

struct SmearGeom {
    long long V;
    int L[4];
    int S[4];   // lex strides 1, L0, L0 L1, L0 L1 L2
};

// One staple pass for output direction mu through direction nu:
//   T(x) = U_nu(x) M(x+nu) U_nu(x+mu)^+ + U_nu(x-nu)^+ M(x-nu) U_nu(x-nu+mu)
//   F(x) = (init ? cM M(x) : F(x)) + cT T(x) [+ cL * the two-step (Lepage) staple]
// T is stored when T_out is not null.  Un, M, F, T_out: one-direction planar fields.
struct StapleArgs {
    const double2 *Un;
    const double2 *M;
    double2 *F;
    double2 *T_out;
    double cM, cT, cL;
    int init;
    int mu, nu;
};

hipError_t launch_smear_staple(const SmearGeom &g, const StapleArgs &a, hipStream_t s);

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
