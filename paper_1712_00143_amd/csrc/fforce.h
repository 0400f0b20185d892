// Launchers of the HISQ fermion-force kernels (FP64).  Fields are the
// site-planar link fields of smear.h; gradients G of a real scalar Q with
// respect to a link field Y are fields with dQ = sum Re Tr(dY_mu(x) G_mu(x)).
#pragma once
#include <hip/hip_runtime.h>

#include "smear.h"

namespace hisq {

// Gradients of Q = sum_k alpha_k X_k^+ A X_k with respect to the fat and long
// links, from the even vectors X_k and Y_k = D_oe X_k ([n][h][3] complex
// each): with Psi = (X on even, Y on odd sites) and eps = +1 / -1 on even /
// odd sites,
//   OF_mu(x) = -2 eps(x) sum_k alpha_k Psi_k(x+mu) Psi_k(x)^+,
//   OL_mu(x) = -2 eps(x) sum_k alpha_k Psi_k(x+3mu) Psi_k(x)^+.
// fold: write eta_mu(x) OF and cN eta_mu(x) OL instead (the gradients with
// respect to the unphased level-2 sum and the Naik product).
struct OuterArgs {
    const double2 *X, *Y;
    const double *alpha;
    int n;
    long long h;
    double2 *OF, *OL;   // four planar fields each
    int fold;
    double cN;
};
hipError_t launch_ff_outer(const SmearGeom &g, const OuterArgs &a, hipStream_t s);

// Adjoint of the staple of M through direction d for output direction mu,
//   T(x) = sum_s L_s(x) M_s(x+s) L_s(x+mu)^+   (s = +d, -d; L_{+d}(x) = U_d(x),
//                                              L_{-d}(x) = U_d(x-d)^+),
// for the gradient G_s of T (each sign its own field, the sum of G[s][0]
// and, if not null, G[s][1]), scaled by c:
//   GM[s] (= or +=)  the gradient with respect to M_s (GM[0] may equal GM[1]),
//   GUd +=           the gradient with respect to the links U_d.
// Sign index 0 is +d, 1 is -d; M[s] null leaves that sign out; GM[s] and
// GUd may be null.  With one field for both signs (GM[0] == GM[1]) and Gb
// not null, that field also receives gb Gb:
//   GM = (gm_init ? 0 : GM) + gb Gb + c (adjoint),
// the initial share a gradient field takes directly from G (the one-link
// and lower staple terms), so that no separate pass writes it.
struct StapleAdjArgs {
    const double2 *Ud;
    const double2 *M[2];
    const double2 *G[2][2];
    double2 *GM[2];
    double2 *GUd;
    double c;
    int mu, d, gm_init;
    int ord[4];
    const double2 *Gb;
    double gb;
};
hipError_t launch_staple_adjoint(const SmearGeom &g, const StapleAdjArgs &a, hipStream_t s);

// GW += gradient of sum Re Tr(N_mu(x) GN_mu(x)), N_mu(x) = W_mu(x) W_mu(x+mu) W_mu(x+2mu)
// (four-direction planar fields).
hipError_t launch_ff_naik_adjoint(const SmearGeom &g, const double2 *W, const double2 *GN, double2 *GW,
                                  hipStream_t s);

// In place: G <- gradient with respect to V of Re Tr(W(V) G), W = V (V^+ V)^{-1/2},
// four-direction planar fields.
hipError_t launch_ff_unitarize_adjoint(const SmearGeom &g, const double2 *V, double2 *G, hipStream_t s);

// out = a * out + b * in over n double2 (a = 0: out = b * in, out not read).
hipError_t launch_field_axpby(double2 *out, double a, const double2 *in, double b, size_t n, hipStream_t s);

// F_mu(x) = TA[U_mu(x) G_mu(x)] (four-direction planar fields; F may alias G).
hipError_t launch_ff_project(const SmearGeom &g, const double2 *U, const double2 *G, double2 *F, hipStream_t s);

}  // namespace hisq
