/*
 * CPU oracle for the HISQ staggered even-odd solver hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 statement of
 * what the GPU library computes.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the library never does, and the
 * two share no code, headers or tables.
 *
 * The paper (Sections 4 and 4.1) benchmarks the staggered single-mass and
 * multi-shift conjugate gradient of MILC's HISQ action, a matrix-vector
 * stencil at low arithmetic intensity (Section 4.2, the 0.26 flop/byte
 * figure).  It never writes the operator down, so the definitions below are
 * the standard ones, stated here:
 *
 *   geometry  lex(x) = x0 + L0 (x1 + L1 (x2 + L2 x3)), periodic, parity
 *             (x0+x1+x2+x3) mod 2; even-parity vectors are indexed by lex/2.
 *   Dslash    (D psi)(x) = sum_mu [ F_mu(x) psi(x+mu) - F_mu(x-mu)^+ psi(x-mu)
 *                                 + L_mu(x) psi(x+3mu) - L_mu(x-3mu)^+ psi(x-3mu) ]
 *             with the staggered phases already folded into F (fat) and L
 *             (long); no factor 1/2.  M = 2m + D, so on even sites
 *             M^+M = A = 4 m^2 - D_eo D_oe.
 *   CG        Hestenes-Stiefel on A (+ sigma), true-residual restart.
 *   MS-CG     shifted CG with collinear residuals (Jegerlehner,
 *             hep-lat/9612014), base system = smallest shift.
 *   PTC       gauge-covariant parallel-transport convolution layer and its
 *             exact adjoint (input and weight gradients).
 *   FCG       flexible CG with truncation 1 (Notay 2000) with the PTC network
 *             as preconditioner.
 *   smearing  HISQ fat and long links from thin links: two fat7 levels
 *             with a U(3) polar projection between, Lepage and Naik terms
 *             at the second (stated with the code below).
 *   gauge     Symanzik-improved (plaquette, rectangle, parallelogram)
 *   force     gauge action and its force (stated with the code below).
 *   fermion   adjoints (link gradients) of fat7 and of the Naik product
 *   force     for the chain rule of the HISQ fermion force; the rest of that
 *             force is composed in the Python module.
 *
 * Complex numbers are C99 double complex; fields are site-major:
 *   links   [V][4][3][3]          (row-major 3x3)
 *   vectors [V][3] (full) or [V/2][3] (one parity, index lex/2)
 *   PTC activations [C][V][3], weights [Cout][Cin][9] with path
 *   0 = identity, 1+2mu = +mu hop F_mu(x) psi(x+mu),
 *   2+2mu = -mu hop F_mu(x-mu)^+ psi(x-mu).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ---------------------------------------------------------------- geometry */

static long vol(const int d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

static void coords_of(const int d[4], long s, int x[4])
{
    x[0] = (int)(s % d[0]); s /= d[0];
    x[1] = (int)(s % d[1]); s /= d[1];
    x[2] = (int)(s % d[2]); s /= d[2];
    x[3] = (int)s;
}

static long lex_of(const int d[4], const int x[4])
{
    return x[0] + (long)d[0] * (x[1] + (long)d[1] * (x[2] + (long)d[2] * x[3]));
}

/* site reached from s by k steps along mu, periodic */
static long hop(const int d[4], long s, int mu, int k)
{
    int x[4];
    coords_of(d, s, x);
    x[mu] = ((x[mu] + k) % d[mu] + d[mu]) % d[mu];
    return lex_of(d, x);
}

static int parity_of(const int d[4], long s)
{
    int x[4];
    coords_of(d, s, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* ------------------------------------------------------- 3x3 helpers */

/* y += U v */
static void mv_add(cplx *y, const cplx *U, const cplx *v, cplx c)
{
    for (int i = 0; i < 3; i++) {
        cplx a = 0;
        for (int j = 0; j < 3; j++) a += U[3 * i + j] * v[j];
        y[i] += c * a;
    }
}

/* y += U^+ v */
static void mhv_add(cplx *y, const cplx *U, const cplx *v, cplx c)
{
    for (int i = 0; i < 3; i++) {
        cplx a = 0;
        for (int j = 0; j < 3; j++) a += conj(U[3 * j + i]) * v[j];
        y[i] += c * a;
    }
}

static const cplx *link(const cplx *f, long s, int mu) { return f + (s * 4 + mu) * 9; }

/* ------------------------------------------------------------- Dslash */

/* Full-lattice D (eq. above).  in, out: [V][3]. */
void orc_dslash_full(const int d[4], const cplx *fat, const cplx *lng,
                     const cplx *in, cplx *out)
{
    long V = vol(d);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx acc[3] = {0, 0, 0};
        for (int mu = 0; mu < 4; mu++) {
            long sp1 = hop(d, s, mu, 1), sm1 = hop(d, s, mu, -1);
            long sp3 = hop(d, s, mu, 3), sm3 = hop(d, s, mu, -3);
            mv_add(acc, link(fat, s, mu), in + 3 * sp1, 1.0);
            mhv_add(acc, link(fat, sm1, mu), in + 3 * sm1, -1.0);
            mv_add(acc, link(lng, s, mu), in + 3 * sp3, 1.0);
            mhv_add(acc, link(lng, sm3, mu), in + 3 * sm3, -1.0);
        }
        for (int c = 0; c < 3; c++) out[3 * s + c] = acc[c];
    }
}

/* Half-lattice D restricted to output parity `par` (0: D_eo, 1: D_oe).
 * in_half: [V/2][3] on parity 1-par, out_half: [V/2][3] on parity par,
 * both indexed by lex/2. */
void orc_dslash_half(const int d[4], const cplx *fat, const cplx *lng, int par,
                     const cplx *in_half, cplx *out_half)
{
    long V = vol(d);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        if (parity_of(d, s) != par) continue;
        cplx acc[3] = {0, 0, 0};
        for (int mu = 0; mu < 4; mu++) {
            long sp1 = hop(d, s, mu, 1), sm1 = hop(d, s, mu, -1);
            long sp3 = hop(d, s, mu, 3), sm3 = hop(d, s, mu, -3);
            mv_add(acc, link(fat, s, mu), in_half + 3 * (sp1 / 2), 1.0);
            mhv_add(acc, link(fat, sm1, mu), in_half + 3 * (sm1 / 2), -1.0);
            mv_add(acc, link(lng, s, mu), in_half + 3 * (sp3 / 2), 1.0);
            mhv_add(acc, link(lng, sm3, mu), in_half + 3 * (sm3 / 2), -1.0);
        }
        for (int c = 0; c < 3; c++) out_half[3 * (s / 2) + c] = acc[c];
    }
}

/* out = (4 m^2 + sigma) in - D_eo D_oe in, on even vectors */
void orc_apply_A(const int d[4], const cplx *fat, const cplx *lng, double mass,
                 double sigma, const cplx *in, cplx *out)
{
    long h3 = vol(d) / 2 * 3;
    cplx *t = malloc(sizeof(cplx) * h3);
    orc_dslash_half(d, fat, lng, 1, in, t);
    orc_dslash_half(d, fat, lng, 0, t, out);
    double diag = 4.0 * mass * mass + sigma;
    for (long i = 0; i < h3; i++) out[i] = diag * in[i] - out[i];
    free(t);
}

/* ------------------------------------------------------- vector helpers */

static double nrm2(const cplx *a, long n)
{
    double s = 0;
    for (long i = 0; i < n; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

static cplx dotc(const cplx *a, const cplx *b, long n) /* a^+ b */
{
    cplx s = 0;
    for (long i = 0; i < n; i++) s += conj(a[i]) * b[i];
    return s;
}

/* ||b - (A+sigma) x|| / ||b|| */
double orc_true_residual(const int d[4], const cplx *fat, const cplx *lng, double mass,
                         double sigma, const cplx *b, const cplx *x)
{
    long n = vol(d) / 2 * 3;
    cplx *Ax = malloc(sizeof(cplx) * n);
    orc_apply_A(d, fat, lng, mass, sigma, x, Ax);
    double rr = 0;
    for (long i = 0; i < n; i++) {
        cplx r = b[i] - Ax[i];
        rr += creal(r) * creal(r) + cimag(r) * cimag(r);
    }
    free(Ax);
    return sqrt(rr / nrm2(b, n));
}

/* ------------------------------------------------------------------ CG */

/* Conjugate gradient on (A + sigma) x = b.  x is the initial guess on entry
 * (pass zeros for a cold start).  Stops when the recursive residual reaches
 * tol*||b||, then recomputes the true residual and restarts from x if that is
 * still above tol.  Returns 0 on convergence, 1 otherwise; *iters is the
 * total iteration count and *true_rel the final true relative residual. */
int orc_cg(const int d[4], const cplx *fat, const cplx *lng, double mass, double sigma,
           const cplx *b, cplx *x, double tol, int maxiter, int *iters, double *true_rel)
{
    long n = vol(d) / 2 * 3;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n),
         *Ap = malloc(sizeof(cplx) * n);
    double bb = nrm2(b, n);
    int it = 0, ok = 0;
    for (int restart = 0; restart < 10 && it < maxiter; restart++) {
        orc_apply_A(d, fat, lng, mass, sigma, x, Ap);
        for (long i = 0; i < n; i++) r[i] = b[i] - Ap[i];
        double rr = nrm2(r, n);
        if (rr <= tol * tol * bb) { ok = 1; break; }
        memcpy(p, r, sizeof(cplx) * n);
        while (it < maxiter) {
            orc_apply_A(d, fat, lng, mass, sigma, p, Ap);
            double pAp = creal(dotc(p, Ap, n));
            double alpha = rr / pAp;
            for (long i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
            double rr_new = nrm2(r, n);
            it++;
            if (rr_new <= tol * tol * bb) break;
            double beta = rr_new / rr;
            for (long i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
            rr = rr_new;
        }
        double tr = orc_true_residual(d, fat, lng, mass, sigma, b, x);
        if (tr <= tol) { ok = 1; break; }
    }
    *iters = it;
    *true_rel = orc_true_residual(d, fat, lng, mass, sigma, b, x);
    free(r); free(p); free(Ap);
    return ok ? 0 : 1;
}

/* ---------------------------------------------------------- multi-shift CG */

/* Solves (A + shifts[k]) x_k = b for all k with one Krylov space built on the
 * smallest shift.  x: [nshift][V/2][3] (overwritten; cold start).  Shift k
 * stops updating once |zeta_k| ||r|| <= tol ||b||.  Afterwards each shift
 * whose true residual is above tol is refined with orc_cg from its x_k.
 * iters[k]: Krylov iterations that updated shift k (plus refinement);
 * rel[k]: final true relative residual. */
int orc_multishift(const int d[4], const cplx *fat, const cplx *lng, double mass,
                   int nshift, const double *shifts, const cplx *b, cplx *x,
                   double tol, int maxiter, int *iters, double *rel)
{
    long n = vol(d) / 2 * 3;
    int k0 = 0;
    for (int k = 1; k < nshift; k++) if (shifts[k] < shifts[k0]) k0 = k;
    double s0 = shifts[k0];
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n),
         *Ap = malloc(sizeof(cplx) * n), *ps = malloc(sizeof(cplx) * n * nshift);
    double *zeta = malloc(sizeof(double) * nshift), *zeta_old = malloc(sizeof(double) * nshift);
    int *active = malloc(sizeof(int) * nshift);
    double bb = nrm2(b, n);
    memcpy(r, b, sizeof(cplx) * n);
    memcpy(p, b, sizeof(cplx) * n);
    for (int k = 0; k < nshift; k++) {
        memcpy(ps + k * n, b, sizeof(cplx) * n);
        memset(x + k * n, 0, sizeof(cplx) * n);
        zeta[k] = zeta_old[k] = 1.0;
        active[k] = 1;
        iters[k] = 0;
    }
    double rr = bb, alpha_old = 1.0, beta_old = 0.0;
    int it = 0;
    while (it < maxiter) {
        orc_apply_A(d, fat, lng, mass, s0, p, Ap);
        double alpha = rr / creal(dotc(p, Ap, n));
        for (long i = 0; i < n; i++) r[i] -= alpha * Ap[i];
        double rr_new = nrm2(r, n);
        double beta = rr_new / rr;
        int any = 0;
        for (int k = 0; k < nshift; k++) {
            if (!active[k]) continue;
            double dk = shifts[k] - s0;
            double z = zeta[k], zo = zeta_old[k];
            double zn = z * zo * alpha_old /
                        (alpha * beta_old * (zo - z) + zo * alpha_old * (1.0 + dk * alpha));
            double ak = alpha * zn / z;
            double bk = beta * (zn / z) * (zn / z);
            cplx *xk = x + k * n, *pk = ps + k * n;
            for (long i = 0; i < n; i++) {
                xk[i] += ak * pk[i];
                pk[i] = zn * r[i] + bk * pk[i];
            }
            zeta_old[k] = z;
            zeta[k] = zn;
            iters[k]++;
            if (fabs(zn) * sqrt(rr_new) <= tol * sqrt(bb)) active[k] = 0;
            else any = 1;
        }
        for (long i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        alpha_old = alpha;
        beta_old = beta;
        it++;
        if (!any) break;
    }
    int ok = 1;
    for (int k = 0; k < nshift; k++) {
        double tr = orc_true_residual(d, fat, lng, mass, shifts[k], b, x + k * n);
        if (tr > tol) {
            int more = 0;
            double tr2;
            if (orc_cg(d, fat, lng, mass, shifts[k], b, x + k * n, tol, maxiter, &more, &tr2))
                ok = 0;
            iters[k] += more;
        }
        rel[k] = orc_true_residual(d, fat, lng, mass, shifts[k], b, x + k * n);
    }
    free(r); free(p); free(Ap); free(ps); free(zeta); free(zeta_old); free(active);
    return ok ? 0 : 1;
}

/* ------------------------------------------------------------ PTC layer */

/* out[c](x) = sum_{c'} sum_k w[c][c'][k] (T_k in[c'])(x),
 *   T_0 psi = psi, T_{1+2mu} psi(x) = F_mu(x) psi(x+mu),
 *   T_{2+2mu} psi(x) = F_mu(x-mu)^+ psi(x-mu).
 * in: [cin][V][3], out: [cout][V][3], w: [cout][cin][9]. */
void orc_ptc_layer(const int d[4], const cplx *fat, int cin, int cout, const cplx *w,
                   const cplx *in, cplx *out)
{
    long V = vol(d);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        for (int c = 0; c < cout; c++) {
            cplx acc[3] = {0, 0, 0};
            for (int cp = 0; cp < cin; cp++) {
                const cplx *wk = w + ((long)c * cin + cp) * 9;
                const cplx *ps = in + (long)cp * V * 3;
                for (int j = 0; j < 3; j++) acc[j] += wk[0] * ps[3 * s + j];
                for (int mu = 0; mu < 4; mu++) {
                    long sp = hop(d, s, mu, 1), sm = hop(d, s, mu, -1);
                    mv_add(acc, link(fat, s, mu), ps + 3 * sp, wk[1 + 2 * mu]);
                    mhv_add(acc, link(fat, sm, mu), ps + 3 * sm, wk[2 + 2 * mu]);
                }
            }
            for (int j = 0; j < 3; j++) out[((long)c * V + s) * 3 + j] = acc[j];
        }
    }
}

/* Adjoint of orc_ptc_layer for a real loss.  With g_out = dL/dRe(out) +
 * i dL/dIm(out):
 *   g_in[c'](y) = sum_c [ conj(w0) g_c(y) + sum_mu conj(w_{+mu}) F_mu(y-mu)^+ g_c(y-mu)
 *                                        + conj(w_{-mu}) F_mu(y) g_c(y+mu) ]
 *   g_w[c][c'][k] = sum_x (T_k in[c'])(x)^+ g_c(x).
 * g_in may be NULL (first layer). */
void orc_ptc_layer_adj(const int d[4], const cplx *fat, int cin, int cout, const cplx *w,
                       const cplx *in, const cplx *gout, cplx *gin, cplx *gw)
{
    long V = vol(d);
    if (gin) {
#pragma omp parallel for schedule(static)
        for (long s = 0; s < V; s++) {
            for (int cp = 0; cp < cin; cp++) {
                cplx acc[3] = {0, 0, 0};
                for (int c = 0; c < cout; c++) {
                    const cplx *wk = w + ((long)c * cin + cp) * 9;
                    const cplx *g = gout + (long)c * V * 3;
                    for (int j = 0; j < 3; j++) acc[j] += conj(wk[0]) * g[3 * s + j];
                    for (int mu = 0; mu < 4; mu++) {
                        long sp = hop(d, s, mu, 1), sm = hop(d, s, mu, -1);
                        mhv_add(acc, link(fat, sm, mu), g + 3 * sm, conj(wk[1 + 2 * mu]));
                        mv_add(acc, link(fat, s, mu), g + 3 * sp, conj(wk[2 + 2 * mu]));
                    }
                }
                for (int j = 0; j < 3; j++) gin[((long)cp * V + s) * 3 + j] = acc[j];
            }
        }
    }
    if (!gw) return;
    for (int c = 0; c < cout; c++)
        for (int cp = 0; cp < cin; cp++) {
            cplx sum[9] = {0};
            const cplx *ps = in + (long)cp * V * 3;
            const cplx *g = gout + (long)c * V * 3;
            for (long s = 0; s < V; s++) {
                cplx t[9][3];
                memset(t, 0, sizeof t);
                for (int j = 0; j < 3; j++) t[0][j] = ps[3 * s + j];
                for (int mu = 0; mu < 4; mu++) {
                    long sp = hop(d, s, mu, 1), sm = hop(d, s, mu, -1);
                    mv_add(t[1 + 2 * mu], link(fat, s, mu), ps + 3 * sp, 1.0);
                    mhv_add(t[2 + 2 * mu], link(fat, sm, mu), ps + 3 * sm, 1.0);
                }
                for (int k = 0; k < 9; k++)
                    for (int j = 0; j < 3; j++) sum[k] += conj(t[k][j]) * g[3 * s + j];
            }
            for (int k = 0; k < 9; k++) gw[((long)c * cin + cp) * 9 + k] = sum[k];
        }
}

/* -------------------------------------------------- PTC network + FCG */

/* Preconditioner z = M(r) on even vectors, M = 1 + E^+ K^+ K E: embed r on
 * even sites (zeros on odd), apply the nlayer PTC layers K = L_n ... L_1
 * (channel counts chans[0..nlayer], chans[0] = 1), then their adjoints in
 * reverse order, project the output onto even sites and add r.  M is
 * Hermitian positive definite by construction, as the inverse it
 * approximates is, and M = 1 (plain CG) when the weights vanish.  weights:
 * concatenation of every layer's [Cout][Cin][9] block. */
void orc_ptc_apply(const int d[4], const cplx *fat, int nlayer, const int *chans,
                   const cplx *weights, const cplx *r_even, cplx *z_even)
{
    long V = vol(d);
    int cmax = 1;
    for (int l = 0; l <= nlayer; l++) if (chans[l] > cmax) cmax = chans[l];
    cplx *a = calloc((size_t)cmax * V * 3, sizeof(cplx));
    cplx *b = calloc((size_t)cmax * V * 3, sizeof(cplx));
    for (long s = 0; s < V; s++)
        if (parity_of(d, s) == 0)
            for (int j = 0; j < 3; j++) a[3 * s + j] = r_even[3 * (s / 2) + j];
    const cplx *w = weights;
    for (int l = 0; l < nlayer; l++) {
        orc_ptc_layer(d, fat, chans[l], chans[l + 1], w, a, b);
        w += (long)chans[l] * chans[l + 1] * 9;
        cplx *t = a; a = b; b = t;
    }
    for (int l = nlayer - 1; l >= 0; l--) {
        w -= (long)chans[l] * chans[l + 1] * 9;
        orc_ptc_layer_adj(d, fat, chans[l], chans[l + 1], w, NULL, a, b, NULL);
        cplx *t = a; a = b; b = t;
    }
    for (long s = 0; s < V; s++)
        if (parity_of(d, s) == 0)
            for (int j = 0; j < 3; j++)
                z_even[3 * (s / 2) + j] = r_even[3 * (s / 2) + j] + a[3 * s + j];
    free(a); free(b);
}

/* Flexible CG, truncation 1, on A x = b with z = M(r) (M = the PTC network
 * above, or the identity when nlayer == 0):
 *   r = b - A x, z = M(r), p = z; repeat { q = A p; alpha = (p,r)/(p,q);
 *   x += alpha p; r -= alpha q; z = M(r); beta = -(q,z)/(q,p); p = z + beta p },
 * with (a,b) = a^+ b.  beta makes the new p A-orthogonal to the old one,
 * (p_new, A p_old) = 0; for complex vectors that puts q in the first slot.
 * Stop on the recursive residual, then check the true residual and restart
 * from x if needed.  Returns 0 on convergence. */
int orc_fcg(const int d[4], const cplx *fat, const cplx *lng, double mass, int nlayer,
            const int *chans, const cplx *weights, const cplx *b, cplx *x, double tol,
            int maxiter, int *iters, double *true_rel)
{
    long n = vol(d) / 2 * 3;
    cplx *r = malloc(sizeof(cplx) * n), *z = malloc(sizeof(cplx) * n),
         *p = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    double bb = nrm2(b, n);
    int it = 0, ok = 0;
    for (int restart = 0; restart < 10 && it < maxiter; restart++) {
        orc_apply_A(d, fat, lng, mass, 0.0, x, q);
        for (long i = 0; i < n; i++) r[i] = b[i] - q[i];
        if (nrm2(r, n) <= tol * tol * bb) { ok = 1; break; }
        if (nlayer > 0) orc_ptc_apply(d, fat, nlayer, chans, weights, r, z);
        else memcpy(z, r, sizeof(cplx) * n);
        memcpy(p, z, sizeof(cplx) * n);
        while (it < maxiter) {
            orc_apply_A(d, fat, lng, mass, 0.0, p, q);
            cplx pq = dotc(p, q, n);
            cplx alpha = dotc(p, r, n) / pq;
            for (long i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            it++;
            if (nrm2(r, n) <= tol * tol * bb) break;
            if (nlayer > 0) orc_ptc_apply(d, fat, nlayer, chans, weights, r, z);
            else memcpy(z, r, sizeof(cplx) * n);
            cplx beta = -dotc(q, z, n) / conj(pq);
            for (long i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        }
        if (orc_true_residual(d, fat, lng, mass, 0.0, b, x) <= tol) { ok = 1; break; }
    }
    *iters = it;
    *true_rel = orc_true_residual(d, fat, lng, mass, 0.0, b, x);
    free(r); free(z); free(p); free(q);
    return ok ? 0 : 1;
}

/* ------------------------------------------------------------ link smearing
 *
 * HISQ fat and long links from thin SU(3) links U (the smearing the paper's
 * run-time breakdown lists beside the forces, Section 2; its definition is
 * that of the HISQ action, Follana et al., hep-lat/0610092):
 *
 *   level 1   V = fat7(U; 1/8, 1/16, 1/64, 1/384; Lepage 0)
 *   project   W = V (V^+ V)^{-1/2}, the unitary factor of the polar
 *             decomposition (the nearest U(3) matrix)
 *   level 2   X = fat7(W; 5/8, 1/16, 1/64, 1/384; Lepage -1/16)
 *             N_mu(x) = W_mu(x) W_mu(x+mu) W_mu(x+2mu)
 *   output    F_mu(x) = eta_mu(x) X_mu(x),  L_mu(x) = -(1/24) eta_mu(x) N_mu(x)
 *
 * fat7(U; c1, c3, c5, c7; cL)_mu(x) = c1 U_mu(x) + sum over the paths from x to
 * x+mu listed below, each weighted by its class coefficient, of the product of
 * the links along the path:
 *   3-staples  (s nu, mu, -s nu)                           6 paths, c3
 *   5-staples  (s nu, t rho, mu, -t rho, -s nu)            24 paths, c5
 *   7-staples  (s nu, t rho, u sig, mu, -u sig, -t rho, -s nu)  48 paths, c7
 *   Lepage     (s nu, s nu, mu, -s nu, -s nu)              6 paths, cL
 * with nu, rho, sig distinct directions other than mu and s, t, u = +-1.  A
 * step +nu from y multiplies by U_nu(y) and moves to y+nu; a step -nu moves to
 * y-nu and multiplies by U_nu(y-nu)^+.  With unit links X = 9/8 and the Naik
 * coefficient -1/24 makes the free derivative exact to O(p^4).
 */

/* c = a b */
static void mm(cplx *c, const cplx *a, const cplx *b)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = s;
        }
}

/* Product of the links along a path of n signed steps (+(mu+1) or -(mu+1))
 * starting at site s; P receives the 3x3 product. */
static void path_product(const int d[4], const cplx *U, long s, const int *steps, int n, cplx *P)
{
    for (int i = 0; i < 9; i++) P[i] = (i % 4 == 0) ? 1.0 : 0.0;
    long cur = s;
    for (int k = 0; k < n; k++) {
        int mu = abs(steps[k]) - 1;
        cplx M[9], T[9];
        if (steps[k] > 0) {
            memcpy(M, link(U, cur, mu), sizeof M);
            cur = hop(d, cur, mu, 1);
        } else {
            cur = hop(d, cur, mu, -1);
            const cplx *u = link(U, cur, mu);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) M[3 * i + j] = conj(u[3 * j + i]);
        }
        mm(T, P, M);
        memcpy(P, T, sizeof T);
    }
}

static void acc_path(const int d[4], const cplx *U, long s, const int *steps, int n, double c, cplx *out)
{
    cplx P[9];
    path_product(d, U, s, steps, n, P);
    for (int i = 0; i < 9; i++) out[i] += c * P[i];
}

/* fat7 with coefficients c = {c1, c3, c5, c7, cL}; U, out: [V][4][3][3]. */
void orc_fat7(const int d[4], const double c[5], const cplx *U, cplx *out)
{
    const long V = vol(d);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++)
        for (int mu = 0; mu < 4; mu++) {
            cplx *o = out + (s * 4 + mu) * 9;
            const cplx *u = link(U, s, mu);
            for (int i = 0; i < 9; i++) o[i] = c[0] * u[i];
            const int M = mu + 1;
            for (int nu = 0; nu < 4; nu++) {
                if (nu == mu) continue;
                for (int sn = -1; sn <= 1; sn += 2) {
                    const int N = sn * (nu + 1);
                    const int p3[3] = {N, M, -N};
                    acc_path(d, U, s, p3, 3, c[1], o);
                    const int pl[5] = {N, N, M, -N, -N};
                    if (c[4] != 0.0) acc_path(d, U, s, pl, 5, c[4], o);
                    for (int rho = 0; rho < 4; rho++) {
                        if (rho == mu || rho == nu) continue;
                        for (int sr = -1; sr <= 1; sr += 2) {
                            const int R = sr * (rho + 1);
                            const int p5[5] = {N, R, M, -R, -N};
                            acc_path(d, U, s, p5, 5, c[2], o);
                            for (int sig = 0; sig < 4; sig++) {
                                if (sig == mu || sig == nu || sig == rho) continue;
                                for (int ss = -1; ss <= 1; ss += 2) {
                                    const int S = ss * (sig + 1);
                                    const int p7[7] = {N, R, S, M, -S, -R, -N};
                                    acc_path(d, U, s, p7, 7, c[3], o);
                                }
                            }
                        }
                    }
                }
            }
        }
}

/* inverse of a 3x3 complex matrix by cofactors; returns the determinant */
static cplx inv3(const cplx *a, cplx *r)
{
    cplx c[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            c[3 * i + j] = a[3 * i1 + j1] * a[3 * i2 + j2] - a[3 * i1 + j2] * a[3 * i2 + j1];
        }
    cplx det = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r[3 * i + j] = c[3 * j + i] / det;
    return det;
}

/* Unitary polar factor of each of n 3x3 matrices by Newton's iteration
 * X <- (X + X^{-+}) / 2 (Higham, Functions of Matrices, ch. 8), which
 * converges quadratically to V (V^+ V)^{-1/2} for non-singular V.  Returns
 * the number of matrices that did not converge in 100 steps (0 on success). */
int orc_unitarize(long n, const cplx *in, cplx *out)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long m = 0; m < n; m++) {
        cplx X[9], Y[9];
        memcpy(X, in + m * 9, sizeof X);
        int ok = 0;
        for (int it = 0; it < 100; it++) {
            cplx det = inv3(X, Y);
            if (cabs(det) == 0.0 || !isfinite(creal(det)) || !isfinite(cimag(det))) break;
            double dx = 0, nx = 0;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    cplx nxt = 0.5 * (X[3 * i + j] + conj(Y[3 * j + i]));
                    dx += creal((nxt - X[3 * i + j]) * conj(nxt - X[3 * i + j]));
                    nx += creal(nxt * conj(nxt));
                    X[3 * i + j] = nxt;
                }
            if (dx <= 1e-30 * nx) { ok = 1; break; }
        }
        memcpy(out + m * 9, X, sizeof X);
        bad += !ok;
    }
    return bad;
}

/* Three-link product N_mu(x) = W_mu(x) W_mu(x+mu) W_mu(x+2mu). */
void orc_naik_product(const int d[4], const cplx *W, cplx *out)
{
    const long V = vol(d);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++)
        for (int mu = 0; mu < 4; mu++) {
            const int p[3] = {mu + 1, mu + 1, mu + 1};
            path_product(d, W, s, p, 3, out + (s * 4 + mu) * 9);
        }
}

/* eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}) */
static double eta(const int d[4], long s, int mu)
{
    int x[4];
    coords_of(d, s, x);
    int k = 0;
    for (int nu = 0; nu < mu; nu++) k += x[nu];
    return (k & 1) ? -1.0 : 1.0;
}

/* The HISQ links (eq. above) from thin links; fat, lng: [V][4][3][3] with the
 * phases folded in.  Returns orc_unitarize's count of failures. */
int orc_hisq_smear(const int d[4], const cplx *thin, cplx *fat, cplx *lng)
{
    const long V = vol(d), n = V * 4 * 9;
    const double lv1[5] = {1.0 / 8, 1.0 / 16, 1.0 / 64, 1.0 / 384, 0.0};
    const double lv2[5] = {5.0 / 8, 1.0 / 16, 1.0 / 64, 1.0 / 384, -1.0 / 16};
    cplx *Vf = malloc(sizeof(cplx) * n), *W = malloc(sizeof(cplx) * n);
    orc_fat7(d, lv1, thin, Vf);
    int bad = orc_unitarize(V * 4, Vf, W);
    orc_fat7(d, lv2, W, fat);
    orc_naik_product(d, W, lng);
    for (long s = 0; s < V; s++)
        for (int mu = 0; mu < 4; mu++) {
            const double e = eta(d, s, mu);
            for (int i = 0; i < 9; i++) {
                fat[(s * 4 + mu) * 9 + i] *= e;
                lng[(s * 4 + mu) * 9 + i] *= -e / 24.0;
            }
        }
    free(Vf);
    free(W);
    return bad;
}

/* --------------------------------------------------------- gauge force
 *
 * Symanzik-improved gauge action and its force (the gauge-field part of the
 * HISQ RHMC step, Section 4.2).  The paper does not write the action out;
 * it is the Luescher-Weisz action, a sum over three loop shapes:
 *
 *   S = beta sum over loops L of c_L (1 - Re Tr U_L / 3)
 *
 * with c_L = c[0] for the 1x1 plaquettes, c[1] for the 1x2 and 2x1
 * rectangles and c[2] for the six-link parallelograms (mu, a, b, -mu, -a,
 * -b: three orthogonal signed steps and back), each loop counted once.
 *
 * The force on the link U_mu(x) is
 *   F_mu(x) = (beta/3) TA[ U_mu(x) A_mu(x) ],   TA(M) = (M - M^+)/2 - Tr(M - M^+)/6,
 * A_mu(x) = sum over the loops through the link of c_L times the product of
 * the loop's other links, from x+mu back to x.  For U_mu(x) -> exp(eps X)
 * U_mu(x) with X traceless anti-Hermitian, dS/deps = -Re Tr(X F_mu(x)).
 * The loops through (x, mu), written as the steps after the first (+mu):
 *   plaquette     (s nu, -mu, -s nu)                          6
 *   rectangle     (s nu, s nu, -mu, -s nu, -s nu)             6
 *                 (mu, s nu, -mu, -mu, -s nu)                 6
 *                 (s nu, -mu, -mu, -s nu, mu)                 6
 *   parallelogram (a, b, -mu, -a, -b)                        24
 * (nu != mu, s = +-1; a, b signed steps along two distinct axes other
 * than mu).  Every loop through the link appears exactly once when all
 * extents are >= 4, which the functions below require.
 */

static int gf_rest(int mu, int cls, int k, int *st)
{
    /* the k-th loop of class cls through (x, mu): writes its steps after the
     * first and returns their number, or 0 past the end of the class */
    const int M = mu + 1;
    int ax[3], na = 0;
    for (int d = 0; d < 4; d++)
        if (d != mu) ax[na++] = d + 1;
    if (cls == 0) {
        if (k >= 6) return 0;
        const int N = (k & 1 ? -1 : 1) * ax[k >> 1];
        st[0] = N; st[1] = -M; st[2] = -N;
        return 3;
    }
    if (cls == 1) {
        if (k >= 18) return 0;
        const int N = (k & 1 ? -1 : 1) * ax[(k >> 1) % 3], shape = k / 6;
        if (shape == 0) { st[0] = N; st[1] = N; st[2] = -M; st[3] = -N; st[4] = -N; }
        else if (shape == 1) { st[0] = M; st[1] = N; st[2] = -M; st[3] = -M; st[4] = -N; }
        else { st[0] = N; st[1] = -M; st[2] = -M; st[3] = -N; st[4] = M; }
        return 5;
    }
    if (k >= 24) return 0;
    /* ordered pair of distinct transverse axes (6) x signs (4) */
    const int pair = k >> 2, sa = (k & 1) ? -1 : 1, sb = (k & 2) ? -1 : 1;
    const int ia = pair >> 1, ib = (ia + 1 + (pair & 1)) % 3;
    const int A = sa * ax[ia], B = sb * ax[ib];
    st[0] = A; st[1] = B; st[2] = -M; st[3] = -A; st[4] = -B;
    return 5;
}

static int gf_extents_ok(const int d[4])
{
    return d[0] >= 4 && d[1] >= 4 && d[2] >= 4 && d[3] >= 4;
}

/* A_mu(x) for class weights w[3] */
static void gf_staple_sum(const int d[4], const cplx *U, long s, int mu, const double w[3], cplx *A)
{
    for (int i = 0; i < 9; i++) A[i] = 0;
    const long s1 = hop(d, s, mu, 1);
    int st[5];
    for (int cls = 0; cls < 3; cls++) {
        if (w[cls] == 0.0) continue;
        int n;
        for (int k = 0; (n = gf_rest(mu, cls, k, st)) > 0; k++) acc_path(d, U, s1, st, n, w[cls], A);
    }
}

/* F: [V][4][3][3] traceless anti-Hermitian.  Returns 1 (F untouched) if an
 * extent is below 4. */
int orc_gauge_force(const int d[4], const cplx *U, double beta, const double c[3], cplx *F)
{
    if (!gf_extents_ok(d)) return 1;
    const long V = vol(d);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++)
        for (int mu = 0; mu < 4; mu++) {
            cplx A[9], M[9];
            gf_staple_sum(d, U, s, mu, c, A);
            mm(M, link(U, s, mu), A);
            cplx tr = 0;
            for (int i = 0; i < 3; i++) tr += M[4 * i] - conj(M[4 * i]);
            cplx *f = F + (s * 4 + mu) * 9;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++)
                    f[3 * i + j] = (beta / 3.0) * (0.5 * (M[3 * i + j] - conj(M[3 * j + i])) - (i == j ? tr / 6.0 : 0.0));
        }
    return 0;
}

/* S (the definition above): every loop is met once per link it contains,
 * so summing Re Tr U_mu(x) A_mu(x) with the class weights divided by the
 * loop lengths (4, 6, 6) counts each loop once; there are 6, 12 and 16
 * loops of the three classes per site.  Returns NaN if an extent is below 4. */
double orc_gauge_action(const int d[4], const cplx *U, double beta, const double c[3])
{
    if (!gf_extents_ok(d)) return NAN;
    const long V = vol(d);
    const double w[3] = {c[0] / 4.0, c[1] / 6.0, c[2] / 6.0};
    double re = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : re)
    for (long s = 0; s < V; s++)
        for (int mu = 0; mu < 4; mu++) {
            cplx A[9], M[9];
            gf_staple_sum(d, U, s, mu, w, A);
            mm(M, link(U, s, mu), A);
            re += creal(M[0] + M[4] + M[8]);
        }
    return beta * ((double)V * (6.0 * c[0] + 12.0 * c[1] + 16.0 * c[2]) - re / 3.0);
}

/* ------------------------------------------------------- fermion force
 *
 * Chain rule of the HISQ fermion force (Section 4.2's fermion force, the
 * derivative of the pseudofermion action through the link smearing).  For a
 * scalar Q of the smeared links with gradient G (dQ = sum Re Tr(dY G) over
 * every output link Y), the gradient with respect to the input links of a
 * path sum Y = sum_P c_P L_1 ... L_n follows link by link:
 *   Re Tr(L_1 .. dL_k .. L_n G) = Re Tr(dL_k R_k),  R_k = L_{k+1}..L_n G L_1..L_{k-1},
 * and a link met daggered (L_k = U^+) receives R_k^+.  The functions below
 * walk the same path lists as orc_fat7 and orc_naik_product.
 */

static void adj_path(const int d[4], const cplx *U, long s, const int *steps, int n, double c, const cplx *G,
                     cplx *GU)
{
    cplx L[7][9], pre[8][9], suf[8][9];
    long addr[7];
    int dg[7];
    long cur = s;
    for (int k = 0; k < n; k++) {
        const int mu = abs(steps[k]) - 1;
        if (steps[k] > 0) {
            memcpy(L[k], link(U, cur, mu), sizeof L[k]);
            addr[k] = cur * 4 + mu;
            dg[k] = 0;
            cur = hop(d, cur, mu, 1);
        } else {
            cur = hop(d, cur, mu, -1);
            const cplx *u = link(U, cur, mu);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) L[k][3 * i + j] = conj(u[3 * j + i]);
            addr[k] = cur * 4 + mu;
            dg[k] = 1;
        }
    }
    for (int i = 0; i < 9; i++) pre[0][i] = suf[n][i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int k = 0; k < n; k++) mm(pre[k + 1], pre[k], L[k]);            /* pre[k] = L_1..L_k */
    for (int k = n - 1; k >= 0; k--) mm(suf[k], L[k], suf[k + 1]);       /* suf[k] = L_{k+1}..L_n (0-based) */
    for (int k = 0; k < n; k++) {
        cplx T[9], R[9];
        mm(T, suf[k + 1], G);
        mm(R, T, pre[k]);
        cplx *g = GU + addr[k] * 9;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) g[3 * i + j] += c * (dg[k] ? conj(R[3 * j + i]) : R[3 * i + j]);
    }
}

/* GU += gradient of sum Re Tr(fat7(U; c)_mu(x) G_mu(x)) with respect to U
 * (the path list of orc_fat7).  Serial: contributions scatter to links. */
void orc_fat7_adjoint(const int d[4], const double c[5], const cplx *U, const cplx *G, cplx *GU)
{
    const long V = vol(d);
    for (long s = 0; s < V; s++)
        for (int mu = 0; mu < 4; mu++) {
            const cplx *g = G + (s * 4 + mu) * 9;
            cplx *gu = GU + (s * 4 + mu) * 9;
            for (int i = 0; i < 9; i++) gu[i] += c[0] * g[i];
            const int M = mu + 1;
            for (int nu = 0; nu < 4; nu++) {
                if (nu == mu) continue;
                for (int sn = -1; sn <= 1; sn += 2) {
                    const int N = sn * (nu + 1);
                    const int p3[3] = {N, M, -N};
                    adj_path(d, U, s, p3, 3, c[1], g, GU);
                    const int pl[5] = {N, N, M, -N, -N};
                    if (c[4] != 0.0) adj_path(d, U, s, pl, 5, c[4], g, GU);
                    for (int rho = 0; rho < 4; rho++) {
                        if (rho == mu || rho == nu) continue;
                        for (int sr = -1; sr <= 1; sr += 2) {
                            const int R = sr * (rho + 1);
                            const int p5[5] = {N, R, M, -R, -N};
                            adj_path(d, U, s, p5, 5, c[2], g, GU);
                            for (int sig = 0; sig < 4; sig++) {
                                if (sig == mu || sig == nu || sig == rho) continue;
                                for (int ss = -1; ss <= 1; ss += 2) {
                                    const int S = ss * (sig + 1);
                                    const int p7[7] = {N, R, S, M, -S, -R, -N};
                                    adj_path(d, U, s, p7, 7, c[3], g, GU);
                                }
                            }
                        }
                    }
                }
            }
        }
}

/* GW += gradient of sum Re Tr(N_mu(x) G_mu(x)), N = W_mu(x) W_mu(x+mu) W_mu(x+2mu). */
void orc_naik_adjoint(const int d[4], const cplx *W, const cplx *G, cplx *GW)
{
    const long V = vol(d);
    for (long s = 0; s < V; s++)
        for (int mu = 0; mu < 4; mu++) {
            const int p[3] = {mu + 1, mu + 1, mu + 1};
            adj_path(d, W, s, p, 3, 1.0, G + (s * 4 + mu) * 9, GW);
        }
}
