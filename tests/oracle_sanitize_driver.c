/* Drives every entry point of the oracle once on a small lattice, for the
 * AddressSanitizer / UndefinedBehaviorSanitizer build of the oracle (test
 * infrastructure: built and run by test_oracle_sanitizers.py).  Exit status 0
 * when every result is finite and the solvers converge. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

void orc_dslash_full(const int d[4], const cplx *fat, const cplx *lng, const cplx *in, cplx *out);
void orc_dslash_half(const int d[4], const cplx *fat, const cplx *lng, int par, const cplx *in_half,
                     cplx *out_half);
double orc_true_residual(const int d[4], const cplx *fat, const cplx *lng, double mass, double sigma,
                         const cplx *b, const cplx *x);
int orc_cg(const int d[4], const cplx *fat, const cplx *lng, double mass, double sigma, const cplx *b, cplx *x,
           double tol, int maxiter, int *iters, double *true_rel);
int orc_multishift(const int d[4], const cplx *fat, const cplx *lng, double mass, int nshift,
                   const double *shifts, const cplx *b, cplx *x, double tol, int maxiter, int *iters,
                   double *rel);
void orc_ptc_layer(const int d[4], const cplx *fat, int cin, int cout, const cplx *w, const cplx *in, cplx *out);
void orc_ptc_layer_adj(const int d[4], const cplx *fat, int cin, int cout, const cplx *w, const cplx *in,
                       const cplx *gout, cplx *gin, cplx *gw);
void orc_ptc_apply(const int d[4], const cplx *fat, int nlayer, const int *chans, const cplx *weights,
                   const cplx *r_even, cplx *z_even);
int orc_fcg(const int d[4], const cplx *fat, const cplx *lng, double mass, int nlayer, const int *chans,
            const cplx *weights, const cplx *b, cplx *x, double tol, int maxiter, int *iters, double *true_rel);

static double urand(unsigned long long *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0 - 0.5;
}

static int finite_all(const cplx *v, long n)
{
    for (long i = 0; i < n; i++)
        if (!isfinite(creal(v[i])) || !isfinite(cimag(v[i]))) return 0;
    return 1;
}

int main(void)
{
    const int d[4] = {4, 2, 4, 6};
    const long V = 4L * 2 * 4 * 6, h = V / 2;
    unsigned long long seed = 12345;
    /* links near the identity (the generic form the oracle accepts) */
    cplx *fat = malloc(sizeof(cplx) * V * 4 * 9), *lng = malloc(sizeof(cplx) * V * 4 * 9);
    for (long i = 0; i < V * 4; i++)
        for (int a = 0; a < 3; a++)
            for (int c = 0; c < 3; c++) {
                fat[i * 9 + 3 * a + c] = (a == c) + 0.2 * (urand(&seed) + I * urand(&seed));
                lng[i * 9 + 3 * a + c] = -(a == c) / 24.0 + 0.02 * (urand(&seed) + I * urand(&seed));
            }
    cplx *full = malloc(sizeof(cplx) * V * 3), *fout = malloc(sizeof(cplx) * V * 3);
    cplx *b = malloc(sizeof(cplx) * h * 3), *x = calloc(h * 3, sizeof(cplx)), *t = malloc(sizeof(cplx) * h * 3);
    for (long i = 0; i < V * 3; i++) full[i] = urand(&seed) + I * urand(&seed);
    for (long i = 0; i < h * 3; i++) b[i] = urand(&seed) + I * urand(&seed);
    orc_dslash_full(d, fat, lng, full, fout);
    orc_dslash_half(d, fat, lng, 0, b, t);
    orc_dslash_half(d, fat, lng, 1, t, x);
    int ok = finite_all(fout, V * 3) && finite_all(t, h * 3) && finite_all(x, h * 3);
    for (long i = 0; i < h * 3; i++) x[i] = 0;
    int it = 0;
    double tr = 0;
    ok = ok && orc_cg(d, fat, lng, 0.2, 0.0, b, x, 1e-10, 5000, &it, &tr) == 0 && tr <= 1e-10;
    ok = ok && fabs(orc_true_residual(d, fat, lng, 0.2, 0.0, b, x) - tr) <= 1e-12;
    const double shifts[2] = {0.0, 0.3};
    cplx *xs = calloc(2 * h * 3, sizeof(cplx));
    int its[2];
    double rel[2];
    ok = ok && orc_multishift(d, fat, lng, 0.2, 2, shifts, b, xs, 1e-10, 5000, its, rel) == 0;
    ok = ok && rel[0] <= 1e-10 && rel[1] <= 1e-10;
    /* a 1 -> 2 -> 1 network: layer, adjoint with both gradients, apply, FCG */
    const int chans[3] = {1, 2, 1};
    cplx *w = malloc(sizeof(cplx) * (2 * 9 + 2 * 9));
    for (int i = 0; i < 36; i++) w[i] = 0.1 * (urand(&seed) + I * urand(&seed));
    cplx *a1 = malloc(sizeof(cplx) * 2 * V * 3), *g1 = malloc(sizeof(cplx) * 2 * V * 3);
    cplx *gin = malloc(sizeof(cplx) * V * 3), *gw = malloc(sizeof(cplx) * 18);
    orc_ptc_layer(d, fat, 1, 2, w, full, a1);
    for (long i = 0; i < 2 * V * 3; i++) g1[i] = urand(&seed) + I * urand(&seed);
    orc_ptc_layer_adj(d, fat, 1, 2, w, full, g1, gin, gw);
    ok = ok && finite_all(a1, 2 * V * 3) && finite_all(gin, V * 3) && finite_all(gw, 18);
    orc_ptc_apply(d, fat, 2, chans, w, b, t);
    ok = ok && finite_all(t, h * 3);
    for (long i = 0; i < h * 3; i++) x[i] = 0;
    ok = ok && orc_fcg(d, fat, lng, 0.2, 2, chans, w, b, x, 1e-10, 5000, &it, &tr) == 0 && tr <= 1e-10;
    free(fat); free(lng); free(full); free(fout); free(b); free(x); free(t); free(xs);
    free(w); free(a1); free(g1); free(gin); free(gw);
    printf(ok ? "oracle driver ok\n" : "oracle driver FAILED\n");
    return ok ? 0 : 1;
}
