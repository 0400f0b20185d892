/*
 * hisq.h -- C ABI of the MI355X HISQ staggered Dslash / CG library.
 *
 * What it computes.  The paper (DeTar, Gottlieb, Li, Toussaint, "MILC Code
 * Performance on High End CPU and GPU Supercomputer Clusters", Lattice 2017)
 * benchmarks MILC's staggered multi-shift and single-mass conjugate gradient
 * for HISQ quarks (Section 4, Section 4.1), whose inner work is the
 * matrix-vector stencil (Section 4.2).  The operator is the standard even-odd
 * HISQ staggered Dslash on a periodic local lattice:
 *
 *   (D psi)(x) = sum_mu [ F_mu(x) psi(x+mu) - F_mu(x-mu)^+ psi(x-mu)
 *                       + L_mu(x) psi(x+3mu) - L_mu(x-3mu)^+ psi(x-3mu) ],
 *
 * with fat links F and long (Naik) links L that already carry the staggered
 * phases eta_mu(x) = (-1)^(x_0+...+x_{mu-1}).  M = 2m + D, and the solvers
 * work on even sites with A = M^+M|_even = 4m^2 - D_eo D_oe (+ sigma).
 *
 * Conventions shared by every entry point:
 *   - lattice extents L0..L3 are even and >= 2; lex(x) = x0 + L0(x1 + L1(x2 + L2 x3));
 *   - links: complex FP64 [V][4][3][3] (re, im interleaved, row-major 3x3),
 *     V = L0 L1 L2 L3 sites in lex order, mu = 0..3 <-> x, y, z, t;
 *   - a parity vector holds V/2 sites, site index lex(x)/2 over the sites of
 *     that parity, 3 colours per site: complex [V/2][3];
 *     device vectors may be FP64 (16 B per complex), FP32 (8 B) or FP16:
 *     an FP16 vector is [V/2][3] half2 followed immediately by [V/2] float
 *     per-site scales (value = half * scale); nrhs vectors are stored back to
 *     back;
 *   - every function returns a hisq_status; nothing throws or aborts across
 *     the ABI.  Details of the last error: hisq_last_error().
 *   - ownership: the caller owns every pointer it passes; the library copies
 *     what it needs before returning (solvers) or before the enqueued work
 *     completes (hisq_dslash with device pointers) and keeps no caller
 *     pointer.  hisq_destroy frees everything the handle allocated.
 *   - streams: all device work of a handle goes to its stream.  Solvers return
 *     synchronised; hisq_dslash on device pointers is asynchronous.
 *   - threads: one handle per host thread at a time.
 */
#ifndef HISQ_H
#define HISQ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hisq_lattice_s *hisq_lattice;
typedef struct hisq_ptc_s *hisq_ptc;

typedef enum {
    HISQ_OK = 0,
    HISQ_ERR_ARG = -1,            /* invalid argument (extents, mass, tol, sizes, null pointers) */
    HISQ_ERR_HIP = -2,            /* a HIP runtime call failed */
    HISQ_ERR_OOM = -3,            /* device allocation failed */
    HISQ_ERR_STATE = -4,          /* call out of order (e.g. no links loaded) */
    HISQ_ERR_RECON = -5,          /* links are not a * sign * SU(3): recon-12 impossible */
    HISQ_ERR_NOT_CONVERGED = -6,  /* maxiter reached; x and info hold the best iterate */
    HISQ_ERR_BREAKDOWN = -7,      /* non-positive p.Ap or non-finite scalar */
    HISQ_ERR_IO = -8              /* a file could not be written or read, or holds no matching network */
} hisq_status;

typedef enum { HISQ_F64 = 0, HISQ_F32 = 1, HISQ_F16 = 2 } hisq_prec;
typedef enum { HISQ_RECON_18 = 18, HISQ_RECON_12 = 12 } hisq_recon;
typedef enum { HISQ_EVEN = 0, HISQ_ODD = 1 } hisq_parity;

enum {
    HISQ_DEVICE_PTR = 1,   /* vector / link pointers are device pointers */
    HISQ_X_IS_GUESS = 2,   /* solvers: x holds an initial guess (else cold start) */
    HISQ_USE_GRAPH = 4,    /* solvers: replay captured HIP graphs of iteration chunks */
    HISQ_NO_TUNE = 8,      /* use default launch shapes, skip the autotuner */
    HISQ_STOP_STAGNATION = 16,  /* CG solvers: give up (HISQ_ERR_NOT_CONVERGED, x the last
                                   reliable update's iterate) when three reliable updates in a
                                   row bring no FP64 true residual below the one before them */
    HISQ_STREAM_LINKS = 32,     /* hisq_dslash (one right-hand side): stream every link past the
                                   caches (no part kept in the Infinity Cache between calls), in
                                   the block shape the autotuner found fastest that way; the rate
                                   is then an HBM rate whatever the operator's size */
    HISQ_LOAD_RESULT = 64       /* hisq_smear_links: the smeared links become the lattice's
                                   links, as if passed to hisq_load_links */
};
/* Environment: HISQ_TUNE=0 gives every call the default launch shapes (as
 * HISQ_NO_TUNE does for one call); HISQ_TUNE_CACHE=<file> appends every tuned
 * choice to a text file (one "key W remap cache-policy us" line each; W is
 * the waves per block, plus 256 for the variant compiled for at most two
 * waves per SIMD) and reads it back at start-up, so a later process skips the
 * timing. */

typedef struct {
    double tol;          /* target FP64 true relative residual ||b - A x|| / ||b|| */
    int maxiter;         /* iteration cap (Krylov iterations, all precisions) */
    hisq_prec sloppy;    /* precision of the iteration: F64 = plain CG; F32 / F16 = mixed
                            precision with FP64 reliable updates */
    hisq_recon recon;    /* link reconstruction of the sloppy operator */
    double delta;        /* reliable update when ||r|| < delta * max ||r|| since the last one
                            (FP32 sloppy at small mass: 0.01 halves the updates of 0.1 at the
                            same iteration count; FP16 keeps 0.1) */
    int check_every;     /* most iterations launched between host status checks; a single
                            solve sizes each chunk from the residual's decay to end near the
                            next reliable update, a batch launches check_every at a time (the
                            chunk lengths never change the result) */
    int flags;           /* HISQ_DEVICE_PTR | HISQ_X_IS_GUESS | HISQ_USE_GRAPH | HISQ_NO_TUNE |
                            HISQ_STOP_STAGNATION */
} hisq_solver_params;

typedef struct {
    int iters;               /* Krylov iterations */
    int reliable_updates;    /* FP64 true-residual recomputations */
    int converged;           /* 1 if the FP64 true residual reached tol */
    int status;              /* hisq_status of this solve */
    double true_residual;    /* final FP64 ||b - A x|| / ||b|| */
    double time_s;           /* wall time of the solve call (excludes link loading) */
    double dslash_bytes;     /* algorithmic bytes moved by the Dslash applications */
    double flops;            /* algorithmic flops (1146 per half-Dslash output site) */
    double t_done_s;         /* batch solves: device time from start to convergence */
    int fell_back;           /* learned solver: 1 if it handed over to plain CG */
    int fcg_iters;           /* learned solver: flexible-CG iterations before any hand-over */
    int restarts;            /* reliable updates that restarted the search direction (p = r)
                                because the FP64 residual exceeded twice the sloppy one */
    int refine_iters;        /* multi-shift: iterations of this shift's refinement (part of iters) */
} hisq_solver_info;

/* Fill params with defaults: tol 1e-10, maxiter 100000, F64, recon 18,
 * delta 0.1, check_every 16, flags 0. */
void hisq_default_params(hisq_solver_params *p);

const char *hisq_status_string(hisq_status s);

/* Last error message of the handle (or of the last failed hisq_create when
 * lat is NULL), copied into buf (n bytes, NUL-terminated). */
hisq_status hisq_last_error(hisq_lattice lat, char *buf, size_t n);

/* Create a handle for one periodic local lattice on `device`.  stream: a
 * hipStream_t to enqueue on, or NULL for a stream the handle creates (default
 * priority).  Errors: HISQ_ERR_ARG for extents that are odd or < 2. */
hisq_status hisq_create(const int dims[4], int device, void *stream, hisq_lattice *out);
hisq_status hisq_destroy(hisq_lattice lat);

/* Load fat and long links (layout above, phases folded; host pointers, or
 * device pointers with HISQ_DEVICE_PTR).  Keeps a device FP64 copy and packs
 * the FP64 recon-18 operator (errors of that packing as hisq_prepare_links).
 * Discards earlier link sets. */
hisq_status hisq_load_links(hisq_lattice lat, const double *fat, const double *lng, int flags);

/* Build the packed operator in precision `prec` with reconstruction `recon`
 * from the loaded FP64 links (on the device).  Recon-12 requires each link to
 * be c * SU(3), c = s * eta_mu(x) * a with one a > 0 and one s = +-1 per
 * field; it returns HISQ_ERR_RECON if row 3 is not recovered to 1e-10 * a.
 * The packed links of one direction are addressed with 32-bit offsets:
 * HISQ_ERR_ARG if one direction block (about V/2 sites x the link's bytes,
 * 144 in FP64 recon-18) would reach 2 GiB, i.e. V above about 29.8 million
 * sites in FP64 recon-18 (59.6 million in FP32). */
hisq_status hisq_prepare_links(hisq_lattice lat, hisq_prec prec, hisq_recon recon);

/* out = D_{out_parity, 1-out_parity} in, i.e. D_eo (HISQ_EVEN) or D_oe
 * (HISQ_ODD).  `prec` is the precision of links and vectors; the link set
 * (prec, recon) must have been prepared (FP64 recon-18 always is).  With
 * HISQ_DEVICE_PTR, in/out are device vectors in precision prec, nrhs of them
 * back to back (nrhs > 1 uses the multi-right-hand-side kernel, FP32/FP16
 * only); without it they are host FP64 vectors, converted by the library.
 * Asynchronous on device pointers.  The first call for a (lattice shape,
 * precision, recon, nrhs) times the candidate block shapes synchronously
 * (the autotuner); make it before capturing calls into a HIP graph. */
hisq_status hisq_dslash(hisq_lattice lat, hisq_parity out_parity, hisq_prec prec,
                        hisq_recon recon, const void *in, void *out, int nrhs, int flags);

/* The launch shape hisq_dslash (one right-hand side) uses for (prec, recon)
 * on this lattice under `flags` (HISQ_STREAM_LINKS, HISQ_NO_TUNE), running
 * the autotuner first if it has not chosen yet: *waves = wavefronts per block
 * (1, 2, 4, 8, 16; plus 256 for the variant compiled for at most two waves
 * per SIMD), *remap = 1 for the XCD-contiguous tile order, *cache_blocks =
 * link direction blocks (of 16) loaded so that they stay in the Infinity
 * Cache.  For naming the kernel a measurement profiles.  Errors: HISQ_ERR_ARG
 * (null outputs, bad format), HISQ_ERR_STATE (no links, set not prepared). */
hisq_status hisq_dslash_shape(hisq_lattice lat, hisq_prec prec, hisq_recon recon, int flags, int *waves,
                              int *remap, int *cache_blocks);

/* Solve (4m^2 - D_eo D_oe) x = b on even sites (host FP64 vectors, or device
 * FP64 with HISQ_DEVICE_PTR).  Plain FP64 CG when params->sloppy == HISQ_F64;
 * otherwise the iteration runs in FP32 or FP16 storage (FP32 arithmetic) and
 * FP64 reliable updates recompute x and the true residual.  Stops when the
 * FP64 true residual is <= tol.  info may be NULL. */
hisq_status hisq_cg(hisq_lattice lat, double mass, const double *b, double *x,
                    const hisq_solver_params *params, hisq_solver_info *info);

/* hisq_cg for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same iteration and kernels, with every work vector, reduction partial, the
 * solver state and the problem descriptor in one static device buffer of
 * 64 MiB per GPU (held until the process ends), so the call performs no
 * hipMalloc, hipFree or other allocation on the device.  The launch shape is
 * the autotuner's cached choice for this lattice if one exists (made by an
 * earlier hisq_cg or hisq_dslash), else the default; nothing is timed.
 * Requirements: b and x are device FP64 vectors (HISQ_DEVICE_PTR); no
 * HISQ_USE_GRAPH (instantiating a graph allocates); the FP64 and the sloppy
 * link sets are already prepared (hisq_prepare_links allocates).  The buffer
 * holds 4 FP64 vectors, 3 accumulators (FP64 plain, FP32 mixed) and 2 sloppy
 * vectors of V/2 sites plus per-tile partials: V/2 up to about 155 000 sites
 * in plain FP64 (16^3x32 fits, 24^4 does not), 215 000 in mixed FP32 (24^4
 * fits, 32^4 does not), 226 000 in mixed FP16.  Every call on a GPU shares that GPU's buffer and its
 * contents from the last call (everything a solve reads is written first by
 * that solve); calls that overlap on one GPU, from any handle or thread, race.
 * Errors: as hisq_cg, plus HISQ_ERR_ARG for host vectors, HISQ_USE_GRAPH or a
 * lattice whose work set exceeds the buffer, HISQ_ERR_STATE for link sets not
 * prepared. */
hisq_status hisq_cg_noalloc(hisq_lattice lat, double mass, const double *b, double *x,
                            const hisq_solver_params *params, hisq_solver_info *info);

/* Multi-shift CG (Section 4.1): solve (A + shifts[k]) x_{j,k} = b_j for
 * nshift <= 64 shifts and nrhs right-hand sides with one Krylov space per
 * right-hand side (base system = smallest shift, FP64 zeta/alpha/beta
 * recurrences on the device), the nrhs spaces sharing one multi-RHS Dslash.
 * b: nrhs host FP64 vectors back to back; x: nrhs*nshift vectors, index
 * j*nshift + k.  Each shift stops when |zeta_k| ||r|| <= tol ||b||; shifts
 * whose FP64 true residual is above tol are then refined with mixed CG
 * (all nrhs*nshift refinements advance together, sharing link reads; their
 * status is checked every min(check_every, 4) iterations).
 * info: nrhs*nshift entries (or NULL). */
hisq_status hisq_multishift_cg(hisq_lattice lat, double mass, int nshift, const double *shifts,
                               int nrhs, const double *b, double *x,
                               const hisq_solver_params *params, hisq_solver_info *info);

/* Batched solve of nprob independent systems, one per handle (each with its
 * own links, extents and mass), all advanced by the same kernel launches over
 * a flattened tile list, with per-problem FP64 scalars and a device status
 * mask.  b[k], x[k]: host FP64 vectors of problem k.  All handles must be on
 * the same device; the first handle's stream is used.  info: nprob entries. */
hisq_status hisq_batch_cg(int nprob, const hisq_lattice *lats, const double *masses,
                          const double *const *b, double *const *x,
                          const hisq_solver_params *params, hisq_solver_info *info);

/* ---- learned preconditioner: gauge-covariant parallel-transport network ----
 *
 * Layer l maps C_in to C_out channels of full-lattice colour vectors:
 *   out_c(x) = sum_{c'} [ w0 psi_c'(x) + sum_mu ( w_{+mu} F_mu(x) psi_c'(x+mu)
 *                                         + w_{-mu} F_mu(x-mu)^+ psi_c'(x-mu) ) ]
 * with 9 complex weights per (c, c') (path order: 0 = identity,
 * 1+2mu = +mu, 2+2mu = -mu) and the fat links F; no bias, which would break
 * gauge covariance.  With K = L_n ... L_1 the layer stack and E the embedding
 * of an even vector on the full lattice (zeros on odd sites), the
 * preconditioner of the flexible CG is z = M(r), M = 1 + E^+ K^+ K E: the
 * layers, then their exact adjoints in reverse order, the even projection,
 * plus the identity.  M is Hermitian positive definite by construction, like
 * the A^-1 it approximates, and M = 1 (plain CG) for zero weights.
 *
 * Activation layout of the layer calls (device FP32): channel c is
 * [2 parities][V/2 sites][3 colours] complex, even sites first, each parity in
 * lex(x)/2 order.
 */

/* nlayer layers (<= 8), chans[0..nlayer] channel counts (chans[0] = 1; each
 * 1, 2, 4 or 8).  Weights start at zero (M = 1). */
hisq_status hisq_ptc_create(hisq_lattice lat, int nlayer, const int *chans, hisq_ptc *out);
/* Frees the network and its stored pairs.  It may be called after the
 * lattice handles are destroyed; every other network call needs the handle
 * it was created on (and, for training, the handles the pairs came from). */
hisq_status hisq_ptc_destroy(hisq_ptc net);
/* Weights as complex FP64, layer by layer [Cout][Cin][9]; set writes the
 * FP32 master copy and the FP16 inference copy. */
hisq_status hisq_ptc_set_weights(hisq_ptc net, const double *w);
hisq_status hisq_ptc_get_weights(hisq_ptc net, double *w);
/* Checkpoint of a network: its shape, the FP32 master weights, the Adam
 * moments and step count, in a small binary file (an 8-byte magic
 * "HISQPTC1", then little-endian int32 version 1, nlayer, chans[0..nlayer],
 * the complex weight count nw and the Adam step; then 2 nw float32 weights,
 * 2 nw float32 first moments and 2 nw float32 second moments).  Load
 * requires a network of the same shape, restores weights and Adam state
 * exactly (training continues as if uninterrupted) and refreshes the FP16
 * copies.  Stored pairs are not saved.  Errors: HISQ_ERR_ARG (null
 * arguments), HISQ_ERR_IO (the file cannot be written or read, is not such a
 * file, or was saved from a network of another shape). */
hisq_status hisq_ptc_save(hisq_ptc net, const char *path);
hisq_status hisq_ptc_load(hisq_ptc net, const char *path);
/* Polynomial starting weights (a starting point for training, or a
 * preconditioner of its own): K = a (1 + c D_f^2 / lambda) on even vectors,
 * with D_f the one-hop fat-link part of D (the PTC transports with weights
 * +1 forward, -1 backward).  On an eigenvector of -D_f^2 with eigenvalue t,
 * M = 1 + a^2 (1 - c t/lambda)^2: the low modes of A are enlarged up to
 * 1 + a^2 times against the upper spectrum (c slightly above 1 puts the zero
 * of K inside the spectrum, which lowers the condition number further;
 * c = 1.2 is a good choice on the fields tested).  lambda, the largest
 * eigenvalue of -D_f^2 on even sites, is estimated with `iters` power
 * iterations on D_f^4 (FP32 transports, a fixed seeded start vector) and
 * returned in *lambda (may be NULL).  Needs >= 2 layers and >= 2 channels
 * after every layer but the last; all other weights are zero.  Adam state is
 * reset.  Errors: HISQ_ERR_ARG (a <= 0, c outside (0, 4], iters outside
 * [1, 1000], a network too small), HISQ_ERR_STATE (no links),
 * HISQ_ERR_BREAKDOWN (no positive spectrum estimate). */
hisq_status hisq_ptc_init_polynomial(hisq_ptc net, double a, double c, int iters, double *lambda);
/* One layer on device FP32 activations (layout above, HISQ_DEVICE_PTR
 * required): forward out = L_l(in); backward gin = L_l^+(gout) (gin may be
 * NULL) and gw = sum_x (T_k in)^+ gout (complex FP64 [Cout][Cin][9], host). */
hisq_status hisq_ptc_layer_forward(hisq_ptc net, int layer, const void *in, void *out, int flags);
hisq_status hisq_ptc_layer_backward(hisq_ptc net, int layer, const void *in, const void *gout,
                                    void *gin, double *gw, int flags);
/* z = M(r) on device even vectors (FP32 complex), using the FP16 weights and
 * the network's transport links (hisq_ptc_set_transport; HISQ_DEVICE_PTR
 * required). */
hisq_status hisq_ptc_apply(hisq_ptc net, const void *r, void *z, int flags);
/* Generate training pairs: plain FP32/FP64 CG on b (host FP64), storing the
 * residual r_i and error e_i = x* - x_i every `every` iterations, at most
 * maxpairs.  Pairs are appended to the network's device pair store.
 * Returns the number of pairs stored in *npairs. */
hisq_status hisq_ptc_harvest(hisq_ptc net, hisq_lattice lat, double mass, const double *b,
                             int every, int maxpairs, int *npairs);
/* Number of stored pairs, and pair `index` (in storage order) as host FP64
 * even vectors r, e ([V/2][3] complex each, as stored: FP32 values). */
hisq_status hisq_ptc_pair_count(hisq_ptc net, int *count);
hisq_status hisq_ptc_get_pair(hisq_ptc net, int index, double *r, double *e);
/* Training loss (hisq_ptc_set_loss).  For a minibatch of B pairs (r_b, e_b),
 * A e_b = r_b, and z_b = M r_b, the misfit of z_b ~ c e_b with one common
 * complex c, minimised over c and normalised (invariant to the scale of M,
 * which the flexible CG does not see):
 *   HISQ_LOSS_ENERGY (default): in the energy norm |v|_A^2 = <v, A v> that CG
 *     minimises, L = 1 - |S|^2/(B Q), S = sum_b <z_b, r_b>/w_b,
 *     Q = sum_b <z_b, A z_b>/w_b, w_b = <e_b, r_b>; each step applies the
 *     FP32 operator of the pairs' lattice to the batch;
 *   HISQ_LOSS_EUCLIDEAN: in the Euclidean norm, S = sum_b <z_b, e_b>/|e_b|^2,
 *     Q = sum_b |z_b|^2/|e_b|^2.  It weights the low modes of the error by
 *     1/lambda^2 and drifts away from good preconditioners. */
enum { HISQ_LOSS_ENERGY = 0, HISQ_LOSS_EUCLIDEAN = 1 };
hisq_status hisq_ptc_set_loss(hisq_ptc net, int loss);
/* Link format of the network's transports F_mu: HISQ_F32 with HISQ_RECON_18
 * (the default) or HISQ_F16 with HISQ_RECON_12 (fat links stored as FP16
 * rows 1-2 over the field scale, row 3 rebuilt; requires links that are
 * scale * sign * SU(3), else the first call that needs them returns
 * HISQ_ERR_RECON).  Every later call of the network uses it -- the layer
 * calls, hisq_ptc_apply, hisq_ptc_train, hisq_ptc_init_polynomial's spectrum
 * estimate and hisq_cg_learned -- so that a network is trained and applied on
 * the same operator; the link set is prepared on the lattice on first use.
 * Arithmetic stays FP32.  Errors: HISQ_ERR_ARG (null net, another format).
 * get_transport returns the current format (prec, recon). */
hisq_status hisq_ptc_set_transport(hisq_ptc net, hisq_prec prec, hisq_recon recon);
hisq_status hisq_ptc_get_transport(hisq_ptc net, int *prec, int *recon);
/* Storage precision of the activations between the layers of z = M(r) in
 * hisq_ptc_apply and hisq_cg_learned: HISQ_F32 (the default; channel-major
 * FP32 activations) or HISQ_F16 (site-major, channel-interleaved IEEE
 * binary16 values over one FP32 scale per site, the site's largest |entry|;
 * about half the activation bytes per layer).  Arithmetic stays FP32 and the
 * input r and output z stay FP32; training keeps FP32 activations (it needs
 * them for the gradients).  FP16 storage rounds each stored activation entry
 * to 2^-11 of its site's scale, so M is applied to about 1e-3 relative; the
 * flexible CG tolerates a preconditioner that inexact.  Errors: HISQ_ERR_ARG
 * (null net, another precision). */
hisq_status hisq_ptc_set_activations(hisq_ptc net, hisq_prec prec);
/* Train on the stored pairs (all from lattices whose links are those of the
 * handle each pair was harvested on): `steps` Adam steps (lr, beta1 0.9,
 * beta2 0.999, eps 1e-8) on minibatches of `batch` pairs of one lattice,
 * drawn with `seed`, on the loss set above.  losses: steps entries or NULL. */
hisq_status hisq_ptc_train(hisq_ptc net, int steps, int batch, double lr, unsigned long long seed,
                           double *losses);
/* Flexible CG (truncation 1) with z = M(r), FP32 iteration and FP64 true
 * residual; falls back to hisq_cg from the current x on breakdown or if the
 * iteration count exceeds params->maxiter / 2. */
hisq_status hisq_cg_learned(hisq_lattice lat, hisq_ptc net, double mass, const double *b,
                            double *x, const hisq_solver_params *params, hisq_solver_info *info);

/* FP64 true relative residuals ||b - A x|| / ||b|| at each reliable update
 * (the last one is the final convergence check) of the last solve led by this
 * handle: hisq_cg (problem 0), hisq_batch_cg led by it (problem = index in
 * that call's arrays), the refinement of hisq_multishift_cg (problem = shift *
 * nrhs + rhs), or hisq_cg_learned (problem 0; after a hand-over, the plain
 * CG that finished the solve).  Writes min(count, cap) values to out and the
 * number recorded to *count.  Errors: HISQ_ERR_STATE (no solve yet),
 * HISQ_ERR_ARG (problem out of range, null count, cap < 0). */
hisq_status hisq_residual_history(hisq_lattice lat, int problem, double *out, int cap, int *count);

/* ---- link smearing ----
 *
 * The HISQ fat and long links from thin SU(3) links (the link smearing the
 * paper's run-time breakdown reports beside the fermion and gauge forces,
 * Section 2 and Fig. 1; the construction is that of the HISQ action,
 * Follana et al., hep-lat/0610092):
 *   V = fat7(U; 1/8, 1/16, 1/64, 1/384; Lepage 0)
 *   W = V (V^+ V)^{-1/2}                         (projection onto U(3))
 *   fat_mu(x) = eta_mu(x) fat7(W; 5/8, 1/16, 1/64, 1/384; Lepage -1/16)_mu(x)
 *   lng_mu(x) = -(1/24) eta_mu(x) W_mu(x) W_mu(x+mu) W_mu(x+2mu)
 * fat7(U; c1, c3, c5, c7; cL)_mu(x) is c1 U_mu(x) plus, over the directions
 * nu, rho, sig (distinct, != mu) and both signs of each, c3 times the
 * 3-link staples (nu, mu, -nu), c5 the 5-link staples (nu, rho, mu, -rho,
 * -nu), c7 the 7-link staples (nu, rho, sig, mu, -sig, -rho, -nu) and cL the
 * Lepage paths (nu, nu, mu, -nu, -nu), each the product of the links along
 * the path (a step -nu from y multiplies by U_nu(y-nu)^+).  Unit thin links
 * give fat = 9/8 eta, lng = -1/24 eta.
 *
 * Arrays use the link layout above ([V][4][3][3] complex FP64, site-major;
 * thin links without phases), host pointers or, with HISQ_DEVICE_PTR, device
 * pointers.  FP64 throughout; synchronous.  The library keeps a device
 * workspace of 51 link-direction fields (59 with host outputs that are not
 * loaded; 144 P bytes each, P = V rounded up to 8 plus 296 sites of padding:
 * 7.7 GB at 32^4) per lattice until hisq_destroy.
 *
 * hisq_smear_links: thin -> (fat, lng).  With HISQ_LOAD_RESULT the result
 * also becomes the lattice's links (fat and lng may then be NULL), ready for
 * the solvers; its fat links are not a scaled SU(3), so hisq_prepare_links
 * with recon-12 returns HISQ_ERR_RECON for them.  Errors: HISQ_ERR_ARG (null
 * arguments), HISQ_ERR_BREAKDOWN (some V^+ V singular: no projection; with
 * HISQ_LOAD_RESULT the lattice is then left without links),
 * HISQ_ERR_OOM / HISQ_ERR_HIP. */
hisq_status hisq_smear_links(hisq_lattice lat, const double *thin, double *fat, double *lng, int flags);

/* One fat7 level alone: out = fat7(in; coef[0..4] = c1, c3, c5, c7, cL), no
 * phases, no projection (with the asqtad coefficients 5/8, 1/16, 1/64, 1/384,
 * -1/16 on thin links: the asqtad fat links before their phases).  Errors:
 * HISQ_ERR_ARG (null arguments), HISQ_ERR_OOM / HISQ_ERR_HIP. */
hisq_status hisq_fat7(hisq_lattice lat, const double coef[5], const double *in, double *out, int flags);

/* The U(3) projection alone: out = in (in^+ in)^{-1/2} for each of the 4 V
 * links.  Errors: HISQ_ERR_ARG, HISQ_ERR_BREAKDOWN (a singular link; out
 * still written, non-finite there). */
hisq_status hisq_unitarize(hisq_lattice lat, const double *in, double *out, int flags);

/* ---- gauge force ----
 *
 * The Symanzik-improved gauge action and force, the gauge-field part of the
 * RHMC molecular-dynamics step (the paper's second benchmark, Section 4.2):
 *   S = beta sum over loops L of c_L (1 - Re Tr U_L / 3)
 * over the 1x1 plaquettes (c_L = coef[0]), the 1x2 and 2x1 rectangles
 * (coef[1]) and the six-link parallelograms mu, a, b, -mu, -a, -b around 3-cubes
 * (coef[2]), each loop once.  (The tadpole-improved one-loop choice is
 * coef = {1, -(1 + 0.4805 alpha_s) / (20 u0^2), -0.03325 alpha_s / u0^2}.)
 * Thin links U in the link layout above, no phases; host pointers or, with
 * HISQ_DEVICE_PTR, device pointers.  FP64, synchronous; every extent must be
 * >= 4 (HISQ_ERR_ARG otherwise; on smaller extents loops wrap onto
 * themselves).
 *
 * hisq_gauge_force: F_mu(x) = (beta/3) TA[U_mu(x) A_mu(x)], the traceless
 * anti-Hermitian part TA(M) = (M - M^+)/2 - Tr(M - M^+)/6, A_mu(x) the sum
 * over the loops through the link of c_L times the product of its other
 * links from x+mu back to x; so that U_mu(x) -> exp(eps X) U_mu(x) (X in
 * su(3)) changes S at the rate -Re Tr(X F_mu(x)).  F: [V][4][3][3]. */
hisq_status hisq_gauge_force(hisq_lattice lat, const double *U, double beta, const double coef[3], double *F,
                             int flags);

/* hisq_gauge_action: *S (a host double) as defined above; the site sums
 * are reduced in a fixed order (the same bits on every call). */
hisq_status hisq_gauge_action(hisq_lattice lat, const double *U, double beta, const double coef[3], double *S,
                              int flags);

/* ---- fermion force ----
 *
 * The HISQ fermion force of the RHMD step (Section 4.2), for the rational
 * pseudofermion action S = Phi^+ (a0 + sum_k alpha_k (A + sigma_k)^-1) Phi
 * with the multi-shift solutions X_k = (A + sigma_k)^-1 Phi: at fixed X_k
 * dS = -dQ, where
 *   Q = sum_k alpha_k X_k^+ A X_k,   A = 4 m^2 - D_eo D_oe
 * (n terms, 1 <= n <= 64; X: n even FP64 vectors back to back, [n][V/2][3]
 * complex; alpha: n host doubles).  Gradients are taken in the sense
 * dQ = sum Re Tr(dY_mu(x) G_mu(x)) over the links Y; arrays in the link
 * layout above, host pointers or, with HISQ_DEVICE_PTR, device pointers
 * (alpha is always a host array).  FP64, synchronous.
 *
 * hisq_fermion_force_links: the gradients OF, OL of Q with respect to the
 * lattice's loaded (phased) fat and long links:
 *   OF_mu(x) = -2 eps(x) sum_k alpha_k Psi_k(x+mu) Psi_k(x)^+,
 *   OL_mu(x) = -2 eps(x) sum_k alpha_k Psi_k(x+3mu) Psi_k(x)^+,
 * Psi_k = X_k on even and D_oe X_k on odd sites, eps = +1 (-1) on even (odd)
 * sites.  Errors: HISQ_ERR_ARG, HISQ_ERR_STATE (no links loaded). */
hisq_status hisq_fermion_force_links(hisq_lattice lat, int n, const double *alpha, const double *X, double *OF,
                                     double *OL, int flags);

/* hisq_fermion_force: the force on the thin links U of the HISQ links
 * (hisq_smear_links), F_mu(x) = TA[U_mu(x) G_mu(x)], G the gradient of Q with
 * respect to U, so that U_mu(x) -> exp(eps X) U_mu(x) (X in su(3)) changes Q
 * at the rate Re Tr(X F_mu(x)) (and S at minus that rate).  The chain rule
 * runs through the Naik product, the second fat7 level, the U(3) projection
 * and the first level.  U is smeared first and the result loaded as the
 * lattice's links (as hisq_smear_links with HISQ_LOAD_RESULT would).
 * Workspace: 106 link-direction fields (144 P bytes each, P as for
 * hisq_smear_links: 16.0 GB at 32^4)
 * and 2 n V/2 vectors, kept until hisq_destroy.  Errors: HISQ_ERR_ARG, HISQ_ERR_BREAKDOWN (a level-1 link
 * has no U(3) projection; the lattice keeps the links it had),
 * HISQ_ERR_OOM / HISQ_ERR_HIP. */
hisq_status hisq_fermion_force(hisq_lattice lat, const double *U, int n, const double *alpha, const double *X,
                               double *F, int flags);

/* ---- measurement ----
 *
 * Practical HBM ceilings of `device`, measured on `stream` (NULL: the null
 * stream) with the library's own streaming kernels over a buffer of `bytes`
 * (>= 1 MiB; two such buffers are allocated and freed): *read_gbs from a
 * read-only pass of non-temporal 16-byte loads (the access the Dslash makes
 * for its links), *copy_gbs from a copy (bytes read + written), each the
 * average over `reps` launches after one warm-up.  Synchronous. */
hisq_status hisq_stream_bandwidth(int device, void *stream, size_t bytes, int reps, double *read_gbs,
                                  double *copy_gbs);

#ifdef __cplusplus
}
#endif
#endif /* HISQ_H */
