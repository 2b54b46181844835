/*
 * crsolve.h -- C ABI of the MI355X (gfx950) solver for the multi-resolution
 * Wiener-filter / constrained-realization system of Seljebotn et al.,
 * "Multi-resolution Bayesian CMB component separation through
 * Wiener-filtering with a pseudo-inverse preconditioner" (arXiv:1710.00621).
 *
 * The library solves A x = b with (Sect. 2.3, eq:A)
 *     A = S^-1 + sum_nu P_nu^T N_nu^-1 P_nu,   P_nu = Y_nu B_nu q_{nu,k}  (eq:P)
 * by preconditioned conjugate gradients, preconditioned either with the
 * pseudo-inverse preconditioner M_PI = U^+ T^+ (U^+)^T (Sect. 3.3,
 * eq:fullmodel-preconditioner) or with the block-diagonal comparison
 * preconditioner M_diag = (U^T diag(T) U)^-1 (Sect. 5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns CRS_OK (0) or a negative CRS_E* code and
 *   never throws.  On failure a message is kept per thread (crs_last_error).
 *   Arguments are validated on the host before anything is launched.
 * Precision: float64 throughout.  Architecture: gfx950 only.
 * Harmonic vectors: real orthonormal spherical harmonics (no Condon-Shortley
 *   sign; Y^c_lm = sqrt2 lambda_lm cos m phi, Y^s_lm = sqrt2 lambda_lm sin m phi)
 *   packed m-major: [m=0: l=0..L] then for m=1..L [cos: l=m..L][sin: l=m..L];
 *   (L+1)^2 doubles.  A component vector is the concatenation over
 *   components k of their (L_k+1)^2 blocks; n = sum_k (L_k+1)^2.
 * Maps: ring-major pixel order (HEALPix RING order), north to south.
 * Memory: "device" pointers are HIP device memory owned by the caller; the
 *   library never frees them nor keeps them past the call.  "host" pointers
 *   are ordinary host memory.  Handles own their tables and workspaces.
 * Streams: work is enqueued on the given stream (0 = null stream).  Calls
 *   on one handle must not overlap in time (the handle's workspace is
 *   shared); distinct handles are independent.
 * Allocation: create calls allocate; apply/solve calls allocate nothing
 *   once a handle has seen the largest nrhs it is used with (workspaces grow
 *   on the first call with a larger nrhs).  sht_synth / sht_adjoint allocate
 *   per-(grid, lmax) tables on their first call for that pair and grow the
 *   grid's transform workspace on a call with more maps; crs_sht_reserve
 *   does both up front.
 */
#ifndef CRSOLVE_H
#define CRSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* crs_stream;   /* hipStream_t */

typedef struct crs_grid_s*  crs_grid;
typedef struct crs_model_s* crs_model;
typedef struct crs_batch_s* crs_batch;

enum {
  CRS_OK = 0,
  CRS_EINVAL = -1,        /* invalid argument (message says which) */
  CRS_ENOMEM = -2,        /* device or host allocation failed */
  CRS_EHIP = -3,          /* a HIP runtime call failed */
  CRS_ENOTCONV = -4,      /* PCG hit maxiter; x holds the last iterate */
  CRS_EBREAKDOWN = -5,    /* PCG breakdown: p.Ap <= 0, r.z <= 0 or non-finite */
  CRS_EUNSUPPORTED = -6   /* valid request outside what the library supports */
};

enum { CRS_PRECOND_NONE = 0, CRS_PRECOND_DIAG = 1, CRS_PRECOND_PINV = 2, CRS_PRECOND_ADD = 3 };
enum { CRS_MODE_WF = 0, CRS_MODE_CR = 1 };

const char* crs_strerror(int status);
/* Copies the calling thread's last error message into buf (NUL-terminated,
 * truncated to n bytes).  Returns the status code of that error. */
int crs_last_error(char* buf, size_t n);
/* Library version string (static storage). */
const char* crs_version(void);

/* ------------------------------------------------------------------ grids
 * Ring grids of Sect. 2.1 / 2.2: HEALPix RING (Gorski et al. 2005) for sky
 * maps and Gauss-Legendre (roots of P_nrings, north to south, phi0 = 0).
 * Ring lengths are limited to 8192 pixels (Nside <= 2048, nphi <= 8192); an
 * odd nphi above 4096 must have no prime factor above 7.  Outside these
 * limits the constructors return CRS_EUNSUPPORTED.
 */
int crs_grid_healpix(int nside, crs_grid* out);
int crs_grid_gauss_legendre(int nrings, int nphi, crs_grid* out);
/* host out-params; either may be NULL */
int crs_grid_info(crs_grid g, int* nrings, int64_t* npix);
/* Pixel centres (z = cos theta, phi) in ring order; host arrays of npix. */
int crs_grid_pixel_centres(crs_grid g, double* z, double* phi);
/* Quadrature weights, the diagonal of W (Sect. 2.1); host array of npix.
 * HEALPix: 4 pi / Npix.  Gauss-Legendre: w_r 2 pi / nphi. */
int crs_grid_weights(crs_grid g, double* w);
int crs_grid_destroy(crs_grid g);

/* -------------------------------------------------------------- transforms
 * sht_synth: map = Y alm, spherical harmonic synthesis (Sect. 2.1).
 * sht_adjoint: alm = Y^T map, the literal transpose of synthesis (adjoint
 *   synthesis, Sect. 3.2; not analysis, which is Y^T W).
 * alm: device, nmaps x alm_stride doubles, each map (lmax+1)^2 packed.
 * map: device, nmaps x map_stride doubles, each map npix pixels.
 * Any lmax >= 0 is accepted on any grid; rings with fewer than 2 lmax + 1
 * pixels alias (m folded modulo nphi), exactly like the dense matrix.
 * Strides must be >= the per-map length.  Errors: CRS_EINVAL on NULL
 * pointers, lmax < 0, nmaps < 1, short strides.
 */
int sht_synth(crs_grid g, int lmax, int nmaps, const double* alm, int64_t alm_stride,
              double* map, int64_t map_stride, crs_stream s);
int sht_adjoint(crs_grid g, int lmax, int nmaps, const double* map, int64_t map_stride,
                double* alm, int64_t alm_stride, crs_stream s);

/* crs_sht_reserve: setup for the transforms of Sect. 2.1 on (g, lmax) with
 * up to nmaps maps: builds the (grid, lmax) Legendre tables and grows the
 * grid's transform workspace (hat vectors, phase array, per-tile partial sums
 * sized for any kernel variant), so that later sht_synth / sht_adjoint calls
 * on this grid with lmax and at most nmaps maps allocate nothing.
 * Synchronises the stream.  Errors: CRS_EINVAL (NULL grid, lmax < 0,
 * nmaps < 1), CRS_ENOMEM. */
int crs_sht_reserve(crs_grid g, int lmax, int nmaps, crs_stream s);

/* sht_adjoint_noalloc: sht_adjoint for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and result as sht_adjoint, but
 * its scratch (the phase array and the per-tile partial sums) lives in one
 * static device array of 64 MiB that the library holds on every GPU it runs
 * on until the process ends; the call itself allocates nothing.
 * Preconditions: the (grid, lmax) Legendre tables already exist (created by
 * any earlier sht_synth / sht_adjoint on that pair, or by a model using it);
 * otherwise CRS_EINVAL.  A request whose scratch exceeds 64 MiB (e.g. more
 * than about two maps at HEALPix Nside 256 / lmax 512) returns CRS_EINVAL
 * with the needed size in the message.  All calls on one GPU share that
 * GPU's array: calls that overlap in time on one GPU (different streams or
 * threads) race and must be serialised by the caller.  Nothing in the array
 * needs clearing between calls: every scratch entry is written before it is
 * read. */
int sht_adjoint_noalloc(crs_grid g, int lmax, int nmaps, const double* map, int64_t map_stride,
                        double* alm, int64_t alm_stride, crs_stream s);

/*
 * Legendre kernel autotuning (the recurrence and contraction of Sect. 2.1,
 * the bulk of every transform).  Both transforms have several kernel
 * variants per shape: the matrix-core contraction (from a few maps on) or
 * vector FP64 code, and the number of ring pairs per lane / 64-pair tiles
 * per wave.  crs_autotune_legendre times every variant for (grid, lmax,
 * nmaps) on the given stream (setup: allocates scratch, synchronises) and
 * records the fastest synthesis and adjoint for that shape; every later
 * transform of that shape in the process (sht_synth, sht_adjoint, and the
 * operators of models and batches created afterwards) uses it.  Batches
 * (crs_batch_create) tune each of their groups themselves.  Without tuning
 * the library uses fixed rules measured on MI355X.
 * crs_legendre_choice writes the variant in use for a shape to out[5]:
 * synthesis on matrix cores (0/1), synthesis ring pairs per lane, adjoint on
 * matrix cores (0/1), adjoint ring pairs per lane, adjoint tiles per wave.
 * Errors: CRS_EINVAL for a NULL grid / out, lmax < 0 or nmaps < 1.
 */
int crs_autotune_legendre(crs_grid g, int lmax, int nmaps, crs_stream s);
int crs_legendre_choice(crs_grid g, int lmax, int nmaps, int* out);

/* ------------------------------------------------------------------ model
 * One band (sky map) nu of Sect. 2.2: grid, band-limit L_nu, beam b_{nu,l}
 * (host, lmax+1; modes above L_nu are not represented), inverse-noise map
 * tau = diag(N_nu^-1) (host, npix, >= 0; 0 marks masked pixels) and the
 * mixing scalars q_{nu,k} (host, ncomp) of the spatially constant mixing
 * Q~_{nu,k} = q_{nu,k} I (Sect. 3.3).  tau, beam and q are copied.
 */
typedef struct {
  crs_grid grid;
  int lmax;
  const double* beam;
  const double* tau;
  const double* q;
} crs_band_desc;

/* The model: ncomp components with band-limits L_k (host array) and prior
 * inverse spectra C_{k,l}^-1 (host pointers, each L_k+1 values >= 0; 0 means
 * no prior for that mode, Sect. 3.3 under eq:U-prior), plus nbands bands.
 * Creation computes alpha_nu (App. A.1, eq:optimal-alpha), the blocks U_l^+
 * (Sect. 3.3) and the T^+ pixel weights alpha^2 w^2 tau^+ (tau^+ = 1/tau where
 * tau > 0, else 0), and with flags & CRS_MODEL_DIAG also the M_diag blocks.
 */
enum { CRS_MODEL_DIAG = 1 };
typedef struct {
  int ncomp;
  const int* lmax_comp;
  const double* const* inv_cl;
  int nbands;
  const crs_band_desc* bands;
  int flags;
} crs_model_desc;

int crs_model_create(const crs_model_desc* d, crs_stream s, crs_model* out);
int crs_model_destroy(crs_model m);
/* n = sum_k (L_k+1)^2 */
int crs_model_size(crs_model m, int64_t* n);
/* Memory plan (host computation, nothing allocated): the model's own
 * device tables (model_bytes) and the operator / solver state for nrhs
 * right-hand sides (exec_bytes: per (grid, L) group the harmonic inputs,
 * phase array, adjoint partial sums and pixel maps, plus the PCG vectors).
 * The first operator call with a new nrhs allocates exec_bytes; it returns
 * CRS_ENOMEM before allocating anything if they exceed the free device
 * memory.  Either pointer may be NULL. */
int crs_model_plan_bytes(crs_model m, int nrhs, int64_t* model_bytes, int64_t* exec_bytes);
/* alpha_nu^2 for every band (host array of nbands). */
int crs_model_alpha2(crs_model m, double* alpha2);
/* Replace the mixing matrix q (host, nbands x ncomp, row = band) and
 * recompute U^+ (and M_diag if present). */
int crs_model_set_mixing(crs_model m, const double* q, crs_stream s);

/* Spatially varying mixing (Sect. 2.2, eq:P, eq:Q): the block (band, comp)
 * of P becomes Y_nu B_nu Q~ with Q~ = Y^T W Q Y, Q = diag(qmap) on grid (any
 * of the library's grids; Gauss-Legendre gives an exact quadrature at the
 * band-limit), applied at the component's band-limit L_k (the product's
 * modes above L_k are dropped).  qmap: host, npix of grid, finite, positive
 * sum; NULL returns the pair to its scalar q.  The pair's scalar in M_PI and
 * M_diag becomes sum q^2 / sum q (App. A.2, eq:optimal-q).  Each varying pair
 * adds four SHTs at L_k on its grid to every application of A (two before the
 * forward mix, two after the transpose), and to build_rhs / project.
 * A model with mask-in-mixing (Sect. 4.1) is the special case qmap = q (1 -
 * mask).  Supported on single models (batches of such models return
 * CRS_EUNSUPPORTED, and so do the mixing gradients apply_dA_dmix /
 * apply_db_dmix).  The grid must outlive the model.  Synchronises the
 * stream; the model's operator state is rebuilt. */
int crs_model_set_mixing_map(crs_model m, int band, int comp, crs_grid grid, const double* qmap,
                             crs_stream s);

/* Observation merging in the pseudo-inverse preconditioner (App. A.3):
 * group: host array of nbands, the merge group of each band (-1 = not
 * merged; NULL clears all merging).  Bands of one group must share grid and
 * band-limit.  In each group the lowest band index keeps a row of U, scaled
 * by sqrt(1 + sum gamma_l^2) with gamma_l the least-squares scale of each
 * other member's row onto it at multipole l (the printed (gamma + 1)^{1/2}
 * read as (1 + gamma^2)^{1/2}); the other members drop out of U^+ and T^+,
 * so M_PI runs their SHTs no longer.  A and M_diag are unchanged.  Exact
 * for bands whose rows are proportional and whose normalised inverse noise
 * agrees (detector sub-sets of one channel); a compromise otherwise.
 * Synchronises the stream; the model's operator state is rebuilt. */
int crs_model_merge_observations(crs_model m, const int* group, crs_stream s);

/* ------------------------------------------------ mask-restricted preconditioner
 * M_mask = Z^T (Z S^-1 Z^T)^-1 Z (Sect. 4.2, eq:M_mask), Z = synthesis to the
 * masked pixels of a HEALPix grid after the low-pass r_l = exp(-beta l^2
 * (l+1)^2) with r_{L/2}^2 = lowpass_r2 (Sect. 4.3, eq:rl), L the components'
 * band-limit; (Z S^-1 Z^T)^-1 approximated by the multigrid V-cycle of
 * Sect. 4.4 (fig:code:mg, J taken as I): HEALPix levels with Nside and L
 * halved, a coarse pixel masked when its four children are, Gaussian
 * restriction of one coarse pixel FWHM, smoother omega / diag(G), bottom at
 * the first level with fewer than nbottom masked pixels solved by the
 * pseudo-inverse of its dense G (eigenvalues below rcond * max dropped).
 * Each component with a prior gets its own cycle; those components must
 * share one band-limit (else CRS_EUNSUPPORTED).  The preconditioner
 * CRS_PRECOND_ADD is M_add = M_PI + M_mask (Sect. 4.2).
 * crs_model_set_mask: grid: HEALPix; mask: host, npix bytes, nonzero =
 * masked; opts: NULL or fields 0 for the defaults (0.05, 0.2, 1000, 1e-6,
 * J taken as I).
 * The grid must outlive the model.  Setup: allocates, builds the level grids
 * and tables, eigendecomposes the bottom level on the device (rocSOLVER),
 * synchronises the stream.
 * crs_model_mask_info: number of levels and, per level, (Nside, L, masked
 * pixels) into out (host, n ints; as many levels as fit).
 * apply_mask_precond: z = M_mask r (device, nrhs x n). */
typedef struct {
  double lowpass_r2;
  double omega;
  int nbottom;
  double rcond;
  int exact_j;  /* nonzero: apply J = Y_h^T W_h Y_h (masked pixels) exactly in
                   the cycle, four more transforms per level; the cycle is then
                   the textbook V-cycle, symmetric (J taken as I otherwise) */
} crs_mask_opts;
int crs_model_set_mask(crs_model m, crs_grid grid, const uint8_t* mask, const crs_mask_opts* opts,
                       crs_stream s);
int crs_model_mask_info(crs_model m, int* nlevels, int* out, int n);
int apply_mask_precond(crs_model m, int nrhs, const double* r, double* z, crs_stream s);

/* Operators on nrhs stacked component vectors (device, nrhs x n, contiguous).
 * apply_A: y = A x (eq:A).  apply_pinv_precond: z = M_PI r.
 * apply_diag_precond: z = M_diag r (needs CRS_MODEL_DIAG). */
int apply_A(crs_model m, int nrhs, const double* x, double* y, crs_stream s);
int apply_pinv_precond(crs_model m, int nrhs, const double* r, double* z, crs_stream s);
int apply_diag_precond(crs_model m, int nrhs, const double* r, double* z, crs_stream s);

/* Preconditioned CG (Sect. 2.3) on nrhs independent right-hand sides.
 * b: device nrhs x n.  x: device nrhs x n, initial guess on entry (use zeros
 * for the paper's x_1 = 0), solution on exit.  Each RHS stops when its
 * recursive residual |r|/|b| <= rtol; the true residual is then formed once
 * and the RHS restarts from its iterate if that fails rtol.
 * iters, relres: host arrays of nrhs (iterations used, final true relative
 * residual), may be NULL.  The host reads one scalar per iteration to test
 * convergence.  Returns CRS_ENOTCONV if any RHS hit maxiter, CRS_EBREAKDOWN
 * on breakdown (x then holds the last good iterate of that RHS).
 * history: optional host array of maxiter * nrhs recursive relative residuals
 * (row = iteration), may be NULL. */
int pcg_solve(crs_model m, int precond, int nrhs, const double* b, double* x,
              double rtol, int maxiter, int* iters, double* relres, double* history,
              crs_stream s);

/* Right-hand side (Sect. 2.3, with S^-1 omega_2 read as S^-1/2 omega_2):
 *   b = sum_nu P_nu^T (tau_nu d_nu + tau_nu^1/2 omega1_nu) + C^-1/2 omega2.
 * d, omega1: host arrays of nbands device pointers, each nrhs x npix_nu
 * (the array itself or any entry may be NULL = zero).  omega2: device
 * nrhs x n or NULL.  b: device nrhs x n. */
int build_rhs(crs_model m, int nrhs, const double* const* d, const double* const* omega1,
              const double* omega2, double* b, crs_stream s);

/* Constrained realization (mode CRS_MODE_CR) or Wiener filter (CRS_MODE_WF):
 * draws omega_1, omega_2 on the device with Philox4x64-10 (key = (seed,
 * stream id), counter = (i/4, rhs, 0, 0), Box-Muller), builds b and runs
 * pcg_solve from x = 0.  d as in build_rhs.  x: device nrhs x n. */
int constrained_realization(crs_model m, int nrhs, const double* const* d, uint64_t seed,
                            int mode, int precond, double rtol, int maxiter, double* x,
                            int* iters, double* relres, crs_stream s);

/* P_nu x for every band (eq:P): maps is a host array of nbands device
 * pointers, each receiving nrhs x npix_nu doubles.  x: device nrhs x n.
 * (Used to synthesise data d = P s + n.) */
int crs_model_project(crs_model m, int nrhs, const double* x, double* const* maps, crs_stream s);

/* ------------------------------------------------------ differentiation
 * Building blocks of implicit gradients through the solve (Sect. 2.3 with
 * the mixing q_{nu,k} of Sect. 3.3 as parameters).  All vectors are device
 * nrhs x n; dq is device nrhs x nbands x ncomp (row-major), overwritten.
 *
 * apply_prior_inv: y = S^-1 x (C_{k,l}^-1 per coefficient).
 * apply_dA_dmix:   dq[r][nu][k] = -lam_r^T (dA/dq_{nu,k}) x_r
 *                  = -(lam_{r,k} . B_nu Y^T tau Y B_nu u^x_nu + x_{r,k} . B_nu Y^T tau Y B_nu u^lam_nu),
 *                  u^v_nu = sum_k' q_{nu,k'} v_k'  (two SHT round trips per band).
 * apply_db_dmix:   dq[r][nu][k] = lam_r^T (db/dq_{nu,k}) for b = sum_nu P_nu^T tau d_nu
 *                  = lam_{r,k} . B_nu Y^T (tau d_{r,nu}); d as in build_rhs (host array of
 *                  nbands device pointers, each nrhs x npix_nu; NULL entries are zero).
 */
int apply_prior_inv(crs_model m, int nrhs, const double* x, double* y, crs_stream s);
/* The terms of a Wiener-filter loss L = 1/2 x^T S^-1 x + chi^2 (the prior
 * term and the data misfit of the posterior of Sect. 2.3) and its gradient
 * with respect to the data maps:
 * crs_prior_quad:   y = S^-1 x and val[r] = 1/2 x_r^T S^-1 x_r (val: device, nrhs).
 * crs_chi2:         res_nu = d_nu - P_nu x (res: host array of nbands device
 *                   pointers, each nrhs x npix_nu, written) and
 *                   val[r] = sum_nu res_nu^T N_nu^-1 res_nu (device, nrhs);
 *                   d as in build_rhs (NULL entries are zero).
 * crs_noise_weight: out_nu = scale N_nu^-1 in_nu, per band (in / out as res;
 *                   NULL in entries are zero).  With in = P lam it gives
 *                   dL/dd through the right-hand side; with in = res and
 *                   scale 2 the chi-square's own dL/dd.
 * These calls synchronise the stream before returning. */
int crs_prior_quad(crs_model m, int nrhs, const double* x, double* y, double* val, crs_stream s);
int crs_chi2(crs_model m, int nrhs, const double* x, const double* const* d, double* const* res,
             double* val, crs_stream s);
int crs_noise_weight(crs_model m, int nrhs, double scale, const double* const* in, double* const* out,
                     crs_stream s);
int apply_dA_dmix(crs_model m, int nrhs, const double* lam, const double* x, double* dq,
                  crs_stream s);
int apply_db_dmix(crs_model m, int nrhs, const double* lam, const double* const* d, double* dq,
                  crs_stream s);

/* Device normals of the library's Philox stream (the omega draws of
 * constrained_realization): out[i] for i < n, device array. */
int crs_philox_normals(uint64_t seed, uint64_t stream, uint64_t rhs, int64_t n, double* out,
                       crs_stream s);

/* ------------------------------------------------------------------ batch
 * Many independent problems (models) solved together: the batch stacks
 * their component vectors, merges the bands of all problems that share
 * (grid, L_nu) into one group per transform launch, and advances every
 * problem's PCG (each with its own scalars and stopping test) in lockstep.
 * models: host array of nprob model handles; the models must outlive the
 * batch and must not be modified while it exists.  Allocates the batch's
 * workspaces.
 */
int crs_batch_create(const crs_model* models, int nprob, crs_stream s, crs_batch* out);
int crs_batch_destroy(crs_batch b);
/* Number of problems and total stacked vector length (host scalars). */
int crs_batch_info(crs_batch b, int* nprob, int64_t* ntot);
/* Wiener filter (CRS_MODE_WF) or constrained realization (CRS_MODE_CR) of
 * every problem from x = 0.  d: host array of nprob entries, each NULL or a
 * host array of the problem's nbands device map pointers (NULL = zero data),
 * each npix_nu doubles.  seeds: host array of nprob Philox seeds (CR mode;
 * problem p draws exactly the omegas of constrained_realization with seed
 * seeds[p]).  x: host array of nprob device pointers receiving n_p doubles.
 * iters, relres: host arrays of nprob, may be NULL.  use_graph != 0 runs the
 * PCG (Sect. 2.3) in chunks of 8 iterations, each chunk one captured hipGraph
 * launch: every iteration stops the problems whose recursive residual passes
 * rtol on the device, and between chunks the host checks their true
 * residuals and restarts the ones that fail; transform groups whose problems
 * have all finished are left out of the graph (graphs are captured per set of
 * live groups and kept for later solves).  use_graph = 0 runs one iteration
 * at a time with a host decision after each.  Returns as pcg_solve. */
int crs_batch_solve(crs_batch b, int mode, const double* const* const* d, const uint64_t* seeds,
                    int precond, double rtol, int maxiter, double* const* x, int* iters,
                    double* relres, int use_graph, crs_stream s);
/* Counters of the batch's last solve (host array out[4]): iterations of the
 * slowest problem, graph launches, graphs captured, host reads of the PCG
 * flags. */
int crs_batch_stats(crs_batch b, int* out);
/* Runs the batch's transform groups (the bands sharing a grid and
 * band-limit) on up to nstreams HIP streams (1..8; default 1, or the
 * environment variable CRS_GROUP_STREAMS at creation): the groups of one
 * operator application are independent until the back-mix (eq:A sums over
 * bands), so their launches may overlap, forked from and joined back into the
 * solve's stream by events (graph edges inside the captured chunks).  The
 * extra streams have the default priority and are created here; results do
 * not depend on nstreams.  CRS_EINVAL outside 1..8. */
int crs_batch_set_streams(crs_batch b, int nstreams);

/* ------------------------------------------------------------- profiling
 * With profiling on, every Legendre-stage kernel launch is bracketed by HIP
 * events on its stream; crs_kernel_stats synchronises on those events and
 * reports, per kernel family ("legendre_synth", "legendre_adjoint",
 * "ring_fft"), launches, summed device time and summed algorithmic work
 * (flops for Legendre, bytes for ring_fft). */
int crs_set_profiling(int on);
int crs_kernel_stats(const char* family, int64_t* launches, double* total_ms,
                     double* total_work);
/* The summed work of a family counted three ways (work3, host array of 3):
 * [0] Legendre flops over the (ring pair, l, m) triples whose |lambda_lm|
 * reaches the float64 normal range (the figure crs_kernel_stats reports),
 * [1] over all triples (nominal), [2] over the triples the kernels evaluate
 * (|lambda_lm| >= 2^-100).  Legendre flops per triple: 4 for the recurrence
 * plus 4 per map.  Launches on finished systems are credited with the work
 * of the maps still active.  ring_fft: bytes in all three. */
int crs_kernel_work_counts(const char* family, double* work3);
int crs_kernel_stats_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* CRSOLVE_H */
