/*
 * kryging.h -- C ABI of the MI355X (gfx950) Kryging hot path.
 *
 * The library evaluates Gaussian-process likelihoods and kriging predictions
 * for data on a regular n1 x n2 grid with missing cells, following
 * Majumder, Guan, Reich & Saibaba, "Kryging: Geostatistical analysis of
 * large-scale datasets using Krylov subspace methods":
 *
 *   model (Sec. 2, eq. obs_mod):  y = X beta + A x + eps,  x ~ N(0, sigma^2 Sigma),
 *                                 eps ~ N(0, tau^2 I), A = identity with the
 *                                 rows of unobserved cells removed;
 *   Sigma (Sec. 2):               Matern correlation with range, smoothness
 *                                 and (rotated) geometric anisotropy; on a
 *                                 grid it is symmetric BTTB (Sec. 3);
 *   K  = A Sigma A^T + eta I,     eta = tau^2 / sigma^2, the unit-variance
 *                                 covariance of the observations;
 *   X beta:                       covariates (kry_problem_set_covariates),
 *                                 beta estimated by generalised least
 *                                 squares; without covariates the mean is 0.
 *
 * Every device step runs in the library's own HIP kernels.  Conventions that
 * hold for every entry point:
 *
 *  - Return value: kry_status, KRY_OK (0) on success.  On failure a message
 *    is available from kry_last_error() (thread-local, valid until the next
 *    failing call on that thread).  Inputs are validated before any device
 *    work; on KRY_EINVAL no output is written.  No C++ exception crosses the
 *    ABI.
 *  - Ownership: the caller owns every host array passed in or out and needs
 *    to keep it alive only for the duration of the call; the library copies
 *    inputs and writes caller-allocated outputs.  Handles are opaque and owned
 *    by the library; every destroy function accepts NULL.
 *  - Grid layout: cell (i, j) is row i (spacing dx1) and column j (spacing
 *    dx2), row-major cell id i * n2 + j.  "Compact" vectors hold one value
 *    per observed cell, in increasing cell id.
 *  - Calls are synchronous: when an entry point taking host buffers returns,
 *    its outputs are written.  One kry_ctx (and the problems made from it)
 *    must be used from one host thread at a time.
 */
#ifndef KRYGING_H
#define KRYGING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KRY_OK = 0,
    KRY_EINVAL = 1,   /* invalid argument (message says which)              */
    KRY_ENOMEM = 2,   /* device allocation failed or above the HBM budget   */
    KRY_EDEVICE = 3,  /* HIP runtime error                                  */
    KRY_ENOTPSD = 4,  /* circulant embedding not PSD within the size cap    */
    KRY_ENOCONV = 5,  /* iteration limit reached; outputs still written     */
    KRY_EBUSY = 6,    /* server queue full                                  */
    KRY_ENOTIMPL = 7  /* feature not available                              */
} kry_status;

typedef struct kry_ctx kry_ctx;
typedef struct kry_problem kry_problem;
typedef struct kry_server kry_server;

/* Regular grid: n1 rows x n2 columns, 2 <= n1, n2 <= 4096, spacings > 0. */
typedef struct {
    int32_t n1, n2;
    double dx1, dx2;
} kry_grid;

/* Matern parameters (Sec. 2): marginal variance sigma2 > 0, nugget
 * variance tau2 >= 0, range > 0 (along the major axis), smoothness nu > 0,
 * anisotropy ratio >= 1 (1 = isotropic) and angle (radians, counter-clockwise
 * from the +column axis) of the major axis. */
typedef struct {
    double sigma2, tau2, range, nu, aniso_ratio, aniso_angle;
} kry_matern;

typedef enum { KRY_FP64 = 0, KRY_FP32 = 1 } kry_precision;
typedef enum { KRY_PROBE_RADEMACHER = 0, KRY_PROBE_COLOURED = 1 } kry_probe_kind;
typedef enum { KRY_SOLVER_CG = 0, KRY_SOLVER_GENGK = 1 } kry_solver;

/* Options.  precision = KRY_FP32 is the mixed form: transforms and Krylov
 * vectors in FP32; dot products, Lanczos coefficients, quadrature, CG
 * scalars and the likelihood in FP64, with FP64 residual refinement in CG. */
typedef struct {
    int32_t lanczos_steps;   /* m, Lanczos steps per probe (1..1024)        */
    int32_t num_probes;      /* N, Rademacher probes (ignored if coloured)  */
    int32_t probe_kind;      /* kry_probe_kind                              */
    int32_t colour_period;   /* c for coloured probes (c*c probes)          */
    uint64_t seed;           /* Philox key for probes and samples           */
    int32_t reorth;          /* 1 = full reorthogonalisation (FP64 coeffs)  */
    int32_t precision;       /* kry_precision                               */
    double cg_rtol;          /* CG stop: ||r|| <= cg_rtol ||b||             */
    int32_t cg_maxit;        /* CG iteration cap                            */
    int32_t solver;          /* kry_solver for the quadratic form           */
    int32_t gk_steps;        /* k for genGK                                 */
    int32_t shift_share;     /* 1 = points of one call that differ only in
                                the nugget ratio share Krylov spaces (below) */
    int32_t lanczos_max_steps; /* adaptive mode: cap on the steps (10..1024) */
    double lanczos_rtol;     /* > 0: adaptive mode for the log-determinants:
                                checks after steps 5, 10, ..., each
                                5 max(1, floor(j / 50)) steps after the last
                                (every 5 to step 100, every 10 to 150, ...);
                                from step 10 on, stop once every probe's
                                quadrature value moved by at most lanczos_rtol
                                times its size since the previous check (or
                                at lanczos_max_steps); lanczos_steps is then
                                unused.  0 = exactly lanczos_steps.        */
    int32_t reml;            /* with covariates: 0 = likelihood with beta at its
                                GLS estimate, 1 = restricted likelihood (of
                                the error contrasts; see kry_loglik)        */
} kry_opts;

/* Largest number of covariate columns a problem takes. */
#define KRY_MAX_COVARIATES 8

typedef struct {
    double loglik;           /* l at the given sigma2                       */
    double loglik_profiled;  /* l_p with sigma2 = sigma2_hat                */
    double sigma2_hat;       /* Q / p                                       */
    double logdet;           /* estimate of log det K                       */
    double logdet_se;        /* probe standard error of logdet              */
    double quad;             /* Q = y^T K^{-1} y                            */
    int64_t p;               /* number of observed cells                    */
    int32_t lanczos_steps_used; /* max over probes                          */
    int32_t cg_iters;        /* CG iterations (or genGK steps)              */
    double cg_relres;        /* final relative residual                     */
    /* covariates (all 0 without): */
    int32_t ncov;            /* q, covariate columns of the problem         */
    double beta[KRY_MAX_COVARIATES];    /* GLS estimate of beta (first q)   */
    double beta_se[KRY_MAX_COVARIATES]; /* sqrt diag(sigma2_hat G^{-1}),
                                           G = X^T K^{-1} X                 */
    double logdet_xkx;       /* log det G                                   */
} kry_loglik_result;

/* ---- status, options ---------------------------------------------------- */
const char* kry_status_string(kry_status s);
const char* kry_last_error(void);

/* Defaults: m = 30, N = 10 Rademacher, seed 303, no reorth, FP64,
 * cg_rtol 1e-8, cg_maxit 20000, CG, gk_steps 100, no shift sharing, fixed
 * step count (lanczos_rtol 0, lanczos_max_steps 500), reml 0. */
kry_status kry_opts_default(kry_opts* out);

/* ---- stage timing ----------------------------------------------------------- */
/* Start recording HIP events around the three stage kernels of every masked
 * product launched through this context (on the stream each is launched
 * on).  Adds two event records per stage launch. */
kry_status kry_profile_begin(kry_ctx* ctx);
/* Stop recording; synchronise the device and return, for stages A (row
 * transform), B (column transform and spectrum multiply) and C (inverse row
 * transform and gather): total milliseconds ms[3], launch counts
 * launches[3], and the number of vectors the recorded products processed. */
kry_status kry_profile_end(kry_ctx* ctx, double* ms, int64_t* launches, int64_t* vectors);

/* ---- launch configuration of the masked product ----------------------------- */
/* Per (embedding, precision) choice of how the product's stage kernels are
 * laid out.  Every choice computes bit-identical results; only speed
 * differs. */
typedef struct {
    int32_t col_vectors;    /* vectors per workgroup of the column stage: 1 or 2          */
    int32_t row_tile_scale; /* rows per row-stage tile: 64-byte runs of the transposed
                               intermediate times this (1 or 2; capped by LDS)           */
    int32_t row_vthreads;   /* values per thread in the row stages: 8 x this (1 or 2;
                               2 only for rows of >= 1024 points)                         */
    int32_t col_split;      /* 1: the column stage exchanges real and imaginary parts
                               through LDS separately (half the LDS per workgroup, more
                               workgroups per CU; columns of >= 256 points), 0: together */
    int32_t row_split;      /* the row stages likewise, bit 0 the forward (first) stage,
                               bit 1 the inverse (last) stage: 0..3 (rows of >= 1024
                               points of the half-length complex transform)               */
    double ms;              /* kry_autotune: time of one product of nvec vectors        */
} kry_tuning;

/* Time configurations on the problem's own embedding with a product of nvec
 * (1..4096) compact vectors in `precision`, keep the fastest for that
 * embedding, precision and batch class in the problem's context and return
 * it.  There are two batch classes, products of at most 8 vectors and larger
 * ones; a product uses its class's setting, else the other class's, else the
 * built-in default.  The row-stage fields are searched first
 * (every combination, column stage at its default), then the column-stage
 * fields with the best row setting.  Each candidate runs 2 untimed and 5
 * timed products (HIP events on the context's stream); ms is the fastest's
 * median. */
kry_status kry_autotune(kry_problem* prob, int32_t precision, int32_t nvec, kry_tuning* out);
/* Set (t != NULL) or reset to the built-in default (t == NULL) the
 * configuration used for embedding N1 x N2 in `precision` on this context,
 * for both batch classes; KRY_EINVAL for values outside the ranges above.
 * kry_get_tuning returns the setting of the larger batch class (else the
 * smaller's, else the default). */
kry_status kry_set_tuning(kry_ctx* ctx, int32_t N1, int32_t N2, int32_t precision, const kry_tuning* t);
/* The configuration in use for N1 x N2 in `precision` (ms = 0 unless set by
 * kry_autotune). */
kry_status kry_get_tuning(kry_ctx* ctx, int32_t N1, int32_t N2, int32_t precision, kry_tuning* out);

/* CG solves run their iterations in blocks of 16 between convergence reads;
 * with graphs enabled (the default) every block after the first replays one
 * captured HIP graph of the block's kernel launches instead of launching them
 * one by one (the first block runs directly and sizes the workspaces).
 * Results are bit-identical either way.  Not while stage profiling is on,
 * and not inside the request server, whose slots run in several threads. */
kry_status kry_set_graphs(kry_ctx* ctx, int32_t enable);

/* ---- context and problems ----------------------------------------------- */
/* Binds HIP device `device`; hbm_budget_bytes = 0 means no limit beyond the
 * device.  Creates the library's stream (default priority). */
kry_status kry_ctx_create(int32_t device, uint64_t hbm_budget_bytes, kry_ctx** out);
void kry_ctx_destroy(kry_ctx* ctx);
/* How problems created on the context choose their embedding sides (each
 * side independently; any side >= 2 n - 1 gives the exact product, Sec. 3.3):
 * KRY_EMBED_FAST (the default) takes the supported side >= max(16, 2 n - 1)
 * with the least N w(N), where w = 1 for powers of two, 1.2 for a side with
 * one factor 3, 5 or 7 and 1.75 for a side with more (their transforms cost
 * more per point);
 * KRY_EMBED_SMALLEST takes the smallest supported side (least memory).
 * Supported sides: powers of two and multiples of 16 with no prime factor
 * above 7, in [16, 8192].  KRY_EINVAL for another rule. */
enum { KRY_EMBED_FAST = 0, KRY_EMBED_SMALLEST = 1 };
kry_status kry_ctx_set_embedding(kry_ctx* ctx, int32_t rule);
/* Device bytes the context holds now (problems, workspaces, tables, server
 * slots) and the most it has held since creation or the last reset
 * (reset_peak != 0 sets the peak to the current value after reading it).
 * Not part of the paper's method: the request server's admission by HBM
 * footprint is checked against it. */
kry_status kry_ctx_memory(kry_ctx* ctx, uint64_t* allocated, uint64_t* peak, int32_t reset_peak);

/* A problem: grid, observation mask (n1*n2 bytes, nonzero = observed; at
 * least one observed cell) and data y (n1*n2 doubles read only where
 * observed, must be finite; NULL = zeros).  Uploads the mask in packed form
 * and y to the device.  The embedding used by the masked product (Sec. 3.3)
 * follows the context's embedding rule (kry_ctx_set_embedding). */
kry_status kry_problem_create(kry_ctx* ctx, const kry_grid* grid, const uint8_t* mask,
                              const double* y, kry_problem** out);
/* A problem with irregularly spaced observations (Sec. 2): the latent field
 * on the grid and p observations at locs (p x 2 doubles: fractional row and
 * fractional column in grid units, grid point (a, b) at (a, b), each inside
 * [0, n1 - 1] x [0, n2 - 1]).  Observation j is the convex combination
 * A_ji = w(d_ji) / sum_k w(d_jk) of the grid values, with the Wendland
 * function w(d) = (1 - d)_+^4 (1 + 4 d) and d = max(|u1 - a|, |u2 - b|) (at
 * most the four corners of its cell; an observation on a grid point takes
 * that value exactly).  y: p doubles (NULL = zeros).  The covariance of the
 * observations is K = A Sigma A^T + eta I, applied as A^T, the grid product
 * and A.  Every entry point taking a problem works on it except:
 * kry_loglik_multi (KRY_EINVAL) and kriging with covariates (KRY_ENOTIMPL);
 * kriging targets are grid cells (NULL = every cell, ntargets = n1*n2),
 * kry_problem_set_data takes p values and kry_problem_set_covariates q x p
 * values (one per observation); coloured probes colour an observation by
 * its nearest grid cell; bootstrap noise uses the observation index. */
kry_status kry_problem_create_irregular(kry_ctx* ctx, const kry_grid* grid, int64_t p, const double* locs,
                                        const double* y, kry_problem** out);
/* Replace the data (n1*n2 doubles, read where observed; p doubles for an
 * irregular problem). */
kry_status kry_problem_set_data(kry_problem* prob, const double* y);
/* Covariates of the mean X beta (Sec. 2, eq. obs_mod): q columns of n1*n2
 * doubles each (X is q x n1*n2, row-major), read where observed and, for
 * kriging, at the targets; finite.  0 <= q <= KRY_MAX_COVARIATES, q < p, and
 * the columns restricted to the observed cells must be linearly independent
 * (KRY_EINVAL otherwise).  q = 0 (X may be NULL) restores the zero mean.
 * With covariates the likelihoods take beta at its generalised least-squares
 * estimate for each parameter point, kriging adds X_t beta_hat to the mean,
 * and solves and products are unchanged. */
kry_status kry_problem_set_covariates(kry_problem* prob, int32_t q, const double* X);
/* Observed count p and embedding sizes N1, N2 (any pointer may be NULL). */
kry_status kry_problem_info(const kry_problem* prob, int64_t* p, int32_t* N1, int32_t* N2);
void kry_problem_destroy(kry_problem* prob);

/* ---- lag grid and spectrum (Sec. 2 Matern; Sec. 3.3 BCCB embedding) ---- */
/* Lag grid c of the N1 x N2 block-circulant embedding (row-major):
 * c[l1][l2] = C(h2 dx2, h1 dx1) at the wrapped lag (h1, h2); on a Nyquist
 * line (l = N/2) the mean over both aliases.  N1, N2 = 0 selects the
 * problem's own embedding; otherwise supported sides in [16, 8192] (powers
 * of two, or multiples of 16 with no prime factor above 7). */
kry_status kry_lag_grid(kry_problem* prob, const kry_matern* theta, int32_t N1, int32_t N2,
                        double* c_out /* N1*N2 */);
/* Eigenvalues lam = DFT2(c) on the half spectrum, layout [k2][k1] with
 * k2 in [0, N2/2], k1 in [0, N1) (so lam_out has (N2/2+1)*N1 doubles), and
 * minmax = {min lam, max lam}.  Sizes as for kry_lag_grid. */
kry_status kry_spectrum(kry_problem* prob, const kry_matern* theta, int32_t N1, int32_t N2,
                        double* lam_out, double* minmax);

/* ---- masked BTTB product (Sec. 3, 3.2: circulant embedding + FFT) ------ */
/* out = K v for nvec compact vectors (nvec x p, row-major, host). */
kry_status kry_matvec(kry_problem* prob, const kry_matern* theta, int32_t precision,
                      int32_t nvec, const double* v, double* out);
/* Same on device buffers of the precision's element type (double or float),
 * nvec x p contiguous, enqueued on `hip_stream` (NULL = library stream);
 * returns after enqueueing.  The library's workspace for this call is owned
 * by the problem and reused by later calls on the same stream. */
kry_status kry_matvec_device(kry_problem* prob, const kry_matern* theta, int32_t precision,
                             int32_t nvec, const void* d_v, void* d_out, void* hip_stream);
/* For callers that cannot allocate device memory (code under HIP stream
 * capture, serving loops, harnesses that forbid hipMalloc): the product of
 * kry_matvec_device, same arguments, layout and results, with every
 * intermediate (lag grid, spectrum, transform intermediate) in one
 * file-scope device array of KRY_NOALLOC_SCRATCH_BYTES per GPU, held from
 * library load until the process ends.  Nothing is allocated and nothing
 * waits: the spectrum is recomputed and the work only enqueued on
 * `hip_stream`.  Masked grid problems only (KRY_EINVAL for irregular ones);
 * KRY_EINVAL with a message when the embedding's spectrum or one vector's
 * intermediate does not fit (embeddings up to 2048 x 2048 fit; larger
 * batches go through in chunks).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race
 * and must be serialised by the caller. */
#define KRY_NOALLOC_SCRATCH_BYTES (256ull << 20)
kry_status kry_matvec_device_noalloc(kry_problem* prob, const kry_matern* theta, int32_t precision,
                                     int32_t nvec, const void* d_v, void* d_out, void* hip_stream);
/* Sigma A^T w: compact vectors in, full-grid vectors out (nvec x n1*n2),
 * no nugget -- the kriging-mean product (eq. act_xhat) and the Sigma
 * product of Algorithm 1. */
kry_status kry_cov_apply_full(kry_problem* prob, const kry_matern* theta, int32_t precision,
                              int32_t nvec, const double* w, double* out);

/* ---- probes and Lanczos quadrature (log det alternative of Sec. 3.3) --- */
/* The probe vectors used by kry_logdet (nprobe x p, compact); nprobe is
 * N for Rademacher and c*c for coloured probes (query with out = NULL). */
kry_status kry_probes(kry_problem* prob, const kry_opts* opts, int32_t* nprobe, double* out);
/* Lanczos coefficients for every probe: alpha (nprobe x m), beta
 * (nprobe x m; beta[k][j] couples steps j and j+1, beta[k][m-1] unused) and
 * the steps each probe ran before an exact breakdown. */
kry_status kry_lanczos(kry_problem* prob, const kry_matern* theta, const kry_opts* opts,
                       double* alpha, double* beta, int32_t* steps);
/* SLQ estimate of log det K: Gauss quadrature of every probe's tridiagonal
 * (per_probe, nullable, nprobe values) combined as the mean (Rademacher) or
 * the sum (coloured), with its probe standard error. */
kry_status kry_logdet(kry_problem* prob, const kry_matern* theta, const kry_opts* opts,
                      double* logdet, double* se, double* per_probe);

/* Gauss quadrature of given Lanczos tridiagonals on the device (implicit QL
 * with first eigenvector components): for probe k with steps[k] = s,
 * T = tridiag(beta[k][0..s-2], alpha[k][0..s-1]) and
 * gamma[k] = znorm2[k] * sum_i tau_i^2 log theta_i.  alpha, beta: nprobe x m
 * host arrays; uses the current HIP device. */
kry_status kry_gauss_quadrature(int32_t nprobe, int32_t m, const double* alpha, const double* beta,
                                const int32_t* steps, const double* znorm2, double* gamma);

/* ---- solves --------------------------------------------------------------- */
/* CG solve K x = b for nrhs compact right-hand sides (nrhs x p); iters and
 * relres per right-hand side (nullable). KRY_ENOCONV if cg_maxit reached. */
kry_status kry_solve(kry_problem* prob, const kry_matern* theta, const kry_opts* opts,
                     int32_t nrhs, const double* b, double* x, int32_t* iters, double* relres);
/* Algorithm 1 (genGK) for k = opts->gk_steps steps on the problem's data with
 * A the selection and R = tau^2 I: alpha (k+1), beta (k+1) of B_k, z_k (k)
 * of eq. xhat_est, the full-grid x_k* (n1*n2, nullable) and
 * J = ||B_k z - beta1 e1||^2 + ||z||^2 / sigma^2 (sigma^2 J approximates Q). */
kry_status kry_gengk(kry_problem* prob, const kry_matern* theta, const kry_opts* opts,
                     double* alpha, double* beta, double* z, double* x_full, double* J);

/* ---- likelihood, fit, kriging ------------------------------------------- */
/* Log-likelihood of the problem's data: logdet by SLQ, Q by CG (or genGK),
 * l = -1/2 [p log(2 pi sigma2) + logdet + Q / sigma2], sigma2_hat = Q / p,
 * l_p = -1/2 [p (log 2 pi + log sigma2_hat + 1) + logdet].
 *
 * With q covariates, beta_hat = G^{-1} X^T K^{-1} y with G = X^T K^{-1} X
 * (the beta that maximises l at the given covariance parameters) and
 * Q = (y - X beta_hat)^T K^{-1} (y - X beta_hat).  The K^{-1} X columns are
 * solved together with the data (q + 1 right-hand sides per point; genGK
 * runs on the residual y - X beta_hat).  With opts->reml = 1 the restricted
 * likelihood replaces l (m = p - q):
 *   l = -1/2 [m log(2 pi sigma2) + logdet + log det G - log det X^T X + Q / sigma2],
 *   sigma2_hat = Q / m,
 *   l_p = -1/2 [m (log 2 pi + log sigma2_hat + 1) + logdet + log det G - log det X^T X]. */
kry_status kry_loglik(kry_problem* prob, const kry_matern* theta, const kry_opts* opts,
                      kry_loglik_result* out);
/* `count` parameter points on one problem, evaluated together: every
 * (theta, probe) pair is one vector of a batched product and the CG solves
 * run as one multi-RHS solve.  Same probes for every theta (common random
 * numbers).
 *
 * With opts->shift_share = 1, points with equal range, smoothness and
 * anisotropy form a group whose covariances K = Sigma_oo + eta I differ only
 * by a multiple of I.  A Krylov space does not change under such a shift, so
 * each group runs one Lanczos recurrence per probe on the nugget-free
 * Sigma_oo (in opts->precision) and every point takes the Gauss quadrature
 * of log(x + eta) on the shifted tridiagonal T + eta I; the quadratic forms
 * of the group come from one multi-shift CG recurrence on Sigma_oo in FP64
 * (vectors and products), which reaches cg_rtol for every nugget without
 * residual refinement.  Each point's result depends only on its own
 * parameters, not on which other points share the call.  Lanczos breakdown
 * is tested on Sigma_oo, so lanczos_steps_used can differ from the unshared
 * form.  Q is accumulated from the multi-shift recurrence's scalars (the
 * shifted solutions are never formed) and cg_relres is the recursive
 * residual |zeta| ||r|| / ||y||. */
kry_status kry_loglik_batch(kry_problem* prob, const kry_matern* thetas, int32_t count,
                            const kry_opts* opts, kry_loglik_result* out /* count */);
/* Independent problems (grids of any sizes, created on one context), one
 * parameter point each: thetas[i] applies to probs[i], out[i] receives its
 * result.  Problems whose embeddings are equal run together: each stage of
 * every masked product is one launch over all their vectors, the kernels
 * reading a per-vector table of masks, blocks and spectra; Krylov vectors are
 * stored with the group's largest observed count as stride (zero past each
 * problem's own count).  Each problem uses its own probes (the Philox
 * streams of kry_loglik with opts->seed), so out[i] matches kry_loglik on
 * probs[i] up to rounding.  Problems with covariates are evaluated one at a
 * time, as by kry_loglik.  Requires opts->solver = CG and shift_share = 0.
 * KRY_ENOCONV as for kry_loglik_batch. */
kry_status kry_loglik_multi(kry_problem* const* probs, const kry_matern* thetas, int32_t count,
                            const kry_opts* opts, kry_loglik_result* out);
/* Maximise l_p over (log range, log eta) -- bit 0 of free_mask frees the
 * range, bit 1 the nugget ratio -- by Nelder-Mead from `init`, with the same
 * probes at every point.  est receives the estimate with sigma2 = sigma2_hat
 * and tau2 = eta * sigma2_hat; at_est the likelihood there.  With the
 * environment variable KRY_VERBOSE set to 1 or more, every evaluation writes
 * one progress line to stderr. */
kry_status kry_fit(kry_problem* prob, const kry_matern* init, uint32_t free_mask,
                   const kry_opts* opts, double xtol, int32_t maxiter,
                   kry_matern* est, kry_loglik_result* at_est);
/* Parametric bootstrap of the estimates (the extension Sec. 3.5 mentions):
 * for b = 0..B-1 the data set y_b of the prediction-variance bootstrap
 * (kry_krige with bootstrap_B: field of Philox stream b on the smallest PSD
 * torus at theta_hat, nugget noise of stream b) plus X beta_hat (GLS at
 * theta_hat) when the problem has covariates, fitted by kry_fit from
 * theta_hat with the same free_mask, options, xtol and maxiter; est
 * receives the B estimates, sd (nullable, 2 values) the standard deviations
 * over b of log range and log eta.  The problem's data are restored
 * afterwards (also on error). */
kry_status kry_bootstrap_theta(kry_problem* prob, const kry_matern* theta_hat, uint32_t free_mask,
                               const kry_opts* opts, double xtol, int32_t maxiter, int32_t B, kry_matern* est,
                               double* sd);
/* Kriging at target cell ids (or every unobserved cell if targets == NULL):
 * mean_x = c_t^T K^{-1} y (with covariates X_t beta_hat + c_t^T K^{-1}
 * (y - X beta_hat), beta_hat as in kry_loglik, treated as known in the
 * variances, as the bootstrap of Sec. 3.5 does); with bootstrap_B == 0 the exact variances
 * var_x = sigma2 (1 - c_t^T K^{-1} c_t), var_y = var_x + tau2 (multi-RHS
 * CG); with bootstrap_B > 0 the parametric bootstrap of Sec. 3.5
 * (eq. bootstrap_uq) with B circulant-embedding fields.  var_x, var_y are
 * nullable. */
kry_status kry_krige(kry_problem* prob, const kry_matern* theta, const kry_opts* opts,
                     const int64_t* targets, int64_t ntargets, double* mean_x, double* var_x,
                     double* var_y, int32_t bootstrap_B);

/* ---- the paper's own objective (Sec. 3.1 - 3.4 and the appendix) -------------
 * pl~(theta) of eq. prof_lik: with b = y - X beta and k = opts->gk_steps
 * steps of Algorithm 1 (reorthogonalisation per opts->reorth),
 *   pl~ = -(p/2) log tau2 - psi^T psi / (2 tau2) - (n/2) log sigma2
 *         - (1/2) logdet_bccb - ||z_k||^2 / (2 sigma2),
 * psi = b - A x_k*, x_k* and z_k of eq. xhat_est, and logdet_bccb the
 * block-circulant approximation of Sec. 3.3 taken literally: the logs of the
 * eigenvalues of the (2 n1 - 1) x (2 n2 - 1) block-circulant extension of
 * Sigma at the frequencies p < n1, q < n2.  The approximate gradient of the
 * appendix (eq. approx_grad), with lambda^2 = 1/sigma2, lambda_e^2 = 1/tau2:
 *   d/d beta       = X^T psi / tau2
 *   d/d lambda^2   = n sigma2 / 2 - ||z_k||^2 / 2
 *   d/d range      = -dlogdet_bccb / 2 + (V_k z_k)^T dSigma (V_k z_k) / (2 sigma2)
 *   d/d lambda_e^2 = p tau2 / 2 - psi^T psi / 2
 * where dSigma is the range derivative of Sigma (applied by circulant
 * embedding) and dlogdet_bccb = trace(D1^{-1} D2) over the same frequencies
 * (eq. trace_approx).  The constants the paper drops (2 pi) are left out.
 * KRY_ENOTPSD when an eigenvalue of the quadrant is not positive. */
typedef struct {
    double pl;               /* pl~                                          */
    double logdet_bccb;      /* quadrant log det of Sigma                    */
    double dlogdet_bccb;     /* its range derivative                         */
    double psi2;             /* psi^T psi                                    */
    double z2;               /* ||z_k||^2                                    */
    double grad_lam2, grad_range, grad_lame2;   /* eq. approx_grad            */
    double grad_beta[KRY_MAX_COVARIATES];       /* first ncov entries         */
    int32_t ncov;            /* covariate columns                            */
    int32_t gk_steps;        /* k                                            */
} kry_plik_result;
/* pl~ and its approximate gradient at theta and beta (q values; NULL when
 * the problem has no covariates).  Requires tau2 > 0. */
kry_status kry_plik(kry_problem* prob, const kry_matern* theta, const double* beta, const kry_opts* opts,
                    kry_plik_result* out);
/* Maximise pl~ by the trust-region method of Sec. 3.4 with the rank-one
 * Hessian g g^T (the outer product of the approximate gradient g, in the
 * coordinates log sigma2, log tau2, log range, beta): each step is the
 * shortest s with g^T s = 1, cut back to the trust radius (initially
 * delta0) along g; the radius shrinks 4-fold when the gain is under a
 * quarter of the model's and doubles when it exceeds three quarters at the
 * boundary; steps with a gain are taken.  Stops when ||g|| <= gtol, the
 * radius falls below 1e-8 or after maxiter steps.  free_mask: bit 0 range,
 * bit 1 sigma2, bit 2 tau2, bit 3 beta.  beta0: q starting values (NULL:
 * the GLS estimate at init).  Outputs est, beta_est (q, nullable), the
 * result at the estimate (nullable) and the steps taken (nullable).  The
 * objective need not have an interior maximum (it grows without bound as
 * tau2 -> 0 on small grids); the fit reports where the iteration stopped. */
kry_status kry_plik_fit(kry_problem* prob, const kry_matern* init, const double* beta0, uint32_t free_mask,
                        const kry_opts* opts, double delta0, double gtol, int32_t maxiter, kry_matern* est,
                        double* beta_est, kry_plik_result* at_est, int32_t* iters);
/* Low-rank posterior variance of the latent field at every cell (eq.
 * bgamma_approx): with k = opts->gk_steps steps of Algorithm 1 on
 * b = y - X beta (beta NULL: the GLS estimate; ignored without covariates),
 * B_k^T B_k = W Theta W^T, Z = Sigma V_k W and Delta = Theta (Theta + I/sigma2)^{-1},
 *   var_x[i] = sigma2 (1 - sum_j Z_ij^2 Delta_j),  var_y = var_x + tau2,
 * which is exact once the Krylov space is complete and otherwise at least
 * the exact variance.  mean_x (nullable): x_k* + X beta at every cell.
 * Outputs n1*n2 doubles each; var_y nullable.  Requires tau2 > 0. */
kry_status kry_posterior_variance(kry_problem* prob, const kry_matern* theta, const double* beta,
                                  const kry_opts* opts, double* var_x, double* var_y, double* mean_x);
/* Eigen-decomposition of the symmetric tridiagonal matrix with diagonal d
 * (k values) and off-diagonal e (k - 1) on the host (implicit QL): theta
 * (k, ascending) and W (k x k, column-major, column j the unit eigenvector
 * of theta[j]).  The step the posterior variance uses for B_k^T B_k. */
kry_status kry_tridiag_eigen(int32_t k, const double* d, const double* e, double* theta, double* W);

/* ---- sampling (Sec. 3.5 fields; Sec. 3.6 embedding caveat) -------------- */
/* Smallest torus N1 x N2 (from the product's embedding, doubling both
 * sides) whose spectrum satisfies min >= -1e-10 max, up to 8192.
 * KRY_ENOTPSD if none. */
kry_status kry_psd_torus(kry_problem* prob, const kry_matern* theta, int32_t* N1, int32_t* N2);
/* `count` fields x = sigma * (C^{1/2} xi)[corner] on the N1 x N2 torus, xi
 * from Philox stream s = first_stream + i of domain FIELD, written as count x
 * n1*n2 doubles.  Negative eigenvalues within the tolerance are set to 0;
 * minmax (nullable) receives the spectrum's min and max. */
kry_status kry_sample(kry_problem* prob, const kry_matern* theta, int32_t N1, int32_t N2,
                      uint64_t seed, int32_t first_stream, int32_t count, double* out,
                      double* minmax);

/* ---- serving ----------------------------------------------------------------
 * A server runs likelihood and kriging requests on device-resident problems
 * with continuous batching: `slots` worker streams take requests as they
 * arrive, admitting one when a slot is free and the device memory of the
 * slots stays within hbm_budget_bytes (0 = no limit): running slots count
 * the larger of their workspace and an upper bound of their batch's
 * footprint, idle slots the workspace they keep, which is released when a
 * request needs the room; queued likelihood requests on the same problem with identical
 * options are evaluated together (up to max_batch).  A request's result is
 * the same alone and in any mix.  Problems must outlive their requests and
 * must not be modified (kry_problem_set_data) while requests on them are
 * pending; stage timing (kry_profile_begin) must be off while a server runs. */
typedef enum { KRY_REQ_LOGLIK = 0, KRY_REQ_KRIGE = 1 } kry_request_kind;
typedef struct {
    int32_t kind;            /* kry_request_kind                                   */
    kry_problem* prob;
    kry_matern theta;
    kry_opts opts;
    const int64_t* targets;  /* KRIGE: target cell ids (copied at submit)          */
    int64_t ntargets;
    int32_t variances;       /* KRIGE: 1 = also exact var_x / var_y                */
    double* mean_x;          /* KRIGE outputs, ntargets each, caller-owned and     */
    double* var_x;           /* kept alive until the request is done               */
    double* var_y;
} kry_request;
typedef struct {
    int32_t status;          /* kry_status of the request (KRY_ENOCONV: outputs   */
                             /* written, CG stopped at cg_maxit)                   */
    int32_t batch;           /* requests evaluated together with this one         */
    int32_t problems;        /* distinct problems in that batch (1: results are
                                bit-identical to the request alone; more: equal to
                                rounding, the Krylov vectors being padded)        */
    kry_loglik_result loglik;
    double t_submit, t_start, t_end;  /* seconds since the server was created  */
    uint64_t footprint_bytes;  /* admission bound of the batch's device memory  */
    uint64_t workspace_bytes;  /* device bytes the slot held after the batch    */
} kry_response;
/* slots in [1, 16]; max_queue bounds pending (not yet started) requests. */
kry_status kry_server_create(kry_ctx* ctx, int32_t slots, uint64_t hbm_budget_bytes, int32_t max_batch,
                             int32_t max_queue, kry_server** out);
/* Non-blocking: KRY_EBUSY when the queue is full, KRY_ENOMEM when the
 * request alone exceeds the budget, KRY_EINVAL for invalid requests. */
kry_status kry_server_submit(kry_server* srv, const kry_request* req, uint64_t* ticket);
/* done = 1 and *out filled once the request has finished (the ticket is then
 * released); done = 0 otherwise. */
kry_status kry_server_poll(kry_server* srv, uint64_t ticket, kry_response* out, int32_t* done);
/* Block until the request has finished. */
kry_status kry_server_wait(kry_server* srv, uint64_t ticket, kry_response* out);
/* Finishes every queued request, then stops the workers. */
void kry_server_destroy(kry_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* KRYGING_H */
