/*
 * subsmc.h - C ABI of the MI355X Subsampling SMC hot path.
 *
 * Method: Subsampling Sequential Monte Carlo for static Bayesian models
 * (Gunawan, Dang, Quiroz, Kohn, Tran, arXiv:1805.03317). The library runs,
 * on one GPU, the stages of Algorithm 2: the adaptive tempering exponent and
 * reweighting with the annealed likelihood estimator (sections 2.2, 3.3, 3.5),
 * the mass matrix from the particle covariance (Algorithm 2 step d),
 * resampling, and the Markov move of Algorithm 1 (a block pseudo-marginal
 * refresh of the subsample indices u, then HMC on theta given u), with the
 * difference estimator of the log-likelihood, its variance estimate and the
 * second-order Taylor control variates of section 3.2.
 *
 * Conventions
 *  - All functions return an smc_status; SMC_OK is 0. On failure the context
 *    keeps a message readable with smc_last_error().
 *  - "device" pointers are HIP device allocations owned by the caller; the
 *    library never frees them and never allocates device memory: its scratch
 *    comes from the caller's workspace (size from smc_workspace_size).
 *  - "host" pointers are read (or written) before the call returns.
 *  - All device work is enqueued on the stream given to smc_init, in call
 *    order. Functions that return host values (smc_temper, smc_get_*,
 *    smc_init) synchronise that stream; the others only enqueue.
 *  - Matrices are row-major FP64. Subsample indices are 0-based int32.
 *  - A context is used by one host thread at a time.
 *  - Random numbers: Philox4x64-10 keyed by (seed, 0); every draw is a pure
 *    function of (seed, purpose, stage, move index, particle, draw number),
 *    so runs are reproducible and resumable.
 */
#ifndef SUBSMC_H
#define SUBSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SMC_OK = 0,
  SMC_ERR_INVALID_ARG = 1, /* bad size, null pointer, or unsupported combination */
  SMC_ERR_STATE = 2,       /* call out of order (e.g. smc_move before a mass matrix exists) */
  SMC_ERR_DEVICE = 3,      /* a HIP call failed; see smc_last_error */
  SMC_ERR_NOT_PD = 4,      /* covariance not positive definite even after jitter */
  SMC_ERR_NONFINITE = 5,   /* every incremental weight is non-finite */
  SMC_ERR_UNSUPPORTED = 6  /* valid request the library does not implement (e.g. d > 128) */
} smc_status;

typedef enum {
  SMC_LOGISTIC = 0, /* y in {0,1}, l = y eta - log(1 + e^eta)        (Exp. 1)        */
  SMC_POISSON = 1,  /* y in N,     l = y eta - e^eta - log y!        (Exp. 2)        */
  SMC_GAUSSIAN = 2, /* known noise variance gauss_s2; quadratic test family           */
  SMC_STUDENT_T = 3 /* y = x'theta + e, e ~ t_5 (unit scale)              (Exp. 2)        */
} smc_family;

typedef enum {
  SMC_FP64 = 0,  /* data and arithmetic in FP64                                        */
  SMC_MIXED = 1  /* data stored FP32; x'delta and the per-observation terms in FP32;  */
                 /* control variates, reductions, weights and MH ratios in FP64       */
} smc_precision;

typedef enum {
  SMC_MOVE_AUTO = 0,      /* resident when the subsample fits on chip, else streaming */
  SMC_MOVE_STREAMING = 1, /* one wavefront per particle, rows gathered from HBM every pass */
  SMC_MOVE_RESIDENT = 2,  /* one 4-wavefront workgroup per particle, rows gathered once per
                             move and kept in registers and LDS for all L + 1 passes
                             (d <= 24, logistic or Poisson, m rows must fit; else
                             SMC_ERR_UNSUPPORTED from smc_init) */
  SMC_MOVE_RESIDENT_MFMA = 3  /* the resident move with each row's x'delta formed on the matrix
                                 cores (v_mfma_f32_4x4x1f32, FP32 products and sums) beside the
                                 vector work; SMC_MIXED only */
} smc_move_path;

typedef struct smc_ctx_s* smc_ctx;

/*
 * Problem description (copied by smc_init; pointers must stay valid for the
 * context's lifetime where marked "kept").
 */
typedef struct smc_problem {
  int32_t family;      /* smc_family */
  int32_t precision;   /* smc_precision */
  int32_t cv_order;    /* 2: second-order Taylor control variate (section 3.2); 1: first order */
  int32_t d;           /* number of parameters, 1 <= d <= 128 (Gaussian family: d <= 32) */
  int64_t n;           /* number of observations, 1 <= n < 2^31 */
  int32_t ld;          /* pitch of Xy in elements, ld >= d + 1 */
  int32_t xy_fp32;     /* 1: Xy holds float, 0: double */
  const void* Xy;      /* device: n rows [x_k (d) | y_k | ...]; read by smc_init (and smc_set_cv) only */
  double gauss_s2;     /* noise variance for SMC_GAUSSIAN, else ignored */
  int32_t M;           /* particles, 1 <= M <= 8192 */
  int32_t m;           /* subsample size (with replacement), 1 <= m */
  int32_t G;           /* blocks of u for the pseudo-marginal refresh, 1 <= G <= m,
                          ceil(m/G) <= 16384 */
  int32_t move_path;   /* smc_move_path: which move kernel smc_move runs */
  uint64_t seed;       /* Philox key */
  uint32_t dataset;    /* 0..65535: the dataset field of every random-number counter, so
                          that the datasets of one batch draw independent streams under
                          one seed */
  double ess_frac;     /* target ESS = ess_frac * M, 0 < ess_frac <= 1 */
  const double* prior_mean; /* host d: Gaussian prior mean */
  const double* prior_prec; /* host d*d: Gaussian prior precision (SPD) */
  const double* theta_bar;  /* host d: control-variate centre, or NULL: the posterior
                               mode found by Newton's method on the full data */
  /* particle state, device, caller-owned, kept: */
  double* theta;       /* M*d */
  int32_t* u;          /* M*m */
  double* logw;        /* M, normalised log weights */
  double* lhat;        /* M, l_hat at the particle's (theta, u) */
  double* sig2;        /* M, sigma2_hat at the particle's (theta, u) */
  int32_t* accept;     /* M*2, last move's decisions: [u accepted, theta accepted] */
  void* workspace;     /* device, kept: smc_workspace_size bytes, 256-byte aligned */
  size_t workspace_bytes;
} smc_problem;

/* Bytes of device workspace smc_init needs for this problem (0 if invalid). */
size_t smc_workspace_size(const smc_problem* pb);

/*
 * Algorithm 2 step 1. Validates the problem, finds the control-variate centre
 * (Newton's method on the full-data log posterior unless pb->theta_bar is
 * given), builds A, B, C (section 3.2) and the packed per-observation rows in
 * the workspace, draws theta_i ~ prior and u_i ~ uniform (stage 0), sets
 * logw = -log M, and evaluates lhat, sig2 (and the cached gradients) at every
 * particle. Temperature a = 0, log Z = 0, stage 0. `stream` is a hipStream_t
 * (NULL: the default stream). Synchronises.
 */
smc_status smc_init(const smc_problem* pb, void* stream, smc_ctx* out);

/*
 * Algorithm 2 steps a-c. Increments the stage, chooses the next exponent
 * a in (a_prev, 1] with ESS(a) = ess_frac * M (section 2.2, with the target
 * of smc_problem.ess_frac): a = 1 when ESS(1) already meets it, else 60
 * halvings of [a_prev, 1], each keeping the half whose lower end has
 * ESS >= target, and a = the final lower end (the crossing this sequence of
 * halvings selects where the ESS is not monotone in a). Reweights logw with
 * the annealed estimator
 * (a - a_prev) l_hat - (a^2 - a_prev^2) sigma2_hat / 2 (normalised), and adds
 * the log evidence increment log sum_i W_i exp(...) (section 3.5).
 * Host outputs (any may be NULL). Synchronises.
 */
smc_status smc_temper(smc_ctx ctx, double* a_out, double* dlogz_out, double* ess_out);

/*
 * For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation):
 * smc_temper's exponent search, reweighting and evidence increment on
 * caller-held arrays, with no context and no workspace. Device lhat, sig2
 * (M each, read) and logw (M, normalised log weights, overwritten with the
 * reweighted ones); a_prev in [0, 1) is the previous exponent; target
 * ESS = ess_frac * M. Device out (5 doubles) receives [a, log evidence
 * increment, ESS at a, 1 if every incremental weight was non-finite (logw
 * then unchanged) else 0, ESS evaluations]. 1 <= M <= 8192, else
 * SMC_ERR_INVALID_ARG. Only enqueues on `stream` (a hipStream_t, NULL: the
 * default stream); it calls no allocation routine. Its scratch (about 4 KB: the
 * two slots of the exponent search) is a device array of the library, one
 * per GPU, shared by every call on that GPU: calls that overlap on one GPU
 * (on different streams or host threads) race and must be ordered by the
 * caller. Results equal smc_temper's on the same inputs.
 */
smc_status smc_temper_noalloc(int32_t M, const double* lhat, const double* sig2, double* logw, double a_prev,
                              double ess_frac, double* out, void* stream);

/*
 * The same step with the paper's own exponent rule (section 2.2): the ESS is
 * evaluated at the grid points a_j = a_prev + (1 - a_prev) 2^(-j/4),
 * j = 0..grid_points-1 (a_0 = 1), and a is the point above a_prev whose ESS
 * is closest to ess_frac * M (the paper uses ess_frac = 0.8; the first point
 * on ties). grid_points in [1, 256]; ess_frac in (0, 1]. Reweighting and the
 * evidence increment as in smc_temper. ess_grid_out (host, grid_points
 * values, may be NULL) receives the ESS at every grid point. Synchronises.
 */
smc_status smc_temper_grid(smc_ctx ctx, int32_t grid_points, double ess_frac, double* a_out,
                           double* dlogz_out, double* ess_out, double* ess_grid_out);

/* Algorithm 2 step d: weighted particle covariance Sigma (inverse mass matrix),
 * its Cholesky factor and inverse factor (a jitter ladder 1e-10..1e-1 times
 * the mean variance is tried before giving up). Does not wait for the device:
 * a covariance that is not positive definite is reported as SMC_ERR_NOT_PD by
 * the next call that uses the mass matrix (smc_move, smc_recentre without a
 * centre, smc_batch_move), and smc_get_info then shows have_mass = 0. */
smc_status smc_mass(smc_ctx ctx);

/*
 * Algorithm 2 step d as the paper writes it (section 3.2): moves the
 * control-variate centre theta_bar to theta_bar_host (host, d doubles) or,
 * when it is NULL, to the weighted particle mean computed by the last
 * smc_mass of this stage; rebuilds A, B, C and the per-row constants of the
 * packed data at the new centre (a full pass over the n rows) and
 * re-evaluates the cached estimator and gradients of every particle, so the
 * next reweighting and move use the new control variates. SMC_ERR_STATE if
 * theta_bar_host is NULL and there is no mass matrix for this stage.
 * Synchronises.
 */
smc_status smc_recentre(smc_ctx ctx, const double* theta_bar_host);

/* Algorithm 2 step e: systematic resampling with exact integer arithmetic
 * (one Philox offset per stage); copies theta, u and the caches from the
 * ancestors and sets logw = -log M. */
smc_status smc_resample(smc_ctx ctx);

/* Algorithm 2 step e with the paper's multinomial resampling (section 2.1):
 * slot k takes the ancestor of its own uniform (Philox purpose 2, particle k,
 * draw 1) under the integer weights floor(2^48 W_i / max W), i.e. the
 * smallest i whose inclusive prefix sum exceeds floor(r_k S / 2^64). Copies
 * as smc_resample. */
smc_status smc_resample_multinomial(smc_ctx ctx);

/* Algorithm 2 step f: R Markov moves (Algorithm 1) of every particle at the
 * current exponent: block refresh of u (one of G blocks, uniform), then HMC
 * with step eps, L leapfrog steps, momentum ~ N(0, Sigma^{-1}). Requires a
 * mass matrix (smc_mass or smc_set_mass). */
smc_status smc_move(smc_ctx ctx, double eps, int32_t L, int32_t R);

/*
 * Outcome of the last Markov move (Algorithm 1) of smc_move, smc_stage or
 * smc_batch_move on this context: the fraction of particles whose u block
 * refresh was accepted (eq. acc_prop_u) and whose HMC proposal was accepted,
 * and how many of those decisions were near ties, i.e. had
 * |log U - log r| <= tau (1 + |log r|) with tau = 1e-9 (FP64) or 1e-5
 * (mixed): the decisions whose outcome rounding could change. Host outputs,
 * any may be NULL. SMC_ERR_STATE before the first move. Synchronises.
 */
smc_status smc_move_stats(smc_ctx ctx, double* accept_u, double* accept_theta, int64_t* near_ties_u,
                          int64_t* near_ties_theta);

/*
 * The Metropolis-Hastings quantities of every particle's decisions in the last
 * move (eq. acc_prop_u for the u refresh; the HMC energy difference
 * H(theta, p) - H(theta*, p*) for theta): host diag (M*4 doubles) receives,
 * per particle, [log r, log U] of the u refresh, then [log r, log U] of the
 * HMC step; a proposal is accepted iff log U < log r (and log r is finite).
 * SMC_ERR_STATE before the first move. Synchronises.
 */
smc_status smc_move_diag(smc_ctx ctx, double* diag);

/*
 * One whole stage of Algorithm 2 (steps a-f with the default schemes):
 * smc_temper (skipped once a = 1), smc_mass, smc_resample and smc_move(eps,
 * L, R), with the results of those calls (a_out, dlogz_out, ess_out as in
 * smc_temper; a = 1, 0, 0 when no tempering took place). The mass matrix and
 * the resampling are queued before the exponent reaches the host, so the
 * device does not wait for the host between the steps. A tempering failure
 * (SMC_ERR_NONFINITE) leaves the stage counter advanced and the particles
 * resampled.
 */
smc_status smc_stage(smc_ctx ctx, double eps, int32_t L, int32_t R, double* a_out, double* dlogz_out,
                     double* ess_out);

/*
 * Difference estimator (eq. difference_estimator_logl) and its variance
 * estimate (section 3.2) for `count` particles at exponent-free level:
 * device theta (count*d), u (count*m) -> device lhat, sig2, dhat (count each;
 * dhat = (n/m) sum_j d_{u_j}); any output may be NULL.
 */
smc_status loglik_est(smc_ctx ctx, int32_t count, const double* theta, const int32_t* u,
                      double* lhat, double* sig2, double* dhat);

/*
 * Gradients of the same quantities: device grad (count*d) receives
 * g_lhat[i] * grad l_hat + g_sig2[i] * grad sigma2_hat (g_* device, count,
 * NULL meaning 0). grad_l / grad_s (count*d, nullable) receive the two
 * gradients separately.
 */
smc_status loglik_grad(smc_ctx ctx, int32_t count, const double* theta, const int32_t* u,
                       const double* g_lhat, const double* g_sig2, double* grad,
                       double* grad_l, double* grad_s);

/*
 * The annealed log-likelihood estimator of the extended target (section 3.1,
 * eq. tempered_likelihood_estimator): lambda_a = a l_hat - a^2 sigma2_hat / 2
 * at exponent a in [0, 1] for `count` particles: device theta (count*d) and
 * u (count*m) -> device lam (count), and optionally lhat and sig2 (nullable).
 */
smc_status loglik_lambda(smc_ctx ctx, int32_t count, const double* theta, const int32_t* u, double a,
                         double* lam, double* lhat, double* sig2);

/*
 * Picks the move kernel by measurement: times one move (after an untimed
 * one) of every option the problem's move_path allows — the streaming kernel
 * (for FP32 logistic rows with d > 32 in each tile form of its row loop,
 * smc_info.stream_tile) and each resident layout that fits (register rows per
 * lane; for FP32 rows each with x'delta on the vector ALU and on the matrix
 * cores) — from the
 * current state with step eps and L leapfrog steps, restores the particle
 * state, the accept flags and the move counter exactly, and keeps the fastest
 * for later moves (single and batched). *rpl_out (nullable) receives the
 * choice: -1 streaming, else the register rows per lane of the resident
 * kernel (smc_info.res_mfma tells the form of the product); ms_out (nullable,
 * up to 8 entries) the timed durations in the order streaming (when allowed,
 * tile forms 0, 1, 2), then the resident layouts by register rows, the
 * vector form before the matrix-core form. Needs a mass matrix.
 * Uses the resampling buffers of the workspace. Synchronises.
 */
smc_status smc_autotune_move(smc_ctx ctx, double eps, int32_t L, int32_t* rpl_out, float* ms_out);

/*
 * Sets the move kernel directly (a choice smc_autotune_move made on an
 * earlier run, or a test): res_rows = -1 selects the streaming move with tile
 * form stream_tile (0, 1 or 2, where smc_info documents them), else the resident
 * move with res_rows register rows per lane and x'delta on the matrix cores
 * when res_mfma = 1. SMC_ERR_UNSUPPORTED when the option does not exist or
 * does not fit this problem and device, or the problem's move_path excludes it.
 */
smc_status smc_set_move_option(smc_ctx ctx, int32_t res_rows, int32_t res_mfma, int32_t stream_tile);

/* Timing of move launches: with n > 0 (at most 4096) every move launch of
 * smc_move (and smc_stage) is bracketed by a HIP event pair on the context's
 * stream, kept in a ring of the last n; n = 0 stops it. */
smc_status smc_set_move_timing(smc_ctx ctx, int32_t n);

/* Device time in ms of the last moves timed (up to cap, oldest first) into
 * ms; *count receives how many. Waits for their events. */
smc_status smc_move_times(smc_ctx ctx, int32_t cap, float* ms, int32_t* count);

/* Recompute lhat, sig2 and the cached gradients at the current (theta, u),
 * after the caller has written the particle buffers directly. */
smc_status smc_refresh(smc_ctx ctx);

/* Host scalars of the run. */
typedef struct smc_info {
  double a;        /* current tempering exponent */
  double logz;     /* accumulated log evidence estimate */
  int32_t stage;   /* current stage p */
  int32_t move;    /* moves done in this stage */
  int32_t have_mass;
  int32_t newton_iters;
  int32_t move_path;  /* the move kernel in use: SMC_MOVE_STREAMING or SMC_MOVE_RESIDENT */
  int32_t res_rows;   /* resident move: subsample rows each lane keeps in registers (the rest
                         sit in LDS); -1 with the streaming move */
  int32_t res_mfma;   /* resident move: 1 when x'delta is formed on the matrix cores
                         (v_mfma_f32_4x4x1f32), 0 on the vector ALU */
  int32_t stream_tile; /* lane-group streaming move (d > 32): the tile form of its row loop,
                          0 (FP32 logistic rows evaluate each row's remainder once, in one
                          lane of the row's group), 1 (in every lane of the group) or 2
                          (form 0 with 4 consecutive particles per workgroup whose row loops
                          meet at a barrier every 32 iterations, so that resampled copies,
                          which share their subsample, read each row at nearly the same
                          time; offered for every
                          lane-group shape when 4 divides M). Form 1 exists for FP32 logistic
                          rows only. Default: 2 for FP32 logistic rows with d > 60, else 0 */
} smc_info;
smc_status smc_get_info(smc_ctx ctx, smc_info* out);

/* Overwrite the stage counters (checkpoint resume, tests). */
smc_status smc_set_stage(smc_ctx ctx, int32_t stage, int32_t move, double a, double logz);

/*
 * Checkpoint of a run between calls (the state Algorithm 2 carries from one
 * stage to the next): a host blob holding the problem's identity (family,
 * precision, control-variate order, n, d, M, m, G, seed, dataset), the
 * stage counters (stage, move, a, log Z), the control-variate centre, the
 * move kernel in use, the mass matrix of the stage if there is one, and the
 * particle state (theta, u, log W, the cached l_hat, sigma2_hat and both
 * gradients, the last accept flags). With blob = NULL, *bytes receives the
 * size; otherwise *bytes must be at least that size and receives it.
 * Synchronises.
 */
smc_status smc_get_state(smc_ctx ctx, void* blob, size_t* bytes);

/*
 * Restores a blob written by smc_get_state into a context made by smc_init
 * for the same problem (SMC_ERR_INVALID_ARG if the identity or the size
 * differs). A different control-variate centre is rebuilt from the blob's
 * (the same kernels on the same rows, so A, B, C and the packed row
 * constants come back bit for bit). The run then continues exactly as the
 * one that wrote the blob. Synchronises.
 */
smc_status smc_set_state(smc_ctx ctx, const void* blob, size_t bytes);

/* Host d*d covariance -> device Sigma, factor and inverse factor. */
smc_status smc_set_mass(smc_ctx ctx, const double* sigma_host);

/* Host copies of Sigma, its lower Cholesky factor and its inverse (nullable). */
smc_status smc_get_mass(smc_ctx ctx, double* sigma, double* chol, double* chol_inv);

/* Host copies of theta_bar (d), A (1), B (d), C (d*d) (nullable). */
smc_status smc_get_cv(smc_ctx ctx, double* theta_bar, double* A, double* B, double* C);

/* Full-data log-likelihood, gradient and Hessian at a host theta (FP64,
 * host outputs, nullable). Synchronises. */
smc_status smc_full_loglik(smc_ctx ctx, const double* theta, double* A, double* B, double* C);

/* Release the context (device buffers stay with the caller). */
void smc_destroy(smc_ctx ctx);

/*
 * Batches: many independent datasets (each its own context, with its own n, d,
 * family, precision, M, m and G) advanced together, every per-stage step of
 * Algorithm 2 issued once for all of them: one launch per kernel, and for the
 * move one launch per kernel shape present among the members (the shape is
 * fixed by precision, family, padded d and the move path). A member's result
 * is the one its own context gives with the single-context calls; members
 * should differ in seed or in smc_problem.dataset to draw independent streams.
 *
 * All members must share the stream given to smc_init. The batch keeps
 * pointers to the contexts; destroy the batch before them.
 */
typedef struct smc_batch_s* smc_batch;

/* Device workspace bytes for a batch of `count` members (0 if count is not
 * in [1, 65536]). */
size_t smc_batch_workspace_size(int32_t count);

/* ctxs: host array of `count` distinct contexts; workspace: device, 256-byte
 * aligned, at least smc_batch_workspace_size(count) bytes, kept. Also takes a
 * pinned host mirror of the workspace. */
smc_status smc_batch_create(const smc_ctx* ctxs, int32_t count, void* workspace, size_t workspace_bytes,
                            smc_batch* out);

/* smc_temper for every member whose exponent is still below 1 (the members
 * active in this stage); the others are left as they are. Host outputs of
 * `count` entries each (nullable): the member's exponent after the call, its
 * log evidence increment and ESS (0 for inactive members) and 1 for an
 * active member. SMC_ERR_STATE when every member has reached a = 1.
 * Synchronises. */
smc_status smc_batch_temper(smc_batch b, double* a_out, double* dlogz_out, double* ess_out, int32_t* active_out);

/* smc_mass for the active members. Synchronises. */
smc_status smc_batch_mass(smc_batch b);

/* smc_resample (multinomial = 0) or smc_resample_multinomial (1) for the
 * active members. */
smc_status smc_batch_resample(smc_batch b, int32_t multinomial);

/* smc_move for the active members: eps is a host array of `count` step sizes
 * (entries of inactive members are ignored); L and R as in smc_move. */
smc_status smc_batch_move(smc_batch b, const double* eps, int32_t L, int32_t R);

/* Number of move launches per move of the current stage (distinct kernel
 * shapes among the active members). */
int32_t smc_batch_launches(smc_batch b);

/* Concurrency of the move's launches: smc_batch_move spreads its launches
 * (one per kernel shape) over n streams (1 <= n <= 8, default 8): the
 * batch's stream and n - 1 private streams that fork from it before the
 * launches and join it after them, so that launches too small to fill the
 * GPU run side by side; the costliest launches are placed first, each on the
 * least loaded stream. Results do not depend on n (every member is moved by
 * exactly one launch). n = 1 issues everything on the batch's stream. With
 * timing on, the launches run one after another on the batch's stream. */
smc_status smc_batch_set_streams(smc_batch b, int32_t n);

/* Graph replay of the move: with on = 1, smc_batch_move captures its
 * launches into a HIP graph (they take their arguments from tables uploaded
 * before each move) and replays it for every move with the same launch
 * structure, capturing again when the structure changes (a member reaching
 * a = 1). Results are those of the direct launches. Ignored while timing is
 * on. */
smc_status smc_batch_set_graph(smc_batch b, int32_t on);

/* Persistent move (section 2.1: the particles of every dataset move
 * independently under Algorithm 1): with on = 1, smc_batch_move moves all
 * members whose rows share a row type and family in ONE launch. Its grid is
 * what the GPU holds at once; each workgroup takes work items from a device
 * queue (in the caller's workspace) until it is empty: one particle of a
 * member that uses the resident kernel, or four consecutive particles of a
 * member that uses a streaming kernel, costliest member first. A member whose
 * resident layout needs more registers or LDS than the launch allows (14
 * register rows per lane, the matrix-core form, or more LDS than two
 * workgroups per CU leave with float rows) moves with its streaming kernel;
 * smc_batch_member_kernels reports which. Each particle's result is bit for
 * bit that of the member's own context moved with the same kernel. The
 * launches honour graph replay and timing; the stream setting is unused
 * (one launch per row type and family, on the batch's stream). on = 0 (the
 * default): one launch per kernel shape. */
smc_status smc_batch_set_persistent(smc_batch b, int32_t on);

/* The kernel each member's last move ran: kind[k] = 0 narrow streaming,
 * 1 lane-group streaming, 2 resident, -1 not moved (inactive member or no
 * move yet). kind holds one entry per member (host). */
smc_status smc_batch_member_kernels(smc_batch b, int32_t* kind);

/* Number of graph captures smc_batch_move has made. */
int32_t smc_batch_graph_captures(smc_batch b);

/* Timing of the move launches: with on = 1, smc_batch_move records a HIP
 * event pair on the batch's stream around each of its launches. */
smc_status smc_batch_set_timing(smc_batch b, int32_t on);

/* The launches of the last smc_batch_move: their number (*launches), and for
 * each (up to cap) its kernel (0 narrow streaming, 1 lane-group streaming,
 * 2 resident) and its device time in ms summed over the R moves (0 unless
 * timing was on), and per member (count entries) the launch that moved it
 * (-1: inactive). Waits for the recorded events. */
smc_status smc_batch_move_timing(smc_batch b, int32_t cap, int32_t* launches, int32_t* kind, double* ms,
                                 int32_t* member_launch);

void smc_batch_destroy(smc_batch b);
const char* smc_batch_last_error(smc_batch b);

const char* smc_status_string(smc_status s);
const char* smc_last_error(smc_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* SUBSMC_H */
