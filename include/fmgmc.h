/*
 * fmgmc.h - C ABI of the MI355X (gfx950) library for the full-multigrid
 * multilevel (quasi-)Monte Carlo method for single-phase Darcy flow with a
 * log-normal random permeability (Liu, Li, Sun, Yu, arXiv:1910.04727).
 *
 * Problem solved per sample (Section 2.1 Eq. (1); Table 1):
 *   -div(k grad p) = 0 on the unit square. Case II: p = p_west on x = 0,
 *   p = p_east on x = 1, no flow on y = 0 and y = 1; QoI = outflow through
 *   x = 1. Case I: p = p_west / p_east / p_south / p_north on x = 0 / x = 1 /
 *   y = 0 / y = 1; QoI = p(1/2, 1/2).
 *   Cell-centred finite volumes on an n x n grid with harmonic-mean face
 *   transmissibilities (Section 3.1 (1)).
 * Field (Section 3.1 (2)): k = exp(g), g a truncated Karhunen-Loeve expansion
 *   of the separable exponential covariance sigma^2 exp(-|dx|/l - |dy|/l),
 *   sampled at cell lower-left corners; xi (the KL coordinates) are inputs.
 * Hierarchy (Section 3.1 (1), Section 2.5): MLMC level l solves on the grid
 *   n_l = n0 * 2^l; the coarse-mesh QoI Q^c_l is read from the full-multigrid
 *   stage on n_l / 2 of the same pass that yields Q^f_l (Algorithm 3), with
 *   the coefficient coarsened by injection (Section 2.5, Coarsening).
 * Estimators (Section 2.1 Eqs. (2)-(5); Section 2.4): per-level means and
 *   variances of Y_l = Q^f_l - Q^c_l, MLMC sum and its variance; randomised
 *   QMC by per-shift means.
 *
 * Conventions for every call:
 *   - returns FMGMC_OK (0) on success or a negative FMGMC_E* code; the
 *     message of the last error on the calling thread is fmgmc_last_error().
 *   - array pointers may be host or device memory (detected per call); all
 *     arrays are dense, C order. No pointer is retained after a call returns.
 *   - `stream` is a hipStream_t (NULL = the null stream). Device work is
 *     enqueued on it. fmgmc_solve_level and fmgmc_estimate synchronise the
 *     stream (they read per-sample convergence counters / results back);
 *     fmgmc_synthesize_field returns without synchronising when both arrays
 *     are in device memory.
 *   - one context per host thread; a context is bound to one device.
 */
#ifndef FMGMC_H
#define FMGMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FMGMC_OK = 0,
    FMGMC_EINVAL = -1,     /* bad argument */
    FMGMC_ENOMEM = -2,     /* device or host allocation failed */
    FMGMC_EHIP = -3,       /* HIP runtime error */
    FMGMC_ENOTCONV = -4,   /* some sample did not reach rel_tol (outputs are written, flags set) */
    FMGMC_ENONFINITE = -5  /* some sample produced a non-finite residual (flags set) */
};

/* per-sample flag bits */
enum {
    FMGMC_FLAG_NOTCONV = 1,    /* a QoI stage stopped at max_cycles above rel_tol */
    FMGMC_FLAG_NONFINITE = 2,  /* non-finite residual or coefficient */
    FMGMC_FLAG_FP64 = 4,          /* FP32_IR: the sample missed rel_tol within max_cycles and was
                                     solved again by the FP64 FMG pass, whose outputs (Q, cycles,
                                     the other flag bits) replace the FP32_IR ones */
    FMGMC_FLAG_WARM_REJECTED = 8  /* the learned start was worse than the FMG start and was discarded */
};

enum { FMGMC_COV_SEPARABLE_EXP = 0 };
enum { FMGMC_SOLVER_FP64 = 0, FMGMC_SOLVER_FP32_IR = 1 };
/* KL synthesis arithmetic. FP64: the separable factorisation (two FP64 MFMA
 * contractions through the per-sample 1-D coefficient matrix) on grids n >= 64
 * with at most 64 1-D modes per axis, else the dense contraction. FP32, BF16:
 * the dense samples x modes x cells contraction with FP32 accumulation.
 * FP64_DENSE: the dense contraction in FP64. All forms compute the same sum
 * (Section 3.1 (2)) up to rounding. */
enum { FMGMC_KL_FP64 = 0, FMGMC_KL_FP32 = 1, FMGMC_KL_BF16 = 2, FMGMC_KL_FP64_DENSE = 3 };

/* Random field (Section 3.1 (2)). */
typedef struct {
    double sigma2;     /* variance of g, > 0 */
    double corr_len;   /* correlation length l of exp(-|dx|/l - |dy|/l), > 0 */
    int32_t n_modes;   /* M, number of 2-D KL modes kept (largest first), 1..4096 */
    int32_t cov_kind;  /* FMGMC_COV_SEPARABLE_EXP */
} fmgmc_field;

/* Boundary conditions and QoI (Table 1). MIXED, Case II: Dirichlet pressure on
 * the west and east sides, no flow through the south and north sides, QoI =
 * outflow through the east side. DIRICHLET, Case I: Dirichlet pressure on all
 * four sides, QoI = u(1/2, 1/2), the mean of the four centre cells (the point
 * is their shared corner). */
enum { FMGMC_BC_MIXED = 0, FMGMC_BC_DIRICHLET = 1 };

/* Level hierarchy and boundary data (Section 3.1 (1), Table 1). */
typedef struct {
    int32_t n_levels;    /* MLMC levels 0 .. n_levels-1 */
    int32_t n0;          /* fine grid of level 0 (power of two); level l uses n0 << l */
    int32_t n_coarsest;  /* multigrid coarsest grid, 4; n0 >= n_coarsest */
    int32_t boundary;    /* FMGMC_BC_MIXED (0) or FMGMC_BC_DIRICHLET */
    double p_west;       /* Dirichlet pressure at x = 0 */
    double p_east;       /* Dirichlet pressure at x = 1 */
    double p_south;      /* Dirichlet pressure at y = 0 (FMGMC_BC_DIRICHLET only) */
    double p_north;      /* Dirichlet pressure at y = 1 (FMGMC_BC_DIRICHLET only) */
} fmgmc_hier;

/* Solver options. */
typedef struct {
    int32_t solver;        /* FMGMC_SOLVER_FP64 or FMGMC_SOLVER_FP32_IR */
    int32_t kl_prec;       /* FMGMC_KL_FP64 / FP32 / BF16 (arithmetic of the KL contraction) */
    int32_t nu1, nu2;      /* pre/post red-black Gauss-Seidel sweeps per V-cycle: 1..2 (FP64),
                              1..4 (FP32_IR, whose cycles run in FP32) */
    int32_t max_cycles;    /* cap on V-cycles per QoI stage (>= 1) */
    int32_t inner_cycles;  /* FP32 V-cycles per FP64 refinement step (FP32_IR), >= 1 */
    int32_t max_batch;     /* samples resident on the device at once (0 = library default) */
    int32_t w_max_n;       /* coarse-grid corrections on grids with n <= w_max_n (other than the
                              coarsest) are two cycles in succession (W-cycle); 0 = V-cycles only */
    double rel_tol;        /* stop when ||b - A p||_2 <= rel_tol ||b||_2 at a QoI stage */
    int32_t inner_first;   /* FP32 V-cycles before the first FP64 refinement of a QoI stage
                              (FP32_IR; 0 = inner_cycles) */
    int32_t separate_coarse; /* 0: Q^c_l from the FMG pass that yields Q^f_l (FMG-MLMC,
                                Section 2.5); 1: Q^c_l from a separate FMG solve on n_l/2, as in
                                standard MLMC (the comparator of the paper's saving) */
    int32_t fuse_cycles;   /* FP32_IR: 1 = where FP32 V-cycles follow each other with no
                              refinement between them, the post-smoothing pass of one cycle and
                              the pre-smoothing pass of the next run as one pass over the stage
                              grid (the same sweeps in the same order, with x, K and b read
                              once instead of twice); needs nu1 + nu2 <= 4. With nu1 <= 2,
                              each FP64 refinement pass also does the pre-smoothing and
                              restriction of the FP32 cycle after it (its residual is that
                              cycle's right-hand side). 0 = separate passes. Converged
                              results agree to the stopping tolerance; the FP32 iterates may
                              differ in rounding. */
    int32_t warm;          /* FMGMC_WARM_NONE, or FMGMC_WARM_CNN: fmgmc_create loads the network
                              file cnn_weights into a network the context owns and warm-starts
                              every QoI stage with n >= warm_min_n from it (as
                              fmgmc_set_warm_start); needs FMGMC_SOLVER_FP32_IR and Case II */
    int32_t warm_min_n;    /* smallest QoI stage grid the network starts (0 = 256) */
    int32_t warm_max_n;    /* largest QoI stage grid the network starts (0 = no bound) */
    const char *cnn_weights; /* network file (fmgmc_cnn_save format) for FMGMC_WARM_CNN, else NULL */
    const char *tune_cache;  /* NULL, or a schedule file: fmgmc_create reads the per-level schedules
                                from it when it exists and was written for the same hierarchy and
                                solver; fmgmc_autotune rewrites it with every level's schedule */
} fmgmc_opts;

enum { FMGMC_WARM_NONE = 0, FMGMC_WARM_CNN = 1 };

typedef struct fmgmc_ctx fmgmc_ctx;

/*
 * Creates a context on HIP device `device`: builds the KL mode table
 * (Section 3.1 (2): 1-D roots, eigenvalues sigma^2 theta_a theta_b sorted
 * descending, exact ties by (a, b) ascending) and reserves device memory for
 * opts->max_batch samples of the finest level. The structs are copied.
 * Errors: EINVAL (inconsistent sizes), ENOMEM, EHIP.
 */
int fmgmc_create(fmgmc_ctx **out, const fmgmc_field *field, const fmgmc_hier *hier,
                 const fmgmc_opts *opts, int device);

/* Releases every resource of the context. NULL is accepted. */
int fmgmc_destroy(fmgmc_ctx *ctx);

/*
 * Copies the KL mode table in xi-column order: a[m], b[m] = 0-based 1-D mode
 * indices along x and y, lambda[m] = sigma^2 theta_a theta_b (host arrays of
 * at least `cap` entries). Returns the number of modes written (>= 0) or an
 * error code.
 */
int fmgmc_mode_table(const fmgmc_ctx *ctx, int32_t *a, int32_t *b, double *lambda, int32_t cap);

/*
 * Synthesises the permeability k = exp(g) on the n x n grid of MLMC level
 * `level` for n_samples samples (Section 3.1 (2), corner sampling) with the
 * context's kl_prec. xi is [n_samples][n_modes]; k_out is [n_samples][n][n]
 * (double). Errors: EINVAL, EHIP.
 */
int fmgmc_synthesize_field(fmgmc_ctx *ctx, int32_t level, int64_t n_samples, const double *xi,
                double *k_out, void *stream);

/*
 * Batched FMG-MLMC solve of one MLMC level (Algorithm 3): per sample, the
 * field from xi[s][:], its injected pyramid, one full-multigrid pass whose
 * stage on n_l/2 gives q_coarse[s] (0 on level 0) and whose stage on n_l gives
 * q_fine[s], each driven to rel_tol.
 *   xi      [n_samples][n_modes] double
 *   q_fine, q_coarse  [n_samples] double
 *   cycles  [n_samples][2] int32: V-cycles at the coarse / fine QoI stage (nullable)
 *   flags   [n_samples] uint8, FMGMC_FLAG_* bits (nullable)
 * FP32_IR: a finite sample that misses rel_tol within max_cycles is solved
 * again by the FP64 FMG pass (same field and stopping rule; an FP64 context
 * the library creates on first need, 64 samples at a time) and carries its
 * outputs, with FMGMC_FLAG_FP64 set; ENOTCONV is reported only if that pass
 * misses rel_tol too.
 * Returns OK, ENOTCONV or ENONFINITE (outputs written in all three cases),
 * or EINVAL / ENOMEM / EHIP.
 */
int fmgmc_solve_level(fmgmc_ctx *ctx, int32_t level, int64_t n_samples, const double *xi,
                      double *q_fine, double *q_coarse, int32_t *cycles, uint8_t *flags,
                      void *stream);

/*
 * All MLMC levels of one estimate at once (Algorithm 3, the loop over levels
 * with dN_l > 0): level l solves n_samples[l] samples with xi[l]
 * ([n_samples[l]][n_modes]) into q_fine[l], q_coarse[l] (and cycles[l],
 * flags[l] if those tables and entries are non-NULL), as fmgmc_solve_level
 * would. Each level has its own device workspace (allocated on first use:
 * the finest-level workspace's memory budget per level). The levels run on up
 * to four concurrent lanes (a host thread and a stream each, so that each lane
 * keeps a hardware queue of its own), assigned longest first to the least
 * loaded lane; the levels of one lane run one after another. Small grids thus
 * overlap the large ones. Results are identical to per-level
 * fmgmc_solve_level calls. `stream` is synchronised first (inputs may be
 * produced on it); the call returns when every level is done. Returns as
 * fmgmc_solve_level, over all levels.
 */
int fmgmc_solve_levels(fmgmc_ctx *ctx, int32_t n_lev, const int64_t *n_samples,
                       const double *const *xi, double *const *q_fine,
                       double *const *q_coarse, int32_t *const *cycles,
                       uint8_t *const *flags, void *stream);

/*
 * Schedule of one level: params[0] = cycles per host check of convergence
 * (G >= 1; a converged sample still stops after its own cycle because every
 * cycle is followed by the on-device check), params[1] = replay each block of
 * G cycles from a captured HIP graph (0/1; blocks on the null stream always
 * run eagerly), params[2] = samples per device chunk (0 = workspace capacity).
 * A schedule never changes results.
 *
 * fmgmc_autotune measures every schedule in {1,2,4,8} x {eager, graph} x
 * {capacity, 1/2, 1/4} on n_pilot samples of level `level` (xi host or
 * device), keeps the fastest for that level and writes it to params (nullable,
 * 3 entries). fmgmc_set_schedule sets it directly.
 */
int fmgmc_autotune(fmgmc_ctx *ctx, int32_t level, int64_t n_pilot, const double *xi,
                   int32_t *params);
int fmgmc_set_schedule(fmgmc_ctx *ctx, int32_t level, const int32_t *params);
/* The level's current schedule (3 entries, as above). */
int fmgmc_get_schedule(const fmgmc_ctx *ctx, int32_t level, int32_t *params);

/* Per-level statistics of the estimators. */
typedef struct {
    int64_t n;        /* samples */
    double mean_y;    /* mean of Y = Q^f - Q^c (the level term of Eq. (3)) */
    double var_y;     /* sample variance of Y (N - 1), or for RQMC the variance of mean_y */
    double mean_qf;
    double var_qf;
    double mean_qc;
} fmgmc_level_est;

#define FMGMC_MAX_LEVELS 16
/* MLMC / MLQMC estimate over up to FMGMC_MAX_LEVELS levels. */
typedef struct {
    int32_t n_levels;                          /* levels filled in `level` */
    fmgmc_level_est level[FMGMC_MAX_LEVELS];
    double mean;                               /* sum_l mean_y[l] (Eq. (5)'s estimator) */
    double var_of_mean;                        /* its variance (Eq. (4)-(5); Section 2.4 for RQMC) */
} fmgmc_est;

/*
 * MLMC / MLQMC estimator (Section 2.1 Eqs. (2)-(5), Section 2.4) with
 * compensated (Neumaier) sums in a fixed order, computed on the device.
 *   qf[l], qc[l]: n[l] samples of level l (host or device).
 *   n_shifts == 1: Monte Carlo; var_y is the sample variance of Y_l and
 *     var_of_mean = sum_l var_y[l] / n[l].
 *   n_shifts  > 1 (at most 4096): randomised QMC, samples grouped shift-major
 *     [shift][point] (n[l] a multiple of n_shifts); mean_y is the mean of the
 *     per-shift means and var_y is sum_r (Ybar_r - mean_y)^2 / (R (R - 1));
 *     var_of_mean = sum_l var_y[l].
 * fmgmc_estimate fills the aggregate *out (n_lev <= FMGMC_MAX_LEVELS) and runs
 * on the null stream. fmgmc_estimate_levels writes levels[l] (n_lev entries,
 * nullable), *mean and *var_of_mean (nullable) and runs on `stream`; both
 * return after the results are on the host. Errors: EINVAL (sizes, NULL
 * arrays), ENOMEM, EHIP.
 */
int fmgmc_estimate(int32_t n_lev, const int64_t *n, const double *const *qf,
                   const double *const *qc, int32_t n_shifts, fmgmc_est *out);
int fmgmc_estimate_levels(int32_t n_lev, const int64_t *n, const double *const *qf,
                          const double *const *qc, int32_t n_shifts, fmgmc_level_est *levels,
                          double *mean, double *var_of_mean, void *stream);

/*
 * For callers that cannot allocate device memory (work recorded under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * estimate of fmgmc_estimate_levels, bit for bit, with no allocation of any
 * kind. qf[l] and qc[l] must be device arrays (EINVAL for host arrays, which
 * would need a staging buffer). Its kernel works in a fixed per-device scratch
 * array of the library (8 + 4096 doubles, 32.8 KB, held by each device the
 * library runs on until the process ends), so n_shifts is limited to 4096
 * (EINVAL above). The scratch keeps the last call's contents; every value is
 * written before it is read. Calls that overlap on one device (different host
 * threads or streams) race on that array: serialise them.
 */
int fmgmc_estimate_levels_noalloc(int32_t n_lev, const int64_t *n, const double *const *qf,
                                  const double *const *qc, int32_t n_shifts,
                                  fmgmc_level_est *levels, double *mean, double *var_of_mean,
                                  void *stream);

/*
 * Host-only (no device needed): the KL mode table of fmgmc_create for the
 * given field, written to host arrays of n_modes entries (same layout as
 * fmgmc_mode_table). Errors: EINVAL.
 */
int fmgmc_kl_modes(double sigma2, double corr_len, int32_t n_modes, int32_t *a, int32_t *b,
                   double *lambda);

/*
 * Measurement hooks (not part of the method). With profiling enabled, every
 * launch of the kernel classes below on the finest grid of a solve is
 * bracketed by HIP events recorded on the launch stream, and its algorithmic
 * traffic (each operand read once, each result written once; flops for the
 * KL contraction) is accumulated from the number of samples still iterating.
 * Kinds: 0 pre-smoothing + residual + restriction pass, 1 prolongation +
 * post-smoothing pass (+ residual norm, QoI), 2 FP64 refinement pass,
 * 3 KL synthesis (flops of the path taken: 2 M n^2 per sample for the dense
 * contraction, 2 A n (A + n) for the separable one with A 1-D modes per
 * axis), 4 coarse-grid V-cycle in LDS, 5 warm-start network
 * inference (flops; all its layers, every QoI stage it runs on), 6 fused
 * prolongation + post-smoothing + pre-smoothing + residual + restriction pass
 * (fuse_cycles), 7 FP64 refinement pass that also does the next FP32 cycle's
 * pre-smoothing + residual + restriction (fuse_cycles).
 * fmgmc_profile_read synchronises, returns the summed kernel time in ms,
 * the launch count and the algorithmic bytes (flops for kind 3), and clears
 * the kind's record.
 */
enum { FMGMC_PROF_PRE = 0, FMGMC_PROF_POST = 1, FMGMC_PROF_IR = 2, FMGMC_PROF_KL = 3,
       FMGMC_PROF_SMALL = 4, FMGMC_PROF_CNN = 5, FMGMC_PROF_FUSED = 6, FMGMC_PROF_IRPRE = 7,
       FMGMC_PROF_KINDS = 8 };
int fmgmc_profile_enable(fmgmc_ctx *ctx, int32_t enable);
int fmgmc_profile_read(fmgmc_ctx *ctx, int32_t kind, double *ms, int64_t *launches, double *alg);

/*
 * ---------------------------------------------------------------------------
 * Learned warm start of the FMG pass. The paper has no network: its FMG pass
 * (Section 2.5) starts each stage from the bilinear interpolation p~ of the
 * stage below. A small residual convolutional network proposes a correction
 * of that start on a QoI stage grid; the stage then iterates to rel_tol as
 * before, so every Q still meets the same stopping rule, and the plain start
 * is kept whenever the proposal does not lower ||b - A p||_2 (flag bit
 * FMGMC_FLAG_WARM_REJECTED).
 *
 * Network (fixed shape, FMGMC_CNN_PARAMS parameters): 3x3 zero-padded
 * cross-correlations, input x = (log K, r / rms(r)) with r = b - A p~ and
 * rms(r) = ||r||_2 / n; h0 = relu(conv(x) + b0) with 32 channels; four
 * residual layers h_k = h_{k-1} + relu(conv(h_{k-1}) + b_k); output
 * y = conv(h_4) + b_5 (1 channel); the start becomes p~ + rms(r) y.
 * Parameters are FP32, flattened per layer as W[c_out][c_in][3][3] then
 * b[c_out], layers in order. Training: FP32 forward/backward and Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) on one of two losses over a batch of B
 * samples: the residual loss (1 / (B n^2)) sum (x1 - A y)^2, A the stage
 * operator built from K = exp(x0), i.e. the normalised residual of the
 * corrected start (what the stopping rule measures; the training loop uses
 * it), or the error loss (1 / (B n^2)) sum (y - t)^2 against targets t.
 * Inference in the solver: BF16 on the matrix cores with FP32 accumulation.
 * ---------------------------------------------------------------------------
 */
#define FMGMC_CNN_PARAMS 37889
enum { FMGMC_CNN_FP32 = 0, FMGMC_CNN_BF16 = 1, FMGMC_CNN_BF16_FUSED = 2 };
enum { FMGMC_CNN_LOSS_ERROR = 0, FMGMC_CNN_LOSS_RESIDUAL = 1 };
typedef struct fmgmc_cnn fmgmc_cnn;

/* New network on `device`: He-normal weights from `seed` (deterministic), zero biases. */
int fmgmc_cnn_create(fmgmc_cnn **out, uint64_t seed, int32_t device);
int fmgmc_cnn_destroy(fmgmc_cnn *cnn);
/* Parameter copy out / in (FMGMC_CNN_PARAMS floats, host or device). set resets Adam. */
int fmgmc_cnn_get_params(const fmgmc_cnn *cnn, float *theta);
int fmgmc_cnn_set_params(fmgmc_cnn *cnn, const float *theta);
/* Flat file: 8-byte tag "FMGCNN01", int32 {2, 32, 4, 0}, then the FP32 parameters. */
int fmgmc_cnn_save(const fmgmc_cnn *cnn, const char *path);
int fmgmc_cnn_load(fmgmc_cnn *cnn, const char *path);

/*
 * Forward pass on device buffers: x [batch][2][n][n] float (channel 0 = log K,
 * channel 1 = the normalised residual), y [batch][n][n] float. n a power of
 * two in [16, 1024]. prec FMGMC_CNN_FP32 (training kernels), FMGMC_CNN_BF16
 * (BF16 matrix-core inference, one launch per layer, activations through
 * device memory) or FMGMC_CNN_BF16_FUSED (the solver's inference: all layers
 * in one pass over row strips with the activations on chip; the same results
 * as FMGMC_CNN_BF16, batch at most 65535).
 */
int fmgmc_cnn_forward(fmgmc_cnn *cnn, int32_t n, int64_t batch, const float *x, float *y, int32_t prec,
                      void *stream);
/*
 * Loss (loss_kind FMGMC_CNN_LOSS_RESIDUAL, t may be NULL; or
 * FMGMC_CNN_LOSS_ERROR with targets t [batch][n][n], device) into *loss (host)
 * and, if grad is non-NULL, the gradient (FMGMC_CNN_PARAMS floats, host or
 * device). The gradient is also kept for fmgmc_cnn_adam, which applies one
 * Adam step.
 */
int fmgmc_cnn_grad(fmgmc_cnn *cnn, int32_t n, int64_t batch, const float *x, const float *t, int32_t loss_kind,
                   double *loss, float *grad, void *stream);
int fmgmc_cnn_adam(fmgmc_cnn *cnn, double lr, void *stream);

/*
 * Training pairs generated by the method itself: solves n_samples samples of
 * `level` (FP32_IR solver) and, on each QoI stage, writes the network input
 * x at the FMG start and the target t = (p - p~) / rms(r), p the converged
 * stage solution. Coarse-stage buffers ([n][2][n_l/2]^2 and [n][n_l/2]^2) are
 * written for level >= 1 only (nullable); fine-stage ones ([n][2][n_l]^2,
 * [n][n_l]^2) always. Outputs are device buffers; xi host or device.
 */
int fmgmc_cnn_make_data(fmgmc_ctx *ctx, int32_t level, int64_t n_samples, const double *xi, float *x_coarse,
                        float *t_coarse, float *x_fine, float *t_fine, void *stream);
/*
 * Trains on inputs from `level` with the residual loss: for each batch of
 * `batch` samples of xi, one Adam step on the fine-stage inputs, then
 * (level >= 1, n_l/2 >= 16) one on the coarse-stage inputs. loss_hist
 * (nullable, host) receives the losses in that order.
 */
int fmgmc_cnn_train(fmgmc_ctx *ctx, fmgmc_cnn *cnn, int32_t level, int64_t n_samples, const double *xi,
                    int32_t batch, double lr, double *loss_hist);
/*
 * Uses `cnn` (NULL: off) to warm-start every QoI stage with n >= min_n in the
 * FP32_IR solver. The context keeps the pointer; the caller keeps the
 * network alive and does not train it while the context solves.
 * The network calls (make_data, train, set_warm_start) take Case II
 * contexts only (FMGMC_EINVAL otherwise): its residual loss is that operator.
 */
int fmgmc_set_warm_start(fmgmc_ctx *ctx, const fmgmc_cnn *cnn, int32_t min_n);
/* The same for the QoI stages with min_n <= n <= max_n (max_n = 0: no bound). */
int fmgmc_set_warm_range(fmgmc_ctx *ctx, const fmgmc_cnn *cnn, int32_t min_n, int32_t max_n);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *fmgmc_last_error(void);

/* ABI version (major * 10000 + minor * 100 + patch). */
int fmgmc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FMGMC_H */
