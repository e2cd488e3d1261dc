/*
 * pdnqp.h -- C ABI of the MI355X (gfx950) PDNQP hot path.
 *
 * PDNQP finds stationary (KKT) points of sparse, possibly nonconvex QPs
 *
 *     min 1/2 x'Qx + c'x   s.t.  rl <= A x <= ru,   xl <= x <= xu
 *
 * (paper: Section 2, problem (qp) and stationarity (kkt-stationarity)) by a
 * proximal augmented-Lagrangian outer loop (Algorithm "practical outer
 * iteration", Section 3.2) whose strongly convex residual-form subproblems
 * (eq. (inner-qp)) are solved by a diagonal, adaptive, restarted accelerated
 * PDHG (Algorithm "practical diagonal PDHG", Section 3.3).  Every iteration
 * of both loops runs as HIP kernels on one GPU; the host only issues
 * launches and reads back a few scalars per check.
 *
 * Conventions for every function below:
 *  - Functions returning int return PDNQP_OK (0) on success and a negative
 *    PDNQP_E_* code on error; they never throw and never abort.  After an
 *    error, pdnqp_last_error() describes it.
 *  - All array arguments are HOST pointers, read (or written) only during
 *    the call; the library copies what it keeps.  Sizes are element counts.
 *  - Sparse matrices are CSR with int32 row pointers (length rows+1,
 *    starting at 0, nondecreasing) and int32 column indices (sorted
 *    strictly increasing within each row, in range), FP64 values.
 *  - A solver handle is not thread-safe; distinct handles may be used from
 *    distinct threads concurrently (each owns its HIP stream).
 */
#ifndef PDNQP_H
#define PDNQP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes (return values). */
enum {
  PDNQP_OK = 0,
  PDNQP_E_INVALID = -1, /* bad argument: shape, index, ordering, symmetry, non-finite data, bounds */
  PDNQP_E_NOMEM = -2,   /* device or host allocation failed */
  PDNQP_E_DEVICE = -3,  /* a HIP runtime call failed */
  PDNQP_E_STATE = -4    /* operation not valid for this handle (e.g. no trace recorded) */
};

/* Solver outcomes (pdnqp_info.status).  Algorithm "practical outer
 * iteration": termination (outer-termination), iteration limit, and the
 * inner solver's numerical-error exit (rejection limit). */
enum {
  PDNQP_SOLVED = 1,
  PDNQP_MAX_ITER = 2,
  PDNQP_TIME_LIMIT = 3,
  PDNQP_NUMERICAL_ERROR = 4,
  /* 5 and 6 are kept for primal and dual infeasibility, which the paper
   * mentions without formulas or thresholds; no solve returns them. */
  /* The scaled test passed at the smallest internal tolerances of the
   * calibration (settings.external_halvings) but the KKT test on the
   * caller's unscaled problem did not (Section 4, termination and tolerance
   * calibration: such a point counts as a failure). */
  PDNQP_INACCURATE = 7
};

/* Outer scaling modes (Section 3.1, eq. (scaled-problem)). */
enum {
  PDNQP_SCALE_RUIZ_A = 0,  /* Ruiz sweeps on the combined constraint matrix [A_E; A_I] (the paper's) */
  PDNQP_SCALE_NONE = 1,    /* no outer scaling (D_c = D_x = 1; the objective scalar still applies) */
  PDNQP_SCALE_RUIZ_QA = 2  /* Ruiz sweeps where a column's norm also counts the symmetric Q */
};

/* Arithmetic of the inner iteration (settings.precision). */
enum {
  PDNQP_FP64 = 0,
  PDNQP_FP32 = 1
};

/* Largest Anderson memory (settings.anderson_mem). */
enum { PDNQP_ANDERSON_MAX = 8 };

/* Solver parameters.  Obtain defaults with pdnqp_default_settings() and
 * override fields.  Fields marked [paper] take the defaults of the paper's
 * parameter table; fields marked [reading] fix points the paper leaves
 * open (each documented where it is used). */
typedef struct pdnqp_settings {
  int64_t max_outer;       /* [paper] outer iteration limit K_out, 2^31-1 */
  int32_t max_inner;       /* [paper] accepted inner iterations per outer call K_in, 40000 */
  int32_t ruiz_sweeps;     /* [paper] outer and inner Ruiz sweeps, 8 */
  double time_limit_s;     /* [paper] wall-clock limit, +inf */
  double sigma_init;       /* [paper] initial row-penalty scale, 20 */
  double theta_sigma;      /* [paper] residual-reduction threshold of the penalty update, 0.25 */
  double delta_gamma;      /* [paper] margin of the proximal step (R-choice), 1e-2 */
  double rho_in_min;       /* [paper] fast inner-tolerance factor, 0.3 */
  double rho_in_max;       /* [paper] slow inner-tolerance factor, 0.95 */
  double rho_z;            /* [paper] centre-tolerance factor, 0.95 */
  int32_t check_every;     /* [reading] accepted trials between inner stopping/restart checks, 64 */
  int32_t max_rejects;     /* [reading] consecutive rejected trials => numerical error, 50 */
  double restart_suff;     /* [reading] sufficient KKT decay for a restart, 0.2 */
  double restart_nec;      /* [reading] necessary KKT decay (with no progress), 0.8 */
  double restart_art;      /* [reading] artificial restart: epoch >= this * inner count, 0.36 */
  double shrink_safety;    /* [reading] rejected-trial step factor clamp(safety*L/R, min, max): 0.95 */
  double shrink_min;       /*   0.1 */
  double shrink_max;       /*   0.9 */
  double omega0;           /* [reading] initial primal weight, 1 */
  double sigma_growth;     /* [reading] penalty growth multiplier, 10 */
  double sigma_max;        /* [reading] penalty cap, 1e4 (the upper clamp of the initial penalty) */
  double sigma0_min;       /* [reading] clamp of the initial penalty, 1e-4 */
  double sigma0_max;       /*   1e4 */
  int32_t penalty_gate;    /* [reading] rows already within the outer tolerance are not penalised further, 1 */
  int32_t lanczos_iters;   /* [reading] Lanczos steps for the smallest eigenvalue of Q, 100 */
  double gamma_override;   /* > 0: use this proximal step instead of the Lanczos rule; 0 (default) */
  double step_boost;       /* multiplies the diagonal steps at every rebuild; 1 (testing knob) */
  int32_t outer_scaling;   /* PDNQP_SCALE_*, default PDNQP_SCALE_RUIZ_A */
  int32_t profile;         /* P > 0: time the per-trial kernels of one trial slot in every P
                              (pdnqp_kernel_stats); 0: off */
  int32_t trace_iters;     /* record unscaled inner (w, y) after each of the first N accepted trials */
  int32_t trace_trials;    /* record (L, R, accepted) of the first N trials and the first N checks */
  int32_t verbose;         /* 1: one line per outer iteration on stderr; 2: also one line per
                              inner call that ends at the max_inner limit */
  int32_t center_floor;    /* [reading] centre-update tolerances never fall below eps_abs, eps_rel; 1 */
  int32_t precision;       /* PDNQP_FP64 (default) or PDNQP_FP32: FP32 matrix values and inner
                              vectors, FP64 reductions, FP64 outer update and final check */
  int32_t graph;           /* 1: each outer step captures its chunk of trial slots and the check
                              in a hipGraph and replays it (same kernels, same results); 0 (default):
                              plain stream launches */
  int32_t anderson_mem;    /* memory m_A of the Anderson acceleration of (lambda_E, lambda_I, z)
                              (Section 3.2, "Anderson acceleration"; the paper's table: 5);
                              0 (default): off; at most PDNQP_ANDERSON_MAX */
  double anderson_reg;     /* [reading] Tikhonov weight of the Anderson least-squares problem,
                              relative to the mean diagonal of its Gram matrix; 1e-10 */
  int32_t controller;      /* 0 (default): the adaptive inner-tolerance rule (inner-tolerance-factor);
                              1: the learned controller loaded by pdnqp_set_controller sets the
                              next inner tolerance, inner iteration budget and primal weight,
                              falling back to the adaptive rule after 3 outer steps without
                              progress of the outer KKT measure */
  int32_t outer_log;       /* record the controller features of the first N outer steps
                              (pdnqp_get_outer_log); 0 (default): none */
  double fp32_promote;     /* with PDNQP_FP32: once the inner tolerances (max of the absolute
                              and relative one) fall to this value or below, the rest of the solve
                              runs the FP64 inner iteration (FP32 storage bounds the inner
                              residual it can reach); 1e-5 (default); 0: never */
  double delta_floor;      /* [reading] the inner tolerances never fall below delta_floor times
                              eps_abs, eps_rel (inner-tolerance-factor states no floor); 1;
                              0: no floor (the paper's rule as stated) */
  int32_t fp32_stall;      /* with PDNQP_FP32: after this many outer steps without a 10% gain of
                              the outer KKT measure max(r_p/(eps_abs+eps_rel s_p),
                              r_d/(eps_abs+eps_rel s_d)), the rest of the solve runs the FP64 inner
                              iteration (FP32 rounding of the iterate can stall the outer
                              iteration above the tolerance); 50 (default); 0: never */
  int32_t external_halvings; /* [reading] the experimental protocol's tolerance calibration,
                              run as a continuation (Section 4, termination and tolerance
                              calibration): when the scaled test (outer-termination) passes
                              but the same test on the caller's unscaled problem (primal
                              residual with bound violation, projected stationarity) does
                              not, every internal use of eps_abs, eps_rel (scaled test,
                              penalty gate, inner-tolerance and centre floors, Anderson) is
                              halved and the outer iteration continues; after this many
                              halvings such a point ends the solve with PDNQP_INACCURATE.
                              7 (default: 1/128, the protocol's limit); 0: stop on the
                              scaled test alone */
  void *hip_stream;        /* hipStream_t to run on; NULL: the library creates its own */
  /* Device memory provider.  NULL: hipMalloc/hipFree.  Called only from
   * pdnqp_create / pdnqp_destroy (and pdnqp_solve when tracing). */
  void *(*dev_alloc)(size_t bytes, void *user);
  void (*dev_free)(void *ptr, void *user);
  void *alloc_user;
  double delta0;           /* [paper] initial inner tolerances delta_{a,0} = delta_{r,0}, 1
                              (Section 3.1, outer-loop initialization) */
  int32_t col_panels;      /* the first sparse product of a trial (Q and A times the trial x)
                              split into two column panels, each gathered by the workgroups of
                              half of the XCDs, with a second launch adding the two partial
                              row sums (same arithmetic up to the order of the two halves'
                              sums): 0 (default) when the gathered vector exceeds one XCD's L2
                              (4 MiB), 1 never, 2 always */
  int32_t stream_grid;     /* workgroups of the pipelined CSR-stream product launches of a
                              trial (the first product, in its one-launch or column-panel
                              form, and the A' product; a launch tuning knob: it changes only
                              the order in which per-workgroup acceptance sums are added):
                              0 (default) 1024, else 2..4096 */
  double kkt_pass_limit;   /* [paper] KKT pass limit: cumulative inner matrix passes, +inf
                              (parameter table).  One pass = one inner trial (one product
                              each with H_k, B and B'), counted over the whole solve and
                              tested at the periodic checks of the inner iteration; reaching it
                              ends the solve with PDNQP_MAX_ITER.  Must be >= 1 */
} pdnqp_settings;

/* Per-solve report. */
typedef struct pdnqp_info {
  int32_t status;          /* PDNQP_SOLVED ... */
  int32_t anderson_steps;  /* outer steps that took an Anderson extrapolation */
  int64_t outer_iters;     /* outer iterations performed */
  int64_t inner_trials;    /* trial steps (accepted + rejected) */
  int64_t inner_accepted;  /* accepted inner iterations */
  int64_t inner_rejected;
  int64_t restarts;
  int64_t checks;
  /* Final KKT test on the ORIGINAL (unscaled) problem: primal residual
   * including bound violation, projected stationarity, and their scales
   * (outer-residuals)/(outer-scales) evaluated on the caller's data. */
  double r_p, r_d, s_p, s_d;
  /* The same four quantities on the scaled problem at the last outer step
   * (what the termination test used). */
  double r_p_scaled, r_d_scaled, s_p_scaled, s_d_scaled;
  double objective;        /* 1/2 x'Qx + c'x at the returned x */
  double gamma;            /* proximal step used (scaled problem) */
  double lambda_hat;       /* Lanczos estimate of the smallest eigenvalue of the scaled Q */
  double omega;            /* final primal weight */
  double setup_s;          /* seconds in scaling/Lanczos/penalty set-up inside pdnqp_solve */
  double solve_s;          /* seconds of the whole pdnqp_solve call */
  int32_t controller_fallback;  /* 1 if the learned controller handed over to the adaptive rule */
  int32_t outer_logged;    /* outer steps recorded for pdnqp_get_outer_log */
  int32_t promoted_outer;  /* with PDNQP_FP32: the outer step from which the inner iteration ran
                              in FP64 (settings.fp32_promote); 0: none */
  int32_t halvings;        /* internal tolerance halvings taken by the calibration
                              (settings.external_halvings) */
} pdnqp_info;

/* Writes the defaults into *s.  Never fails. */
void pdnqp_default_settings(pdnqp_settings *s);

/* Size in bytes of pdnqp_settings / pdnqp_info as compiled into the library
 * (lets bindings check their struct layout). */
size_t pdnqp_settings_size(void);
size_t pdnqp_info_size(void);

typedef struct pdnqp_solver pdnqp_solver;

/* Creates a solver for one QP and uploads it to the current HIP device.
 *  n >= 1 variables, m >= 0 rows.
 *  Q:   n x n CSR (Qp, Qi, Qx), symmetric with both triangles stored.
 *  A:   m x n CSR (Ap, Ai, Ax).
 *  c, xl, xu: length n; xl <= xu, xl may be -INFINITY, xu +INFINITY.
 *  rl, ru:    length m; rl <= ru.  rl == ru is an equality row; a row with
 *             only rl finite is A_I x >= rl; only ru finite is negated into
 *             that form; both finite is split into two such rows; both
 *             infinite is ignored.
 *  settings:  NULL for defaults.  Copied.
 * On success *out owns all device memory it allocated (released by
 * pdnqp_destroy).  On error *out is NULL.  Errors: PDNQP_E_INVALID for any
 * malformed input (checked before any device call), PDNQP_E_NOMEM,
 * PDNQP_E_DEVICE. */
int pdnqp_create(pdnqp_solver **out, int32_t n, int32_t m,
                 const int32_t *Qp, const int32_t *Qi, const double *Qx,
                 const int32_t *Ap, const int32_t *Ai, const double *Ax,
                 const double *c, const double *xl, const double *xu,
                 const double *rl, const double *ru,
                 const pdnqp_settings *settings);

/* Solves to  r_p <= eps_abs + eps_rel*s_p  and  r_d <= eps_abs + eps_rel*s_d
 * (outer-termination) on the scaled problem.
 *  x0 (length n) and lambda0 (length m, caller's rows) are optional warm
 *  starts (NULL: zero); x0 is clipped into [xl, xu].
 *  x_out (length n), lambda_out (length m): caller-owned host buffers,
 *  written on PDNQP_OK whatever the solver outcome; lambda follows the
 *  sign convention  Qx + c + A'lambda + N_[xl,xu](x) contains 0, i.e.
 *  lambda <= 0 on a row at its lower bound and >= 0 at its upper bound.
 *  info: optional (NULL allowed).
 * The call blocks until the solve ends (it synchronises its stream). */
int pdnqp_solve(pdnqp_solver *s, double eps_abs, double eps_rel,
                const double *x0, const double *lambda0,
                double *x_out, double *lambda_out, pdnqp_info *info);

/* Solves `count` independent QPs (each with its own handle) from zero
 * starts in one persistent kernel launch.  Each workgroup runs the whole
 * method for one instance at a time -- outer scaling, Lanczos proximal
 * step, initial penalties, then the outer iterations of Algorithm
 * "practical outer iteration" with their inner rAPDHG solves, and the
 * unscaling -- and then takes the next instance (largest first) from a
 * device queue.  The steps, readings and stopping rules are those of
 * pdnqp_solve; each handle keeps its own settings, except that
 * time_limit_s counts from the moment a workgroup starts the instance and
 * an infinite limit is replaced by 3600 s.
 *  All handles must be on the same device and share one precision
 *  (PDNQP_E_INVALID otherwise).  The launch uses the first handle's stream.
 *  x_out[i], lambda_out[i], infos[i]: as for pdnqp_solve (infos may be
 *  NULL); infos[i].setup_s and solve_s are the instance's own device times
 *  (start to end of the set-up, start to end of the solve).  Traces are
 *  recorded per handle as in pdnqp_solve.  Returns the first error; a
 *  solver outcome other than PDNQP_SOLVED is not an error.  Not
 *  thread-safe: handles of one batch must not be used concurrently. */
int pdnqp_solve_batch(int32_t count, pdnqp_solver *const *solvers,
                      double eps_abs, double eps_rel,
                      double *const *x_out, double *const *lambda_out,
                      pdnqp_info *infos);

/* Report of the last pdnqp_solve_batch on this thread. */
typedef struct pdnqp_batch_report {
  int32_t count;
  int32_t block;       /* threads per workgroup */
  int32_t grid;        /* workgroups launched (resident at once) */
  int32_t lds_bytes;   /* dynamic LDS per workgroup */
  int32_t staged;      /* instances whose gathered vectors were staged in LDS */
  int32_t tuned;       /* 1: configuration taken from the autotuner's cache */
  int32_t waves;       /* minimum waves per SIMD the kernel was built for (1 or 4) */
  int32_t reserved;
  double kernel_ms;    /* the persistent kernel (HIP events on the stream) */
  double prepare_s;    /* host: start points, descriptors, uploads */
  double finish_s;     /* host: copies back, unscaling, external KKT checks */
  double wall_s;       /* the whole call */
} pdnqp_batch_report;

/* Copies the report; done_ms (optional, up to `cap` entries, instance order
 * of the call) receives each instance's finish time in milliseconds after
 * the first instance started (device clock). */
int pdnqp_batch_last_report(pdnqp_batch_report *rep, double *done_ms, int32_t cap);

/* Launch configuration for later batched solves in this process: the
 * workgroup size (256, 512, 1024) and the minimum waves per SIMD the kernel
 * variant was built for (1: the compiler's register budget; 4: at most 128
 * registers, more workgroups per CU).  Available pairs: (256,1), (512,1),
 * (1024,1), (256,4), (512,4).  block = 0 returns to the autotuned choice
 * ((256,1) when none is cached). */
int pdnqp_batch_set_config(int32_t block, int32_t waves);

/* Autotuner of the batched solve: runs the batch once per configuration
 * with a short budget per instance (one outer step of at most
 * `probe_inner` accepted inner iterations), keeps the fastest for the
 * batch's class (precision, count and mean nonzeros per instance, each
 * rounded down to a power of two) in a process-wide cache that
 * pdnqp_solve_batch consults, and returns it in *block_out, *waves_out.
 * ms_out (optional, 5 entries) receives the kernel time of each
 * configuration in the order listed above. */
int pdnqp_batch_autotune(int32_t count, pdnqp_solver *const *solvers, int32_t probe_inner,
                         int32_t *block_out, int32_t *waves_out, double *ms_out);

/* ---- Learned outer-step controller --------------------------------------
 * A fully connected network 16 -> 64 -> 64 -> 3 (ReLU after the hidden
 * layers, FP32) maps the features of an outer step to the log of the next
 * inner tolerance, the log of the next inner iteration budget and the log of
 * the next primal weight.  Parameters: PDNQP_MLP_PARAMS floats, in the order
 * W1 (16x64, input index major), b1 (64), W2 (64x64), b2 (64), W3 (64x3),
 * b3 (3).  All arrays are caller-owned host buffers; the network runs on the
 * current device. */
enum { PDNQP_MLP_PARAMS = 5443, PDNQP_FEATURES = 16, PDNQP_OUTER_RECORD = 8 };

/* y (count x 3) = network(theta, x (count x 16)). */
int pdnqp_mlp_forward(const float *theta, const float *x, int32_t count, float *y);

/* Gradient (PDNQP_MLP_PARAMS floats) and value of the mean squared error
 * (1 / (3 count)) sum (network(x) - y)^2 over the batch. */
int pdnqp_mlp_gradient(const float *theta, const float *x, const float *y, int32_t count,
                       float *grad, double *loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * gradient and loss of pdnqp_mlp_gradient on caller-owned DEVICE buffers --
 * theta (PDNQP_MLP_PARAMS floats), x (count x 16), y (count x 3), grad
 * (PDNQP_MLP_PARAMS floats, written), loss (one double, written; may be
 * NULL) -- enqueued on hip_stream (a hipStream_t; NULL: the default stream)
 * of the current device, without synchronising; the results equal those of
 * pdnqp_mlp_gradient bit for bit.  Calls no device allocation: the
 * per-workgroup partial gradients live in a static device array of the
 * library sized for PDNQP_MLP_NOALLOC_MAX samples (5.6 MB, held on each
 * device the function runs on until the process ends; the first call on a
 * device looks up its address).  PDNQP_E_INVALID for count outside
 * [1, PDNQP_MLP_NOALLOC_MAX] or a NULL buffer; PDNQP_E_DEVICE if a launch
 * fails.  Every call on one device shares that array: calls that overlap on
 * one device (concurrent streams or threads) race. */
enum { PDNQP_MLP_NOALLOC_MAX = 16384 };
int pdnqp_mlp_gradient_noalloc(const float *theta, const float *x, const float *y, int32_t count,
                               float *grad, double *loss, void *hip_stream);

/* Adam (step lr, moments 0.9 / 0.999) on that loss over `epochs` passes of
 * shuffled minibatches of `batch` samples (seeded); theta is updated in
 * place; loss_curve (optional, `epochs` entries) gets the full-batch loss
 * after each pass. */
int pdnqp_mlp_train(float *theta, const float *x, const float *y, int32_t count, int32_t epochs,
                    int32_t batch, float lr, uint64_t seed, float *loss_curve);

/* Copies the controller parameters into the handle (used when
 * settings.controller = 1). */
int pdnqp_set_controller(pdnqp_solver *s, const float *theta);

/* Outer steps recorded by the last pdnqp_solve (settings.outer_log): for
 * each, the 16 controller features (log10 of r_p, r_d, s_p, s_d,
 * ||x - z||_inf / gamma, delta_a, eps_a,k, omega, min / mean / max sigma,
 * r_p / r_p,prev, r_d / r_d,prev, and of 1 + the step's accepted inner
 * iterations, 1 + its restarts, 1 + k) and PDNQP_OUTER_RECORD raw values
 * (r_p, r_d, s_p, s_d, omega at the end of the inner solve, its accepted
 * inner iterations, its restarts, the inner tolerance delta_a it used).
 * NULL buffers query the count. */
int pdnqp_get_outer_log(const pdnqp_solver *s, int32_t *steps, double *features, double *record);

/* Releases the handle and its device memory.  NULL is a no-op. */
void pdnqp_destroy(pdnqp_solver *s);

/* Message of the last error on this thread ("" if none).  Valid until the
 * next library call on this thread. */
const char *pdnqp_last_error(void);

/* Internal dimensions after row normalisation: number of equality rows,
 * inequality rows (after splitting two-sided rows) and the inner primal
 * length d_w = n + m_I + m_E + m_I.  Any pointer may be NULL. */
int pdnqp_dims(const pdnqp_solver *s, int32_t *m_e, int32_t *m_i, int32_t *d_w);

/* Copies out what the last pdnqp_solve recorded when trace_iters /
 * trace_trials were set:
 *  iters:  number of recorded accepted iterations (<= trace_iters);
 *  w, y:   if non-NULL, iters*d_w and iters*(m_e+m_i) doubles: the inner
 *          iterate (x, s_I, r_E, r_I) and inner dual (y_E, y_I) after each
 *          accepted trial, in the outer-scaled, penalty- and Ruiz-unscaled
 *          coordinates of (inner-qp), internal row order (equalities first);
 *  trials: number of recorded trials; tr (if non-NULL) gets 3 doubles per
 *          trial: lhs and rhs of (adaptive-condition) and 1.0/0.0 accepted;
 *  checks: number of recorded checks; ck (if non-NULL) gets 4 int32 per
 *          check: kind (0 continue, 1 restart, 2 converged), accepted
 *          count t at the check, candidate (0 current, 1 average), and the
 *          number of trials of the solve so far.
 * Pass NULL buffers first to query counts.  PDNQP_E_STATE if nothing was
 * recorded. */
int pdnqp_get_trace(const pdnqp_solver *s, int32_t *iters, double *w, double *y,
                    int32_t *trials, double *tr, int32_t *checks, int32_t *ck);

/* Per-kernel timings gathered when settings.profile > 0 during the last
 * pdnqp_solve: for each kernel class, the launch count, summed and average
 * duration (HIP events that the sampled dispatches themselves stamp on the
 * solver's stream: the kernel's execution interval, without launch gaps)
 * and the kernel's algorithmic
 * bytes per launch (matrix values and indices once, every vector it reads
 * or writes once).  Writes up to `cap` entries; *count receives the number
 * available. */
typedef struct pdnqp_kernel_stat {
  char name[32];
  int64_t launches;
  double total_ms;
  double avg_us;
  double bytes_per_launch;
} pdnqp_kernel_stat;

int pdnqp_kernel_stats(const pdnqp_solver *s, pdnqp_kernel_stat *out, int32_t cap,
                       int32_t *count);

/* Measurement of the bound of the sparse products (Section 3.4: every inner
 * iteration is a few sparse products whose columns, on the random
 * instance families, are gathered at random positions).  On the current
 * device: a vector of vec_len elements of elem_bytes (4 or 8) bytes and
 * `gathers` seeded uniform positions in it; a kernel with the access
 * pattern of the library's CSR-stream products (unit-stride, non-temporal
 * index loads, then all of a thread's gathers at once) reads x[idx[k]] for
 * every k, once to warm the caches, then `reps` times under HIP events.
 * panels (1, 2, 4 or 8): the positions of each 2048-gather tile come from
 * one of `panels` equal slices of the vector, and the tiles of one slice
 * run on the same XCDs (workgroups are dispatched round-robin over the 8
 * XCDs), as in a column-panel split of a product.  Writes the gathers per
 * second and the average launch time (microseconds).  Allocates and frees
 * its own device buffers.  PDNQP_E_INVALID for a non-positive size or
 * count, elem_bytes other than 4 and 8, or another panel count. */
int pdnqp_probe_gather(int32_t vec_len, int32_t elem_bytes, int64_t gathers, int32_t panels,
                       int32_t reps, uint64_t seed, double *gathers_per_s, double *launch_us);

#ifdef __cplusplus
}
#endif

#endif /* PDNQP_H */
