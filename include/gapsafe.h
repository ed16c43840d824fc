/*
 * gapsafe.h -- C ABI of the MI355X (gfx950) library for the Lasso solved by
 * cyclic coordinate descent with dynamic GAP SAFE sphere screening
 * (Fercoq, Gramfort, Salmon, "Mind the duality gap: safer rules for the
 * Lasso", ICML 2015).
 *
 * Problem (Sec. 1.1, the Lasso):  min_beta 1/2 ||X beta - y||^2 + lambda ||beta||_1,
 * X in R^{n x p} given column-wise, solved over a non-increasing grid of
 * lambdas with warm starts (Algorithm 1; grid of Sec. 3.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers marked [device] are caller-owned device memory (for instance a
 *   torch tensor's data_ptr()); [host] pointers are read during the call only.
 * - X is column-major: entry (i, j) is X[i + j*ldx], ldx >= n.  X and y
 *   share the problem's dtype (FP32 or FP64).  Coefficient vectors (beta_init,
 *   beta_out, screen()'s beta) are always FP64, so that a returned beta is
 *   exactly the iterate whose gap is reported.  All reductions, the residual,
 *   the duality gap and the screening radius are FP64 on the device.
 * - Vectorized 16-byte loads are used when X is 16-byte aligned,
 *   ldx*sizeof(dtype) is a multiple of 16 and n is a multiple of
 *   16/sizeof(dtype); otherwise scalar loads.  No entry beyond row n-1 of a
 *   column is read.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   lasso_path returns when the path is finished on `stream` (it reads the
 *   per-lambda status back); lasso_solve_batch, lasso_batch_run and screen
 *   are stream-ordered and asynchronous: their outputs are valid once the
 *   caller synchronizes the stream.
 * - The library never allocates device memory: every scratch array lives in
 *   the caller's workspace (size from the *_workspace_size queries, any
 *   256-byte-aligned device buffer).  Workspace contents need no
 *   initialisation and are not meaningful after the call.
 * - Host-side argument checks happen before any launch; on error nothing is
 *   launched.  Return codes:
 *     GS_OK             0   every lambda certified (gap <= eps)
 *     GS_NOT_CONVERGED  1   soft: at least one lambda hit max_epochs; its
 *                           outputs hold the last iterate and its gap.
 *                           Returned by the calls that wait for their result
 *                           (lasso_path, lasso_path_learned); the
 *                           asynchronous batch calls report it per lambda in
 *                           status_out only.
 *     GS_EINVAL        -1   bad size, pointer, lambda, eps, f or dtype
 *     GS_EHIP          -2   HIP runtime error (text: lasso_strerror)
 *     GS_EWORKSPACE    -3   workspace NULL or smaller than required
 *     GS_EUNSUPPORTED  -4   n larger than this build handles (2048)
 *     GS_ETOOLARGE     -5   (screen_noalloc) the pass needs more scratch
 *                           than GS_NOALLOC_SCRATCH_BYTES
 */
#ifndef GAPSAFE_H
#define GAPSAFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { GS_F32 = 0, GS_F64 = 1 } gs_dtype;

enum {
  GS_OK = 0,
  GS_NOT_CONVERGED = 1,
  GS_EINVAL = -1,
  GS_EHIP = -2,
  GS_EWORKSPACE = -3,
  GS_EUNSUPPORTED = -4,
  GS_ETOOLARGE = -5
};

/* Per-lambda status written to status_out[t]. */
enum {
  GS_STATUS_CONVERGED = 0,     /* gap <= eps_rel * ||y||^2                      */
  GS_STATUS_NOT_CONVERGED = 1, /* max_epochs reached; gap_out holds the gap of
                                  the returned beta                          */
  GS_STATUS_NONFINITE = 2      /* X or y holds a NaN or Inf; outputs are zero  */
};

/* Schedules (gs_opts.schedule). */
enum {
  GS_SCHED_AUTO = 0,   /* narrow for small n*p, wide above the tuned threshold */
  GS_SCHED_NARROW = 1, /* one wavefront runs the whole path of one problem     */
  GS_SCHED_WIDE = 2    /* sweeps over all CUs, CD on one wavefront (one problem) */
};

/* CD epoch modes of the narrow schedule (gs_opts.cd_mode).  Both run the
 * same cyclic coordinate descent (Algorithm 1) and make the same updates up
 * to the order of rounding. */
enum {
  GS_CD_AUTO = 0,     /* pattern mode: while no coefficient changes sign or
                         leaves/reaches zero, a whole epoch is one triangular
                         solve on the support plus a Gram update of the
                         correlations, checked exactly against that premise;
                         an epoch that fails the check runs in residual mode */
  GS_CD_RESIDUAL = 1  /* residual updates only (rho in registers and LDS)    */
};

/* Safe region of the screening test (gs_opts.rule, screen()'s rule). */
enum {
  GS_RULE_SPHERE = 0, /* GAP SAFE sphere B(theta, sqrt(2 gap)/lambda)
                         (Sec. 3.2, Proposition 1)                        */
  GS_RULE_DOME = 1,   /* the sphere test and the GAP SAFE dome test (Sec. 3.2
                         dome equation, appendix dome support function): the
                         ball of diameter [theta, y/lambda] cut by the plane
                         through its intersection with the sphere of radius
                         r_check[beta] around y/lambda, normal (y/lambda -
                         theta)/||theta - y/lambda||.  Uses x_j^T y, computed
                         once per problem, so it adds no pass over X; every
                         input is replaced by a bound that enlarges the dome
                         under rounding.  A coordinate is dropped when either
                         test drops it.                                    */
  /* The comparison rules of Table 1, sphere tests that replace the GAP SAFE
   * test (the duality gap still decides the stop).  They run on the wide
   * schedule only (lasso_path moves to it; lasso_solve_batch and screen()
   * return GS_EUNSUPPORTED): */
  GS_RULE_STATIC = 2,  /* static SAFE: B(y/lambda, ||y|| |1/lambda -
                          1/lambda_max|) (Sec. 2.1)                         */
  GS_RULE_DYNSAFE = 3, /* Dynamic Safe: B(y/lambda, ||theta_k - y/lambda||)
                          (Sec. 2.3)                                        */
  GS_RULE_ST3 = 4      /* Dynamic ST3: B(y/lambda, R_hat) cut by the plane
                          s* x*^T theta = 1 (x* the column of largest
                          |x_j^T y|, s* its sign), held in the ball around the
                          projection of y/lambda on the plane: center
                          y/lambda - s* (lambda_max/lambda - 1) x* / ||x*||^2,
                          radius (R_hat^2 - d^2)^(1/2), d the distance to the
                          plane (Table 1)                                   */
};

/* Counters of gs_opts.stats (indices). */
enum {
  GS_STAT_PATTERN_EPOCHS = 0, /* epochs committed by the pattern mode         */
  GS_STAT_RESIDUAL_EPOCHS,    /* epochs run by the residual mode              */
  GS_STAT_REJECTED,           /* pattern epochs rejected by the check         */
  GS_STAT_BUILDS,             /* Gram columns computed                        */
  GS_STAT_SETUPS,             /* pattern set-ups                              */
  GS_STAT_SUPPORT_CHANGES,    /* set-ups whose support features changed     */
  GS_STAT_PASSES,             /* screening passes                             */
  GS_STAT_SKIPPED,            /* epochs skipped at an exact fixed point       */
  GS_STAT_EXACT,              /* pattern epochs whose zero coordinates needed
                                 the exact check over the whole active set   */
  GS_STAT_NEAR,               /* pattern epochs where the norm bound left at
                                 most 64 zero coordinates, checked exactly   */
  GS_STAT_WIDE_VISITS,        /* wide schedule: coordinates the CD rounds
                                 visited exactly (the others were proven to
                                 stay at zero)                               */
  GS_STAT_WIDE_ROUNDS,        /* wide schedule: CD rounds                     */
  GS_STAT_WIDE_STOPS,         /* wide schedule: rounds that re-anchored       */
  GS_NSTATS
};

/* One Lasso path (Algorithm 1 inputs X, y and the lambda grid). */
typedef struct gs_problem {
  int32_t n, p;            /* rows and columns of the design, n, p >= 1        */
  int64_t ldx;             /* leading dimension of X (>= n, or >= the largest
                              row index + 1 when `rows` is set)              */
  int32_t dtype;           /* gs_dtype of X and y                              */
  const void* X;           /* [device] design, column-major                    */
  const void* y;           /* [device] response                                */
  const int32_t* rows;     /* [device] optional: n row indices into X and y
                              (a row subsample); NULL = rows 0..n-1          */
  int32_t T;               /* number of lambdas, >= 1                          */
  const double* lambdas;   /* [host] T non-increasing positive values, or NULL */
  int32_t lambda_relative; /* != 0: lambdas[] are multiples of lambda_max      */
  double lambda_min_ratio; /* lambdas == NULL: the grid lambda_t =
                              lambda_max * ratio^(t/(T-1)), t = 0..T-1, so
                              lambda_0 = lambda_max (Sec. 3.3; the paper's
                              10^(-delta) is ratio).  0 < ratio <= 1.        */
  const double* beta_init; /* [device] optional warm start for the first
                              lambda (p values); NULL = 0, the solution at
                              lambda_max (Algorithm 1 initialisation)        */
  double* beta_out;        /* [device] p x T column-major: beta^{lambda_t}     */
  double* gap_out;         /* [device] T: duality gap of the returned beta on
                              the final safe active set (the dual norm is
                              taken over A, Sec. 4.1); it bounds
                              P(beta) - P(beta_hat)                          */
  int32_t* epochs_out;     /* [device] T: CD epochs run at lambda_t           */
  int32_t* nactive_out;    /* [device] T: size of the safe active set at exit */
  int32_t* status_out;     /* [device] T: GS_STATUS_*                          */
  double* lambda_out;      /* [device] optional T: the lambdas used           */
  /* Sparse designs (Sec. 4.1: the paper's second implementation).  With
   * format GS_CSC, X holds the nnz nonzero values (dtype), col_ptr[j] ..
   * col_ptr[j+1]-1 index column j's entries in X and row_idx (rows distinct
   * within a column), and ldx and rows are not used.  A CSC path runs one
   * wavefront per problem with the residual in LDS when 8n bytes fit
   * (else in the workspace), the sweep is the transposed sparse product
   * over the active columns and a CD step touches only column j's rows;
   * rule sphere or dome, the Lasso only (no elastic net), residual-mode
   * epochs.  A batch must be all dense or all CSC. */
  int32_t format;          /* GS_DENSE (0, default) or GS_CSC (1)             */
  const int64_t* col_ptr;  /* [device] CSC: p + 1 non-decreasing offsets,
                              col_ptr[0] = 0                                  */
  const int32_t* row_idx;  /* [device] CSC: col_ptr[p] row indices in [0, n)  */
} gs_problem;

enum { GS_DENSE = 0, GS_CSC = 1 };

typedef struct gs_opts {
  double eps_rel;        /* stop when gap <= eps_rel * ||y||^2 (default 1e-8;
                            the paper's epsilon is absolute)                 */
  int32_t screen_every;  /* f: screening pass every f CD epochs (default 10,
                            Sec. 4.1)                                        */
  int32_t max_epochs;    /* K: CD epochs per lambda (default 100000)         */
  int32_t schedule;      /* GS_SCHED_*                                        */
  int32_t cd_mode;       /* GS_CD_*: how the narrow schedule runs its epochs  */
  int32_t* select_counts;/* [device] optional (batch only): T x p int32
                            counters; count[t*p + j] += 1 for every problem
                            whose beta^{lambda_t}_j != 0 (stability
                            selection).  Requires equal p and T in the batch;
                            the caller zeroes it.                            */
  int64_t* timestamps;   /* [device] optional (batch only): 2*B values, start
                            and end of each problem in device wall-clock
                            ticks (see gs_wallclock_hz)                      */
  int64_t* stats;        /* [device] optional: GS_NSTATS counters of the
                            narrow schedule, incremented (atomically) by the
                            call; the caller zeroes them                     */
  int32_t rule;          /* GS_RULE_*: the safe region (default sphere)       */
  double enet_alpha;     /* elastic net mixing a in (0, 1] (appendix,
                            "Elastic-Net"): minimizes 1/2||X b - y||^2 +
                            a lambda ||b||_1 + (1-a) lambda/2 ||b||^2, solved
                            as the Lasso with parameter a lambda on the
                            augmented design [X; sqrt((1-a) lambda) I] and
                            response [y; 0], kept implicit; the grid starts
                            at ||X^T y||_inf / a and the gap is that of the
                            augmented problem.  1 (default; 0 also means 1)
                            is the Lasso.  a < 1 runs on the wide schedule
                            (lasso_path moves there; lasso_solve_batch and
                            lasso_path_learned return GS_EUNSUPPORTED) and
                            with the GAP SAFE sphere or dome only.         */
} gs_opts;

/* Fill *o with the defaults above. */
void gs_opts_default(gs_opts* o);

/* Device wall-clock frequency used by gs_opts.timestamps, in Hz (0 on error). */
double gs_wallclock_hz(void);

/* Bytes of workspace that lasso_path / lasso_solve_batch need for these
 * problems (0 when an argument is invalid). */
size_t lasso_workspace_size(const gs_problem* probs, int32_t B,
                            const gs_opts* opts);

/* Algorithm 1 for one problem: precompute ||x_j||^2 and lambda_max =
 * ||X^T y||_inf (Sec. 1.2), build the grid, then for each lambda_t warm-start
 * from beta^{lambda_{t-1}}, screen every f epochs with the GAP SAFE sphere
 * (Sec. 3.2: theta = alpha rho from the residual rescaling of Sec. 2.3,
 * radius sqrt(2 gap)/lambda inflated by a rounding bound) and run cyclic CD
 * on the surviving coordinates until the gap is <= eps.  Returns when the
 * path is finished (GS_NOT_CONVERGED if a lambda reached max_epochs). */
int lasso_path(const gs_problem* prob, const gs_opts* opts, void* workspace,
               size_t ws_bytes, void* stream);

/* B independent paths in one persistent launch: problems are ordered by
 * estimated cost and handed to one wavefront each through a device work
 * queue.  Asynchronous; per-problem results in each problem's outputs. */
int lasso_solve_batch(const gs_problem* probs, int32_t B, const gs_opts* opts,
                      void* workspace, size_t ws_bytes, void* stream);

/* A batch recorded once and replayed: lasso_batch_plan checks the problems,
 * uploads their descriptors and lambdas into the workspace (on `stream`,
 * which it synchronizes), and captures the persistent launches of
 * lasso_solve_batch into a HIP graph; lasso_batch_run replays that graph on
 * any stream, each replay solving the whole batch again from the inputs
 * (select_counts keep accumulating over replays; timestamps are
 * overwritten).  The plan refers to the caller's workspace, inputs and
 * outputs, which must stay valid and unchanged in size while it is used;
 * their contents (X, y, beta_init) may change between replays.  The plan is
 * host memory owned by the caller; lasso_batch_plan_free releases it.
 * Returns the codes of lasso_solve_batch, or GS_EHIP when capture fails. */
typedef struct gs_batch_plan gs_batch_plan;
int lasso_batch_plan(const gs_problem* probs, int32_t B, const gs_opts* opts,
                     void* workspace, size_t ws_bytes, void* stream,
                     gs_batch_plan** plan);
int lasso_batch_run(gs_batch_plan* plan, void* stream);
void lasso_batch_plan_free(gs_batch_plan* plan);

/* Tile autotuner of the batched launch.  Problems fall into classes (dtype,
 * row list or not, 16-byte loads or not, and the smallest compiled column
 * layout that holds n rows).  For each class present in probs it times every
 * candidate layout (the smallest one of each lane split S that holds the
 * class) on up to `sample` of its most expensive problems, each solved for
 * its first min(T, max_lambdas) lambdas, and records the fastest; later
 * calls in this process (lasso_path's narrow schedule, lasso_solve_batch,
 * lasso_batch_plan) use the recorded layout.  The sampled problems' outputs
 * are overwritten with those partial runs.  choice_out (optional, host, 2B
 * int32): the chosen (S, NG) of each problem.  Synchronizes `stream`.
 * gs_tune_save / gs_tune_load write and read the recorded choices as JSON
 * (GS_EINVAL when the file cannot be opened or holds no valid entry);
 * gs_tune_reset forgets them. */
int gs_autotune(const gs_problem* probs, int32_t B, const gs_opts* opts,
                void* workspace, size_t ws_bytes, void* stream,
                int32_t max_lambdas, int32_t sample, int32_t* choice_out);

/* Schedule autotuner of lasso_path's "auto" schedule (GS_SCHED_AUTO), which
 * runs a problem on the wide schedule when n*p exceeds a per-dtype threshold
 * (16 Mi by default) and on the narrow one otherwise.  This call times both
 * schedules on prob's first min(T, max_lambdas) lambdas (after one untimed
 * run of each) with opts, records the size n*p and which was faster, and
 * moves the dtype's threshold to the cut between all sizes measured so far
 * in this process that misclassifies the fewest of them (the geometric
 * midpoint of the two sizes around it).  prob's outputs are overwritten with
 * those partial runs; the workspace is lasso_path's.  choice_out (optional,
 * host): 1 if the wide schedule was faster, else 0.  GS_EUNSUPPORTED for a
 * problem only one schedule runs (a row subsample, a CSC design, a
 * comparison rule, the elastic net).  Synchronizes `stream`.
 * gs_wide_threshold returns the dtype's current threshold (-1 for a bad
 * dtype).  gs_tune_save / gs_tune_load also write and read the thresholds;
 * gs_tune_reset restores the default. */
int gs_autotune_schedule(const gs_problem* prob, const gs_opts* opts, void* workspace,
                         size_t ws_bytes, void* stream, int32_t max_lambdas,
                         int32_t* choice_out);
double gs_wide_threshold(int32_t dtype);
int gs_tune_save(const char* path);
int gs_tune_load(const char* path);
void gs_tune_reset(void);

/* Bytes of workspace that screen() needs. */
size_t screen_workspace_size(int32_t n, int32_t p);

/* One GAP SAFE screening pass at (beta, lambda) over the active set A:
 * rho = y - X beta; c_j = x_j^T rho and M = max_{j in A} |c_j| (the dual norm
 * over A, Sec. 4.1); theta = alpha rho with alpha = min(max(y^T rho /
 * (lambda ||rho||^2), -1/M), 1/M) (Sec. 2.3); gap G = P(beta) - D(theta);
 * radius r = sqrt(2 G)/lambda (Proposition 1); keep j iff
 * |x_j^T theta| + r ||x_j|| >= 1 (Sec. 2.1 sphere test) with the rounding
 * inflation, and with rule GS_RULE_DOME also the GAP SAFE dome test (it
 * computes x_j^T y in the same sweep).  Asynchronous.
 *   dtype/X/y/ldx as in gs_problem (no row subsample); beta [device] p FP64
 *   values; active_in [device] q_in ascending column indices or NULL (all p);
 *   active_out [device] capacity q_in (p when active_in is NULL), receives the
 *   kept indices in ascending order; q_out [device] 1 int32; gap_out,
 *   alpha_out, radius_out [device] 1 double each (radius_out is the inflated
 *   radius actually used by the test); c_out [device] optional q_in doubles:
 *   c_j for the j of active_in, in its order. */
int screen(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X,
           const void* y, const double* beta, double lambda, int32_t rule,
           const int32_t* active_in, int32_t q_in, int32_t* active_out,
           int32_t* q_out, double* gap_out, double* alpha_out,
           double* radius_out, double* c_out, void* workspace,
           size_t ws_bytes, void* stream);

/* screen() without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, outputs and semantics as screen(); its
 * scratch arrays live in a static device array of GS_NOALLOC_SCRATCH_BYTES
 * (16 MiB) that the library holds on each GPU it runs on until the process
 * ends, so the call allocates nothing.  The pass fits when
 * screen_workspace_size(n, p) <= GS_NOALLOC_SCRATCH_BYTES (about 48 bytes
 * per column: p up to roughly 347,000 at n = 2048); larger inputs return
 * GS_ETOOLARGE before anything is launched.  Every call on one GPU uses that
 * GPU's array: calls that overlap on one GPU (on different streams or host
 * threads) race and must be serialized by the caller; calls ordered on one
 * stream are fine.  The array keeps the last call's contents; the pass
 * initialises everything it reads. */
#define GS_NOALLOC_SCRATCH_BYTES (16u << 20)
int screen_noalloc(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X,
                   const void* y, const double* beta, double lambda, int32_t rule,
                   const int32_t* active_in, int32_t q_in, int32_t* active_out,
                   int32_t* q_out, double* gap_out, double* alpha_out, double* radius_out,
                   double* c_out, void* stream);

/* ---------------------------------------------------------------------
 * Learned warm start.  A small network proposes, at each lambda_t of a path,
 * a starting point for Algorithm 1 in place of beta^{lambda_{t-1}}.  GAP SAFE
 * screening is safe for any primal point (Theorem 2), so a proposal can only
 * change the time to the certified gap, never the answer; the driver keeps it
 * only when its duality gap is smaller than the plain warm start's.
 *
 * Network: 4 -> 64 -> 64 -> 2 with ReLU hidden layers.  Parameters are one
 * FP32 array of GS_MLP_PARAMS values: W1 (64x4, row-major, row = hidden
 * unit) at 0, b1 at 256, W2 (64x64, row = output unit) at 320, b2 at 4416,
 * W3 (2x64) at 4480, b3 at 4608.  Evaluation rounds W1, W2, W3 and the first
 * hidden layer (the input of the second layer, which runs on the matrix
 * cores) to bfloat16 (nearest, ties to even) and accumulates in FP32.
 * Outputs per feature: o0 = the change of the coefficient from the previous
 * point in units of lambda_t / ||x_j||^2, (beta0_j - beta_prev_j) ||x_j||^2 /
 * lambda_t, o1 = the logit of "beta_j != 0 at lambda_t".  (Predicting the
 * change rather than the value keeps the proposal as precise as the previous
 * point where the network proposes no change: a value passed through BF16
 * weights would carry a relative error of about 2^-8.  In these units the
 * change of a support coefficient is of the order of the relative lambda
 * step, whatever the scale of X and y.)
 * Inputs per feature j at (beta, lambda), with c_j = x_j^T (y - X beta):
 *   u_j = (|c_j| / lambda, lambda / lambda_max, beta_j ||x_j|| / ||y||, bmc_j)
 * where bmc_j is the block max correlation below.
 * All pointers are device pointers unless marked [host]; calls are
 * asynchronous on `stream` unless stated.  Errors: GS_EINVAL for a bad size,
 * pointer or value, GS_EWORKSPACE for a missing or small workspace, GS_EHIP
 * for a launch failure. */
enum { GS_MLP_PARAMS = 4610 };

/* bmc_j = max over k != j in j's block of |x_j^T x_k| / (||x_j|| ||x_k||);
 * blocks are `block` (1..64) contiguous columns, the last one possibly
 * shorter; 0 for a block of one column or a zero column.  X as in gs_problem
 * (column-major, ldx >= n); bmc: p floats.  FP32 accumulation. */
int gs_block_corr(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X,
                  int32_t block, float* bmc, void* stream);

/* Network outputs for m feature rows: U is m x 4 (row-major), out m x 2. */
int gs_mlp_forward(const float* params, const float* U, int32_t m, float* out,
                   void* stream);

/* Training.  targets is m x 3 (row-major): (step target, support target in
 * {0, 1}, mask of the step term).  Loss = (1/m) sum_j [ BCE(o1_j, support_j)
 * + mask_j (o0_j - step_j)^2 ], differentiated through the evaluation above
 * (the bfloat16 roundings pass gradients unchanged).  The workspace holds one
 * partial gradient per 64 rows, summed in a fixed order, so results are
 * deterministic.
 *   gs_mlp_grad: grad (GS_MLP_PARAMS floats) and loss (1 float), either
 *   optional.
 *   gs_mlp_adam: one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias
 *   correction for step t >= 1) of params with moments adam_m, adam_v (each
 *   GS_MLP_PARAMS floats, zero before step 1) from grad.
 *   gs_mlp_train_step: gs_mlp_grad then gs_mlp_adam in two launches; loss
 *   optional. */
size_t gs_mlp_train_workspace_size(int32_t m);
int gs_mlp_grad(const float* params, const float* U, const float* targets, int32_t m,
                float* grad, float* loss, void* workspace, size_t ws_bytes, void* stream);
int gs_mlp_adam(float* params, float* adam_m, float* adam_v, const float* grad, int32_t t,
                float lr, void* stream);
int gs_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t t, float lr,
                      const float* U, const float* targets, int32_t m, float* loss,
                      void* workspace, size_t ws_bytes, void* stream);

/* The network inputs u_j for j < p into U (p x 4): c, beta_prev, nrm2
 * (||x_j||^2) are p FP64 values, bmc p floats; lambda, lambda_max, ynorm
 * (||y||) positive and finite. */
int gs_warm_features(int32_t p, const double* c, const double* beta_prev,
                     const double* nrm2, const float* bmc, double lambda,
                     double lambda_max, double ynorm, float* U, void* stream);

/* A path (Algorithm 1 over the problem's lambda grid) whose warm start at
 * each lambda_t with a previous point comes from the network (t >= 1, and
 * t = 0 when beta_init is given: the previous point is then beta_init, so a
 * path may be run in consecutive pieces):
 *   1. a screening pass at the previous point beta^{lambda_{t-1}} over all
 *      p gives the safe set A_plain and c (coordinates outside A_plain are
 *      zero at the optimum);
 *   2. the network maps u_j to (o0_j, o1_j); the working set W holds the j
 *      of A_plain on the support of beta_prev and those off it that violate
 *      the optimality conditions at beta_prev (|c_j| > lambda_t) with o1_j >
 *      tau (the network's predicted entrants), tau the first of 0, 1, 2, 3,
 *      4, 6, 8 that admits at most min(GS_WS_ADD, (cap - |supp beta_prev|)
 *      / 2) entrants (none if 8 admits more); signs sigma_j =
 *      sign(beta_prev_j) on the previous support and sign(c_j) elsewhere;
 *   3. the restricted solve (gs_restricted_solve below) gives b on W; the
 *      coordinates whose sign disagrees with sigma leave W (those off the
 *      previous support when there are any such, else the others) and W is
 *      solved again (at most GS_WS_DROPS times); beta0 = b on W, 0 elsewhere;
 *   4. at most GS_WS_ROUNDS times: a screening pass at beta0 over A_plain
 *      gives c; the (at most GS_WS_ADD) largest violators |c_j| > lambda_t
 *      outside W join W with sigma_j = sign(c_j), and step 3 runs again;
 *      no violator ends the rounds;
 *   5. when the rounds ended with no violator and that last pass found the
 *      duality gap of beta0 on the problem reduced to A_plain already <= eps
 *      (a certificate for the whole problem: A_plain is safe), lambda_t is
 *      output from it -- beta0, that gap, 0 epochs, the pass's kept count as
 *      nactive -- as Algorithm 1 would stop at its first pass; otherwise
 *   6. the duality gaps of beta0 and of beta^{lambda_{t-1}} on the problem
 *      reduced to A_plain are compared, and the smaller one's point starts
 *      lambda_t (ties keep the plain start), and
 *   7. Algorithm 1 runs for lambda_t from there, exactly as in lasso_path.
 * A working set larger than cap = min(n - 1, p, GS_WS_MAX) or a failed
 * factorization (a pivot that is not positive) leaves lambda_t to the plain
 * start.  The output o0 is not used by the driver (the restricted solve
 * gives the coefficients).
 * With params NULL every lambda starts from the previous point (the plain
 * path, run one lambda at a time).  The problem has no row subsample and all
 * its outputs; block (1..64) is the bmc block width.  learned_out (optional,
 * T int32) receives 1 where the network's start was taken, else 0.
 * Synchronizes `stream` (the lambda grid, the active set and working set
 * sizes are read on the host).  Returns the codes of lasso_path. */
enum { GS_WS_ROUNDS = 4, GS_WS_ADD = 32, GS_WS_DROPS = 4, GS_WS_MAX = 2047 };
size_t lasso_path_learned_workspace_size(const gs_problem* prob);
int lasso_path_learned(const gs_problem* prob, const gs_opts* opts, const float* params,
                       int32_t block, int32_t* learned_out, void* workspace,
                       size_t ws_bytes, void* stream);

/* The restricted solve of the learned start.  On the working set W (m
 * distinct column indices) with signs sigma (+1 or -1), the Lasso's
 * optimality conditions (Sec. 2: the subgradient of ||beta||_1 at a nonzero
 * beta_j is sign(beta_j)) reduce to the linear system
 *     (X_W^T X_W) b = X_W^T y - lambda sigma,
 * whose solution is the Lasso solution at lambda when W holds its support,
 * sigma its signs, b has those signs and |x_j^T (y - X_W b)| <= lambda for
 * every other column.  Solved in FP64 by a blocked Cholesky factorization of
 * the Gram matrix (products of the stored X values, exact in FP64).
 * n, p, ldx, dtype, X, y as in gs_problem (column-major X, no row subsample);
 * W [device] m int32 in [0, p); sigma [device] m doubles; 1 <= m < n, m <= p,
 * m <= GS_WS_MAX (X_W must have full column rank); lambda >= 0 finite;
 * b_out [device] m doubles; info_out [device] 1 int32: 0 on success, k >= 1
 * when the k-th pivot was not a positive normal number (X_W numerically rank
 * deficient; b_out is then not written), -1 for an index of W outside [0, p).
 * workspace: gs_restricted_solve_workspace_size(m) bytes (8 M (M + 64) for
 * the matrix and its right-hand-side tile row, M = m rounded up to 64, plus
 * at most 15 MB of partial sums of the Gram product split over rows), or
 * 0 for an m out of range.  Asynchronous on `stream`.  GS_EINVAL for a bad
 * size, pointer or value, GS_EWORKSPACE for a small workspace. */
size_t gs_restricted_solve_workspace_size(int32_t m);
int gs_restricted_solve(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X,
                        const void* y, const int32_t* W, const double* sigma, int32_t m,
                        double lambda, double* b_out, int32_t* info_out, void* workspace,
                        size_t ws_bytes, void* stream);

/* Optional kernel timing for benchmarks (off by default).  When on, the
 * library records a pair of HIP events on the launch stream around each
 * launch of the named kernels and accumulates their elapsed time:
 *   "sweep"  the X^T rho sweep of the wide schedule and of screen()
 *   "path"   the persistent per-problem path kernel (narrow schedule)
 * gs_timing_query waits for the recorded events, then returns the total in
 * milliseconds and the number of launches (0 / -1 for an unknown name).
 * Not thread-safe; meant for single-threaded benchmark drivers. */
void gs_timing_enable(int on);
void gs_timing_reset(void);
int gs_timing_query(const char* kernel, double* total_ms, int64_t* launches);

/* Human-readable text for a return code (for GS_EHIP, the last HIP error). */
const char* lasso_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* GAPSAFE_H */
