/*
 * ammse.h - C ABI of libammse, a batched GPU solver (AMD MI355X, gfx950) for
 * weighted-sum-rate (WSR) downlink precoding by A-MMMSE, the accelerated
 * mixed weighted-unweighted sum-MSE method of arXiv 2510.20507.
 *
 * Problem (Section II, WSR problem): C base stations (BS) with M antennas;
 * users u, ordered cell by cell, with N receive antennas and d streams;
 * channel H_{u,j} (N x M) from BS j to user u, noise power sigma2_u, weight
 * alpha_u, per-BS sum-power budget P_c.  Find precoders V_u (M x d) that
 * maximise sum_u alpha_u R_u subject to sum_{u in c} ||V_u||_F^2 <= P_c.
 *
 * Method (Algorithm 3): per iteration, receivers U and weights W by exact
 * block minimisation (Section IV equations for U and W; only N x N and d x d
 * factorisations), W = I during the warm-start stage (Section V-B) until the
 * relative WSR change drops to eps1, then one projected-gradient step for V
 * (Section V-A: gradient, projection onto the sum-power ball, adaptive step
 * for the first T_c iterations, extrapolation weight omega^t).  The fixed
 * step after the adaptive window is not given by the paper; by default the
 * second stage uses the bound of Section VI (ammse_options_t.step_rule).
 *
 * Conventions for every entry point:
 *   - All data buffers are caller-owned DEVICE memory unless stated; the
 *     library never frees or reallocates them.  Tables passed to
 *     ammse_validate / ammse_plan_create are HOST memory and are copied.
 *   - Complex numbers are interleaved (re, im): double2 when the plan's
 *     precision is AMMSE_PREC_FP64, float2 for AMMSE_PREC_FP32.
 *   - Calls that take a stream only enqueue work on it and return; outputs
 *     are valid once the stream has synchronised.
 *   - Errors in arguments are reported synchronously by the return code and
 *     nothing is enqueued.  Numerical trouble in one instance (a failed
 *     factorisation, a non-finite value) is reported in that instance's
 *     status word and never aborts the process.  No C++ exception crosses
 *     this interface.
 */
#ifndef AMMSE_H
#define AMMSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AMMSE_VERSION 2

/* Return codes. */
typedef int32_t ammse_status_t;
#define AMMSE_OK 0
#define AMMSE_ERR_NULL 1        /* a required pointer argument is NULL */
#define AMMSE_ERR_SHAPE 2       /* an instance entry has invalid sizes or offsets */
#define AMMSE_ERR_OPTION 3      /* an option is out of range */
#define AMMSE_ERR_WORKSPACE 4   /* workspace smaller than ammse_plan_workspace_size */
#define AMMSE_ERR_HIP 5         /* HIP runtime error (no device, launch failure) */
#define AMMSE_ERR_UNSUPPORTED 6 /* valid but outside this build's limits (see below) */
#define AMMSE_ERR_ALLOC 7       /* the plan could not allocate its device tables */

/* Per-instance status bits written by ammse_solve. */
#define AMMSE_INST_OK 0
#define AMMSE_INST_NONFINITE 1  /* a WSR or step became NaN/Inf; iteration stopped */
#define AMMSE_INST_CHOLESKY 2   /* a covariance factorisation failed; iteration stopped */
#define AMMSE_INST_ZERO_POWER 4 /* some BS ended with zero transmit power */

/* Arithmetic of the channel products (and storage type of H and V). */
#define AMMSE_PREC_FP64 0       /* everything in double */
#define AMMSE_PREC_FP32 1       /* channel products in float; N x N, d x d work,
                                   step size and projection in double */
#define AMMSE_PREC_BF16 2       /* mixed: H and V stored as float; the two channel
                                   products of an iteration run in bfloat16 with float
                                   accumulation, except in the last refine_iters
                                   iterations (the refinement pass), which start by
                                   recomputing G^{t-1} and G^{t-2} in float and then
                                   run as AMMSE_PREC_FP32; the step size, the N x N /
                                   d x d algebra and the projection are as in FP32 */

/* Kernel selection (ammse_options_t.path). */
#define AMMSE_PATH_AUTO 0
#define AMMSE_PATH_GENERAL 1

/* Limits of this build. */
#define AMMSE_MAX_CELLS 16
#define AMMSE_MAX_RX 4          /* N <= 4 (the paper's d <= N <= 4 regime) */
#define AMMSE_MAX_USERS 256     /* users per instance (all cells) */
#define AMMSE_MAX_ANTENNAS 4096

/*
 * One instance (channel realisation).  Offsets index the flat buffers passed
 * to ammse_solve; they may be in any order but blocks must not overlap.
 *   H:       C blocks, block c = stacked channel H_{:,c} = [H_{0,c}; ...;
 *            H_{U-1,c}], (U*N) x M row-major; element offset h_off.
 *   V:       C blocks, block c = V_c = [V_u, u in cell c], M x (U_c*d)
 *            row-major, so V_u[m][s] = V_c[m][i*d + s] for the i-th user of c;
 *            element offset v_off.
 *   sigma2, alpha: U entries at user_off.    P: C entries at bs_off.
 *   cell_users: C entries (users per cell) at cell_off; they sum to U.
 */
typedef struct ammse_instance_t {
  int32_t C;        /* base stations (cells), 1..AMMSE_MAX_CELLS */
  int32_t U;        /* users over all cells, 1..AMMSE_MAX_USERS */
  int32_t M;        /* BS antennas, 1..AMMSE_MAX_ANTENNAS */
  int32_t N;        /* receive antennas per user, 1..AMMSE_MAX_RX */
  int32_t d;        /* streams per user, 1..N */
  int32_t cell_off; /* index of this instance's first entry in cell_users[] */
  int64_t h_off;    /* complex elements */
  int64_t v_off;    /* complex elements */
  int64_t user_off; /* entries of sigma2[] / alpha[] */
  int64_t bs_off;   /* entries of P[] */
} ammse_instance_t;

/* Algorithms (ammse_options_t.algorithm). */
#define AMMSE_ALGO_AMMMSE 0  /* Algorithm 3 (A-MMMSE; A-WMMSE with warm_start = 0) */
#define AMMSE_ALGO_WMMSE 1   /* Algorithm 2 (WMMSE, Section IV): U and W as in
                                Algorithm 3's second stage, V per BS by the exact
                                minimiser (A_c + mu_c I)^{-1} B_c with the dual
                                mu_c >= 0 of the power budget (mu_c = 0 when the
                                unconstrained minimiser meets it).  The comparator
                                of Section VII.  max_iters caps the iterations,
                                eps2 > 0 stops once the relative WSR change of an
                                iteration is <= eps2; T_c, eps1, warm_start,
                                extrapolate, gamma_c are ignored.  FP64 and FP32
                                storage (the M x M solve runs in double); the
                                general kernel only. */
#define AMMSE_ALGO_MMMSE 2   /* Section V-B (mixed weighted-unweighted sum-MSE):
                                WMMSE iterations with W = I (sum-MSE block
                                coordinate descent, V by the same exact minimiser)
                                until the eps1 rule of Algorithm 3 switches to W =
                                E^{-1}; eps2 stops after a second-stage iteration.
                                warm_start = 0 or force_switch_iter as for
                                Algorithm 3; otherwise as AMMSE_ALGO_WMMSE. */
#define AMMSE_ALGO_BCGD 3    /* BCGD-WMMSE, the full block-coordinate gradient
                                method of the Section VII-F ablation: per
                                iteration U_u takes one gradient step of f (step
                                1 / (2 alpha_u ||J_u||_F ||W_u||_F), J_u the
                                receive covariance), W_u one Schulz step
                                W (2I - E_u W) with E_u the MSE matrix at the new
                                U_u, and V Algorithm 3's second-stage projected
                                step (extrapolation, T_c, step_rule, gamma_c as
                                there); U and W start as the MMSE receivers and
                                E^{-1} at V^0.  eps2 stops as for Algorithm 3's
                                second stage; eps1, warm_start, force_switch_iter
                                are ignored.  FP64 and FP32 storage; the general
                                kernel only. */

/* Fixed step after the adaptive window (ammse_options_t.step_rule); the
 * paper leaves gamma_c as an input of Algorithm 3 without a value.
 *   AMMSE_STEP_BOUND: stage I keeps the last adaptive step of each BS; stage
 *     II (after its own re-armed window, see rearm_at_switch) uses
 *     gamma_c = 1 / Lhat_c, Lhat_c = 2 lambda_max(sum_u (alpha_u / sigma2_u)
 *     H_{u,c}^H H_{u,c}) over all users u.  Section VI (proof of Lemma 3)
 *     gives lambda_max(W_u U_u^H U_u) <= 1 / sigma2_u, so Lhat_c bounds the
 *     Lipschitz constant ||2 A_c||_2 of the V-gradient at every iterate and
 *     every stage-II step meets the descent condition of Theorem 1.  Lhat_c
 *     is computed once per solve (Lanczos), when the first such step needs it.
 *   AMMSE_STEP_FROZEN: the last adaptive step of each BS in both stages.
 * A positive gamma_c overrides either rule. */
#define AMMSE_STEP_BOUND 0
#define AMMSE_STEP_FROZEN 1

/* Solver options (Algorithm 3 inputs). */
typedef struct ammse_options_t {
  int32_t precision;         /* AMMSE_PREC_* */
  int32_t max_iters;         /* iterations T (>= 0) */
  int32_t T_c;               /* adaptive-step window (paper: 3) */
  int32_t warm_start;        /* 1: stage I (W = I) until eps1 (A-MMMSE); 0: A-WMMSE */
  int32_t extrapolate;       /* 1: omega^t = max{(t-2)/(t+1),0}; 0: omega = 0 */
  int32_t rearm_at_switch;   /* 1: also use the adaptive step in the first T_c
                                stage-II iterations (default); 0: only t <= T_c */
  int32_t force_switch_iter; /* -1: switch by the eps1 rule; s >= 1: first stage-II
                                iteration is s for every instance */
  int32_t lanczos_steps;     /* Krylov dimension for ||2A_c||_2; 0 = min(M, 64) */
  int32_t path;              /* AMMSE_PATH_AUTO: LDS-resident MFMA kernel when every
                                instance fits it, else the general kernel;
                                AMMSE_PATH_GENERAL: always the general kernel */
  int32_t refine_iters;      /* AMMSE_PREC_BF16: final iterations with float products
                                (the refinement pass); ignored otherwise */
  int32_t algorithm;         /* AMMSE_ALGO_AMMMSE (Algorithm 3), _WMMSE or _MMMSE */
  int32_t tile;              /* output tile shape of the MFMA channel products of the
                                general kernel (FP32 and BF16): 0 = the plan's choice
                                (shape 0 until ammse_autotune picks one per shape
                                class); 1, 2, 3 = force shape 0, 1, 2 (64 x 64,
                                128 x 16, 64 x 32) for every instance.  Applies to
                                products with more than 64 output rows; those with
                                33-64 rows take a 64-row shape and conjugated ones
                                (H^H Z, R^H R) with at most 32 rows a 16- or
                                32-row shape whatever this option says */
  int32_t step_rule;         /* AMMSE_STEP_BOUND (default) or AMMSE_STEP_FROZEN */
  double eps1;               /* stage-switch tolerance (paper: 0.1) */
  double eps2;               /* stop tolerance (0: run exactly max_iters) */
  double gamma_c;            /* > 0: fixed step after the adaptive windows (both
                                stages); <= 0: the step rule above */
} ammse_options_t;

/* Opaque plan: validated copy of the instance table on the device, the
 * per-instance workspace map and the launch order. */
typedef struct ammse_plan_s* ammse_plan_t;

/* HIP stream handle (identical to hipStream_t). */
typedef struct ihipStream_t* ammse_stream_t;

/* Library version (AMMSE_VERSION). */
int32_t ammse_version(void);

/* Human-readable text for a return code; never NULL. */
const char* ammse_status_string(ammse_status_t s);

/* Fill *opt with the paper's defaults: FP32, T = 100, T_c = 3, warm start,
 * extrapolation, re-armed step, step_rule = AMMSE_STEP_BOUND, eps1 = 0.1,
 * eps2 = 0, gamma_c = 0, refine_iters = 10, algorithm = AMMSE_ALGO_AMMMSE. */
void ammse_default_options(ammse_options_t* opt);

/*
 * Host-only validation of an instance table (no GPU needed).  table and
 * cell_users are host arrays of `batch` entries and of the referenced cell
 * counts.  On success the optional outputs receive the minimum lengths the
 * flat buffers must have: complex elements of H and V, entries of
 * sigma2/alpha, entries of P.  opt may be NULL (defaults).
 */
ammse_status_t ammse_validate(const ammse_instance_t* table, const int32_t* cell_users,
                              int32_t batch, const ammse_options_t* opt, int64_t* h_elems,
                              int64_t* v_elems, int64_t* user_elems, int64_t* bs_elems);

/*
 * Create a plan for `batch` instances on HIP device `device`.  Validates the
 * table first (same checks as ammse_validate), then copies it to the device
 * and sorts instances by decreasing work so that uneven batches balance.
 * *plan is set only on success.  Allocates device memory for the tables.
 */
ammse_status_t ammse_plan_create(ammse_plan_t* plan, int32_t device,
                                 const ammse_instance_t* table, const int32_t* cell_users,
                                 int32_t batch, const ammse_options_t* opt);

/* Bytes of device workspace ammse_solve / ammse_wsr need for this plan. */
ammse_status_t ammse_plan_workspace_size(ammse_plan_t plan, size_t* bytes);

/* Kernel a plan launches (AMMSE_KERNEL_*) and its LDS bytes per workgroup. */
#define AMMSE_KERNEL_LDS_MFMA 0  /* LDS-resident, MFMA FP32 channel products */
#define AMMSE_KERNEL_GENERAL 1   /* any shape; workspace-resident state */
ammse_status_t ammse_plan_info(ammse_plan_t plan, int32_t* kernel, size_t* lds_bytes);

/*
 * Tile-shape autotuner of the general kernel's MFMA channel products.  The
 * instances of the plan fall into three shape classes by the widest
 * precoder block of one cell, n = max_c U_c d (the column count of the
 * products G_c = H_{:,c} V_c and 2 H_{:,c}^H Z_c): n <= 16, 16 < n <= 32,
 * n > 32.  For every class present, a sample of at most 64 of its instances
 * is solved (a few iterations, on a scratch copy of V) with each output tile
 * shape (0: 64 x 64, 1: 128 x 16, 2: 64 x 32), timed with HIP events on
 * `stream`, and the fastest shape is kept in the plan for every instance of
 * the class; later ammse_solve / ammse_wsr calls with options.tile = 0 use
 * it (for the products with more than 64 output rows; smaller products take
 * shapes fitted to their row count, see ammse_options_t.tile).  Arguments as for ammse_solve (V is only read); choice: host int32[3]
 * (may be NULL) receives the shape picked per class, -1 for an absent class.
 * Plans without MFMA tile choices (the LDS-resident kernel, FP64) return
 * AMMSE_OK with every choice -1.  Blocks until the trials have run;
 * allocates and frees temporary device memory (AMMSE_ERR_ALLOC on failure).
 * The results of a solve do not depend on the tile shape up to the
 * summation order of the products.
 */
ammse_status_t ammse_autotune(ammse_plan_t plan, const void* H, const double* sigma2,
                              const double* alpha, const double* P, const void* V,
                              void* workspace, size_t workspace_bytes, int32_t* choice,
                              ammse_stream_t stream);

/* Release the plan's device tables.  NULL is accepted. */
ammse_status_t ammse_plan_destroy(ammse_plan_t plan);

/*
 * Run A-MMMSE (Algorithm 3) on every instance of the plan, one workgroup per
 * instance, all iterations in one kernel launch.
 *   H        device, complex, layout above (read only)
 *   sigma2   device double [users]   noise powers (> 0)
 *   alpha    device double [users]   priority weights (>= 0)
 *   P        device double [BSs]     power budgets (>= 0)
 *   V        device, complex: in = feasible V^0, out = final precoders
 *   wsr      device double [batch]   WSR of the returned V, bits/channel use
 *   iters    device int32 [batch]    iterations run (may be NULL)
 *   switch_iter device int32 [batch] first stage-II iteration, -1 if none (may be NULL)
 *   status   device int32 [batch]    AMMSE_INST_* bits (may be NULL)
 *   wsr_trace device double [batch][max_iters+1]: WSR(V^0..V^t), NaN after
 *            the last iteration run (may be NULL)
 *   force_switch device int32 [batch]: per-instance first stage-II iteration,
 *            <= 0 for the eps1 rule (may be NULL; overrides the option)
 *   workspace device, >= ammse_plan_workspace_size bytes, 256-byte aligned
 *   stream   HIP stream (NULL = default stream)
 * Iteration t evaluates receivers, MSE matrices and WSR at V^{t-1}; the
 * gradient at the extrapolated point; WSR(V^{t-1}) drives the stage test.
 */
ammse_status_t ammse_solve(ammse_plan_t plan, const void* H, const double* sigma2,
                           const double* alpha, const double* P, void* V, double* wsr,
                           int32_t* iters, int32_t* switch_iter, int32_t* status,
                           double* wsr_trace, const int32_t* force_switch, void* workspace,
                           size_t workspace_bytes, ammse_stream_t stream);

/*
 * Allocation-free ammse_solve, for callers that cannot allocate device memory
 * around the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Arguments and results as ammse_solve,
 * without the workspace: the kernels use the library's own static device
 * array of AMMSE_SCRATCH_BYTES, one per device, whose address is resolved when
 * the first plan on that device is created (ammse_plan_create).  The call
 * itself allocates and frees nothing.
 *   - Returns AMMSE_ERR_WORKSPACE, enqueuing nothing, when the plan needs more
 *     workspace than AMMSE_SCRATCH_BYTES (ammse_plan_workspace_size).
 *   - Every call on one device shares that device's array, which keeps the
 *     last call's contents; the kernels write every workspace value before
 *     they read it, so nothing needs clearing between calls.  Calls that
 *     overlap in time on one device (several streams, several host threads)
 *     race on the array and give undefined results: serialise them.
 */
#define AMMSE_SCRATCH_BYTES ((size_t)64 << 20)
ammse_status_t ammse_solve_noalloc(ammse_plan_t plan, const void* H, const double* sigma2,
                                   const double* alpha, const double* P, void* V, double* wsr,
                                   int32_t* iters, int32_t* switch_iter, int32_t* status,
                                   double* wsr_trace, const int32_t* force_switch,
                                   ammse_stream_t stream);

/*
 * Weighted sum rate (Section II rate definition, bits) of the precoders V for
 * every instance of the plan; same buffer conventions as ammse_solve.
 */
ammse_status_t ammse_wsr(ammse_plan_t plan, const void* H, const double* sigma2,
                         const double* alpha, const void* V, double* wsr, void* workspace,
                         size_t workspace_bytes, ammse_stream_t stream);

/*
 * Unrolled (differentiable) A-MMMSE.  T = opt.max_iters iterations of
 * Algorithm 3 in which the step size of iteration t is an input,
 * gamma[b * T + t - 1] (the learnable step sizes of an unrolled solver; the
 * adaptive rule of Section V-A and T_c, gamma_c are not used), with the stage
 * switch by the eps1 rule or forced, extrapolation and projection as in
 * ammse_solve; output WSR(V^T).  ammse_unrolled_backward returns the
 * derivatives of sum_b dwsr[b] * WSR_b(V^T) with respect to the step sizes
 * and the channels, the stage switch and the projection branch (active or
 * not) of the forward held fixed.  Supported: plans whose instances are all
 * single-cell (C = 1), algorithm AMMSE_ALGO_AMMMSE, precision FP64 or FP32
 * (else AMMSE_ERR_UNSUPPORTED).
 *
 * Checkpoints: the forward stores (V^t, V^{t-1}) for t = 0, K, 2K, ... (K =
 * ckpt_every >= 1) in `ckpt`; the backward recomputes each segment of K
 * iterations from its checkpoint with the same kernel code and propagates the
 * adjoints backwards through it, so its memory is O(K) iterations.
 */

/* Device bytes of the workspace (shared by forward and backward) and of the
 * checkpoint buffer for this plan and K. */
ammse_status_t ammse_unrolled_workspace_size(ammse_plan_t plan, int32_t ckpt_every,
                                             size_t* ws_bytes, size_t* ckpt_bytes);

/*
 *   H, sigma2, alpha, P, V, wsr, switch_iter, status, wsr_trace, force_switch:
 *            as for ammse_solve (V: in V^0, out V^T; switch_iter is required)
 *   gamma    device double [batch][T], step sizes in the caller's instance order
 *   ckpt     device, ckpt_bytes from ammse_unrolled_workspace_size
 *   workspace device, ws_bytes, 256-byte aligned
 */
ammse_status_t ammse_unrolled_forward(ammse_plan_t plan, const void* H, const double* sigma2,
                                      const double* alpha, const double* P, void* V,
                                      const double* gamma, int32_t ckpt_every, double* wsr,
                                      int32_t* switch_iter, int32_t* status, double* wsr_trace,
                                      const int32_t* force_switch, void* ckpt, void* workspace,
                                      size_t workspace_bytes, ammse_stream_t stream);

/*
 *   gamma, ckpt_every, ckpt: as passed to (and written by) the forward
 *   switch_iter device int32 [batch], the forward's output
 *   dwsr     device double [batch], upstream weight of WSR_b
 *   dH       device, layout of H (complex, storage precision), overwritten with
 *            dL/dRe(H) + i dL/dIm(H), L = sum_b dwsr[b] WSR_b, so that
 *            dL = Re sum(conj(dH) * delta H); channel blocks must not overlap
 *            (else AMMSE_ERR_SHAPE)
 *   dgamma   device double [batch][T], dL/dgamma
 */
ammse_status_t ammse_unrolled_backward(ammse_plan_t plan, const void* H, const double* sigma2,
                                       const double* alpha, const double* P, const double* gamma,
                                       int32_t ckpt_every, const int32_t* switch_iter,
                                       const void* ckpt, const double* dwsr, void* dH,
                                       double* dgamma, void* workspace, size_t workspace_bytes,
                                       ammse_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* AMMSE_H */
