/*
 * tctf2r.h - C ABI of the MI355X (gfx950) TCTF2R completion library.
 *
 * TCTF2R is the separable low-tubal-rank completion method of Ling, Yu, Qi and Xu,
 * "A Parallelizable Method for Missing Internet Traffic Tensor Data" (arXiv:2005.09838).
 * Problem statement (section 3.1, eq. (TETP-optim)):
 *
 *   min  f0 = 1/2 ||X*Y - W||^2 + mu/2 ||W||^2
 *             + rho1/2 ||H unfold(X*Y, 1)||^2 + rho2/2 ||K unfold(W, 2)||^2
 *   s.t. P_Omega(W) = P_Omega(G),
 *
 * with X (n1 x r x n3), Y (r x n2 x n3), W (n1 x n2 x n3) real, "*" the t-product along
 * mode 3, H and K the first-difference matrices of eq. (Toeplitz) along modes 1 and 2.
 * One iteration (section 4.1, algorithm box, steps 1-4 and 7) transforms along the tube,
 * updates every frequency's factors with pseudo-inverse-preconditioned block steps
 * (eq. (updataXYW1)), transforms Z~ = X~Y~ back, solves the per-row W-step (eq. (Wkiom))
 * and transforms W again.
 *
 * Conventions
 *  - Every array pointer is a DEVICE pointer on the device that is current when
 *    tctf_create is called (for instance a torch tensor's data_ptr()).
 *  - Tensors are C-contiguous [n1][n2][n3] (mode 3 fastest): G, the mask, W.
 *    X is [n1][r][n3] and Y is [r][n2][n3].
 *  - The caller owns every buffer, including the workspace; the library never
 *    allocates device memory and never frees caller memory.
 *  - The tube transform uses the paper's root omega = exp(+2 pi i / n3) (eq. (bar BA-k)).
 *  - A context belongs to one HIP stream and must be used from one host thread at a time.
 *    Calls that return results synchronise that stream; tctf_step only enqueues work.
 *  - Errors: every argument check runs before any device work; no call aborts or throws.
 *    On failure a status below is returned and tctf_last_error() holds a detail string.
 */
#ifndef TCTF2R_H
#define TCTF2R_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TCTF_OK = 0,
  TCTF_E_ARG = -1,        /* NULL pointer or parameter out of range                    */
  TCTF_E_SHAPE = -2,      /* sizes out of the supported range (see tctf_params)         */
  TCTF_E_NONFINITE = -3,  /* an observed value of G is NaN/Inf (tctf_create), or a quantity
                             computed from the iterate (f0, the step-6 differences, the
                             stationarity measures) is not finite                         */
  TCTF_E_HIP = -4,        /* a HIP runtime call failed (detail in tctf_last_error())    */
  TCTF_E_WORKSPACE = -5,  /* workspace NULL, too small or misaligned (256 B)            */
  TCTF_E_STATE = -6       /* checkpoint blob of the wrong size or for another problem   */
} tctf_status;

typedef enum {
  TCTF_FP32 = 0,        /* FP32 storage and products; the reduction over n1 of X~^* W~
                           accumulates in FP64; r x r Grams, pseudo-inverses, objective FP64 */
  TCTF_MIXED_BF16 = 1   /* W~ stored in BF16 (half the bytes of its write and reads), rounded
                           stochastically with counter-based rounding bits keyed by the entry
                           and the iteration (deterministic and resumable; unlike
                           round-to-nearest its error does not repeat from one iteration to
                           the next, so the iteration does not accumulate it); the slice
                           products Z~ = X~ Y~ and A = W~ Y~^* run on the BF16 matrix cores
                           with FP32 accumulation, the BF16 W~ as it is and each FP32 factor
                           split into two BF16 parts (hi + lo: three or two products, errors
                           near 2^-17); X~^* W~ accumulates in FP64 (G_X^+ multiplies it);
                           factors, G, Z~ and W stay FP32; r x r Grams, pseudo-inverses and
                           objective FP64                                                    */
} tctf_precision;

typedef struct {
  int32_t n1, n2, n3;   /* G is n1 x n2 x n3; n1, n2 >= 1; n3 in the supported set below    */
  int32_t r;            /* tubal rank of the factorisation, 1 <= r <= min(n1, n2, 32)
                           (section 3.1: X is n1 x r x n3, Y is r x n2 x n3)                */
  double mu;            /* ridge weight on W (eq. (ETP-optim)), >= 0                       */
  double rho1;          /* temporal-stability weight of H along mode 1 (eq. (TETP-optim)), >= 0 */
  double rho2;          /* periodicity weight of K along mode 2 (eq. (TETP-optim)), >= 0   */
  double eta;           /* common step alpha/L = beta/L of eq. (updataXYW1), 0 < eta < 2;
                           1 gives the exact block minimiser                               */
  int32_t precision;    /* tctf_precision                                                  */
  int32_t pinv_mode;    /* 0: inverse by elimination when the Gram provably keeps every
                           eigenvalue, eigen-decomposition otherwise; 1: always eigen     */
  double eps;           /* threshold of the termination test (step 6), default 1e-6        */
  double rank_tol;      /* step 5: keep in each stored frequency the components of
                           Z~_k = X~_k Y~_k whose singular values exceed rank_tol times the
                           largest over all frequencies; >= 0, default 0                  */
  int32_t rank_every;   /* step 5 runs after iterations rank_every, 2 rank_every, ...;
                           0 (default) = never, the rank vector stays r everywhere.  With
                           rank_every > 0 iterations are launched eagerly (no graph replay)
                           and batches refuse the context                                   */
  int32_t autotune;     /* 1: tctf_create times the execution shapes this problem allows (the
                           fusion depth of steps 3, 4 and 7: one fused kernel per OD row with
                           several or one thread per tube, or three launches; columns
                           per X~^* W~ block; columns per Y-step block) and keeps the fastest,
                           remembered per shape and device for the process (later contexts
                           of the shape reuse it); the workspace is sized for every shape.
                           Shapes change summation orders only.  0 (default): fixed rules.
                           tctf_complete_noalloc ignores it                                  */
  int32_t xsolve;       /* X-update, first line of eq. (updataXYW1).  0 (default): where
                           r <= 16 and H_rho1^{-1}'s entries c lambda^|i-j| fall below
                           2^-40 c within 12 rows (rho1 <= 0.15), the A = W~Y~^* launch
                           applies H_rho1^{-1} itself as that short stencil (with the mirror
                           terms of the two end rows); otherwise, and with 1, a separate
                           tridiagonal solve follows it.  The two agree to FP32 rounding   */
} tctf_params;
/* Sizes: n1 <= 8192, n2 <= 1024, n3 <= 8192.  For n3 in 1..16, 20, 24, 28, 32, 40, 48, 56,
 * 64, 84, 96, 112, 128 (the lengths the tube transform is generated for) with one slice
 * (n2 x (n3 + 1) floats) inside 150 KiB, steps 3, 4 and 7 run as one fused kernel per OD
 * row; any other size runs them as three launches through spatial Z and W buffers (direct
 * tube transforms; the workspace grows by 12 n1 n2 n3 bytes). */

typedef struct tctf_ctx tctf_ctx;

/* Fill *p with defaults: mu = rho1 = rho2 = 1e-2, eta = 1, FP32, pinv_mode 0, eps = 1e-6.
 * Sizes and r are set to 0 and must be filled in. */
void tctf_default_params(tctf_params* p);

/* Bytes of device workspace a context with these parameters needs (256-byte aligned). */
tctf_status tctf_workspace_bytes(const tctf_params* p, size_t* bytes);

/* Create a context (algorithm box, "Input" and "Initialize"; section 3.1 for P_Omega).
 *  G      [n1][n2][n3] float, observed values; entries off Omega are ignored.
 *  omega  [n1][n2][n3] uint8, nonzero = observed.
 *  X0     [n1][r][n3] float or NULL (NULL = zeros).
 *  Y0     [r][n2][n3] float or NULL (NULL = standard normal from a counter-based
 *         generator keyed by seed).
 *  W starts as P_Omega(G) (missing entries 0).  X0, Y0 are real, so the transformed
 *  factors satisfy the conjugate symmetry eq. (rcm_3-k+2).
 *  workspace: device memory of tctf_workspace_bytes() bytes, 256-byte aligned, owned by
 *  the caller and used exclusively by this context until tctf_destroy.
 *  hip_stream: the hipStream_t every call of this context runs on (NULL = default).
 *  G, omega, X0, Y0 are copied into the workspace; they may be freed once this returns.
 *  Returns TCTF_E_NONFINITE if an observed value of G is not finite. */
tctf_status tctf_create(const tctf_params* p, const float* G, const uint8_t* omega,
                        const float* X0, const float* Y0, uint64_t seed,
                        void* workspace, size_t ws_bytes, void* hip_stream, tctf_ctx** out);

/* Enqueue `iters` iterations (steps 1-4 and 7 of the algorithm box; step 5 keeps r,
 * step 6 is tctf_termination).  Asynchronous and stream-ordered.  Whole blocks of 10
 * iterations are replayed from a HIP graph that the first call with iters >= 1 captures on
 * a private stream of the context (the results are the same as eager launches); the rest
 * run as eager launches.  Nothing but the iteration runs unless step 6 is tracked. */
tctf_status tctf_step(tctf_ctx* c, int32_t iters);

/* Step 6 tracking (algorithm box, step 6).  With on != 0, every later tctf_step call keeps a
 * copy of X~, Y~ and W~ before its last iteration and evaluates the termination quantities
 * after it (one device copy of the iterate and one reduction per call), so that
 * tctf_termination can report them.  Off by default; tctf_run turns it on while it runs. */
tctf_status tctf_track_termination(tctf_ctx* c, int32_t on);

/* Synchronise and return f0 of eq. (TETP-optim) at the current iterate, accumulated in
 * FP64 (the fit, ridge and K terms from the spatial W-step rows, the H term from the
 * Fourier form eq. (fun-XYW)). */
tctf_status tctf_objective(tctf_ctx* c, double* f0);

/* Synchronise and return the step-6 quantities of the last iteration of the last tracked
 * tctf_step call (tctf_track_termination, tctf_run): out[0] = ||X~+ - X~||_inf (largest
 * entry modulus), out[1] = ||Y~+ - Y~||_inf, out[2] = ||W+ - W||_F, and out[3] = 1 if all
 * three are <= eps.  TCTF_E_STATE when no tracked iteration ran since create or restore;
 * TCTF_E_NONFINITE when the iterate is not finite. */
tctf_status tctf_termination(tctf_ctx* c, double out[4]);

/* Iterate until the step-6 test of the algorithm box holds or max_iters iterations have
 * run: blocks of check_every iterations (tctf_step with step 6 tracked), each followed by
 * tctf_termination on the block's last iteration.  *iters_run = iterations run by this call;
 * *converged = 1 if the test held (then it held on iteration *iters_run).  Synchronises
 * after every block; TCTF_E_NONFINITE if the iterate stops being finite. */
tctf_status tctf_run(tctf_ctx* c, int32_t max_iters, int32_t check_every, int32_t* iters_run,
                     int32_t* converged);

/* Synchronise and return stationarity measures at the current iterate (Theorem ThKKT,
 * eq. (AKKTstar)): out[0] = sqrt(sum_k ||grad_X h_k||^2 + ||grad_Y h_k||^2) /
 * (||W~|| (||X~|| + ||Y~||)) over the full spectrum; out[1] = max over unobserved entries
 * of |(W_k K_{mu rho2} - Z_k)_ij| / ||Z||_inf; out[2] = max over observed |W - G|. */
tctf_status tctf_stationarity(tctf_ctx* c, double out[3]);

/* Synchronise and copy results out (algorithm box, "Output").  Any pointer may be NULL.
 *  W [n1][n2][n3]: the completed tensor W of the last W-step (observed entries equal G).
 *  Z [n1][n2][n3]: X*Y of the current factors.
 *  X [n1][r][n3], Y [r][n2][n3]: the factors in the spatial domain (eq. (barAAk)). */
tctf_status tctf_get_result(tctf_ctx* c, float* W, float* Z, float* X, float* Y);

/* Bytes of a checkpoint blob, and save / restore of the iterate (X~, Y~, W~, iteration
 * count) to / from DEVICE memory.  Restoring continues bit-identically. */
tctf_status tctf_state_bytes(tctf_ctx* c, size_t* bytes);
tctf_status tctf_get_state(tctf_ctx* c, void* dst, size_t bytes);
tctf_status tctf_set_state(tctf_ctx* c, const void* src, size_t bytes);

/* Synchronise and copy the rank vector of step 5 (algorithm box: r^(l+1), one rank per
 * frequency) to the HOST array ranks[nb], nb = n3 / 2 + 1 stored frequencies (the others
 * mirror them).  r everywhere until step 5 has run.  Step 5 (tctf_params.rank_tol,
 * rank_every) rotates each frequency's factors into the singular basis of Z~_k, computed
 * from the r x r Grams in FP64, and zeroes the dropped components; f0's fit, ridge and K
 * terms after an adjusting iteration are those of its W-step (taken before the truncation). */
tctf_status tctf_rank_vector(tctf_ctx* c, int32_t* ranks);

/* The execution shape in use: out[0] = slice path (1 fused, several threads per tube;
 * 2 fused, one thread per tube; 3 three launches), out[1] = columns per X~^* W~ block,
 * out[2] = columns per Y-step block, out[3] = 1 if it came from the process's tuning cache,
 * out[4] = half-width of the H_rho1^{-1} stencil in the X-update, -1 for the separate solve. */
tctf_status tctf_tuning(tctf_ctx* c, int32_t out[5]);

/* Iterations run since create (or as restored). */
tctf_status tctf_iterations(tctf_ctx* c, int64_t* iters);

/* Destroy a context (the workspace stays the caller's).  NULL is a no-op. */
void tctf_destroy(tctf_ctx* c);

/* One call: create, run `iters` iterations, copy W out, f0 (may be NULL), destroy. */
tctf_status tctf_complete(const tctf_params* p, const float* G, const uint8_t* omega,
                          const float* X0, const float* Y0, uint64_t seed, int32_t iters,
                          void* workspace, size_t ws_bytes, void* hip_stream,
                          float* W_out, double* f0_out);

/* Allocation-free variant of tctf_complete, for callers that cannot allocate device memory
 * (serving loops or harnesses in which hipMalloc is not allowed).  Same arguments and
 * results as tctf_complete minus the workspace: a static scratch array of the library,
 * TCTF_NOALLOC_SCRATCH_BYTES per device (each device the library runs on holds it until the
 * process ends), serves as the workspace.  The call allocates nothing (no hipMalloc or
 * hipFree, no host allocation), creates no stream, event or graph (every launch is eager)
 * and synchronises hip_stream before it returns.  A problem whose workspace
 * (tctf_workspace_bytes) exceeds the scratch is rejected with TCTF_E_WORKSPACE before any
 * device work.  Every call on one device uses that device's one scratch, which keeps the
 * last call's contents (each call clears what must start at zero): calls that overlap on one
 * device, from other threads or on other streams, race and give undefined results. */
#define TCTF_NOALLOC_SCRATCH_BYTES (32u << 20)
tctf_status tctf_complete_noalloc(const tctf_params* p, const float* G, const uint8_t* omega,
                                  const float* X0, const float* Y0, uint64_t seed, int32_t iters,
                                  void* hip_stream, float* W_out, double* f0_out);

/* Time one stage of the iteration: launch it `reps` times back to back on the context's
 * stream between two HIP events and return the mean duration in microseconds.  Stages:
 *   0 slice kernel (inverse tube transform, W-step, forward transform; the W~ stream)
 *   1 Z~ = X~Y~ products
 *   2 A = W~Y~^* products and the X-update: the right-hand side, or with the H_rho1^{-1}
 *     stencil (tctf_params.xsolve) the new X~ itself, written to a scratch buffer
 *   3 tridiagonal H_rho1 solve (no launch where the stencil replaces it)
 *   4 X~^* W~ partials, with G_X, its pseudo-inverse and I - eta P_X
 *   5 Y-step and the column-block partials of G_Y
 *   6 G_Y from its partials, its pseudo-inverse and I - eta P_Y
 *   7 one whole iteration
 * Stages 0-6 recompute from the current state without advancing it (7 does advance). */
tctf_status tctf_time_stage(tctf_ctx* c, int32_t stage, int32_t reps, double* mean_us);

/* Live per-stage timing of tctf_step.  tctf_profile(c, mask) with mask != 0 clears the
 * record and, from then on, brackets every launch of each stage whose bit is set (bit k =
 * stage k of tctf_time_stage, k = 0..6) with a pair of HIP events on the context's stream;
 * mask = 0 stops recording and keeps the record.  While recording, every launch is eager
 * (no graph replay); the kernels themselves are unchanged.
 * tctf_profile_read synchronises the stream and returns, per stage, the summed duration in
 * microseconds of the recorded launches and their number. */
tctf_status tctf_profile(tctf_ctx* c, uint32_t mask);
tctf_status tctf_profile_read(tctf_ctx* c, double total_us[7], int64_t launches[7]);

/* ---- Differentiation (reverse mode) of the iteration (section 4.1: eq. (updataXYW1) with
 * the common step eta, eq. (subquKKT), eq. (bar BA-k) / eq. (barAAk)).  The Grams G_Y and
 * G_X must have full rank (then their pseudo-inverses are inverses, Lemma SVPMPI).  FP32
 * contexts only; the adjoint itself runs in FP64 on the context's stream.
 * Adjoint convention for a real loss L: the adjoint of a complex entry z is
 * dL/dRe z + i dL/dIm z; a stored frequency b = 0..nb-1 carries the adjoint it has in the
 * sum over all n3 frequencies (the conjugate frequencies hold the conjugates).  Adjoint
 * arrays are DEVICE arrays of doubles, complex ones interleaved (re, im):
 *   xt_bar [nb][r][n1] complex (the layout of X~), yt_bar [nb][r][n2] complex, w_bar
 *   [n1][n2][n3] real, theta_bar[3] = adjoints of (mu, rho1, rho2).
 * The adjoint workspace (tctf_adjoint_workspace_bytes, 256-byte aligned) is the caller's. */
tctf_status tctf_adjoint_workspace_bytes(const tctf_params* p, size_t* bytes);

/* Reverse pass of one iteration.  state_in, state_out: checkpoint blobs (tctf_get_state)
 * of this context's iterate before and after one iteration (TCTF_E_STATE otherwise).  On
 * entry xt_bar, yt_bar, w_bar hold the adjoints of X~, Y~ and W after the iteration; on
 * return those before it (of X~, Y~ and of the W whose transform the iteration read);
 * the weights' adjoints are ADDED to theta_bar.  Synchronises; TCTF_E_STATE if a Gram is
 * rank deficient. */
tctf_status tctf_adjoint_step(tctf_ctx* c, const void* state_in, const void* state_out, double* xt_bar,
                              double* yt_bar, double* w_bar, double* theta_bar, void* workspace,
                              size_t ws_bytes);

/* Adjoint of the set-up transforms X~0 = dft(X0), Y~0 = dft(Y0) (eq. (bar BA-k)): the
 * gradients of L with respect to the real initial factors, x0_bar [n1][r][n3] and y0_bar
 * [r][n2][n3] (either may be NULL). */
tctf_status tctf_adjoint_initial(tctf_ctx* c, const double* xt_bar, const double* yt_bar, double* x0_bar,
                                 double* y0_bar);

/* Gradients of f0 (eq. (TETP-optim)) with respect to the real spatial factors at the
 * current iterate: through eq. (fun-XYW) and eq. (bar BA-k), d f0 / d X = Re idft(grad_X h)
 * with grad_X h_k of eq. (hkXYDer), likewise for Y.  x_grad [n1][r][n3], y_grad [r][n2][n3]
 * doubles.  Uses the adjoint workspace; synchronises. */
tctf_status tctf_objective_gradient(tctf_ctx* c, double* x_grad, double* y_grad, void* workspace,
                                    size_t ws_bytes);

/* ---- Batches of independent completions (one level above the per-frequency and per-row
 * separability of one completion, section 3.2).  A batch owns n contexts of possibly
 * different sizes, ranks and parameters, carved from one caller-owned workspace in member
 * order (each member's part 256-byte aligned).  Pointer arguments are HOST arrays of n
 * DEVICE pointers (X0, Y0 and seeds may be NULL, or hold NULL entries, as in tctf_create).
 * tctf_batch_step enqueues `iters` iterations of every member, all inside graph launches:
 * blocks of 10 iterations of all members run as ONE graph launch in which each member's
 * chain is an independent branch (members are spread over 16 branches), and the remaining
 * iterations as launches of a one-iteration graph of the same form.  Results are the same
 * as running every member alone.  Step 6 is not evaluated inside a batch step.
 * tctf_batch_member gives member k's context for the per-completion calls (objective,
 * termination, results, checkpoints); it stays owned by the batch. */
typedef struct tctf_batch tctf_batch;
tctf_status tctf_batch_workspace_bytes(int32_t n, const tctf_params* p, size_t* bytes);
tctf_status tctf_batch_create(int32_t n, const tctf_params* p, const float* const* G,
                              const uint8_t* const* omega, const float* const* X0,
                              const float* const* Y0, const uint64_t* seeds, void* workspace,
                              size_t ws_bytes, void* hip_stream, tctf_batch** out);
tctf_status tctf_batch_step(tctf_batch* b, int32_t iters);
tctf_status tctf_batch_size(tctf_batch* b, int32_t* n);
tctf_status tctf_batch_member(tctf_batch* b, int32_t k, tctf_ctx** member);
void tctf_batch_destroy(tctf_batch* b);   /* destroys the members too; NULL is a no-op */

const char* tctf_status_string(tctf_status s);
const char* tctf_last_error(void);  /* thread-local detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* TCTF2R_H */
