/*
 * prgd.h -- C ABI of the MI355X (gfx950) library for low-TT-rank tensor
 * completion by preconditioned Riemannian gradient descent (PRGD).
 *
 * Method: Bian, Cai, Zhang & Zhang, "Fast and Provable Tensor-Train Format
 * Tensor Completion via Preconditioned Riemannian Gradient Descent".
 *
 *   Problem (section 1, completion model): find T of TT rank r minimising
 *     f(T) = 1/2 <T - T*, P_Omega(T - T*)>, given the entries y_j of T* (plus
 *     noise) at the observed multi-indices x^(j) in Omega.
 *   TT format (section 2.1): T(x) = T_1(x_1,:) T_2(:,x_2,:) ... T_m(:,x_m),
 *     core T_k of shape r_{k-1} x n_k x r_k with r_0 = r_m = 1.
 *   Iteration (Algorithm 2, trimming skipped as section 3.2.2 allows):
 *     G_l = P_Omega(T_l - T*); metric weights G_{l,i} = eps I +
 *     diag(M_i(G_l) M_i(G_l)^T) (section 3.2.1); direction
 *     xi = P~_T W^{-1} G_l (Lemma 3); W_l = T_l - alpha_l xi;
 *     T_{l+1} = TT-SVD_r(W_l) (Algorithm 1).
 *
 * Conventions shared by every call
 *   - All integers are int32 unless stated; sizes that can exceed 2^31 are int64.
 *   - Cores are passed "packed": core k = 1..m as a row-major array of shape
 *     (r_{k-1}, n_k, r_k) (index (a, x, b) -> a*n_k*r_k + x*r_k + b), the m cores
 *     concatenated in order; prgd_cores_numel() gives the total length.
 *   - Multi-indices are 0-based, structure of arrays: indices[k*N + j] is the
 *     mode-(k+1) index of sample j, 0 <= indices[k*N+j] < n_k.
 *   - Host pointers are read only during the call that receives them; the
 *     library copies what it keeps.  Device pointers (mem_device = 1) must be
 *     device memory of the current HIP device, readable for the duration of
 *     the call; they are validated on the device (no copy to the host).
 *   - Return codes: prgd_status values below.  No exception crosses the ABI.
 *     A negative code leaves output buffers unspecified; prgd_last_error()
 *     returns a thread-local message for the last failing call.
 *   - A solver handle must not be used from two threads at once.
 *   - Limits of this build: order m in [2, 32]; TT ranks <= 16; mode sizes
 *     in [1, 2^31); N in [1, 2^31).
 */
#ifndef PRGD_H
#define PRGD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t prgd_status;

#define PRGD_OK              0   /* success; for prgd_run: stopping rule met          */
#define PRGD_NOT_CONVERGED   1   /* max_iter reached; cores are the last iterate      */
#define PRGD_PENDING         2   /* server: request not finished yet                  */
#define PRGD_EINVAL         -1   /* invalid shape, rank, index, value, tolerance       */
#define PRGD_EDUPLICATE     -2   /* a multi-index occurs twice in Omega               */
#define PRGD_ENOMEM         -3   /* host or device allocation failed / over budget    */
#define PRGD_EDEVICE        -4   /* HIP runtime error                                  */
#define PRGD_EBREAKDOWN     -5   /* non-positive-definite Gram, non-finite residual,   */
                                 /* or rank-deficient truncation                       */
#define PRGD_ESTATE         -6   /* null or destroyed handle, wrong call order         */
#define PRGD_ENOTSUP        -7   /* outside the limits of this build                   */

/* precision */
#define PRGD_PREC_FP64   0   /* every step in float64                                        */
#define PRGD_PREC_MIXED  1   /* sampled pass (evaluation, residual, weights, gradient
                                scatter) in float32 arithmetic.  Its sums accumulate in
                                float32, except in the order-3 grouped kernel, whose
                                boundary-core gradients and slice sums accumulate in
                                float64 (LDS), and ||R||^2, always summed in float64.
                                Grams, factorisations, retraction, stopping test in
                                float64                                                     */
#define PRGD_PREC_MIXED_BF16 2 /* as PRGD_PREC_MIXED, and the tangent components
                                (the three R x R slice products of Lemma 3's projection,
                                X = omega^{-1} GL^{-1} Y H^{-1} - T Psi) on bfloat16
                                matrix-core operations with float32 accumulation; every
                                operand scaled by a power of two (per core for GL^{-1},
                                H^{-1}, Psi; per slice for Y, T and GL^{-1} Y) so that it
                                sits near unit size                                         */
/* step policy (section 3.2.2 and Theorem 1) */
#define PRGD_STEP_THEORY 0   /* alpha_l = step * eps_l^{1/2} / p, p = N / (n_1...n_m);
                                Theorem 1 uses step = 1.001                                 */
#define PRGD_STEP_CONST  1   /* alpha_l = step for every l; with the data-driven metric it
                                requires eps_fixed > 0                                      */
#define PRGD_STEP_ADAPTIVE 2 /* steepest step along the direction in the tangent space
                                (equation of the PRGD step size, section 3.2.2; for the
                                Euclidean metric the RGD step of section 3.1):
                                alpha_l = ||xi||_W^2 / ||P_Omega xi||_F^2, evaluated as
                                <G_l, xi> / ||P_Omega xi||^2 by a second pass over Omega  */
/* metric of the tangent space */
#define PRGD_METRIC_DATA      0 /* data-driven metric G_{l,i} = eps I + diag(M_i M_i^T)
                                   (section 3.2.1): PRGD                                    */
#define PRGD_METRIC_EUCLIDEAN 1 /* Euclidean metric: Riemannian gradient descent (RGD,
                                   section 3.1); THEORY then means alpha_l = step / p       */
/* stopping rule, tested with tolerance tol */
#define PRGD_STOP_RESIDUAL 0 /* ||P_Omega(T_l) - y||_2 / ||y||_2 <= tol, tested on T_l      */
#define PRGD_STOP_CHANGE   1 /* ||T_{l+1} - T_l||_F <= tol * max(1, ||T_l||_F)
                                (section 5.1, noise experiment)                             */
#define PRGD_STOP_ERROR    2 /* ||T_{l+1} - T*||_F / ||T*||_F <= tol; needs truth_cores     */
#define PRGD_STOP_NONE     3 /* run exactly max_iter iterations                             */

typedef struct prgd_solver_s *prgd_solver;

typedef struct {
  int32_t order;               /* m >= 2                                                   */
  const int32_t *mode_sizes;   /* host [m], n_k >= 1                                       */
  const int32_t *tt_ranks;     /* host [m+1], r_0 = r_m = 1, 1 <= r_k <=
                                  min(n_1...n_k, n_{k+1}...n_m), r_k <= 16                 */
  int64_t n_obs;               /* N = |Omega| >= 1; multi-indices must be distinct         */
  const int32_t *indices;      /* [m*N] SoA multi-indices (host or device, see mem_device) */
  const void *values;          /* [N] observed values y_j, float64 or float32              */
  int32_t values_fp64;         /* 1: values are double; 0: float                           */
  int32_t mem_device;          /* 1: indices and values are device pointers                */
  const double *init_cores;    /* host, packed T_0 (required; any TT of ranks tt_ranks)    */
  const double *truth_cores;   /* host, packed T* or NULL; enables STOP_ERROR and the
                                  relative error in reports                                */
  int32_t precision;           /* PRGD_PREC_*                                              */
  int32_t step_policy;         /* PRGD_STEP_*                                              */
  double step;                 /* step constant c (THEORY) or step alpha (CONST), > 0      */
  double eps_fixed;            /* > 0: fixed eps in G_{l,i}; <= 0: eps_l = ||G_l||_vee^2,
                                  the largest squared mode-slice norm of G_l (Appendix B)  */
  int32_t stop_rule;           /* PRGD_STOP_*                                              */
  double tol;                  /* >= 0                                                     */
  int32_t max_iter;            /* >= 0                                                     */
  int32_t sort_mode;           /* mode (0-based) by which Omega is grouped on the device;
                                  -1 chooses the mode with the largest r_{k-1} r_k         */
  void *stream;                /* hipStream_t to run on; NULL: a stream owned by the solver */
  int32_t metric;              /* PRGD_METRIC_* (0 = PRGD)                                  */
  int32_t mode_interfaces;     /* orders whose sampled pass runs mode by mode: 1 = one
                                  pass forms every sample's left and right interfaces and
                                  residual and the mode passes read them, -1 = every mode
                                  pass re-evaluates them, 0 = choose (1 for orders >= 6
                                  and ranks <= 8 with |Omega| >= 65536 when the stored
                                  interfaces take at most 8 GiB).  Results agree to
                                  rounding either way.                                      */
  int32_t pass_kind;           /* sampled pass for orders >= 4 (section 2.1 evaluation,
                                  section 3.2.1 slice norms, the gradient of f):
                                  PRGD_PASS_AUTO = the one-pass chain kernel when every
                                  core from some split on has n_k <= (16/R)^2 (R the
                                  rank padded to 2, 4 or 8; n_k <= 16 at R = 2) and the
                                  modes before the split leave >= 1024 samples per
                                  prefix, else the choice above; PRGD_PASS_CHAIN
                                  requires the chain kernel (PRGD_ENOTSUP if it does not
                                  apply); PRGD_PASS_MODES never uses it                     */
} prgd_desc;

/* pass_kind */
#define PRGD_PASS_AUTO  0
#define PRGD_PASS_CHAIN 1
#define PRGD_PASS_MODES 2

/* One row of the per-iteration record kept on the device. */
typedef struct {
  int32_t iter;                /* l: the record describes the step T_l -> T_{l+1}          */
  int32_t flags;               /* bit0: rel_change valid, bit1: rel_error valid            */
  double rel_residual;         /* ||P_Omega T_l - y|| / ||y||                               */
  double rel_change;           /* ||T_{l+1} - T_l|| / max(1, ||T_l||)                       */
  double rel_error;            /* ||T_{l+1} - T*|| / ||T*||                                 */
  double eps;                  /* eps_l used in the metric                                  */
  double alpha;                /* alpha_l                                                   */
} prgd_iter_info;

typedef struct {
  int32_t iterations;          /* completed iterations l                                    */
  int32_t status;              /* PRGD_OK / PRGD_NOT_CONVERGED / negative error             */
  double rel_residual;         /* of the returned iterate's last evaluated residual         */
  double rel_change;           /* last computed relative change (NaN if never)             */
  double rel_error;            /* relative error of the returned iterate (NaN if no truth) */
  double seconds;              /* device-synchronised wall time of the iteration loop      */
} prgd_report;

/* Total length of the packed cores for shape n[m] and ranks r[m+1] (-1 if invalid). */
int64_t prgd_cores_numel(int32_t m, const int32_t *n, const int32_t *r);

/* Set up one completion problem (section 1: observed entries y_j of T* at the
   multi-indices of Omega; TT cores of the ranks tt_ranks, section 2.1) for
   Algorithm 2 started at T_0 = init_cores, which Algorithm 2 requires to lie on
   the rank-r manifold.  Validate the problem on the host, copy it to the
   device, group Omega by sort_mode, left-orthogonalise T_0 (Algorithm 1 applied
   to T_0 at its own ranks) and prepare the iteration.  Validation
   (shapes, ranks, index ranges, duplicate multi-indices, finite values) runs
   before any GPU work.  On success *out owns all device memory of the solve. */
prgd_status prgd_create(const prgd_desc *desc, prgd_solver *out);

/* Enqueue exactly `iters` iterations of Algorithm 2 (one iteration: residual
   G_l on Omega, metric weights of section 3.2.1, direction P~_T W^{-1} G_l by
   Lemma 3, step of section 3.2.2, W_l = T_l - alpha_l xi, T_{l+1} =
   TT-SVD_r(W_l) by Algorithm 1) without synchronising; fewer if the stopping
   rule fires or max_iter is reached (later iterations become no-ops on the
   device).  Returns PRGD_OK once enqueued, PRGD_ESTATE for a null handle,
   PRGD_EINVAL for iters < 0, PRGD_EDEVICE on a launch failure.  A breakdown
   found on the device is reported by prgd_get_report / prgd_run. */
prgd_status prgd_iterate(prgd_solver s, int32_t iters);

/* Number of phases reported by prgd_iterate_profiled. */
#define PRGD_NPHASES 6

/* Like prgd_iterate, with HIP events recorded on the solver's stream around
   each phase of every iteration; waits for completion and writes the summed
   elapsed milliseconds per phase into phase_ms[PRGD_NPHASES]:
     0 sampled pass, main kernel (evaluation, residual, slice sums, gradient
       scatter)
     1 sampled pass, reduction of the partials and the weights/step finish
     2 metric-weighted Gram sweeps and tangent components (projection)
     3 retraction sweeps (right Grams of W_l, truncated left sweep); for
       padded ranks <= 8 with at most 16 slices per core one launch also
       forms the new cores and runs the stopping test, so phase 4 is then
       part of phase 3
     4 new cores and stopping-test reductions
     5 relative error against the truth (0 without truth_cores)            */
prgd_status prgd_iterate_profiled(prgd_solver s, int32_t iters, double *phase_ms);

/* Runs `iters` iterations exactly as prgd_iterate does, timed on the device
   with HIP events: the sampled pass's main kernel of every iteration `it` with
   it % stride == 0 is bracketed by two events (the interval of phase 0 of
   prgd_iterate_profiled), and *main_ms receives the mean of those intervals
   in milliseconds per bracketed launch; *total_ms receives the device
   milliseconds from the start of the first iteration to the end of the last.
   Each recorded event idles the device for a few microseconds between
   kernels, so a stride above 1 keeps that cost out of most iterations.
   Waits for the solver's stream.  Both outputs are host pointers and
   required.  Errors: PRGD_EINVAL (iters < 0, stride < 1 or a null output),
   PRGD_EDEVICE. */
prgd_status prgd_iterate_timed(prgd_solver s, int32_t iters, int32_t stride, double *main_ms, double *total_ms);

/* Wait for the solver's stream. */
prgd_status prgd_sync(prgd_solver s);

/* Iterate Algorithm 2 until the stopping rule (stop_rule, tol: the rules of
   section 5.1) holds or max_iter iterations, then fill *report (may be NULL).
   Returns PRGD_OK, PRGD_NOT_CONVERGED (cores hold the last iterate) or an
   error: PRGD_EBREAKDOWN (non-positive-definite Gram, non-finite residual,
   or a truncation whose kept singular values span more than 1e6, the
   resolution of the Gram-form retraction), PRGD_EDEVICE, PRGD_ESTATE. */
prgd_status prgd_run(prgd_solver s, prgd_report *report);

/* Current state without iterating (synchronises). */
prgd_status prgd_get_report(prgd_solver s, prgd_report *report);

/* Copy the current iterate T_l (the output of Algorithm 2 once the run has
   stopped), packed, into host memory out[cap]; cap >= prgd_cores_numel or
   PRGD_EINVAL.  Cores 1..m-1 are left-orthogonal (Algorithm 1's output form)
   after any completed iteration. */
prgd_status prgd_get_cores(prgd_solver s, double *out, int64_t cap);

/* Copy up to cap per-iteration records into out; *count receives the number
   of records written (one per completed or stopped iteration). */
prgd_status prgd_get_history(prgd_solver s, prgd_iter_info *out, int32_t cap, int32_t *count);

/* Hot path in isolation (rows a1-a3 of the iteration): evaluate the current
   iterate on Omega, form the residual R_j = T_l(x^(j)) - y_j, and return
   (host arrays, any may be NULL)
     grad[numel]   packed like the cores: df/dT_k(:,x,:) = sum_{j: x_k=x} R_j
                   T^{<=k-1}(x^(j))^T T^{>=k+1}(x^(j))^T  (chain rule on the TT format)
     slice_sq[sum n_k]  s_k(x) = sum_{j: x_k = x} R_j^2, mode after mode
                   (squared row norms of the mode unfoldings of G_l, section 3.2.1)
     res_sq        sum_j R_j^2.
   Arithmetic follows the solver's precision.  Does not advance the iteration. */
prgd_status prgd_sampled_pass(prgd_solver s, double *grad, double *slice_sq, double *res_sq);

/* Evaluate a TT (section 2.1, TT format) at N multi-indices on the GPU:
   out[j] = T(x^(j)).  cores: host packed float64; indices: SoA [m*N]
   (device if mem_device, else host); out: float64 [N] in the same memory
   kind as indices.  stream: hipStream_t or NULL (default stream); the call
   returns after the result is written. */
prgd_status prgd_eval(int32_t m, const int32_t *n, const int32_t *r, const double *cores,
                      int64_t n_obs, const int32_t *indices, double *out, int32_t mem_device,
                      void *stream);

/* Sketched spectral initialisation T_0 ~ SVD^tt_r(P_Omega(y) / p), p =
   |Omega| / prod n_k: the starting point the convergence analysis assumes
   (Theorem 1; the spectral choice is Algorithm 1 applied to the rescaled
   sampled tensor).  Algorithm 1's projected unfolding A_i at split i
   (i = 1..m-1) is replaced by the sketch Y_i = A_i Psi_i, where the row of
   Psi_i for the later indices (x_{i+1}, ..., x_m) is the elementwise product
   of the rows Gamma_{i,k}[x_k, :] of the caller's standard-normal test
   matrices; core i is the top r_i left singular vectors of Y_i (so cores
   1..m-1 are left-orthonormal) and core m is A_m.  For an exact TT-rank-r
   tensor observed in full the result reproduces the tensor.
     m, n[m], r[m+1]  order, mode sizes, TT ranks (r_0 = r_m = 1, r_k <= 16)
     indices   host int32 SoA [m * n_obs], values host float64 [n_obs]
     sketch    columns of every test matrix, max(r) <= sketch <= 32
     gauss     host float64: for i = 1..m-1 and k = i+1..m, Gamma_{i,k}
               (n_k x sketch, row-major) in that order
     cores_out host float64, packed like prgd_eval's cores (prgd_cores_numel)
     stream    hipStream_t or NULL; returns after cores_out is written.
   Multi-indices are not required to be distinct (repeats add up).  Device
   memory is allocated for the call and freed before it returns.
   Errors: PRGD_EINVAL (arguments, index range, non-finite values),
   PRGD_ENOTSUP (ranks above 16), PRGD_EBREAKDOWN (a sketch whose r_i-th
   singular value is not above 1e-7 of its largest: too few samples for the
   ranks), PRGD_EDEVICE. */
prgd_status prgd_spectral_init(int32_t m, const int32_t *n, const int32_t *r, int64_t n_obs,
                               const int32_t *indices, const double *values, int32_t sketch,
                               const double *gauss, double *cores_out, void *stream);

/* prgd_eval for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc): the
   same values as prgd_eval with mem_device = 1, computed by the same kernel,
   but every argument is device memory and nothing is allocated.
     cores_dev    device float64, packed like prgd_eval's cores
     indices_dev  device int32 SoA [m * n_obs]; indices must be in range (not
                  checked: checking would need a copy to the host)
     out_dev      device float64 [n_obs]
     stream       hipStream_t or NULL; the work is queued on it and the call
                  returns at once (no synchronisation): out_dev is valid once
                  the stream has reached this point.
   The padded cores are staged in a fixed 4 MiB workspace that each GPU holds
   for the life of the process: sum_k n_k R^2 + 64 <= 2^19 doubles, R the
   largest TT rank padded up to 2, 4, 6, 8, 10, 12 or 16, else PRGD_ENOMEM.
   Calls that overlap on one GPU (two streams, two threads) share that
   workspace and race; serialise them.  Errors: PRGD_EINVAL, PRGD_ENOTSUP
   (ranks above 16), PRGD_ENOMEM (workspace too small), PRGD_EDEVICE. */
prgd_status prgd_eval_noalloc(int32_t m, const int32_t *n, const int32_t *r, const double *cores_dev,
                              int64_t n_obs, const int32_t *indices_dev, double *out_dev, void *stream);

prgd_status prgd_destroy(prgd_solver s);

/* ------------------------------------------------------------------------
 * Request server: many independent completion problems on one device.
 *
 * Serves callers that solve streams of independent problems (different
 * orders, mode sizes, ranks and |Omega|).  Each request is one PRGD solve with
 * exactly the semantics of prgd_create + prgd_run on the same descriptor.  A
 * scheduler thread owned by the server admits queued requests in arrival
 * order while their device footprint fits the memory budget and a slot is
 * free, keeps every admitted solve's cores, observations and preconditioner
 * state resident, and advances all live solves that share order, padded rank,
 * precision and sampled-pass variant with the same kernel launches (one
 * launch serves every member, blockIdx.y selecting the solve).  Finished
 * solves leave the batch between rounds and queued requests join as memory
 * frees up (continuous batching).  Results do not depend on which other
 * requests were live: every kernel computes each solve from its own data only.
 * ------------------------------------------------------------------------ */
typedef struct prgd_server_s *prgd_server;

typedef struct {
  int64_t hbm_budget_bytes;    /* device bytes the live solves may hold together;
                                  <= 0: three quarters of the free device memory        */
  int32_t max_slots;           /* live solves at once, 1..4096                            */
  int32_t iters_per_tick;      /* iterations launched for the live solves per scheduling
                                  round; <= 0: 4.  Does not change any result.            */
} prgd_server_desc;

typedef struct {
  prgd_report report;          /* as prgd_run's; seconds = admission to completion       */
  double submit_s;             /* server clock (seconds since prgd_server_create)        */
  double admit_s;              /* solve created on the device                             */
  double finish_s;             /* completion observed by the scheduler                    */
  int64_t footprint_bytes;     /* admission estimate of the device bytes it held          */
} prgd_ticket_info;

/* Start a server on the current HIP device.  *out owns a scheduler thread and
   every device buffer of the solves it admits. */
prgd_status prgd_server_create(const prgd_server_desc *desc, prgd_server *out);

/* Queue one problem.  desc is read during the call only: host or device
   inputs are copied into server-owned host memory; desc->stream is ignored.
   Shapes, ranks, sizes and options are checked here (PRGD_EINVAL,
   PRGD_ENOTSUP); a request whose footprint exceeds the whole budget returns
   PRGD_ENOMEM.  Index ranges, duplicates and values are checked at admission
   and reported by poll.  *ticket identifies the request (thread-safe). */
prgd_status prgd_server_submit(prgd_server sv, const prgd_desc *desc, uint64_t *ticket);

/* Non-blocking.  PRGD_PENDING while the request is queued or running.  Once it
   has finished: fills *info (may be NULL), copies the packed final cores into
   cores[cap] (may be NULL; cap >= prgd_cores_numel or PRGD_EINVAL and the
   result is kept), releases the ticket and returns the solve's status
   (PRGD_OK, PRGD_NOT_CONVERGED or a negative error).  Unknown or released
   ticket: PRGD_ESTATE.  Thread-safe. */
prgd_status prgd_server_poll(prgd_server sv, uint64_t ticket, prgd_ticket_info *info, double *cores,
                             int64_t cap);

/* Block until the request has finished (PRGD_OK) or timeout_s seconds have
   passed (PRGD_PENDING); timeout_s < 0 waits without limit.  Does not release
   the ticket.  Thread-safe. */
prgd_status prgd_server_wait(prgd_server sv, uint64_t ticket, double timeout_s);

/* Counters: requests queued, live on the device, finished and not yet polled,
   and the device bytes the live solves hold by their admission estimates. */
prgd_status prgd_server_stats(prgd_server sv, int32_t *queued, int32_t *live, int32_t *finished,
                              int64_t *bytes_in_use);

/* Stop the scheduler, wait for the device, free everything.  Requests still
   queued or running are abandoned. */
prgd_status prgd_server_destroy(prgd_server sv);

const char *prgd_status_str(prgd_status st);
const char *prgd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PRGD_H */
