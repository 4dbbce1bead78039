/*
 * skipm — sketch-preconditioned infeasible interior-point LP solver for AMD
 * Instinct MI355X (gfx950).
 *
 * Solves  min c^T x  s.t.  A x = b, x >= 0   (primal, eq. "primal" of Sec. 1)
 * and     max b^T y  s.t.  A^T y + s = c, s >= 0   (dual, eq. "dual")
 * for short-and-fat A (m << n) with the infeasible long-step path-following
 * IPM of Alg. 2 (Sec. 4).  Every iteration solves the normal equations
 * A D^2 A^T dy = p (eq. "normal", p of eq. "pdef", D^2 = X S^{-1}) by conjugate
 * gradients preconditioned with Q = (A D W)(A D W)^T (eq. "pdprecond"), where W
 * is a sparse embedding (Sec. 2), then applies the correction vector v of eq.
 * "compv" so that the residuals stay on the segment between r^0 and 0
 * (eq. "addl", Lemma 3), and takes the step of Alg. 2 steps (e)-(g).
 *
 * Conventions for every entry point:
 *  - Return value: SKIPM_OK (0) or a negative SKIPM_E* code; nothing throws.
 *    skipm_last_error() returns a message for the last failing call on the
 *    calling thread.
 *  - Array arguments are DEVICE pointers (HIP device memory of the current
 *    device) unless the comment says "host".  The library never frees caller
 *    memory.
 *  - Work is ordered on the given stream (NULL = the default stream).  Calls
 *    that return host info (ipm_step, lp_solve, pcg_solve) synchronise that
 *    stream before returning.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - All floating-point state of the IPM (x, y, s, residuals, p, v, the step)
 *    is FP64.  SKIPM_PREC_MIXED / SKIPM_PREC_BF16 only let the CG
 *    matrix-vector products read an FP32 / BF16 copy of A (FP64 accumulation);
 *    the normal-equation residual that decides convergence is recomputed from
 *    the FP64 A.
 */
#ifndef SKIPM_H
#define SKIPM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SKIPM_OK        0
#define SKIPM_EINVAL   (-1)  /* bad argument (sizes, null pointers, parameter ranges) */
#define SKIPM_ENOMEM   (-2)  /* device allocation failed */
#define SKIPM_EDEVICE  (-3)  /* a HIP runtime call failed */
#define SKIPM_ERANK    (-4)  /* the Gram matrix of the sketch A D W kept a non-positive Cholesky
                                pivot (Lemma 3's failure event, rank(A D W) < m) through 3 fresh
                                sketches (new salts) and then 3 growing diagonal shifts */
#define SKIPM_ENOTCONV (-5)  /* max_outer iterations reached without meeting the stopping test */
#define SKIPM_ESTALL   (-6)  /* step length below 1e-12 three times in a row */
#define SKIPM_ENAN     (-7)  /* non-finite iterate */

/* storage of A */
#define SKIPM_DENSE 0        /* column-major, leading dimension lda >= m */
#define SKIPM_CSR   1        /* compressed sparse rows, int32 row pointers / column indices */

/* element type of A's values as handed in */
#define SKIPM_F64 0
#define SKIPM_F32 1

/* arithmetic of the CG solve */
#define SKIPM_INNER_CG         0  /* preconditioned CG (Alg. 1 step 3) */
#define SKIPM_INNER_SD         1  /* preconditioned steepest descent (App. B, Alg. 4) */
#define SKIPM_INNER_RICHARDSON 2  /* preconditioned Richardson iteration (App. A, Alg. 3) */
#define SKIPM_SKETCH_COUNT     0  /* block CountSketch (sparse embedding of Sec. 2) */
#define SKIPM_SKETCH_GAUSSIAN  1  /* dense N(0,1) sketch W_G (Sec. 5) */
#define SKIPM_PREC_FP64  0   /* everything FP64 */
#define SKIPM_PREC_MIXED 1   /* CG products read an FP32 copy of A (FP64 accumulation) inside
                                an iterative refinement on FP64 residuals; residuals, v,
                                step length and preconditioner FP64.  Escalates to FP64
                                products (tier SKIPM_TIER_FP64) when the refinement needs
                                too many steps. */
#define SKIPM_PREC_BF16  2   /* as SKIPM_PREC_MIXED, starting one tier lower: CG products read
                                a BF16 copy of A, then escalate BF16 -> FP32 -> FP64 */

/* precision tier of the CG products of one IPM iteration */
#define SKIPM_TIER_FP64 0
#define SKIPM_TIER_FP32 1
#define SKIPM_TIER_BF16 2

typedef struct skipm_lp_s* skipm_lp_t;

/* The LP (eq. "primal"/"dual").  All pointers are device pointers; lp_create
 * copies everything into library-owned buffers, so the caller may free them
 * after lp_create returns. */
typedef struct {
  int64_t m;               /* rows (constraints), 1 <= m <= min(n, 2048) */
  int64_t n;               /* columns (variables) */
  int64_t nnz;             /* CSR only: number of stored entries */
  int32_t format;          /* SKIPM_DENSE or SKIPM_CSR */
  int32_t a_dtype;         /* SKIPM_F64 or SKIPM_F32 */
  const void* a_vals;      /* dense: lda*n values, column j at a_vals + j*lda;
                              CSR: nnz values in row order */
  int64_t lda;             /* dense only (0 means m) */
  const int32_t* a_rowptr; /* CSR: m+1 offsets, a_rowptr[0] = 0, non-decreasing */
  const int32_t* a_colidx; /* CSR: nnz column indices in [0, n), strictly increasing per row */
  const double* b;         /* m */
  const double* c;         /* n */
} skipm_problem;

/* Parameters of Alg. 1 / Alg. 2.  skipm_params_default() fills the defaults
 * given in brackets. */
typedef struct {
  double sigma;      /* centring parameter, in (0, 0.8)  [0.5] (Alg. 2 input)        */
  double gamma;      /* neighbourhood N(gamma), in (0, 1)  [0.999]                    */
  double tol_cg;     /* relative CG tolerance ||f^(j)|| <= tol ||f^(0)||  [1e-5]      */
  double eps_gap;    /* stop: relative duality gap and x^T s / max(1,|c^T x|)  [1e-6] */
  double eps_feas;   /* stop: ||r_p|| <= eps_feas ||b||, ||r_d|| <= eps_feas ||c||  [1e-8] */
  double guard;      /* step <= (1-guard) x distance to the boundary of x, s > 0  [1e-3] */
  int32_t w;         /* sketch width, m <= w  [0 = 4m]                                 */
  int32_t s;         /* non-zeros per row of W, s divides w  [1]                       */
  int32_t max_cg;    /* CG iteration cap per normal-equation solve, counted over all the
                        inner CG runs of the refinement in SKIPM_PREC_MIXED / _BF16  [1000] */
  int32_t max_outer; /* IPM iteration cap  [300]                                       */
  int32_t resketch;  /* 1: fresh W every IPM iteration (salt = iteration), 0: one W  [1] */
  int32_t precision; /* SKIPM_PREC_FP64, SKIPM_PREC_MIXED or SKIPM_PREC_BF16  [FP64]   */
  uint64_t seed;     /* sketch seed  [0]                                               */
  int32_t inner;     /* solver of Alg. 2 step (c): SKIPM_INNER_CG (Alg. 1), _SD (steepest
                        descent, App. B Alg. 4) or _RICHARDSON (App. A Alg. 3)  [CG]   */
  int32_t sketch;    /* SKIPM_SKETCH_COUNT: the sparse embedding of Sec. 2 (s non-zeros
                        per row); SKIPM_SKETCH_GAUSSIAN: the dense Gaussian W_G of
                        Sec. 5 (dense FP64 A only; s is ignored)  [COUNT]            */
} skipm_params;

/* Result of lp_solve (host struct). */
typedef struct {
  int32_t status;    /* SKIPM_OK when the stopping test holds */
  int32_t iters;     /* IPM iterations taken */
  int32_t cg_total;  /* CG iterations summed over the solve */
  int32_t cg_max;    /* largest CG iteration count of one solve */
  double obj_p;      /* c^T x */
  double obj_d;      /* b^T y */
  double rel_gap;    /* |c^T x - b^T y| / max(1, |c^T x|) */
  double rp_norm;    /* ||A x - b|| */
  double rd_norm;    /* ||A^T y + s - c|| */
  double mu;         /* x^T s / n */
  int32_t demote_iter;  /* first IPM iteration whose CG products moved up a precision tier
                           (SKIPM_PREC_MIXED / _BF16), -1 if none did */
  int32_t tier_final;   /* SKIPM_TIER_* of the CG products at the end of the run */
  int32_t resketches;   /* fresh sketches drawn after a non-positive Gram pivot, summed */
  int32_t shifts;       /* diagonally shifted factorisations after those, summed */
} skipm_result;

/* Diagnostics of one IPM iteration (host struct). */
typedef struct {
  double mu;         /* duality measure at the start of the iteration */
  double rp_norm;    /* ||r_p|| at the start */
  double rd_norm;    /* ||r_d|| at the start */
  double rel_gap;    /* at the start */
  double eta;        /* ||r^k|| / ||r^0|| */
  double alpha_max;  /* Alg. 2 step (e) */
  double alpha;      /* Alg. 2 step (f) */
  double f_norm;     /* ||f^(t)||, final preconditioned CG residual */
  double f0_norm;    /* ||f^(0)|| = ||Q^{-1/2} p|| */
  double v_norm;     /* ||v|| */
  double v_resid;    /* ||B t - g|| / ||g|| with t = (A D W)^+ g: how exactly v meets eq. addl */
  int32_t cg_iters;  /* CG iterations of this solve */
  int32_t v_iters;   /* refinement steps of the FP64 solve for t inside v */
  int32_t converged; /* 1: the stopping test held at the start, nothing was done */
  int32_t status;    /* SKIPM_OK or an error code */
  int32_t tier;      /* SKIPM_TIER_* of the CG products when this iteration's solve ended */
  int32_t refine_steps; /* outer refinement steps of the normal-equation solve (1 in FP64) */
  int32_t resketches;   /* fresh sketches drawn after a non-positive Gram pivot */
  int32_t shifts;       /* diagonally shifted factorisations after those */
} skipm_step_info;

/* Result of pcg_solve (host struct). */
typedef struct {
  int32_t iters;
  double f0_norm;    /* ||f^(0)|| */
  double f_norm;     /* ||f^(iters)|| (from the CG recurrence) */
} skipm_pcg_info;

/* Fill *out with the default parameters.  Returns SKIPM_EINVAL if out is NULL. */
int skipm_params_default(skipm_params* out);

/* Create a solver handle for one LP (device buffers are allocated and the problem
 * copied).  Validates sizes and, for CSR, row pointers and column indices
 * (SKIPM_EINVAL on a bad entry).  The iterate starts at x = s = 1, y = 0
 * (the experiments' all-ones start with y = 0).  Synchronises `stream`.
 * Dense FP64 LPs with m <= 64 whose A takes at most 1 MiB run each CG solve
 * in one workgroup (one launch); the environment variable
 * SKIPM_CG_SMALL_BYTES, read here, sets that limit in bytes (0: never).
 * LPs with n <= 1024 run the step tail of Alg. 2 (steps d-g) in one
 * workgroup; SKIPM_STEP_ONE=0, read here, keeps the multi-launch tail, which
 * computes the same sums in the same order. */
int lp_create(skipm_lp_t* out, const skipm_problem* prob, const skipm_params* prm,
              hipStream_t stream);

/* Free the handle and all its device memory.  NULL is accepted. */
int lp_destroy(skipm_lp_t lp);

/* Reset the iterate to x = s = 1, y = 0 and the iteration counter to 0. */
int lp_reset(skipm_lp_t lp, hipStream_t stream);

/* Overwrite the iterate (device pointers x: n, y: m, s: n; x, s > 0 is the
 * caller's responsibility).  With reset_origin != 0 this point becomes the
 * origin r^0, mu_0 of the neighbourhood N(gamma); otherwise the origin of the
 * current run is kept (resuming from a checkpoint). */
int lp_set_iterate(skipm_lp_t lp, const double* x, const double* y, const double* s,
                   int32_t reset_origin, hipStream_t stream);

/* Copy the current iterate out (device pointers; any may be NULL). */
int lp_get_iterate(skipm_lp_t lp, double* x, double* y, double* s, hipStream_t stream);

/* Copy the last computed direction (dx, ds, v: n; dy: m) out (device pointers;
 * any may be NULL).  Valid after ipm_step. */
int lp_get_direction(skipm_lp_t lp, double* dx, double* dy, double* ds, double* v,
                     hipStream_t stream);

/* Copy the vectors of the last ipm_step out (device pointers; any may be
 * NULL): the prologue's residuals r_p = A x - b (m) and r_d = A^T y + s - c (n)
 * (eqs. "primalres", "dualres") and right-hand side p (m, eq. "pdef"), and the
 * epilogue's g = A D^2 A^T dy - p (m), the residual that the correction vector
 * v of eq. "compv" cancels (eq. "addl").  pcg_solve leaves its right-hand side
 * in g. */
int lp_get_residuals(skipm_lp_t lp, double* rp, double* rd, double* p, double* g,
                     hipStream_t stream);

/* The sparse embedding W used at IPM iteration (salt) k: for every row j < n
 * and block r < s, bucket[j*s + r] in [r*w/s, (r+1)*w/s) and sign[j*s + r] in
 * {-1, +1} (Sec. 2's sparse embedding, made concrete as a block CountSketch
 * with a SplitMix64 counter hash).  bucket and sign are device arrays of n*s
 * entries.  Needs 1 <= s, s | w. */
int sketch_hash(uint64_t seed, int64_t k, int32_t s, int64_t n, int32_t w,
                int32_t* bucket, int8_t* sign, hipStream_t stream);

/* The sketch B = A diag(d) W_k (Alg. 1 step 1 with D = diag(d)), W_k the embedding
 * of sketch_hash(prm.seed, k, prm.s, n, prm.w) (or W_G of Sec. 5 with
 * SKIPM_SKETCH_GAUSSIAN).  d: n (device).  B: device buffer of m*w values of
 * out_dtype (SKIPM_F64, or SKIPM_F32: the FP64 sketch rounded to nearest),
 * column-major with leading dimension m.  Another out_dtype: SKIPM_EINVAL. */
int sketch_apply(skipm_lp_t lp, const double* d, int64_t k, void* B, int32_t out_dtype,
                 hipStream_t stream);

/* Alg. 1 as used in Alg. 2 step (c): with D^2 = diag(d2), build Q from the
 * sketch with salt k and solve A D^2 A^T dy = p by CG preconditioned with Q,
 * from dy = 0, until ||f^(j)|| <= tol ||f^(0)|| or max_it iterations (tol <= 0:
 * run exactly max_it iterations).  d2: n, p: m, dy: m (device).  info: host. */
int pcg_solve(skipm_lp_t lp, const double* d2, const double* p, int64_t k, double* dy,
              double tol, int32_t max_it, skipm_pcg_info* info, hipStream_t stream);

/* out = A D^2 A^T u with the handle's current D^2 (as left by the last prologue
 * of ipm_step / lp_solve or by pcg_solve): the operator of eq. "normal" applied
 * by the same fused one-pass kernel CG uses, reading the copy of A of the
 * handle's current precision tier (FP32 or BF16 values, FP64 accumulation, in
 * SKIPM_PREC_MIXED / _BF16 until the run escalates).  The pass is launched
 * `reps` >= 1 times (to time it); u: m, out: m (device). */
int normal_matvec(skipm_lp_t lp, const double* u, double* out, int32_t reps,
                  hipStream_t stream);

/* As normal_matvec, and *ms_per_pass (host) receives the mean duration of one
 * fused pass, from HIP events recorded on `stream` immediately before the first
 * and after the last of the `reps` back-to-back passes.  Synchronises `stream`. */
int normal_matvec_timed(skipm_lp_t lp, const double* u, double* out, int32_t reps,
                        float* ms_per_pass, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the product
 * of normal_matvec, out = A D^2 A^T u, on the caller's own A and D^2, with no
 * handle and no allocation of any kind.  The same kernels as normal_matvec
 * (one fused pass over A, then a fixed-order sum of per-workgroup partials),
 * so the result is bitwise that of normal_matvec on a handle holding the same
 * A and D^2.  The partials and a zero-padded copy of u live in a static device
 * buffer of the library (8 MiB + 16 KiB on each device it runs on, held until
 * the process ends, its address looked up on the first call on a device).
 *   A: dense column-major, a_dtype SKIPM_F64 or SKIPM_F32, 16-byte aligned,
 *      leading dimension lda with m <= lda <= 2048 and lda a multiple of 4;
 *      rows m..lda-1 are read and must hold finite values (lp_create's own
 *      layout holds zeros there).
 *   d2: n FP64 (NULL: D = I); u: m FP64; out: m FP64.  1 <= m <= 2048, n >= 1.
 * SKIPM_EINVAL outside these limits (checked before any device work).  Every
 * call on a device shares that device's buffer: calls that overlap on one
 * device (different streams or threads without ordering) race; calls ordered
 * on one stream do not.  Nothing is synchronised. */
int normal_matvec_noalloc(const void* A, int32_t a_dtype, int64_t m, int64_t n, int64_t lda,
                          const double* d2, const double* u, double* out, hipStream_t stream);

/* Sampled timing of the CG's normal-equation product A D^2 A^T d inside
 * ipm_step / lp_solve / pcg_solve (the solver's dominant kernel: the fused
 * column pass for dense A, the column + row passes for CSR).  every > 0: a HIP
 * event pair on the solve's stream brackets the product of every `every`-th CG
 * iteration; pairs are read at the CG's host checks, and those of products
 * that the done flag skipped are dropped.  every = 0 turns sampling off.
 * Either call clears the accumulated samples. */
int lp_kernel_timing(skipm_lp_t lp, int32_t every);

/* Mean duration (ms, host) of the sampled products and their number. */
int lp_kernel_time(skipm_lp_t lp, double* avg_ms, int64_t* samples);

/* As lp_kernel_time, over the sampled products that read the copy of A of one
 * precision tier (SKIPM_TIER_*), so that each mean has one byte count. */
int lp_kernel_time_tier(skipm_lp_t lp, int32_t tier, double* avg_ms, int64_t* samples);

/* While lp_kernel_timing is on (every > 0), a second HIP event pair brackets
 * the sketch product B = A D W of each IPM iteration (Alg. 2 step (a)): for
 * the Gaussian sketch the FP64 GEMM with its slice sum, after the fill of
 * D W_G; for the count sketch the sketch kernel.  Mean duration (ms, host)
 * and the number of samples since timing was last switched on. */
int lp_sketch_time(skipm_lp_t lp, double* avg_ms, int64_t* samples);

/* One iteration of Alg. 2 on the handle's iterate (steps a-g), or nothing if
 * the stopping test already holds (info->converged = 1).  info: host, may be NULL. */
int ipm_step(skipm_lp_t lp, skipm_step_info* info, hipStream_t stream);

/* Run Alg. 2 from the current iterate until the stopping test holds or
 * max_outer iterations.  res: host. */
int lp_solve(skipm_lp_t lp, skipm_result* res, hipStream_t stream);

/* ---- many LPs ------------------------------------------------------------ */

/* Device bytes that lp_create and a following lp_solve allocate for this
 * problem (an upper bound, counted the way the library allocates; what the
 * request server admits against its budget).  prob's pointers are not read.
 * *bytes: host. */
int lp_footprint(const skipm_problem* prob, const skipm_params* prm, int64_t* bytes);

/* Device bytes the handle holds now.  *bytes: host. */
int lp_device_bytes(skipm_lp_t lp, int64_t* bytes);

/* Solve `count` independent LPs (handles from lp_create, each from its
 * current iterate, as lp_solve).  Dense LPs with FP64 CG products go through
 * the grouped engine: `workers` host threads (<= 0: min(count, 8)), each with
 * its own non-blocking stream of default priority, take the LPs through the
 * per-LP steps of their IPM iterations (stopping test, sketch, factorisation;
 * epilogue, correction vector, step), while one executor runs the CG of every
 * LP that is ready in grouped launches: one launch per CG pass and lane-group
 * shape, whose work list is the (LP, workgroup) pairs of its LPs, each LP at
 * its own CG iteration; an LP joins when its factorisation is done and leaves
 * at the first host check after its CG has converged (Alg. 1 / Alg. 2 per LP,
 * unchanged).  The other LPs (CSR, FP32/BF16 CG copies) run lp_solve on
 * `workers` further threads.  Every LP keeps the arithmetic of a lone solve,
 * so res[i] (and its final iterate) is bitwise that of lp_solve alone.  The
 * call first waits for all work queued on the device and returns when every
 * LP has finished.  res: host array of `count`.  Returns SKIPM_OK when every
 * solve ran, an LP's outcome (OK, ENOTCONV, ESTALL, ERANK, ENAN) being
 * res[i].status; an argument, memory or device error stops the batch and is
 * returned. */
int lp_solve_batch(skipm_lp_t* lps, int32_t count, skipm_result* res, int32_t workers);

/* Request server: a FIFO of LP solves admitted by device-memory footprint.
 * srv_create starts `slots` slot threads (each with its own non-blocking
 * stream) and a grouped engine like lp_solve_batch's.  A slot takes the request
 * at the head of the queue once at most `slots` requests are in flight and its
 * footprint (lp_footprint) fits in hbm_budget minus the footprints of those in
 * flight, and creates the LP from the request's buffers.  A dense LP with FP64
 * CG products joins the engine: its CG iterations run in the same grouped
 * launches as those of every other request in flight, whatever their sizes,
 * and the slot moves on to the next admission; any other LP is solved on the
 * slot (lp_solve).  At the end the final x is copied out if asked and the LP
 * freed.  Every request's arithmetic is that of lp_solve alone. */
typedef struct skipm_server_s* skipm_server_t;

#define SKIPM_REQ_QUEUED  0
#define SKIPM_REQ_RUNNING 1
#define SKIPM_REQ_DONE    2

typedef struct {
  skipm_result res;      /* as lp_solve; res.status also carries a create error */
  int32_t state;         /* SKIPM_REQ_* */
  int32_t rc;            /* SKIPM_OK, or the argument/memory/device error of the request */
  int64_t footprint;     /* bytes reserved against the budget */
  int64_t device_bytes;  /* bytes the LP actually held at the end of its solve */
  double t_submit;       /* server clock (seconds since srv_create) */
  double t_start;        /* admitted: a worker began creating the LP */
  double t_done;         /* result available */
} skipm_request_info;

typedef struct {
  int64_t budget, in_use, peak_in_use;
  int32_t slots, running, queued;
  int64_t completed;
} skipm_server_stats;

/* hbm_budget > 0 bytes; slots in [1, 64].  Uses the current device. */
int srv_create(skipm_server_t* srv, int64_t hbm_budget, int32_t slots);

/* Queue one solve.  prob's device buffers (A, b, c) are read when the request
 * is admitted, after the work queued on `producer` at the time of this call:
 * they must stay valid until the request is SKIPM_REQ_DONE.  x_out: device,
 * n doubles, receives the final x (may be NULL).  *ticket: host.  Returns
 * SKIPM_ENOMEM at once if the footprint exceeds the whole budget. */
int srv_submit(skipm_server_t srv, const skipm_problem* prob, const skipm_params* prm,
               double* x_out, hipStream_t producer, uint64_t* ticket);

/* Current state of a request, without waiting.  info: host. */
int srv_poll(skipm_server_t srv, uint64_t ticket, skipm_request_info* info);

/* Wait until the request is done.  info: host. */
int srv_wait(skipm_server_t srv, uint64_t ticket, skipm_request_info* info);

/* Seconds since srv_create on the server's clock.  *t: host. */
int srv_now(skipm_server_t srv, double* t);

int srv_stats(skipm_server_t srv, skipm_server_stats* stats);

/* Finish every queued and running request, stop the workers, free the server. */
int srv_destroy(skipm_server_t srv);

/* Message of the last failing call on this thread ("" if none). */
const char* skipm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SKIPM_H */
