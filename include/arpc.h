/*
 * arpc.h - C ABI of the MI355X (gfx950) accelerated randomly pivoted Cholesky library.
 *
 * The operation follows Epperly, Tropp & Webber, "Embrace rejection: kernel
 * matrix approximation by accelerated randomly pivoted Cholesky" (arXiv
 * 2410.03969):
 *   - the problem statement of Section 1 (low-rank psd approximation: given a
 *     psd N x N matrix A and a rank k, return F (N x k) with A ~ F F^T),
 *   - the kernel matrix A(i,j) = kappa(x_i, x_j) built from points (Section 1.2),
 *   - accelerated RPCholesky, standard implementation (Alg. 2, Section 2.3),
 *     with RejectionSampleSubmatrix (Alg. 1, Section 2.2) inside every round.
 *
 * Every call returns an arpc_status; nothing throws or aborts across the ABI.
 * Pointers documented as "device" must point to memory of the current HIP
 * device; the library never frees memory it did not allocate.
 */
#ifndef ARPC_H
#define ARPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum arpc_status {
  ARPC_OK = 0,           /* k pivots produced */
  ARPC_EARLY_STOP = 1,   /* informational: the residual became (numerically) zero
                            before k pivots; k_out < k, see arpc_factor */
  ARPC_INCOMPLETE = 2,   /* informational (arpc_factor_query): the rounds enqueued so far
                            ended before k pivots; arpc_factor_continue adds more */
  ARPC_EINVAL = -1,      /* invalid argument (sizes, pointers, alignment, workspace) */
  ARPC_ENOMEM = -2,      /* an allocation or admission could not be satisfied */
  ARPC_EBUSY = -3,       /* a queue or slot table is full */
  ARPC_EDEVICE = -4,     /* a HIP runtime call failed */
  ARPC_ENUMERIC = -5,    /* the points contain NaN or Inf */
  ARPC_ECANCELED = -6    /* the job was cancelled */
} arpc_status;

/* Kernel functions (Section 1.2 and Section 3).  The Laplace kernel uses the
 * l2 distance; Matern-3/2 is (1 + sqrt3 r/s) exp(-sqrt3 r/s). */
typedef enum arpc_kernel {
  ARPC_GAUSSIAN = 0,     /* exp(-|x-y|^2 / (2 s^2)) */
  ARPC_LAPLACE_L2 = 1,   /* exp(-|x-y| / s) */
  ARPC_MATERN32 = 2,
  ARPC_MATERN52 = 3      /* (1 + sqrt5 r/s + 5 r^2/(3 s^2)) exp(-sqrt5 r/s) */
} arpc_kernel;

/* Arithmetic of the N-sized steps.  In every mode the residual diagonal, the
 * b x b residual submatrix, its Cholesky factor and the acceptance tests are
 * FP64. */
typedef enum arpc_prec {
  ARPC_FP64 = 0,    /* F stored FP64; update GEMM and triangular solve in FP64 */
  ARPC_FP32 = 1,    /* F stored FP32; update GEMM and solve in FP32 */
  ARPC_BF16X3 = 2,  /* F stored FP32; update GEMM on BF16 matrix cores with a
                       hi/lo split of both operands (three products), FP32 accumulation */
  ARPC_BF16 = 3,    /* F stored FP32; update GEMM with BF16-rounded operands, FP32 accumulation */
  ARPC_FP8 = 4      /* the kernel matrix of the points rounded to FP8 e4m3 (OCP: 3 fraction
                       bits, exponent bias 7, ties to even, saturating at +-448), factored as
                       in ARPC_BF16; the distances of the kernel columns contract the e4m3
                       coordinates on FP8 matrix cores with FP32 accumulation (exact products),
                       the b x b steps use the same rounded points in FP64.  Workspace holds
                       the rounded copy (8 N d bytes). */
} arpc_prec;

/* The rule that picks each round's pivots from its b proposals. */
typedef enum arpc_method {
  ARPC_ACCEL = 0,   /* accelerated RPCholesky (Alg. 2): RejectionSampleSubmatrix (Alg. 1) keeps
                       proposal i with probability h_ii / u_i.  With b = 1 every proposal with a
                       positive residual is kept: simple RPCholesky (Alg. 6, Section 1.3.1). */
  ARPC_BLOCK = 1    /* block RPCholesky (Alg. 7, Section 1.3.2): every distinct proposal is kept
                       (the test of Alg. 1 with V = 0, so a proposal whose residual is not
                       positive is still skipped).  A baseline: its columns can be wasted on
                       near-duplicate proposals. */
} arpc_method;

typedef struct arpc_problem {
  int64_t N;          /* number of points, 1 <= N <= 2^31 - 1 */
  int64_t d;          /* dimension, 1 <= d <= 4096 */
  int64_t k;          /* target rank, 1 <= k <= N */
  int64_t b;          /* proposals per round (block size), 1 <= b <= 1024 */
  int32_t kernel;     /* arpc_kernel */
  int32_t prec;       /* arpc_prec */
  double bandwidth;   /* sigma (length scale), finite and > 0 */
  uint64_t seed;      /* key of the uniform stream */
  int64_t max_rounds; /* 0: run until k pivots; > 0: stop after this many rounds */
  int32_t method;     /* arpc_method */
  int32_t reserved;   /* must be 0 */
} arpc_problem;

enum {
  ARPC_KC_INIT = 0, ARPC_KC_PROPOSE, ARPC_KC_GATHER, ARPC_KC_REJECT, ARPC_KC_PREP,
  ARPC_KC_COLGEMM, ARPC_KC_TRSM, ARPC_KC_DIAG, ARPC_KC_FINISH, ARPC_NUM_KC
};

typedef struct arpc_stats {
  int64_t k_out;        /* pivots produced */
  int64_t rounds;       /* rounds run */
  int64_t proposals;    /* b * rounds */
  int32_t status;       /* ARPC_OK or ARPC_EARLY_STOP */
  int32_t fused;        /* 1: each round's update GEMM, solve and stores ran as one
                           kernel (ARPC_BF16X3 / ARPC_BF16 with b <= 256, d <= 16;
                           ARPC_BF16 with b <= 208, d <= 32),
                           timed under the colgemm class; 0: two kernels */
  double trace_A;       /* sum of diag A */
  double trace_resid;   /* sum of the final residual diagonal */
  double ms_total;      /* host wall time of the call */
  double ms_kernel[ARPC_NUM_KC];   /* summed kernel time per class (profiling on) */
  int64_t launches[ARPC_NUM_KC];   /* launches per class (profiling on) */
  double flops_colgemm; /* algorithmic flops of the update GEMM, sum_r 2 N k_r s_r */
  double flops_trsm;    /* algorithmic flops of the triangular solve, sum_r N s_r^2 */
  double bytes_colgemm; /* algorithmic HBM bytes of the update GEMM: F read over k_r columns at
                           the contraction precision, C written, X read (fused: F and X read,
                           G written once to F at its storage precision, row norms written) */
  double bytes_trsm;    /* algorithmic HBM bytes of the triangular solve: C read, G written
                           to F, row norms (0 when fused) */
  double bytes_blocked; /* HBM bytes of G written into the panel-blocked copy of F that the
                           matrix-core contraction of later rounds reads (not counted above) */
} arpc_stats;

/* Human-readable name of a status code (static storage). */
const char* arpc_status_str(int status);

/* Library version string (static storage). */
const char* arpc_version(void);

/* Bytes of device workspace that arpc_factor needs for *problem.
 * Returns ARPC_EINVAL for an invalid problem. */
arpc_status arpc_workspace_size(const arpc_problem* problem, size_t* bytes);

/* Accelerated RPCholesky (Alg. 2 with Alg. 1) of the kernel matrix of X.
 *
 *  X       device, N x d row-major FP64 points (read only).
 *  F       device, N x k column-major output, FP64 for ARPC_FP64 and FP32 for
 *          the other modes; column j belongs to pivots[j].  Caller-allocated.
 *  pivots  device, k int64 outputs, 0-based row indices in acceptance order.
 *  ws      device workspace of at least arpc_workspace_size bytes, 256-byte aligned.
 *  stream  hipStream_t (NULL = default stream) on which all work is enqueued.
 *  stats   host, may be NULL.
 *
 * Round r draws its b proposals from uniform words 2br..2br+b-1 and its b
 * acceptance tests from words 2br+b..2br+2b-1 of the Philox4x64-10 stream
 * keyed by problem->seed (block q of four words at counter q+1, uniform =
 * (word >> 11) * 2^-53).
 *
 * Blocks the calling thread until the factorization is complete.  The host
 * reads the device-side round state back after the rejection step of the
 * last round of each batch and enqueues the next rounds, or the end of the
 * run, while that round finishes, so the stream does not drain between
 * rounds.  Uses a pinned host buffer per calling thread (a few KB, grown to
 * the round history's size, kept until the process ends).  Returns
 * ARPC_OK, or ARPC_EARLY_STOP when the residual trace reached zero or a round
 * accepted nothing; then columns k_out..k-1 of F are zero and
 * pivots[k_out..k-1] = -1.  Errors: ARPC_EINVAL, ARPC_ENUMERIC (non-finite
 * point), ARPC_EDEVICE. */
arpc_status arpc_factor(const arpc_problem* problem, const double* X, void* F,
                        int64_t* pivots, void* ws, size_t ws_bytes, void* stream,
                        arpc_stats* stats);

/* Same as arpc_factor with the uniform stream replaced by an explicit device
 * array U of nU FP64 values in [0,1) (word p = U[p]).  If the run needs more
 * than nU words it stops after the last complete round and returns
 * ARPC_EINVAL. */
arpc_status arpc_factor_uniforms(const arpc_problem* problem, const double* X, void* F,
                                 int64_t* pivots, void* ws, size_t ws_bytes, void* stream,
                                 const double* U, int64_t nU, arpc_stats* stats);

/* Asynchronous form of arpc_factor (the same factorization, kernels and
 * results): enqueues on `stream` the initialisation, `rounds` rounds of Alg. 2
 * and the end of the run, and returns without waiting for the device.
 * Every round reads the round state kept in ws, so rounds past the end of the
 * run (k pivots held, or the residual exhausted) exit on the device at once;
 * the end of the run writes the residual trace into ws and, after an early
 * stop, zero columns k_out..k-1 of F and pivots[k_out..k-1] = -1.
 *
 *  problem, X, F, pivots, ws, ws_bytes, stream   as for arpc_factor.
 *  rounds  rounds to enqueue; 0: problem->max_rounds if set, else
 *          ceil(k/b) + ceil(k/b)/2 + 4 (at most k).  Every round that runs
 *          accepts at least one pivot, so k rounds always suffice.
 *
 * F, pivots and the statistics (arpc_factor_query) are valid once the stream
 * has passed the enqueued work; the caller must keep X, F, pivots and ws
 * untouched until then.  Returns ARPC_OK when the work was enqueued,
 * ARPC_EINVAL / ARPC_EDEVICE otherwise. */
arpc_status arpc_factor_async(const arpc_problem* problem, const double* X, void* F, int64_t* pivots,
                              void* ws, size_t ws_bytes, void* stream, int64_t rounds);

/* Enqueue `rounds` (>= 1) more rounds and the end of the run for a
 * factorization started by arpc_factor_async on the same problem, X, F,
 * pivots and ws (after arpc_factor_query returned ARPC_INCOMPLETE, or without
 * asking: rounds past the end exit at once).  Asynchronous like
 * arpc_factor_async. */
arpc_status arpc_factor_continue(const arpc_problem* problem, const double* X, void* F, int64_t* pivots,
                                 void* ws, size_t ws_bytes, void* stream, int64_t rounds);

/* Outcome of the work enqueued by arpc_factor_async / arpc_factor_continue,
 * read from ws (host memory copies; call after the stream has passed that
 * work).  Returns what arpc_factor would have returned (ARPC_OK,
 * ARPC_EARLY_STOP, ARPC_ENUMERIC, ARPC_EINVAL for an exhausted uniform array),
 * or ARPC_INCOMPLETE when the run needs more rounds; stats (may be NULL) as
 * for arpc_factor, without kernel times and with ms_total = 0. */
arpc_status arpc_factor_query(const arpc_problem* problem, const void* ws, size_t ws_bytes, arpc_stats* stats);

/* Bytes of device workspace that arpc_factor_lowmem needs for *problem:
 * O(N ceil(b/64) + k (2d + 3b) + b^2) doubles, against the N k of arpc_factor's F.
 * Returns ARPC_EINVAL for a problem arpc_factor_lowmem does not take. */
arpc_status arpc_lowmem_workspace_size(const arpc_problem* problem, size_t* bytes);

/* Accelerated RPCholesky, low-memory implementation (Alg. 3, Section 2.4): the
 * same rounds, uniform words and pivots as arpc_factor (Alg. 2 with Alg. 1), but
 * no N x k factor is stored.  The output is the pivot set S and the lower
 * Cholesky factor L of A(S,S), which define the approximation
 * A(:,S) L^{-*} L^{-1} A(S,:); the kernel entries A(R,S) are regenerated in
 * every round, so the arithmetic grows to O(N k^2) kernel evaluations.
 * Requirements: prec ARPC_FP64, method ARPC_ACCEL, k <= 4096, b <= 512,
 * d <= 256.
 *
 *  X       device, N x d row-major FP64 points (read only).
 *  L       device, k x k column-major FP64 output: L(i, j) for j <= i < k_out;
 *          every other entry is zero.  Caller-allocated.
 *  pivots  device, k int64 outputs in acceptance order (-1 past k_out).
 *  ws      device workspace of at least arpc_lowmem_workspace_size bytes,
 *          256-byte aligned.
 *  stream  hipStream_t (NULL = default stream).
 *  stats   host, may be NULL; k_out, rounds, proposals, status, trace_A,
 *          trace_resid, ms_total and the per-class kernel times are filled.
 *
 * Returns ARPC_OK or ARPC_EARLY_STOP as arpc_factor does; errors ARPC_EINVAL,
 * ARPC_ENUMERIC, ARPC_EDEVICE. */
arpc_status arpc_factor_lowmem(const arpc_problem* problem, const double* X, double* L,
                               int64_t* pivots, void* ws, size_t ws_bytes, void* stream,
                               arpc_stats* stats);

/* Bytes of device workspace that arpc_qr_factor needs: O(N + M b + k b + b^2)
 * doubles.  Returns ARPC_EINVAL for sizes arpc_qr_factor does not take. */
arpc_status arpc_qr_workspace_size(int64_t M, int64_t N, int64_t k, int64_t b, size_t* bytes);

/* Accelerated randomly pivoted QR (Alg. 5, Section 5) of a general matrix B:
 * column pivots proposed from the residual squared column norms and filtered
 * by RejectionSampleSubmatrix (Alg. 1) on the residual Gram matrix C^* C of the
 * proposals, so the pivots are those accelerated RPCholesky takes on B^* B
 * (Proposition qr_cholesky) from the same uniform words (the stream of
 * arpc_factor keyed by seed).  Output: Q with orthonormal columns and
 * F = B^* Q, B_hat = Q F^*; each round's new columns of Q are orthonormalized
 * after one extra Gram-Schmidt pass, by the QR factorization with a positive
 * diagonal in R.  FP64; every product on the library's FP64 matrix-core GEMM.
 *
 *  M, N    rows and columns of B, 1 <= k <= min(M, N), 1 <= b <= 512.
 *  B       device, M x N column-major FP64 (read only).
 *  Q       device, M x k column-major FP64 output.
 *  F       device, N x k column-major FP64 output.
 *  pivots  device, k int64 column indices in acceptance order (-1 past k_out).
 *  ws      device workspace of at least arpc_qr_workspace_size bytes, 256-byte
 *          aligned.  stream: hipStream_t (NULL = default).  stats: host, may be
 *          NULL (trace_A is |B|_F^2 and trace_resid the residual's).
 *
 * Returns ARPC_OK or ARPC_EARLY_STOP (the residual reached zero or a round
 * accepted nothing; Q and F columns k_out..k-1 are zero); errors ARPC_EINVAL,
 * ARPC_ENUMERIC (a non-finite entry of B), ARPC_EDEVICE. */
arpc_status arpc_qr_factor(int64_t M, int64_t N, int64_t k, int64_t b, uint64_t seed, int64_t max_rounds,
                           const double* B, double* Q, double* F, int64_t* pivots, void* ws,
                           size_t ws_bytes, void* stream, arpc_stats* stats);

/* ------------------------------------------------------- kernel ridge regression
 * (A + mu I) beta = y for the kernel matrix A of the points X (Section 3.2), by
 * preconditioned conjugate gradients with the low-rank preconditioner
 * P = F F^* + mu I, F the N x k factor of arpc_factor (k = 0: P = mu I). */
typedef struct arpc_krr_stats {
  int64_t iterations;   /* PCG iterations run */
  double rel_residual;  /* |y - (A + mu I) beta| / |y| as tracked by the recurrence */
  double ms_total;      /* host wall time of the call */
  double ms_setup;      /* forming and factoring mu I + F^* F */
  double ms_matvec;     /* products with A + mu I (device time, HIP events) */
  double ms_precond;    /* applications of P^{-1} (device time, HIP events) */
  int32_t status;       /* ARPC_OK: converged to tol; ARPC_EARLY_STOP: max_iter reached */
  int32_t reserved;
} arpc_krr_stats;

/* Bytes of device workspace of arpc_krr_pcg: O(N + k^2) doubles, plus N k
 * doubles when F is FP32 (converted once). */
arpc_status arpc_krr_workspace_size(int64_t N, int64_t d, int64_t k, int32_t f_prec, size_t* bytes);

/* Solves (A + mu I) beta = y by PCG from beta = 0 (Golub and Van Loan,
 * Alg. 11.5.1), stopping when |r| <= tol |y| or after max_iter iterations.
 * The products with A regenerate the kernel entries in FP64 (direct
 * differences, the diagonal exactly kappa(0)); P^{-1} r is applied through the
 * Woodbury identity (r - F (mu I + F^* F)^{-1} F^* r) / mu.
 *
 *  X       device, N x d row-major FP64 points, 1 <= d <= 128.
 *  kernel, bandwidth  as in arpc_problem; mu > 0.
 *  y       device, N FP64 right-hand side.
 *  F       device, N x k column-major factor, FP64 if f_prec is ARPC_FP64, else
 *          FP32 (the layout arpc_factor writes); unused when k = 0.  k <= 2048.
 *  beta    device, N FP64 output.
 *  ws      device workspace of at least arpc_krr_workspace_size bytes, 256-byte aligned.
 *  stream  hipStream_t.  The PCG scalars stay on the device; the host waits on the
 *          stream once per batch of eight iterations to read the stopping flag.
 *  stats   host, may be NULL.
 *
 * Returns ARPC_OK (converged), ARPC_EARLY_STOP (max_iter reached), ARPC_EINVAL,
 * ARPC_ENUMERIC (mu I + F^* F not positive definite, or a non-finite residual),
 * ARPC_EDEVICE. */
arpc_status arpc_krr_pcg(int64_t N, int64_t d, int32_t kernel, double bandwidth, double mu,
                         const double* X, const double* y, const void* F, int32_t f_prec, int64_t k,
                         double tol, int64_t max_iter, double* beta, void* ws, size_t ws_bytes,
                         void* stream, arpc_krr_stats* stats);

/* Host evaluation of the library's uniform stream: out[i] = uniform of word
 * start + i for key seed.  out is host memory of n doubles. */
arpc_status arpc_stream_uniforms_host(uint64_t seed, int64_t start, int64_t n, double* out);

/* Per-kernel timing with HIP events, recorded into arpc_stats.ms_kernel
 * (process-wide switch; off by default).  on != 0 times every kernel class. */
void arpc_set_profiling(int on);

/* The same switch restricted to the kernel classes whose bit (1 << ARPC_KC_*)
 * is set in mask (0: off).  Timing one class keeps the events of the others
 * off the stream. */
void arpc_set_profiling_classes(unsigned mask);

/* ------------------------------------------------------------------ serving
 * A context serves a stream of factorization jobs (each one arpc_factor's
 * operation: Alg. 2 with Alg. 1) on one device with continuous batching:
 *  - a job is admitted, in submission order, as soon as a slot is free and
 *    its workspace (arpc_workspace_size of its problem, about N*k elements of
 *    the blocked factor copy plus O(N + b*k) more) fits in what is left of the
 *    context's HBM budget;
 *  - jobs in the BF16 modes whose rounds run as one kernel (d <= 16 and
 *    b <= 256; in ARPC_BF16 also d <= 32 and b <= 208)
 *    advance together in ticks: one tick runs one round of every such job,
 *    with one kernel launch per round step serving all of them (the round
 *    product once per group of jobs of the same compiled shape), from a
 *    device table of the jobs' arguments; two ticks are kept in flight, and
 *    a job joins the next tick after its admission;
 *  - every other job runs on a stream of its own slot, one batch of rounds
 *    after another (each round replayed from a HIP graph recorded once), so
 *    its rounds overlap with the ticks and with other slots;
 *  - a finished job frees its slot and memory at once and the next job is
 *    admitted.
 * A job runs the same kernels as arpc_factor on its own data, with the same
 * per-job work decomposition, so its result does not depend on the other
 * jobs.  The environment variable ARPC_SERVE_TICKS=0 turns ticks off (every
 * job on its slot stream) and ARPC_SERVE_GRAPHS=0 the graph replay.
 * The context owns one device allocation of the budget (made by arpc_create),
 * a small device table for the ticks, its streams and a scheduler thread; the
 * caller owns every job's X, F and pivots and must keep them alive and
 * untouched until the job completes.  Calls on one context may come from
 * several threads. */
typedef struct arpc_ctx_s* arpc_ctx;
typedef uint64_t arpc_job;

typedef struct arpc_serving_stats {
  int64_t submitted;     /* jobs submitted so far */
  int64_t completed;     /* jobs finished (any status) */
  int64_t cancelled;     /* jobs that ended with ARPC_ECANCELED */
  int64_t active;        /* jobs holding a slot now */
  int64_t queued;        /* jobs waiting for admission */
  int64_t peak_active;   /* most jobs that held slots at the same time */
  int64_t bytes_in_use;  /* budget bytes held by active jobs now */
  int64_t peak_bytes;    /* most budget bytes held at the same time */
  int64_t budget_bytes;  /* the context's budget */
  int64_t slots;         /* the context's slot count */
  int64_t ticks;         /* ticks launched (one round of every ticked job each) */
  int64_t ticked_jobs;   /* jobs admitted to ticks so far */
} arpc_serving_stats;

/* Create a serving context on HIP device `device` with a budget of
 * hbm_budget_bytes of device memory for job workspaces (allocated here, once)
 * and at most max_slots concurrently active jobs (1..64).  Errors:
 * ARPC_EINVAL (bad arguments), ARPC_EDEVICE (no such device, or the budget
 * could not be allocated). */
arpc_status arpc_create(int device, size_t hbm_budget_bytes, int max_slots, arpc_ctx* out);

/* Cancel queued jobs, let active jobs finish their current batch of rounds
 * and end as cancelled, stop the scheduler and free the context's memory.
 * Job handles of the context become invalid. */
arpc_status arpc_destroy(arpc_ctx ctx);

/* Queue a job.  Arguments as for arpc_factor (the workspace comes from the
 * context).  Returns ARPC_EINVAL for an invalid problem or pointers,
 * ARPC_ENOMEM when the job's workspace exceeds the whole budget, and
 * ARPC_EBUSY when the context already holds its limit of jobs submitted and
 * not yet finished (arpc_serving_set_limit; 65536 by default): the job is not
 * queued and may be submitted again later. */
arpc_status arpc_submit(arpc_ctx ctx, const arpc_problem* problem, const double* X, void* F, int64_t* pivots,
                        arpc_job* job);

/* Non-blocking completion check.  *done = 1 when the job has finished; then
 * *stats (may be NULL) holds its statistics, with ms_total = milliseconds
 * from submission to completion, and the return value is the job's own
 * status (as arpc_factor would return).  The handle stays valid until
 * arpc_wait or a poll that reports completion returns. */
arpc_status arpc_poll(arpc_ctx ctx, arpc_job job, int* done, arpc_stats* stats);

/* Block until the job finishes; returns its status and fills *stats (may be
 * NULL).  ARPC_EINVAL for an unknown handle. */
arpc_status arpc_wait(arpc_ctx ctx, arpc_job job, arpc_stats* stats);

/* Cancel a job: a queued job ends at once, an active one after its current
 * batch of rounds (its F and pivots are then incomplete).  Its status becomes
 * ARPC_ECANCELED unless it had already finished. */
arpc_status arpc_cancel(arpc_ctx ctx, arpc_job job);

/* Largest number of jobs submitted to ctx and not yet finished (queued or
 * active), 1 <= max_outstanding <= 2^31 - 1; a submission beyond it returns
 * ARPC_EBUSY. */
arpc_status arpc_serving_set_limit(arpc_ctx ctx, int64_t max_outstanding);

/* Snapshot of the context's counters. */
arpc_status arpc_serving_info(arpc_ctx ctx, arpc_serving_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* ARPC_H */
