/*
 * sacc - subspace-accelerated Krylov solves for sequences of sparse linear systems
 * A(t_i) x(t_i) = b(t_i), i = 0, 1, 2, ... (Guido, Kressner, Ricci, arXiv 2309.02156,
 * Section 1 eq. (seq)), on AMD Instinct MI355X (gfx950).
 *
 * Per step the library computes an initial guess x0 in the span of the M most recent
 * solutions (Alg. 1 (history, basis and reduced problem); basis from the randomized range finder of Section 2.2
 * orthonormalised by a sketched QR) and then runs CG or restarted GMRES from it
 * (Alg. 1 (Krylov solve)).  All arithmetic of a step runs in HIP kernels on the device.
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev are device pointers (hipMalloc'd memory or a torch CUDA
 *     tensor's data_ptr()); everything else is host memory.
 *   - Vectors are dense, contiguous, length n, float64 unless stated otherwise.
 *   - A CSR matrix has int32 row pointers (n + 1) and int32 column indices (nnz),
 *     values float64 or float32 (val_is_fp32).  Columns need not be sorted.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *     device work of a call is enqueued on that stream; pointers must stay valid until
 *     that work has completed.  One sequence is used by one stream at a time.
 *   - Return codes: 0 success; SA_NOTCONV (positive) when maxit was reached (x holds
 *     the last iterate); negative codes are errors and leave no work half-enqueued
 *     on argument errors.  No C++ exception crosses this interface.
 *   - The library allocates device memory only in sa_init_sequence (small control
 *     blocks); the large buffers live in the caller's workspace.
 */
#ifndef SACC_H
#define SACC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------------- */
#define SA_OK 0
#define SA_NOTCONV 1       /* maxit reached; x holds the last iterate                  */
#define SA_EINVAL (-1)     /* bad argument: shape, size, dtype, m > M, s < M, ...       */
#define SA_ENOMEM (-2)     /* workspace smaller than sa_workspace_bytes reports         */
#define SA_EHIP (-3)       /* a HIP runtime call failed                                 */
#define SA_ESTATE (-4)     /* call out of order (e.g. push before init)                 */
#define SA_EBREAKDOWN (-5) /* CG: p^T A p <= 0 or not finite; GMRES: non-finite residual */
#define SA_ETOOBIG (-6)    /* the problem needs more than the fixed device scratch of an
                              allocation-free call (sa_solve_static)                      */

/* ---- enumerations (stored as int32 in the structs) ----------------------------- */
#define SA_FP64 0          /* every vector and reduction in float64                     */
#define SA_MIXED 1         /* float32 matrix values (val_is_fp32 = 1), history, basis and
                              inner Krylov vectors; float64 arithmetic in registers, the
                              small dense solves and the outer iterative refinement; the
                              Gaussian sketch in BF16 on the matrix cores: its normals G
                              rounded to BF16 once, kept in the workspace
                              (ceil(s / 16) 16 x ceil(n / 64) 64 x 2 bytes), applied to
                              BF16(float32(x)) with FP32 accumulation, S = G / sqrt(s)  */
#define SA_MIXED_KRYLOV 2  /* as SA_MIXED but history and basis in float64: the initial
                              guess keeps FP64 accuracy (float32 storage of the history
                              puts rounding noise of relative size 6e-8 into every guess,
                              amplified by the operator in the residual)                */

#define SA_CG 0            /* conjugate gradients (Hestenes-Stiefel), SPD A             */
#define SA_GMRES 1         /* restarted GMRES(restart), classical Gram-Schmidt twice    */

#define SA_GALERKIN 0      /* reduced problem Q^T A Q y = Q^T b                         */
#define SA_MINRES 1        /* reduced problem min ||A Q y - b||_2 (Section 2): normal
                              equations (A Q)^T (A Q) y = (A Q)^T b from the same SpMM
                              pass, solved by Cholesky                                  */

#define SA_SKETCH_GAUSSIAN 0 /* S[r, j] Gaussian from Philox4x64-10 + Box-Muller      */
#define SA_SKETCH_SRHT 1     /* S = s^-1/2 R H D, n a power of two                     */

#define SA_BASIS_SKETCHED_QR 0 /* QR with column pivoting of the sketch S X (Z), Cholesky finish */
#define SA_PRECOND_NONE 0   /* unpreconditioned Krylov solve                          */
#define SA_PRECOND_JACOBI 1 /* D = diag(A) (zero or missing entries taken as 1): CG on
                               z = D^-1 r, GMRES right-preconditioned on A D^-1, so the
                               stopping test stays on the true residual ||b - A x||   */
#define SA_BASIS_POD 1         /* Alg. 2: the m leading left singular vectors of X, from the
                                  eigen-decomposition of X^T X (FP64); singular values below
                                  1e-7 of the largest are dropped (not resolved through the
                                  Gram); the same Cholesky finish                          */

#define SA_GUESS_PROJECTION 0 /* the method: x0 = Q y                                  */
#define SA_GUESS_ZERO 1       /* x0 = 0                                                 */
#define SA_GUESS_PREVIOUS 2   /* x0 = x(t_{i-1}), the paper's Baseline (Sections 4-5)   */

/* ---- configuration ------------------------------------------------------------- */
typedef struct {
  int64_t n;              /* system size                                              */
  int32_t M;              /* history length (number of previous solutions kept), 1..32 */
  int32_t s;              /* sketch rows, M <= s <= 256, s*M <= 8192; SRHT: s <= n     */
  int32_t sketch;         /* SA_SKETCH_*                                               */
  int32_t projection;     /* SA_GALERKIN or SA_MINRES                                   */
  int32_t solver;         /* SA_CG or SA_GMRES                                         */
  int32_t restart;        /* GMRES restart length, 1..32                               */
  double tol;             /* stop when ||b - A x||_2 <= tol ||b||_2                   */
  int32_t maxit;          /* iteration cap (A-products for CG, Arnoldi steps GMRES)    */
  int32_t precision;      /* SA_FP64, SA_MIXED or SA_MIXED_KRYLOV                      */
  double inner_tol;       /* mixed: inner solve tolerance relative to the current
                             residual, in (0, 1)                                      */
  int32_t max_refine;     /* mixed: cap on refinement sweeps, >= 1                     */
  int32_t guess;          /* SA_GUESS_*                                                */
  double rank_tol_sketch; /* QRCP truncation |R_jj| > tau |R_11| (<= 0: default)      */
  double rank_tol_chol;   /* pivoted-Cholesky truncation relative to max diag (<= 0: default) */
  uint64_t seed;          /* key of the sketch's random entries                        */
  int32_t poll;           /* Krylov steps the host may enqueue ahead of the device (<= 0: default 8) */
  int32_t inner_maxit;    /* mixed: iteration cap of one inner solve (<= 0: 10 GMRES
                             cycles, or 1000 CG iterations)                          */
  int32_t m;              /* range finder (Section 2.2, Alg. 3): 1 <= m < M multiplies the
                             history by an M x m Gaussian Z (each column keeps the row of Z
                             it was given, Alg. 3), so the basis spans X Z; 0 or M: Z = I */
  int32_t refresh;        /* with 1 <= m < M: a new Z every `refresh` pushes once the
                             window is full (<= 0: 50, Section 4)                        */
  int32_t basis;          /* SA_BASIS_SKETCHED_QR, or SA_BASIS_POD (m: the POD dimension,
                             0 = M)                                                      */
  int32_t precond;        /* SA_PRECOND_NONE or SA_PRECOND_JACOBI (mixed modes: from the
                             FP32 operator, stored in FP32)                          */
} sa_config;

typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t *rowptr_dev; /* n + 1 entries, rowptr[0] = 0, non-decreasing          */
  const int32_t *col_dev;    /* nnz entries in [0, n)                                 */
  const void *val_dev;       /* nnz values, float64 or float32                        */
  int32_t val_is_fp32;
  int32_t reserved;
} sa_csr;

typedef struct {
  int32_t iters;         /* Krylov iterations of the last solve (summed over restarts, inner sweeps) */
  int32_t restarts;      /* GMRES restarts / CG restarts after a failed true-residual check */
  int32_t refinements;   /* mixed: outer refinement sweeps                             */
  int32_t k_eff;         /* basis dimension used by the last initial guess             */
  int32_t k_sketch;      /* rank kept by the sketched QRCP                            */
  int32_t used_fallback; /* 1 if the guess fell back to x(t_{i-1}) (non-finite basis)  */
  int32_t status;        /* return code of the last solve                             */
  int32_t history;       /* number of history columns used (min(pushes, M))            */
  double relres0;        /* ||b - A x0|| / ||b|| at the start of the last solve        */
  double relres;         /* final ||b - A x|| / ||b|| (true residual)                  */
  float ms_guess;        /* device time of the last initial guess (segmented batch
                            step: wall time of the batch's whole guess phase)         */
  float ms_solve;        /* device time of the last solve (segmented batch step: wall
                            time of the engine's solve of the whole batch)            */
  int32_t used_learned;  /* 1 if the last guess kept the learned prediction            */
  int32_t reserved;
} sa_info;

/* Timing record of one kernel (sa_profile_read). */
typedef struct {
  char name[48];     /* kernel and template arguments, e.g. "k_gm_f<double, double, 32>" */
  int64_t launches;  /* launches that did their work (early-exit launches excluded)      */
  double ms;         /* summed device time between HIP events around each launch        */
  double bytes;      /* summed algorithmic HBM bytes (each operand byte counted once)     */
} sa_kernel_prof;

typedef struct sa_seq sa_seq;

/* Bytes of device workspace one sequence with this configuration needs.
 * Errors: SA_EINVAL for an invalid configuration. */
int sa_workspace_bytes(const sa_config *cfg, size_t *bytes);

/* Create a sequence with an empty history (Section 2: X holds the M most recent
 * solutions).  dev_ws (caller-owned, >= sa_workspace_bytes, 256-byte aligned) must
 * outlive the sequence.  The sketch's row sample (SRHT) is drawn here on the host.
 * Errors: SA_EINVAL, SA_ENOMEM (ws_bytes too small), SA_EHIP. */
int sa_init_sequence(const sa_config *cfg, void *dev_ws, size_t ws_bytes, void *stream,
                     sa_seq **out);

/* Append the solution x(t_{i-1}) to the history, dropping the oldest one when M are
 * held (the sliding window of Section 2.1), and sketch it (S x) for the next QR.
 * x_dev: n float64 values; SA_MIXED stores them rounded to float32 and sketches the
 * stored values (SA_FP64 and SA_MIXED_KRYLOV keep them in float64).
 * Asynchronous.  Errors: SA_EINVAL (null), SA_ESTATE (destroyed sequence). */
int sa_push_solution(sa_seq *q, const void *x_dev, void *stream);

/* Initial guess of Alg. 1 for the system (A, b): basis Q of span(history) from the
 * sketched QR (the basis of Alg. 1, Section 2.2), reduced problem (the reduced problem
 * of Alg. 1; Galerkin or minimum residual per the config) and x0 = Q y.  Empty history gives x0 = 0.
 * b_dev, x0_dev: float64, length n.  Asynchronous; if info is non-NULL the call waits
 * for the stream and fills k_eff, k_sketch, history, used_fallback, ms_guess.
 * Errors: SA_EINVAL (shape mismatch), SA_EHIP. */
int sa_initial_guess(sa_seq *q, const sa_csr *A, const void *b_dev, void *x0_dev,
                     sa_info *info, void *stream);

/* Krylov solve of A x = b from the iterate in x_dev (Alg. 1 (Krylov solve)): CG or GMRES per
 * the config, stopping on ||b - A x||_2 <= tol ||b||_2 checked before the first
 * iteration and confirmed with the true residual.  x_dev: float64, in = x0, out = x.
 * SA_MIXED, SA_MIXED_KRYLOV: A must carry float32 values; each refinement sweep forms r = b - A x in
 * float64, stops on the test above, else solves A d = fl32(r) with float32-stored
 * vectors until the solver's own residual estimate is below inner_tol ||fl32(r)|| (no
 * true-residual confirmation: the next sweep's residual checks the result) or
 * inner_maxit iterations, and updates x += d (iters sums the inner iterations).
 * CG tunes its SpMV tile shape on the first solve of an operator shape (n, nnz, value
 * and vector types) by timing a few launches that change no solver state (cached for
 * the process; the environment variable SACC_CG_CHUNK = 5, 7 or 9 pins it).  Mixed CG
 * reads the column indices as 16-bit offsets from the row when every offset fits and
 * 2 nnz bytes fit in the workspace region of the basis (n M words): packed once per
 * solve into that region, so the next guess recomputes its basis (the same products in
 * the same order: results as with the 32-bit indices; SACC_NO_COL16 turns it off).
 * Waits for the stream; fills info if non-NULL (iters, restarts, refinements,
 * relres0, relres, status, ms_solve).  Returns SA_OK, SA_NOTCONV or an error code. */
int sa_solve(sa_seq *q, const sa_csr *A, const void *b_dev, void *x_dev, sa_info *info,
             void *stream);

/* One step of Alg. 1 for the system (A, b): initial guess into x_dev, solve from it,
 * push of the solution, in one call (the same work as sa_initial_guess, sa_solve and
 * sa_push_solution in turn, without waiting for the stream between them).  x_dev:
 * float64, length n, out = x.  Fills info if non-NULL (the fields of both calls).
 * The solution is pushed also when the solve reports SA_NOTCONV or SA_EBREAKDOWN.  With
 * GMRES in float64 the push is enqueued before the host reads the solve's final state
 * and the call returns once that state has been read: the push, the sketched QR that
 * follows it and the next step's basis Q1 = X T1 (projection guess; it depends on the
 * history only) may still be running on the stream, and the next guess skips the basis.  Returns the solve's status, or
 * the first error (an error the host detects only from the final state, SA_EHIP, then
 * comes after the push). */
int sa_step(sa_seq *q, const sa_csr *A, const void *b_dev, void *x_dev, sa_info *info, void *stream);

/* Release the sequence's host state and control blocks (not the workspace). */
int sa_destroy_sequence(sa_seq *q);

/* Human-readable name of a status code (static string). */
const char *sa_status_string(int code);

/* y = A x, the building block of every Krylov iteration (Section 1).  x_dev, y_dev:
 * float64, length n; A values float64 or float32.  Asynchronous.
 * Errors: SA_EINVAL, SA_EHIP. */
int sa_spmv(const sa_csr *A, const void *x_dev, void *y_dev, void *stream);

/* Measurement of the Krylov solve's dominant kernels (the SpMV-carrying kernel of
 * each GMRES Arnoldi step and of each CG iteration): with enable = 1, every later
 * sa_solve launches those kernels with HIP start/stop events recorded by the launch
 * itself (hipExtLaunchKernel) on its stream and keeps the launches that did their
 * work, with their algorithmic bytes.  Enabling (or disabling) clears the records.
 * Intended for measurement runs.  Errors: SA_ESTATE, SA_EHIP. */
int sa_profile_enable(sa_seq *q, int enable);

/* Copy up to max records to out; *count = number of records held.
 * Errors: SA_ESTATE, SA_EINVAL. */
int sa_profile_read(sa_seq *q, sa_kernel_prof *out, int max, int *count);

/* ---- learned coefficient predictor (not in the paper) ------------------------------
 * A small MLP that predicts the coefficients of the next solution in the history
 * basis from the coefficients of the previous steps (see sa_learned_attach).  Weights
 * are float32 masters used in bfloat16 (round to nearest even); products accumulate in
 * float32; SiLU hidden activations; mean-squared-error loss; Adam. */
typedef struct sa_mlp sa_mlp;
typedef struct {
  int32_t n_in;      /* inputs (n_hist * M + 2 for the learned guess)                  */
  int32_t n_hidden;  /* width of every hidden layer                                    */
  int32_t n_layers;  /* hidden layers (n_layers + 1 linear layers, at most 8)          */
  int32_t n_out;     /* outputs (M for the learned guess)                              */
  int32_t max_batch; /* rows per forward / training call                               */
  float lr, beta1, beta2, eps;  /* Adam                                                */
  int32_t reserved;
} sa_mlp_config;

/* Create an MLP with initial parameters (host, float32, layer by layer: W_l row-major
 * out x in, then b_l).  Allocates its device memory.  Scaling starts as identity.
 * Errors: SA_EINVAL, SA_ENOMEM, SA_EHIP. */
int sa_mlp_create(const sa_mlp_config *cfg, const float *init_params, sa_mlp **out);
int sa_mlp_destroy(sa_mlp *m);

/* Standardisation of inputs and outputs: the network sees (x - mu_in) / sd_in and is
 * trained on (t - mu_out) / sd_out; predictions are mapped back.  Host float32 arrays
 * of n_in and n_out entries, sd > 0.  Synchronous.  Errors: SA_EINVAL, SA_EHIP. */
int sa_mlp_set_scaling(sa_mlp *m, const float *mu_in, const float *sd_in, const float *mu_out,
                       const float *sd_out);

/* Forward pass of batch rows x_dev (device, float32, batch x n_in, raw) into y_dev
 * (device, float32, batch x n_out, standardised outputs).  Asynchronous. */
int sa_mlp_forward(sa_mlp *m, const float *x_dev, int batch, float *y_dev, void *stream);

/* One Adam step on the batch (x_dev raw inputs, t_dev raw targets, device float32);
 * loss_dev (device float, may be NULL) receives the standardised mean squared error
 * before the step.  Asynchronous.  Errors: SA_EINVAL, SA_EHIP. */
int sa_mlp_train_step(sa_mlp *m, const float *x_dev, const float *t_dev, int batch, float *loss_dev,
                      void *stream);

/* Copy parameters (what = 0), the last gradients (1) or the Adam moments (2, 3) to host
 * (count >= number of parameters).  Waits for the stream. */
int sa_mlp_get(sa_mlp *m, int what, float *host, size_t count, void *stream);

/* Attach a predictor to a fresh sequence (before its first push; guess must be
 * SA_GUESS_PROJECTION).  From then on every push records the step's target, the
 * sketched least-squares coordinates (lag order) of the pushed solution in the history
 * that step used, and once n_hist targets exist every initial guess also evaluates the
 * MLP on the last n_hist targets and sin t, cos t (t from sa_set_time), forms
 * x_pred = X c_pred and keeps it instead of the projection when ||b - A x_pred|| is
 * smaller (info->used_learned).  m = NULL detaches.  m must have n_in = n_hist M + 2 and
 * n_out = M.  Errors: SA_EINVAL, SA_ESTATE. */
int sa_learned_attach(sa_seq *q, sa_mlp *m, int n_hist);

/* Time t of the next system, for the learned guess's inputs.  Errors: SA_ESTATE. */
int sa_set_time(sa_seq *q, double t);

/* ---- batches of independent sequences (Section 5: many plane sequences at once) ----
 * One step of every sequence of the batch (initial guess into x[i], solve, push of the
 * solution), the sequences spread over up to max_streams HIP streams owned by the batch
 * (one host thread each) so that small sequences run concurrently; sequences go to
 * streams longest-first by the estimated cost nnz x (iterations of their last step +
 * 10).  The plan (streams used, Krylov steps enqueued ahead) is tuned on the steps after the
 * first tune_warmup ones: each step from then on times one candidate plan, per Krylov
 * iteration of the batch, until all candidates are timed; the fastest is kept. */
typedef struct sa_batch sa_batch;

/* seqs: nseq sequences created by sa_init_sequence (not owned; each must not be used
 * elsewhere while the batch steps).  Creates the streams and host threads and, when every
 * sequence is SA_MIXED or SA_MIXED_KRYLOV without a preconditioner, the segmented
 * engine's device and pinned memory (descriptors, states, and one partial row of 34
 * float64 per 1024 rows); steps allocate nothing.  Errors: SA_EINVAL, SA_ENOMEM,
 * SA_EHIP. */
int sa_batch_create(sa_seq *const *seqs, int nseq, int max_streams, int tune_warmup, sa_batch **out);
int sa_batch_destroy(sa_batch *b);

/* A[i], rhs[i] (float64, device), x[i] (float64, device; out: the solution); info
 * (nseq entries, may be NULL) receives each sequence's solve info.  Synchronous.
 * Returns SA_OK when every sequence's guess, solve and push ran (a solve that stopped
 * at maxit or broke down is reported in its info.status), else the first error. */
int sa_batch_step(sa_batch *b, const sa_csr *const *A, const void *const *rhs, void *const *x,
                  sa_info *info);

/* The plan in use, whether tuning has finished (always, in a fixed mode) and whether the
 * solves run in the segmented engine: *segmented = 0, or the rows of the engine's work
 * items (512 or 1024, picked by the tuner; 1024 in the fixed segmented modes). */
int sa_batch_plan(const sa_batch *b, int *streams, int *poll, int *tuned, int *segmented);

/* Execution of a batch's solves.
 *   SA_BATCH_AUTO: the tuner times the stream plans and, where every sequence is
 *     SA_MIXED or SA_MIXED_KRYLOV without a preconditioner, the segmented ones (host
 *     threads for the guesses, the engine's grid size), and keeps the fastest (the
 *     default);
 *   SA_BATCH_STREAMS: every sequence's solve on its own stream (max_streams threads);
 *   SA_BATCH_SEGMENTED: the solves of all sequences advanced together by the
 *     segmented engine: per engine step one launch over the rows of every unfinished
 *     system and one launch with a block per system that reduces its partial sums and
 *     picks its next phase (residual, CG or GMRES inner step, update), the systems'
 *     phases and scalars kept in device memory; the host replays a captured hipGraph of
 *     16 engine steps until every system has stopped.  Same method, stopping rules and
 *     counts as sa_solve's mixed mode (GMRES with classical Gram-Schmidt twice), with
 *     its own reduction order;
 *   SA_BATCH_SEGMENTED_EAGER: the same launches without the graph (bitwise the same
 *     results).
 * The guesses and pushes of a segmented step run on the batch's streams, except the
 * sketched QR of every push and the column sums, reduced solve and x0 of every
 * projection guess, which run as one launch each on the first stream (the same code as
 * one sequence's).  A step whose
 * matrices include one without nonzeros runs on streams.  Errors: SA_EINVAL (segmented
 * modes for a batch with an FP64 or preconditioned sequence). */
#define SA_BATCH_AUTO 0
#define SA_BATCH_STREAMS 1
#define SA_BATCH_SEGMENTED 2
#define SA_BATCH_SEGMENTED_EAGER 3
int sa_batch_set_mode(sa_batch *b, int mode);

/* The last step's segmented solve: its algorithmic bytes (the CSR arrays once and every
 * Krylov vector read or written once per phase of each system; FP64 x and b, float32
 * values and columns) and its host wall time in ms, from the first engine launch to the
 * end of the last; both 0 when the last step ran on streams.  Errors: SA_EINVAL. */
int sa_batch_solve_stats(const sa_batch *b, double *bytes, double *ms);

/* Copy internal state to host memory for inspection:
 *   what = 0: SX, s x M float64 column-major, columns in ring-slot order;
 *   what = 1: X, n x M column-major in ring-slot order, float32 for SA_MIXED, else
 *             float64;
 *   what = 2: coefficients c of the last guess in history (ring-slot) coordinates,
 *             M float64 (x0 = X c);
 *   what = 3: ring order, M int32: slot of the oldest .. newest column (-1 unused);
 *   what = 4: the learned target of the last push, M float64 in lag order
 *             (SA_ESTATE without an attached predictor or before the first push).
 * Waits for the stream.  Errors: SA_EINVAL (bytes too small or unknown what). */
int sa_copy_state(sa_seq *q, int what, void *host_dst, size_t bytes, void *stream);

/* ---- checkpoint / resume -------------------------------------------------------------
 * The state a sequence carries between steps (Section 2: the window of the M most recent
 * solutions; the sketch S X and the sketched QR of the window; the learned predictor's
 * recent targets), so that a run can stop and resume: after sa_import_state a fresh
 * sequence of the same configuration computes bit for bit the guesses and solves the
 * exporting one would have.  The image is host memory in this library's own layout: a
 * header (a magic word, the configuration, the push count), X (n x M in ring-slot
 * order, float32 for SA_MIXED, else float64), S X (s x M float64), the projection part
 * of the control block.  The predictor's weights are not part of it (sa_mlp_get).
 *
 * sa_state_bytes: size of the image.  Errors: SA_ESTATE, SA_EINVAL.
 * sa_export_state: writes the image to host_dst (>= sa_state_bytes); waits for the
 *   stream.  Errors: SA_ESTATE, SA_EINVAL (too small), SA_EHIP.
 * sa_import_state: loads an image into q, which must have the configuration the image
 *   was exported with (n, M, s, sketch, precision and seed equal; solver settings may
 *   differ); waits for the stream.  Errors: SA_ESTATE, SA_EINVAL (not an image of this
 *   library, another configuration, too small), SA_EHIP. */
int sa_state_bytes(const sa_seq *q, size_t *bytes);
int sa_export_state(sa_seq *q, void *host_dst, size_t bytes, void *stream);
int sa_import_state(sa_seq *q, const void *host_src, size_t bytes, void *stream);

/* ---- allocation-free solve ----------------------------------------------------------
 * For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): the Krylov solve of sa_solve for one
 * system, without a sequence.  Its control block, partial sums and Krylov vectors live
 * in one fixed device array inside the library (32 MiB per device, held by each device
 * the library runs on until the process ends); nothing is allocated, by the library or
 * through any other library, during the call.  The caller passes the inputs and the
 * output only.
 *
 * cfg: as for sa_init_sequence, precision SA_FP64 (history fields unused: no initial
 * guess is formed; x_dev holds x0 on entry and x on return).  A, b_dev, x_dev, info,
 * stream: as for sa_solve.  The call waits for the stream (the host keeps cfg->poll
 * Krylov steps in flight, then reads the solver state with a synchronous copy).
 * Results equal sa_solve's on a fresh sequence of the same configuration: the same
 * kernels run in the same order on the same partial-sum layout.
 *
 * Every call on one device shares that device's array and leaves its last contents
 * there (each call resets the control block first): calls that overlap on one device,
 * from several host threads or streams, race and give undefined results.
 *
 * Errors: SA_EINVAL (invalid configuration, precision other than SA_FP64, null
 * pointers, shape mismatch), SA_ETOOBIG (the Krylov vectors, partial sums and control
 * block need more than the array holds; sa_static_scratch_bytes reports both sizes),
 * SA_EHIP.  Returns SA_OK, SA_NOTCONV or SA_EBREAKDOWN as sa_solve does. */
int sa_solve_static(const sa_config *cfg, const sa_csr *A, const void *b_dev, void *x_dev, sa_info *info,
                    void *stream);

/* Bytes of the fixed array a configuration needs (*need) and what the array holds
 * (*capacity).  Host only.  Errors: SA_EINVAL. */
int sa_static_scratch_bytes(const sa_config *cfg, size_t *need, size_t *capacity);

#ifdef __cplusplus
}
#endif

#endif /* SACC_H */
