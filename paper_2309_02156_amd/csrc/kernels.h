// Host-callable launchers of the device kernels (one sequence, FP64 vectors).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace sacc {

struct CsrView {
  int64_t n, nnz;
  const int *rowptr, *col;
  const void *val;
  int fp32;
  // optional: col[p] - row(p) for every entry, all within 16 bits (the CG kernels then
  // read these instead of col)
  const short *col16 = nullptr;
};

// y = A x
hipError_t launch_spmv(const CsrView &A, const double *x, double *y, hipStream_t st);

// history push: X[:, slot] = x and SX[:, slot] = S x  (Gaussian or SRHT sketch)
// TX = storage type of the history X and basis Q1 (double, or float in the mixed mode)
// zero_rhs != 0: push zero instead of x when ctl's solve ended in the zero right-hand side
// state (for a push enqueued before the host has read that state)
// srht_signs: the sign words of launch_srht_signs (SRHT sketch only)
template <typename TX>
hipError_t launch_push(const double *x, TX *X, double *SX, int64_t n, int64_t ld, int slot, int s, int sketch,
                       uint64_t seed, const long long *srht_rows, const unsigned long long *srht_signs,
                       double *partials, const Ctl *ctl, int zero_rhs, hipStream_t st);

// BF16 Gaussian sketch (mixed mode): G = BF16(normals), s rounded up to 16 rows of
// sketch_bf16_ld(n) entries, generated once; the push streams it through the matrix
// cores and leaves the same partial rows as launch_push (scale 1 / sqrt(s) applied by
// the reduction)
int64_t sketch_bf16_ld(int64_t n);
int sketch_bf16_rows(int s);
hipError_t launch_gen_sketch_bf16(unsigned short *G, int64_t n, int s, uint64_t seed, hipStream_t st);
template <typename TX>
hipError_t launch_push_bf16(const double *x, TX *X, const unsigned short *G, double *SX, int64_t n, int64_t ld,
                            int slot, int s, double *partials, const Ctl *ctl, int zero_rhs, hipStream_t st);

// the SRHT sign words of a sequence (ceil(n / 64) words), once at creation
hipError_t launch_srht_signs(unsigned long long *words, int64_t n, uint64_t seed, hipStream_t st);

// blocks along n of the push kernel (its partial rows per row group)
int push_blocks_x(int64_t n, int s);

// Rows of the range finder's Gaussian stream carried by the history columns (ring-slot
// order) and the stream's epoch; m = 0: no range finder (Z = I)
struct ZRows {
  int row[MAXM];
  int m;
  unsigned epoch;
};

// finish the push (reduce the sketch partials into SX[:, newest]), then QR with column
// pivoting of SX[:, 0:cnt] (or of SX[:, 0:cnt] Z with the range finder) -> k, T1 (in ctl)
hipError_t launch_qrcp(double *SX, int s, int cnt, int newest, double tau, const double *partials, int64_t n,
                       Ctl *ctl, const ZRows &zr, uint64_t seed, hipStream_t st);

// One sequence's QRCP (the arguments of launch_qrcp), for a batched launch
struct QrcpJob {
  double *SX;
  int s, cnt, newest;
  double tau;
  const double *partials;
  int nbx;  // the push kernel's blocks along n (push_blocks_x)
  Ctl *ctl;
  ZRows zr;
  uint64_t seed;
};
// whether the job takes the small instantiation (a batch lists those first)
bool qrcp_job_small(const QrcpJob &j);
// jobs_dev: device copy of jobs_host[0..njobs); block b of a launch runs job b, with the
// same code and results as launch_qrcp of that job
hipError_t launch_qrcp_batch(const QrcpJob *jobs_dev, const QrcpJob *jobs_host, int njobs, hipStream_t st);

// Q1 = X T1 (first ctl->k columns)
template <typename TX>
hipError_t launch_basis(const TX *X, TX *Q1, int64_t n, int64_t ld, int cnt, Ctl *ctl, hipStream_t st);

// partials of Q1^T [Q1 | A Q1 | b] (and [A Q1]^T [A Q1 | b] for minimum residual)
template <typename TX>
hipError_t launch_spmm_gram(const CsrView &A, const TX *Q1, int64_t ld, const double *b, int cnt, int minres,
                            double *partials, int *nblk_out, Ctl *ctl, hipStream_t st);

// entries of one partial row of launch_spmm_gram (Galerkin block, then the minimum-residual one)
int gram_width(int cnt, int minres);

// POD (Alg. 2): partial rows of G = X^T X (cnt x cnt), then, after k_colsum, the
// eigen-decomposition of G and T1 = V_k diag(lam_k)^(-1/2) for the k <= m leading
// eigenvalues above tau lam_1 (in ctl)
template <typename TX>
hipError_t launch_gram_x(const TX *X, int64_t n, int64_t ld, int cnt, double *partials, int *nblk_out,
                         hipStream_t st);
hipError_t launch_pod_eig(int cnt, int m, double tau, Ctl *ctl, hipStream_t st);

// column sums of partials[nblk][W] -> ctl->gram
hipError_t launch_colsum(const double *partials, int nblk, int W, Ctl *ctl, hipStream_t st);

// pivoted Cholesky of G, reduced solve -> c, cX, k2, fallback
hipError_t launch_small_solve(int cnt, int minres, int spd, double tau_c, Ctl *ctl, hipStream_t st);
// one sequence's column sums and reduced solve (the arguments of launch_colsum and
// launch_small_solve), for batched launches
struct SolveJob {
  int cnt, minres, spd;
  double tau_c;
  Ctl *ctl;
  const double *partials;  // the SpMM + Gram kernel's partial rows: nblk rows of W entries
  int nblk, W;
};
hipError_t launch_colsum_batch(const SolveJob *jobs_dev, const SolveJob *jobs_host, int njobs, hipStream_t st);
hipError_t launch_small_solve_batch(const SolveJob *jobs_dev, const SolveJob *jobs_host, int njobs, hipStream_t st);

// x0 = Q1 c (or the fallback)
template <typename TX>
hipError_t launch_x0(const TX *Q1, const TX *X, double *x0, int64_t n, int64_t ld, Ctl *ctl, hipStream_t st);
// one sequence's x0 (the arguments of launch_x0; Q1 and X of the batch's storage type)
struct X0Job {
  const void *Q1, *X;
  double *x0;
  int64_t n, ld;
  const Ctl *ctl;
};
template <typename TX>
hipError_t launch_x0_batch(const X0Job *jobs_dev, const X0Job *jobs_host, int njobs, hipStream_t st);
template <typename TX>
hipError_t launch_to_double(const TX *x, double *y, int64_t n, hipStream_t st);

// mixed mode: outer FP64 residual (r32 = fl32(b - A x)) with its stopping test, and
// the refinement update x += d
hipError_t launch_ir_resid(const CsrView &A, const double *b, const double *x, float *r32, double *partials,
                           int sweep, int max_refine, Ctl *ctl, hipStream_t st);
hipError_t launch_ir_update(double *x, const float *d, int64_t n, hipStream_t st);

// Optional timing of one launch: HIP start/stop events recorded by the launch itself
// (hipExtLaunchKernel), and the index under which the kernel logs that it did its
// work (Ctl::work_log).
struct KTiming {
  hipEvent_t e0, e1;
  int lidx;
};

// Krylov kernels (device-driven: every kernel returns at once unless the control
// block says there is work, so batches may be enqueued ahead of a poll).
// TV = vector storage type (double, or float for the inner solves of the mixed mode).
//
// CG: start(mode) [+ one-block close]; then iterations (two kernels each); after a
// batch, start(mode 1) confirms a recursive-residual stop (no-op unless CHECK).
//   mode 0 start, 1 true-residual confirmation, 2 final residual only.
// p2 holds the two alternating direction vectors (p2 and p2 + padded_ld(n)).
template <typename TV>
hipError_t launch_cg_start_k(const CsrView &A, const TV *b, const TV *x, TV *r, int mode, double *partials,
                             Ctl *ctl, hipStream_t st, int serial = 0, const TV *dinv = nullptr, int chunk = 0);
// tm (may be null) times the direction/SpMV kernel of the iteration.  serial > 0: the
// step's kernel reports serial and what it saw in the control block's progress word.
// dinv (may be null): Jacobi preconditioning, z = dinv * r (the start kernel then also
// forms r^T z); the stopping test stays on ||r||.
template <typename TV>
hipError_t launch_cg_iter(const CsrView &A, TV *x, TV *r, TV *p2, TV *q, double *partials, Ctl *ctl,
                          hipStream_t st, const KTiming *tm = nullptr, int serial = 0, const TV *dinv = nullptr,
                          int chunk = 0);
// The x / r kernel leaves x += alpha p pending (the next p / q kernel applies it for its
// rows); launch_cg_xfix applies it on its own and must precede a true-residual start
// (mode 1 or 2) and the end of a solve.  p2: the two direction buffers.
template <typename TV>
hipError_t launch_cg_xfix(const CsrView &A, TV *x, TV *p2, Ctl *ctl, hipStream_t st);
// chunk: gathers per lane and step of the wave tiles (5, 7 or 9; 0: the heuristic
// cg_tile_chunk).  cg_tile_tune picks it for an operator by timing the start kernel's
// SpMV (mode 2, only partial rows written: b and x are read, r is not written) for each
// value, cached per (n, nnz, value type, vector type); the first call for a shape waits
// for its timing launches.
template <typename TV>
int cg_tile_tune(const CsrView &A, const TV *b, const TV *x, TV *r, double *partials, Ctl *ctl, hipStream_t st);
// dinv[i] = 1 / (sum of row i's entries in column i), 1 where that sum is zero
template <typename TV>
hipError_t launch_jacobi_dinv(const CsrView &A, TV *dinv, hipStream_t st);

// GMRES(m), classical Gram-Schmidt applied twice.  A cycle: start (residual into
// V[:, 0]), steps j = 0..m-1 (first_mode 0 for the first cycle of a solve, 1 for a
// restart), finish (closes step m - 1), update (x += V y).  T is a scratch vector.
template <typename TV>
hipError_t launch_gm_start(const CsrView &A, const TV *b, const TV *x, TV *V, int restart_mode, double *partials,
                           Ctl *ctl, hipStream_t st);
// tm (may be null) times the step's first kernel (SpMV, finalisation, first dots).
// dinv (may be null): right preconditioning, the step's product is A (dinv * v_j)
template <typename TV>
hipError_t launch_gm_step(const CsrView &A, TV *V, TV *T, int64_t ld, int j, int first_mode, double *partials,
                          Ctl *ctl, hipStream_t st, const KTiming *tm = nullptr, int serial = 0,
                          bool norm_w = false, const TV *dinv = nullptr);
// end of a full cycle: F(m) finalise-only, and with close the one-block close of step m - 1
template <typename TV>
hipError_t launch_gm_finish(const CsrView &A, TV *V, TV *T, int64_t ld, int m, double *partials, Ctl *ctl,
                            hipStream_t st, bool close = true);
// x += V y at the end of a cycle; close_last: close step m - 1 first (in every block,
// instead of the finish's one-block close) from F(m)'s partial rows, or with from_g from
// G(m - 1)'s (no F(m) needed; only when gm_norm_in_g(m)).  dinv (may be null): right
// preconditioning, x += dinv * (V y)
template <typename TV>
hipError_t launch_gm_update(TV *x, const TV *V, int64_t n, int64_t ld, int restart, Ctl *ctl, hipStream_t st,
                            double *partials = nullptr, bool close_last = false, bool from_g = false,
                            const TV *dinv = nullptr);
bool gm_norm_in_g(int m);
size_t krylov_partials_doubles();
// row tiles per pass of the GMRES kernel F (1 or 2) for n rows and rb column slots
int gm_f_rows_per_thread(int64_t n, int rb);
// gathers per lane and round of the CG kernels' wave-tile SpMV (their template argument)
int cg_tile_chunk(int64_t n, int64_t nnz);

// ---- learned coefficient predictor (MLP) and the learned initial guess
constexpr int MLP_MAXL = 8;  // linear layers at most
struct MlpDims {
  int n_in, n_hidden, n_layers, n_out, max_batch;  // n_layers hidden layers, n_layers + 1 linear layers
};
// device buffers: parameters (per layer W (out x in, row-major) then b), gradients, Adam
// moments, standardised input / target rows, per-layer pre-activations z and outputs act
// (act[n_layers] is the network output), two gradient buffers
struct MlpBuffers {
  float *P, *G, *am, *av, *xs, *ts;
  float *z[MLP_MAXL], *act[MLP_MAXL];
  float *dz[2];
};
size_t mlp_param_count(const MlpDims &d);
hipError_t launch_mlp_forward(const MlpDims &d, const MlpBuffers &m, int B, hipStream_t st);
hipError_t launch_mlp_backward(const MlpDims &d, const MlpBuffers &m, int B, float *loss, hipStream_t st);
hipError_t launch_mlp_adam(const MlpDims &d, const MlpBuffers &m, float lr, float b1, float b2, float eps, int t,
                           hipStream_t st);
hipError_t launch_mlp_scale(const float *X, int B, int D, const float *mu, const float *sd, float *Y, hipStream_t st);
hipError_t launch_learn_target(const double *SX, int s, const double *partials, int nbx, int cnt_old, int newest_old,
                               int M, int pos, Ctl *ctl, hipStream_t st);
hipError_t launch_learn_features(const Ctl *ctl, int H, int M, int pos, double t, const float *mu, const float *sd,
                                 float *xs, hipStream_t st);
template <typename TX>
hipError_t launch_learn_xpred(const TX *X, int64_t n, int64_t ld, int cnt, int newest, int M, const float *y,
                              const float *mu, const float *sd, double *xp, hipStream_t st);
hipError_t launch_learn_pick(const CsrView &A, const double *b, double *x0, const double *xp, double *partials,
                             Ctl *ctl, hipStream_t st);

// control block reset in device memory: every field zero, then the solver settings, the
// initial state ST_CONV and no history (newest = -1); mirror and guess record unset
hipError_t launch_ctl_reset(Ctl *ctl, double tol, int maxit, int restart, int trust_est, hipStream_t st);
// *p = v in stream order, from a kernel (no host-side copy)
hipError_t launch_set_int(int *p, int v, hipStream_t st);

// packed 16-bit column offsets of A (out: nnz entries) for the CG kernels; *ok is set to
// 0 when an offset does not fit (the caller sets it to 1 first)
hipError_t launch_col_rel16(const CsrView &A, short *out, int *ok, hipStream_t st);

// x = 0 by a fill kernel
hipError_t launch_zero(double *x, int64_t n, hipStream_t st);

// leading dimension of the column-major history, basis and Krylov blocks
int64_t padded_ld(int64_t n);

// partial-buffer size (doubles) the launchers above need for a problem of size n
size_t partials_doubles(int64_t n, int M, int s);


// ---- segmented solve of many independent mixed-precision systems (batched step)
// FP64 refinement around float32 CG / GMRES(m) inner solves for every system of a
// batch in lockstep: one data launch over all systems' rows and one close launch (a
// block per system) per engine step; per-system phase and scalars live in device
// memory.  Each system uses its sequence's own float32 work vectors: kry holds
// max(4, m + 2) columns of ld entries (CG: r, p, p', q; GMRES: V_0..V_m, w), r32 and
// d32 one column each.
struct SegDesc {
  const int *rowptr, *col;
  const float *val;   // float32 operator values (at least one nonzero)
  const double *b;
  double *x;          // in: the initial guess; out: the solution
  float *kry, *r32, *d32;
  double *part;       // set by the engine
  int64_t n, ld, nnz;
  int nblk;           // set by the engine
  int solver, m, max_refine, maxit, icap;
  double tol, itol;
};
// state: ST_CONV / ST_MAXIT / ST_BREAK / ST_ZERO_RHS (x is left to the caller to zero)
struct SegResult {
  int state, iters, restarts, sweeps;
  double relres0, relres;
  double bytes;  // algorithmic bytes of the system's row work in the solve
};
struct SegEngine;
// an engine for systems of sizes n[0..nseg) (all its device and pinned memory).  Returns
// 0, or -1 when device or pinned memory is short.
int seg_engine_create(const int64_t *n, int nseg, SegEngine **out);
void seg_engine_destroy(SegEngine *e);
// Solves every system (desc[i].n must equal the engine's n[i]) on stream st, eager
// launches or replays of one captured hipGraph per chunk of steps; synchronous.
// oversub: the data kernel's grid in multiples of the blocks the device holds at once
// (1..64; 0: the default 8); chunk: gathers per lane of its SpMV tiles (5, 7 or 9);
// rows: rows per work item, 512 or 1024 (any other value: 1024).
hipError_t seg_engine_solve(SegEngine *e, const SegDesc *desc, bool graph, int oversub, int chunk, int rows,
                            hipStream_t st, SegResult *res);

}  // namespace sacc
