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
};

// y = A x
hipError_t launch_spmv(const CsrView &A, const double *x, double *y, hipStream_t st);

// history push: X[:, slot] = x and SX[:, slot] = S x  (Gaussian or SRHT sketch)
// TX = storage type of the history X and basis Q1 (double, or float in the mixed mode)
template <typename TX>
hipError_t launch_push(const double *x, TX *X, double *SX, int64_t n, int64_t ld, int slot, int s, int sketch,
                       uint64_t seed, const long long *srht_rows, double *partials, Ctl *ctl, hipStream_t st);

// finish the push (reduce the sketch partials into SX[:, newest]), then QR with column
// pivoting of SX[:, 0:cnt] -> k, T1 (in ctl)
hipError_t launch_qrcp(double *SX, int s, int cnt, int newest, double tau, const double *partials, int64_t n,
                       Ctl *ctl, hipStream_t st);

// Q1 = X T1 (first ctl->k columns)
template <typename TX>
hipError_t launch_basis(const TX *X, TX *Q1, int64_t n, int64_t ld, int cnt, Ctl *ctl, hipStream_t st);

// partials of Q1^T [Q1 | A Q1 | b] (and [A Q1]^T [A Q1 | b] for minimum residual)
template <typename TX>
hipError_t launch_spmm_gram(const CsrView &A, const TX *Q1, int64_t ld, const double *b, int cnt, int minres,
                            double *partials, int *nblk_out, Ctl *ctl, hipStream_t st);

// column sums of partials[nblk][W] -> ctl->gram
hipError_t launch_colsum(const double *partials, int nblk, int W, Ctl *ctl, hipStream_t st);

// pivoted Cholesky of G, reduced solve -> c, cX, k2, fallback
hipError_t launch_small_solve(int cnt, int minres, int spd, double tau_c, Ctl *ctl, hipStream_t st);

// x0 = Q1 c (or the fallback)
template <typename TX>
hipError_t launch_x0(const TX *Q1, const TX *X, double *x0, int64_t n, int64_t ld, Ctl *ctl, hipStream_t st);
template <typename TX>
hipError_t launch_to_double(const TX *x, double *y, int64_t n, hipStream_t st);

// mixed mode: outer FP64 residual (r32 = fl32(b - A x)) with its stopping test, and
// the refinement update x += d
hipError_t launch_ir_resid(const CsrView &A, const double *b, const double *x, float *r32, double *partials,
                           int sweep, int max_refine, Ctl *ctl, hipStream_t st);
hipError_t launch_ir_update(double *x, const float *d, int64_t n, hipStream_t st);

// Krylov kernels.  Cross-block results travel through per-block partial sums that
// the next kernel reduces (kernel boundaries order them); two partial buffers
// alternate.  A 1-block "close" kernel ends each batch so the host can poll.
//
// CG: start(mode) -> start_close; per iteration [dir] qp xr; batch end: close.
//   mode 0 start, 1 true-residual confirmation, 2 final residual only.
// k = iterations completed before the call (start / confirm / final) or the number
// of the iteration being launched (iter, 1-based), or the last one (close).
// TV = vector storage type (double, or float for the inner solves of the mixed mode).
template <typename TV>
hipError_t launch_cg_start_k(const CsrView &A, const TV *b, const TV *x, TV *r, TV *p, int mode, int k,
                             double *partials, Ctl *ctl, hipStream_t st);
// one iteration; with_dir = 0 right after start/confirm (p = r); fresh = 1 when the
// previous iteration has not been closed (dir reduces its partials itself)
template <typename TV>
hipError_t launch_cg_iter_k(const CsrView &A, TV *x, TV *r, TV *p, TV *q, int k, int with_dir, int fresh,
                            double *partials, Ctl *ctl, hipStream_t st);
hipError_t launch_cg_close_k(double *partials, int64_t n, int k, Ctl *ctl, hipStream_t st);

// GMRES(m), classical Gram-Schmidt applied twice.  it = global iteration number.
template <typename TV>
hipError_t launch_gm_start(const CsrView &A, const TV *b, const TV *x, TV *V, int restart_mode, double *partials,
                           Ctl *ctl, hipStream_t st);
template <typename TV>
hipError_t launch_gm_step_it(const CsrView &A, TV *V, int64_t ld, int j, int it, int fresh, double *partials,
                             Ctl *ctl, hipStream_t st);
hipError_t launch_gm_close_it(double *partials, int64_t n, int j, int it, Ctl *ctl, hipStream_t st);
template <typename TV>
hipError_t launch_gm_update(TV *x, const TV *V, int64_t n, int64_t ld, int restart, Ctl *ctl, hipStream_t st);
size_t krylov_partials_doubles();

// leading dimension of the column-major history, basis and Krylov blocks
int64_t padded_ld(int64_t n);

// partial-buffer size (doubles) the launchers above need for a problem of size n
size_t partials_doubles(int64_t n, int M, int s);

}  // namespace sacc
