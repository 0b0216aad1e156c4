// Krylov kernels: CG (Hestenes-Stiefel) and GMRES(m) with classical Gram-Schmidt
// applied twice (Alg. 1 step 4 of arXiv 2309.02156; stopping rule ||b - A x|| <=
// tol ||b||, tested before the first iteration and confirmed with the true residual).
//
// No block waits on another block inside a kernel.  Each streaming kernel writes one
// row of per-block partial sums; the next kernel (or a one-block "close" kernel at the
// end of a polled batch) reduces those rows in a fixed order in every block and
// derives the same scalars everywhere.  Three partial buffers rotate so a kernel
// never overwrites rows that blocks of the same kernel still read.  Within a kernel,
// block 0 persists scalars only into fields that no block of that kernel reads:
// CG keeps rho / beta in rings indexed by the host-supplied iteration number, GMRES
// keeps the raw Hessenberg column, the rotated column and the rotated right-hand side
// in separate arrays.  The run flag is read once per block into LDS.
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace sacc {

constexpr int KTPB = 512;
constexpr int KNW = KTPB / WAVE;
constexpr int KMAXBLK = 256;
constexpr int KW = 64;  // stride of a partial row

static inline int kblocks(int64_t n) {
  int64_t b = (n + KTPB - 1) / KTPB;
  if (b < 1) b = 1;
  return (int)(b > KMAXBLK ? KMAXBLK : b);
}
static inline double *PA(double *P) { return P; }
static inline double *PB(double *P) { return P + (size_t)KMAXBLK * KW; }
static inline double *PC(double *P) { return P + (size_t)2 * KMAXBLK * KW; }

#define KROWS(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

template <typename VT>
__device__ inline double krow_dot(const int *__restrict__ rowptr, const int *__restrict__ col,
                                  const VT *__restrict__ val, const double *__restrict__ x, int64_t i) {
  const int p0 = rowptr[i], p1 = rowptr[i + 1];
  double s = 0.0;
  for (int p = p0; p < p1; ++p) s += (double)val[p] * x[col[p]];
  return s;
}

// block sums of K per-thread values -> out[0..kc) (fixed butterfly, fixed wave order)
template <int K>
__device__ inline void kstore(const double (&v)[K], int kc, double *red, double *out) {
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
#pragma unroll
  for (int e = 0; e < K; ++e)
    if (e < kc) {
      const double s = wave_sum(v[e]);
      if (lane == 0) red[wid * K + e] = s;
    }
  __syncthreads();
  for (int e = threadIdx.x; e < kc; e += blockDim.x) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < KNW; ++w) s += red[w * K + e];
    out[e] = s;
  }
}

// run flag of this block: state == RUN (and active, for GMRES); read once into LDS
__device__ inline bool block_running(const Ctl *ctl, bool need_active) {
  __shared__ int s_run;
  if (threadIdx.x == 0) s_run = (ctl->state == ST_RUN) && (!need_active || ctl->active);
  __syncthreads();
  return s_run != 0;
}

// ============================================================================ CG
template <typename VT>
__global__ __launch_bounds__(KTPB) void k_cg_start(const int *rowptr, const int *col, const VT *val,
                                                   const double *b, const double *x, double *r, double *p,
                                                   int64_t n, int mode, double *Pout, const Ctl *ctl) {
  __shared__ double red[KNW * 2];
  __shared__ int s_go;
  if (threadIdx.x == 0) s_go = (mode != 1) || (ctl->state == ST_CHECK);
  __syncthreads();
  if (!s_go) return;
  double acc[2] = {0.0, 0.0};
  KROWS(i, n) {
    const double bi = b[i];
    const double ri = bi - krow_dot(rowptr, col, val, x, i);
    if (mode != 2) {
      r[i] = ri;
      p[i] = ri;
    }
    acc[0] += ri * ri;
    acc[1] += bi * bi;
  }
  kstore<2>(acc, 2, red, Pout + (size_t)blockIdx.x * KW);
}

// one block: the stopping test before iteration 1 (mode 0), the confirmation of a
// recursive-residual stop (mode 1), or the final residual (mode 2).  k = iterations done.
__global__ __launch_bounds__(KTPB) void k_cg_start_close(const double *Pin, int nblk, int mode, int k, Ctl *ctl) {
  __shared__ double outv[2];
  __shared__ double scratch[KTPB];
  __shared__ int s_go;
  if (threadIdx.x == 0) s_go = (mode != 1) || (ctl->state == ST_CHECK);
  __syncthreads();
  if (!s_go) return;
  final_sum(Pin, nblk, KW, 2, outv, scratch);
  if (threadIdx.x != 0) return;
  const double rho = outv[0];
  if (mode == 0) {
    ctl->bnorm = sqrt(outv[1]);
    ctl->iters = 0;
    ctl->restarts = 0;
  }
  const double bn = ctl->bnorm, nr = sqrt(rho);
  const double rel = bn > 0.0 ? nr / bn : 0.0;
  ctl->relres = rel;
  if (mode == 0) ctl->relres0 = rel;
  if (mode == 2) return;
  ctl->rho[k & 3] = rho;
  if (bn == 0.0)
    ctl->state = ST_ZERO_RHS;
  else if (nr <= ctl->tol * bn)
    ctl->state = ST_CONV;
  else if (!isfinite(nr))
    ctl->state = ST_BREAK;
  else {
    if (mode == 1) ctl->restarts += 1;
    ctl->state = (k >= ctl->maxit) ? ST_MAXIT : ST_RUN;
  }
}

template <typename VT>
__global__ __launch_bounds__(KTPB) void k_cg_qp(const int *rowptr, const int *col, const VT *val, const double *p,
                                                double *q, int64_t n, double *Pout, const Ctl *ctl) {
  __shared__ double red[KNW];
  if (!block_running(ctl, false)) return;
  double acc[1] = {0.0};
  KROWS(i, n) {
    const double qi = krow_dot(rowptr, col, val, p, i);
    q[i] = qi;
    acc[0] += p[i] * qi;
  }
  kstore<1>(acc, 1, red, Pout + (size_t)blockIdx.x * KW);
}

// iteration k: alpha = rho_{k-1} / p^T q; x += alpha p; r -= alpha q; partial r^T r
__global__ __launch_bounds__(KTPB) void k_cg_xr(double *x, double *r, const double *p, const double *q, int64_t n,
                                                const double *Pin, int nblk, int k, double *Pout, Ctl *ctl) {
  __shared__ double red[KNW];
  __shared__ double outv[1];
  __shared__ double scratch[KTPB];
  if (!block_running(ctl, false)) return;
  final_sum(Pin, nblk, KW, 1, outv, scratch);
  const double pq = outv[0];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->iters = k - 1;
      ctl->state = ST_BREAK;
    }
    return;
  }
  const double alpha = ctl->rho[(k - 1) & 3] / pq;
  double acc[1] = {0.0};
  KROWS(i, n) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc[0] += ri * ri;
  }
  kstore<1>(acc, 1, red, Pout + (size_t)blockIdx.x * KW);
}

// decision after iteration k from r_k^T r_k; persisted by one thread of block 0 only.
// returns true when iterating stops (state changes).
__device__ inline bool cg_decide(double rn, int k, Ctl *ctl, bool persist, double *beta_out) {
  const double bn = ctl->bnorm;
  int st = ST_RUN;
  double beta = 0.0;
  if (sqrt(rn) <= ctl->tol * bn)
    st = ST_CHECK;
  else if (!isfinite(rn))
    st = ST_BREAK;
  else {
    beta = rn / ctl->rho[(k - 1) & 3];
    if (k >= ctl->maxit) st = ST_MAXIT;
  }
  if (persist) {
    ctl->iters = k;
    ctl->rho[k & 3] = rn;
    ctl->beta[k & 3] = beta;
    if (st != ST_RUN) ctl->state = st;
  }
  *beta_out = beta;
  return st != ST_RUN;
}

// p = r + beta_k p before iteration k + 1.  fresh: iteration k is not closed yet, so
// reduce its r^T r partials here and take the stopping decision (same in every block).
__global__ __launch_bounds__(KTPB) void k_cg_dir(double *p, const double *r, int64_t n, const double *Pin, int nblk,
                                                 int k, int fresh, Ctl *ctl) {
  __shared__ double outv[1];
  __shared__ double scratch[KTPB];
  __shared__ double s_beta;
  __shared__ int s_stop;
  if (!block_running(ctl, false)) return;
  if (fresh) {
    final_sum(Pin, nblk, KW, 1, outv, scratch);
    if (threadIdx.x == 0) {
      double beta;
      s_stop = cg_decide(outv[0], k, ctl, blockIdx.x == 0, &beta);
      s_beta = beta;
    }
    __syncthreads();
    if (s_stop) return;
  } else {
    if (threadIdx.x == 0) s_beta = ctl->beta[k & 3];
    __syncthreads();
  }
  const double beta = s_beta;
  KROWS(i, n) p[i] = r[i] + beta * p[i];
}

__global__ __launch_bounds__(KTPB) void k_cg_close(const double *Pin, int nblk, int k, Ctl *ctl) {
  __shared__ double outv[1];
  __shared__ double scratch[KTPB];
  if (!block_running(ctl, false)) return;
  final_sum(Pin, nblk, KW, 1, outv, scratch);
  if (threadIdx.x == 0) {
    double beta;
    cg_decide(outv[0], k, ctl, true, &beta);
  }
}

hipError_t launch_cg_start_k(const CsrView &A, const double *b, const double *x, double *r, double *p, int mode,
                             int k, double *partials, Ctl *ctl, hipStream_t st) {
  const int nb = kblocks(A.n);
  if (A.fp32)
    hipLaunchKernelGGL(k_cg_start<float>, dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col, (const float *)A.val, b,
                       x, r, p, A.n, mode, PA(partials), ctl);
  else
    hipLaunchKernelGGL(k_cg_start<double>, dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col, (const double *)A.val,
                       b, x, r, p, A.n, mode, PA(partials), ctl);
  hipLaunchKernelGGL(k_cg_start_close, dim3(1), dim3(KTPB), 0, st, PA(partials), nb, mode, k, ctl);
  return hipGetLastError();
}

// iteration k (1-based): [dir] qp xr
hipError_t launch_cg_iter_k(const CsrView &A, double *x, double *r, double *p, double *q, int k, int with_dir,
                            int fresh, double *partials, Ctl *ctl, hipStream_t st) {
  const int nb = kblocks(A.n);
  if (with_dir)
    hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(KTPB), 0, st, p, r, A.n, PB(partials), nb, k - 1, fresh, ctl);
  if (A.fp32)
    hipLaunchKernelGGL(k_cg_qp<float>, dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col, (const float *)A.val, p, q,
                       A.n, PA(partials), ctl);
  else
    hipLaunchKernelGGL(k_cg_qp<double>, dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col, (const double *)A.val, p,
                       q, A.n, PA(partials), ctl);
  hipLaunchKernelGGL(k_cg_xr, dim3(nb), dim3(KTPB), 0, st, x, r, p, q, A.n, PA(partials), nb, k, PB(partials),
                     ctl);
  return hipGetLastError();
}

hipError_t launch_cg_close_k(double *partials, int64_t n, int k, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_close, dim3(1), dim3(KTPB), 0, st, PB(partials), kblocks(n), k, ctl);
  return hipGetLastError();
}

// ============================================================================ GMRES
template <typename VT>
__global__ __launch_bounds__(KTPB) void k_gm_start(const int *rowptr, const int *col, const VT *val,
                                                   const double *b, const double *x, double *V, int64_t n,
                                                   int restart_mode, double *Pout, const Ctl *ctl) {
  __shared__ double red[KNW * 2];
  __shared__ int s_go;
  if (threadIdx.x == 0) s_go = !restart_mode || ctl->state == ST_RUN;
  __syncthreads();
  if (!s_go) return;
  double acc[2] = {0.0, 0.0};
  KROWS(i, n) {
    const double bi = b[i];
    const double ri = bi - krow_dot(rowptr, col, val, x, i);
    V[i] = ri;
    acc[0] += ri * ri;
    acc[1] += bi * bi;
  }
  kstore<2>(acc, 2, red, Pout + (size_t)blockIdx.x * KW);
}

// one block: stopping test on the (true) residual and set-up of a new cycle
__global__ __launch_bounds__(KTPB) void k_gm_start_close(const double *Pin, int nblk, int restart_mode, Ctl *ctl) {
  __shared__ double outv[2];
  __shared__ double scratch[KTPB];
  __shared__ int s_go;
  if (threadIdx.x == 0) s_go = !restart_mode || ctl->state == ST_RUN;
  __syncthreads();
  if (!s_go) return;
  final_sum(Pin, nblk, KW, 2, outv, scratch);
  if (threadIdx.x != 0) return;
  if (!restart_mode) {
    ctl->bnorm = sqrt(outv[1]);
    ctl->iters = 0;
    ctl->restarts = 0;
  }
  const double beta = sqrt(outv[0]), bn = ctl->bnorm;
  const double rel = bn > 0.0 ? beta / bn : 0.0;
  ctl->relres = rel;
  if (!restart_mode) ctl->relres0 = rel;
  if (bn == 0.0)
    ctl->state = ST_ZERO_RHS;
  else if (beta <= ctl->tol * bn)
    ctl->state = ST_CONV;
  else if (!isfinite(beta))
    ctl->state = ST_BREAK;
  else if (ctl->iters >= ctl->maxit)
    ctl->state = ST_MAXIT;
  else {
    if (restart_mode) ctl->restarts += 1;
    ctl->state = ST_RUN;
    ctl->active = 1;
    ctl->jend = 0;
    ctl->gnext[0] = beta;
    ctl->vs[0] = 1.0 / beta;
  }
}

// Close Arnoldi step j given hn = ||w_j||: rotate the raw column j, new Givens
// rotation, rotated right-hand side, cycle-end test.  `it` = global iteration number
// of step j (1-based).  Every block computes this identically; only `persist` writes.
__device__ inline bool gm_close_step(int j, double hn, int it, Ctl *ctl, bool persist, double *vs_next) {
  const int LD = MAXR + 1;
  double col[MAXR + 1];
  for (int l = 0; l <= j; ++l) col[l] = ctl->Hraw[l + j * LD];
  col[j + 1] = hn;
  for (int l = 0; l < j; ++l) {
    const double t = ctl->cs[l] * col[l] + ctl->sn[l] * col[l + 1];
    col[l + 1] = -ctl->sn[l] * col[l] + ctl->cs[l] * col[l + 1];
    col[l] = t;
  }
  const double a = col[j];
  const double rr = hypot(a, hn);
  double c = 1.0, s = 0.0;
  if (rr != 0.0) {
    c = a / rr;
    s = hn / rr;
  }
  col[j] = rr;
  const double gj = ctl->gnext[j];
  const double gam_j = c * gj, gnext = -s * gj;
  const bool end = fabs(gnext) <= ctl->tol * ctl->bnorm || hn == 0.0 || it >= ctl->maxit ||
                   j + 1 >= ctl->restart || !isfinite(gnext);
  *vs_next = hn > 0.0 ? 1.0 / hn : 0.0;
  if (persist) {
    for (int l = 0; l <= j; ++l) ctl->R[l + j * LD] = col[l];
    ctl->cs[j] = c;
    ctl->sn[j] = s;
    ctl->gam[j] = gam_j;
    ctl->gnext[j + 1] = gnext;
    ctl->vs[j + 1] = *vs_next;
    ctl->iters = it;
    ctl->jend = j + 1;
    if (end) {
      const int m = j + 1;
      double y[MAXR];
      for (int i = m - 1; i >= 0; --i) {
        double acc = (i == j) ? gam_j : ctl->gam[i];
        for (int l = i + 1; l < m; ++l) acc -= ((l == j) ? col[i] : ctl->R[i + l * LD]) * y[l];
        y[i] = acc / ((i == j) ? col[j] : ctl->R[i + i * LD]);
      }
      for (int i = 0; i < m; ++i) ctl->y[i] = y[i];
      ctl->active = 0;
    }
  }
  return end;
}

// step j, kernel 1: [close step j-1 if fresh] w = A v_j into V[:, j+1]; partials V_l^T w
template <typename VT, int RB>
__global__ __launch_bounds__(KTPB) void k_gm_a1(const int *rowptr, const int *col, const VT *val, double *V,
                                                int64_t n, int j, int it, int fresh, const double *Pin, int nblk,
                                                double *Pout, Ctl *ctl) {
  __shared__ double red[KNW * RB];
  __shared__ double outv[1];
  __shared__ double scratch[KTPB];
  __shared__ double s_vs;
  __shared__ int s_end;
  if (!block_running(ctl, true)) return;
  if (fresh) {
    final_sum(Pin, nblk, KW, 1, outv, scratch);
    if (threadIdx.x == 0) {
      double vsn;
      s_end = gm_close_step(j - 1, sqrt(outv[0]), it - 1, ctl, blockIdx.x == 0, &vsn);
      s_vs = vsn;
    }
    __syncthreads();
    if (s_end) return;
  } else {
    if (threadIdx.x == 0) s_vs = ctl->vs[j];
    __syncthreads();
  }
  const double vsj = s_vs;
  const double *vj = V + (size_t)j * n;
  double *w = V + (size_t)(j + 1) * n;
  double acc[RB];
#pragma unroll
  for (int l = 0; l < RB; ++l) acc[l] = 0.0;
  KROWS(i, n) {
    const double s = krow_dot(rowptr, col, val, vj, i) * vsj;
    w[i] = s;
#pragma unroll
    for (int l = 0; l < RB; ++l)
      if (l <= j) acc[l] += V[(size_t)l * n + i] * s;
  }
  kstore<RB>(acc, j + 1, red, Pout + (size_t)blockIdx.x * KW);
}

// kernel 2: h1 = reduce(partials) * vs; w -= sum h1_l v_l; partials V_l^T w
template <int RB>
__global__ __launch_bounds__(KTPB) void k_gm_a2(double *V, int64_t n, int j, const double *Pin, int nblk,
                                                double *Pout, Ctl *ctl) {
  __shared__ double red[KNW * RB];
  __shared__ double outv[RB];
  __shared__ double scratch[KTPB];
  __shared__ double coef[RB];
  if (!block_running(ctl, true)) return;
  final_sum(Pin, nblk, KW, j + 1, outv, scratch);
  for (int l = threadIdx.x; l < RB; l += blockDim.x) {
    const double h1 = (l <= j) ? outv[l] * ctl->vs[l] : 0.0;
    coef[l] = h1 * ((l <= j) ? ctl->vs[l] : 0.0);
    if (blockIdx.x == 0 && l <= j) ctl->h1[l] = h1;
  }
  __syncthreads();
  double *w = V + (size_t)(j + 1) * n;
  double acc[RB];
#pragma unroll
  for (int l = 0; l < RB; ++l) acc[l] = 0.0;
  KROWS(i, n) {
    double vl[RB];
    double wi = w[i];
#pragma unroll
    for (int l = 0; l < RB; ++l) {
      vl[l] = (l <= j) ? V[(size_t)l * n + i] : 0.0;
      wi -= coef[l] * vl[l];
    }
    w[i] = wi;
#pragma unroll
    for (int l = 0; l < RB; ++l) acc[l] += vl[l] * wi;
  }
  kstore<RB>(acc, j + 1, red, Pout + (size_t)blockIdx.x * KW);
}

// kernel 3: h2 = reduce(partials) * vs; raw column j = h1 + h2; w -= sum h2_l v_l; partial ||w||^2
template <int RB>
__global__ __launch_bounds__(KTPB) void k_gm_a3(double *V, int64_t n, int j, const double *Pin, int nblk,
                                                double *Pout, Ctl *ctl) {
  __shared__ double red[KNW];
  __shared__ double outv[RB];
  __shared__ double scratch[KTPB];
  __shared__ double coef[RB];
  if (!block_running(ctl, true)) return;
  final_sum(Pin, nblk, KW, j + 1, outv, scratch);
  for (int l = threadIdx.x; l < RB; l += blockDim.x) {
    const double h2 = (l <= j) ? outv[l] * ctl->vs[l] : 0.0;
    coef[l] = h2 * ((l <= j) ? ctl->vs[l] : 0.0);
    if (blockIdx.x == 0 && l <= j) ctl->Hraw[l + j * (MAXR + 1)] = ctl->h1[l] + h2;
  }
  __syncthreads();
  double *w = V + (size_t)(j + 1) * n;
  double acc[1] = {0.0};
  KROWS(i, n) {
    double wi = w[i];
#pragma unroll
    for (int l = 0; l < RB; ++l)
      if (l <= j) wi -= coef[l] * V[(size_t)l * n + i];
    w[i] = wi;
    acc[0] += wi * wi;
  }
  kstore<1>(acc, 1, red, Pout + (size_t)blockIdx.x * KW);
}

__global__ __launch_bounds__(KTPB) void k_gm_close(const double *Pin, int nblk, int j, int it, Ctl *ctl) {
  __shared__ double outv[1];
  __shared__ double scratch[KTPB];
  if (!block_running(ctl, true)) return;
  final_sum(Pin, nblk, KW, 1, outv, scratch);
  if (threadIdx.x == 0) {
    double vsn;
    gm_close_step(j, sqrt(outv[0]), it, ctl, true, &vsn);
  }
}

template <int RB>
__global__ __launch_bounds__(KTPB) void k_gm_update(double *x, const double *V, int64_t n, const Ctl *ctl) {
  __shared__ double coef[RB];
  __shared__ int s_m;
  if (threadIdx.x == 0) s_m = (ctl->state == ST_RUN) ? ctl->jend : -1;
  __syncthreads();
  const int m = s_m;
  if (m < 0) return;
  for (int l = threadIdx.x; l < RB; l += blockDim.x) coef[l] = (l < m) ? ctl->y[l] * ctl->vs[l] : 0.0;
  __syncthreads();
  KROWS(i, n) {
    double s = x[i];
#pragma unroll
    for (int l = 0; l < RB; ++l)
      if (l < m) s += coef[l] * V[(size_t)l * n + i];
    x[i] = s;
  }
}

hipError_t launch_gm_start(const CsrView &A, const double *b, const double *x, double *V, int restart_mode,
                           double *partials, Ctl *ctl, hipStream_t st) {
  const int nb = kblocks(A.n);
  if (A.fp32)
    hipLaunchKernelGGL(k_gm_start<float>, dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col, (const float *)A.val, b,
                       x, V, A.n, restart_mode, PA(partials), ctl);
  else
    hipLaunchKernelGGL(k_gm_start<double>, dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col, (const double *)A.val,
                       b, x, V, A.n, restart_mode, PA(partials), ctl);
  hipLaunchKernelGGL(k_gm_start_close, dim3(1), dim3(KTPB), 0, st, PA(partials), nb, restart_mode, ctl);
  return hipGetLastError();
}

template <int RB>
static void gm_step_rb(const CsrView &A, double *V, int j, int it, int fresh, double *partials, Ctl *ctl,
                       hipStream_t st) {
  const int nb = kblocks(A.n);
  if (A.fp32)
    hipLaunchKernelGGL((k_gm_a1<float, RB>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col, (const float *)A.val,
                       V, A.n, j, it, fresh, PC(partials), nb, PA(partials), ctl);
  else
    hipLaunchKernelGGL((k_gm_a1<double, RB>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const double *)A.val, V, A.n, j, it, fresh, PC(partials), nb, PA(partials), ctl);
  hipLaunchKernelGGL(k_gm_a2<RB>, dim3(nb), dim3(KTPB), 0, st, V, A.n, j, PA(partials), nb, PB(partials), ctl);
  hipLaunchKernelGGL(k_gm_a3<RB>, dim3(nb), dim3(KTPB), 0, st, V, A.n, j, PB(partials), nb, PC(partials), ctl);
}

// it = global iteration number of step j (1-based)
hipError_t launch_gm_step_it(const CsrView &A, double *V, int j, int it, int fresh, double *partials, Ctl *ctl,
                             hipStream_t st) {
  if (j < 16)
    gm_step_rb<16>(A, V, j, it, fresh, partials, ctl, st);
  else if (j < 32)
    gm_step_rb<32>(A, V, j, it, fresh, partials, ctl, st);
  else
    gm_step_rb<64>(A, V, j, it, fresh, partials, ctl, st);
  return hipGetLastError();
}

hipError_t launch_gm_close_it(double *partials, int64_t n, int j, int it, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_close, dim3(1), dim3(KTPB), 0, st, PC(partials), kblocks(n), j, it, ctl);
  return hipGetLastError();
}

hipError_t launch_gm_update(double *x, const double *V, int64_t n, int restart, Ctl *ctl, hipStream_t st) {
  const int nb = kblocks(n);
  if (restart <= 16)
    hipLaunchKernelGGL(k_gm_update<16>, dim3(nb), dim3(KTPB), 0, st, x, V, n, ctl);
  else if (restart <= 32)
    hipLaunchKernelGGL(k_gm_update<32>, dim3(nb), dim3(KTPB), 0, st, x, V, n, ctl);
  else
    hipLaunchKernelGGL(k_gm_update<64>, dim3(nb), dim3(KTPB), 0, st, x, V, n, ctl);
  return hipGetLastError();
}

size_t krylov_partials_doubles() { return (size_t)3 * KMAXBLK * KW; }

}  // namespace sacc
