// Krylov kernels: CG (Hestenes-Stiefel) and GMRES(m) with classical Gram-Schmidt
// applied twice (Alg. 1 step 4 of arXiv 2309.02156; stopping rule ||b - A x|| <=
// tol ||b||, tested before the first iteration and confirmed with the true residual).
//
// Vectors are stored as TV (double, or float for the inner solves of the mixed
// mode); every arithmetic operation is carried out in double from the stored
// operands and rounded to TV only when a vector is stored.
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

// Row tiles of KTPB rows; every thread of a block runs the same number of tiles, so
// the tile SpMV may synchronise the block.
#define KTILES(r0, n) \
  for (int64_t r0 = (int64_t)blockIdx.x * KTPB; r0 < (n); r0 += (int64_t)gridDim.x * KTPB)

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
template <typename VT, typename TV>
__global__ __launch_bounds__(KTPB) void k_cg_start(const int *rowptr, const int *col, const VT *val,
                                                   const TV *b, const TV *x, TV *r, TV *p, int64_t n, int mode,
                                                   double *Pout, const Ctl *ctl) {
  __shared__ double red[KNW * 2];
  __shared__ double prod[SPMV_CAP];
  __shared__ int s_go;
  if (threadIdx.x == 0) s_go = (mode != 1) || (ctl->state == ST_CHECK);
  __syncthreads();
  if (!s_go) return;
  double acc[2] = {0.0, 0.0};
  KTILES(r0, n) {
    const double ax = tile_spmv(rowptr, col, val, x, n, r0, prod);
    const int64_t i = r0 + threadIdx.x;
    if (i < n) {
      const double bi = (double)b[i];
      const TV rs = (TV)(bi - ax);
      if (mode != 2) {
        r[i] = rs;
        p[i] = rs;
      }
      const double ri = (double)rs;
      acc[0] += ri * ri;
      acc[1] += bi * bi;
    }
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

template <typename VT, typename TV>
__global__ __launch_bounds__(KTPB) void k_cg_qp(const int *rowptr, const int *col, const VT *val, const TV *p,
                                                TV *q, int64_t n, double *Pout, const Ctl *ctl) {
  __shared__ double red[KNW];
  __shared__ double prod[SPMV_CAP];
  if (!block_running(ctl, false)) return;
  double acc[1] = {0.0};
  KTILES(r0, n) {
    const double qi = tile_spmv(rowptr, col, val, p, n, r0, prod);
    const int64_t i = r0 + threadIdx.x;
    if (i < n) {
      const TV qs = (TV)qi;
      q[i] = qs;
      acc[0] += (double)p[i] * (double)qs;
    }
  }
  kstore<1>(acc, 1, red, Pout + (size_t)blockIdx.x * KW);
}

// iteration k: alpha = rho_{k-1} / p^T q; x += alpha p; r -= alpha q; partial r^T r
template <typename TV>
__global__ __launch_bounds__(KTPB) void k_cg_xr(TV *x, TV *r, const TV *p, const TV *q, int64_t n,
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
    x[i] = (TV)((double)x[i] + alpha * (double)p[i]);
    const TV rs = (TV)((double)r[i] - alpha * (double)q[i]);
    r[i] = rs;
    const double ri = (double)rs;
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
template <typename TV>
__global__ __launch_bounds__(KTPB) void k_cg_dir(TV *p, const TV *r, int64_t n, const double *Pin, int nblk, int k,
                                                 int fresh, Ctl *ctl) {
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
  KROWS(i, n) p[i] = (TV)((double)r[i] + beta * (double)p[i]);
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

template <typename TV>
hipError_t launch_cg_start_k(const CsrView &A, const TV *b, const TV *x, TV *r, TV *p, int mode, int k,
                             double *partials, Ctl *ctl, hipStream_t st) {
  const int nb = kblocks(A.n);
  if (A.fp32)
    hipLaunchKernelGGL((k_cg_start<float, TV>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const float *)A.val, b, x, r, p, A.n, mode, PA(partials), ctl);
  else
    hipLaunchKernelGGL((k_cg_start<double, TV>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const double *)A.val, b, x, r, p, A.n, mode, PA(partials), ctl);
  hipLaunchKernelGGL(k_cg_start_close, dim3(1), dim3(KTPB), 0, st, PA(partials), nb, mode, k, ctl);
  return hipGetLastError();
}

// iteration k (1-based): [dir] qp xr
template <typename TV>
hipError_t launch_cg_iter_k(const CsrView &A, TV *x, TV *r, TV *p, TV *q, int k, int with_dir, int fresh,
                            double *partials, Ctl *ctl, hipStream_t st) {
  const int nb = kblocks(A.n);
  if (with_dir)
    hipLaunchKernelGGL(k_cg_dir<TV>, dim3(nb), dim3(KTPB), 0, st, p, r, A.n, PB(partials), nb, k - 1, fresh,
                       ctl);
  if (A.fp32)
    hipLaunchKernelGGL((k_cg_qp<float, TV>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col, (const float *)A.val,
                       p, q, A.n, PA(partials), ctl);
  else
    hipLaunchKernelGGL((k_cg_qp<double, TV>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const double *)A.val, p, q, A.n, PA(partials), ctl);
  hipLaunchKernelGGL(k_cg_xr<TV>, dim3(nb), dim3(KTPB), 0, st, x, r, p, q, A.n, PA(partials), nb, k,
                     PB(partials), ctl);
  return hipGetLastError();
}

hipError_t launch_cg_close_k(double *partials, int64_t n, int k, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_close, dim3(1), dim3(KTPB), 0, st, PB(partials), kblocks(n), k, ctl);
  return hipGetLastError();
}

// ============================================================================ GMRES
template <typename VT, typename TV>
__global__ __launch_bounds__(KTPB) void k_gm_start(const int *rowptr, const int *col, const VT *val,
                                                   const TV *b, const TV *x, TV *V, int64_t n, int restart_mode,
                                                   double *Pout, const Ctl *ctl) {
  __shared__ double red[KNW * 2];
  __shared__ double prod[SPMV_CAP];
  __shared__ int s_go;
  if (threadIdx.x == 0) s_go = !restart_mode || ctl->state == ST_RUN;
  __syncthreads();
  if (!s_go) return;
  double acc[2] = {0.0, 0.0};
  KTILES(r0, n) {
    const double ax = tile_spmv(rowptr, col, val, x, n, r0, prod);
    const int64_t i = r0 + threadIdx.x;
    if (i < n) {
      const double bi = (double)b[i];
      const TV rs = (TV)(bi - ax);
      V[i] = rs;
      const double ri = (double)rs;
      acc[0] += ri * ri;
      acc[1] += bi * bi;
    }
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
// of step j (1-based).  Called by all threads of a block: the inputs are staged in
// LDS in parallel, thread 0 does the scalar recurrence from LDS.  Every block computes
// the same result; only `persist` (block 0) writes.  Returns the cycle-end flag; the
// scale of the next basis vector is left in *s_vs (LDS).
__device__ inline bool gm_close_block(int j, double hn, int it, Ctl *ctl, bool persist, double *s_vs) {
  const int LD = MAXR + 1;
  __shared__ double col[MAXR + 1], cs[MAXR], sn[MAXR];
  __shared__ double s_gj;
  __shared__ int s_endf;
  for (int l = threadIdx.x; l <= j; l += blockDim.x) col[l] = ctl->Hraw[l + j * LD];
  for (int l = threadIdx.x; l < j; l += blockDim.x) {
    cs[l] = ctl->cs[l];
    sn[l] = ctl->sn[l];
  }
  if (threadIdx.x == 0) s_gj = ctl->gnext[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    col[j + 1] = hn;
    for (int l = 0; l < j; ++l) {
      const double t = cs[l] * col[l] + sn[l] * col[l + 1];
      col[l + 1] = -sn[l] * col[l] + cs[l] * col[l + 1];
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
    const double gj = s_gj;
    const double gam_j = c * gj, gnext = -s * gj;
    const bool end = fabs(gnext) <= ctl->tol * ctl->bnorm || hn == 0.0 || it >= ctl->maxit ||
                     j + 1 >= ctl->restart || !isfinite(gnext);
    *s_vs = hn > 0.0 ? 1.0 / hn : 0.0;
    s_endf = end ? 1 : 0;
    if (persist) {
      ctl->cs[j] = c;
      ctl->sn[j] = s;
      ctl->gam[j] = gam_j;
      ctl->gnext[j + 1] = gnext;
      ctl->vs[j + 1] = *s_vs;
      ctl->iters = it;
      ctl->jend = j + 1;
      if (end) ctl->active = 0;
    }
  }
  __syncthreads();
  if (persist)
    for (int l = threadIdx.x; l <= j; l += blockDim.x) ctl->R[l + j * LD] = col[l];
  return s_endf != 0;
}

// step j, kernel 1: [close step j-1 if fresh] w = A v_j into V[:, j+1]; partials V_l^T w
template <typename VT, typename TV, int RB>
__global__ __launch_bounds__(KTPB) void k_gm_a1(const int *rowptr, const int *col, const VT *val, TV *V, int64_t n,
                                                int64_t ld, int j, int it, int fresh, const double *Pin, int nblk,
                                                double *Pout, Ctl *ctl) {
  __shared__ double red[KNW * RB];
  __shared__ double outv[1];
  __shared__ double scratch[KTPB];
  __shared__ double prod[SPMV_CAP];
  __shared__ double s_vs;
  if (!block_running(ctl, true)) return;
  if (fresh) {
    final_sum(Pin, nblk, KW, 1, outv, scratch);
    if (gm_close_block(j - 1, sqrt(outv[0]), it - 1, ctl, blockIdx.x == 0, &s_vs)) return;
  } else {
    if (threadIdx.x == 0) s_vs = ctl->vs[j];
    __syncthreads();
  }
  const double vsj = s_vs;
  const TV *vj = V + (size_t)j * ld;
  TV *w = V + (size_t)(j + 1) * ld;
  double acc[RB];
#pragma unroll
  for (int l = 0; l < RB; ++l) acc[l] = 0.0;
  KTILES(r0, n) {
    const double s = tile_spmv(rowptr, col, val, vj, n, r0, prod) * vsj;
    const int64_t i = r0 + threadIdx.x;
    if (i < n) {
      const TV ws = (TV)s;
      w[i] = ws;
      const double wd = (double)ws;
#pragma unroll
      for (int l = 0; l < RB; ++l)
        if (l <= j) acc[l] += (double)V[(size_t)l * ld + i] * wd;
    }
  }
  kstore<RB>(acc, j + 1, red, Pout + (size_t)blockIdx.x * KW);
}

// kernel 2: h1 = reduce(partials) * vs; w -= sum h1_l v_l; partials V_l^T w
template <typename TV, int RB>
__global__ __launch_bounds__(KTPB) void k_gm_a2(TV *V, int64_t n, int64_t ld, int j, const double *Pin, int nblk,
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
  TV *w = V + (size_t)(j + 1) * ld;
  double acc[RB];
#pragma unroll
  for (int l = 0; l < RB; ++l) acc[l] = 0.0;
  KROWS(i, n) {
    double vl[RB];
    double wi = (double)w[i];
#pragma unroll
    for (int l = 0; l < RB; ++l) {
      vl[l] = (l <= j) ? (double)V[(size_t)l * ld + i] : 0.0;
      wi -= coef[l] * vl[l];
    }
    const TV ws = (TV)wi;
    w[i] = ws;
    const double wd = (double)ws;
#pragma unroll
    for (int l = 0; l < RB; ++l) acc[l] += vl[l] * wd;
  }
  kstore<RB>(acc, j + 1, red, Pout + (size_t)blockIdx.x * KW);
}

// kernel 3: h2 = reduce(partials) * vs; raw column j = h1 + h2; w -= sum h2_l v_l; partial ||w||^2
template <typename TV, int RB>
__global__ __launch_bounds__(KTPB) void k_gm_a3(TV *V, int64_t n, int64_t ld, int j, const double *Pin, int nblk,
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
  TV *w = V + (size_t)(j + 1) * ld;
  double acc[1] = {0.0};
  KROWS(i, n) {
    double wi = (double)w[i];
#pragma unroll
    for (int l = 0; l < RB; ++l)
      if (l <= j) wi -= coef[l] * (double)V[(size_t)l * ld + i];
    const TV ws = (TV)wi;
    w[i] = ws;
    const double wd = (double)ws;
    acc[0] += wd * wd;
  }
  kstore<1>(acc, 1, red, Pout + (size_t)blockIdx.x * KW);
}

__global__ __launch_bounds__(KTPB) void k_gm_close(const double *Pin, int nblk, int j, int it, Ctl *ctl) {
  __shared__ double outv[1];
  __shared__ double scratch[KTPB];
  __shared__ double s_vs;
  if (!block_running(ctl, true)) return;
  final_sum(Pin, nblk, KW, 1, outv, scratch);
  gm_close_block(j, sqrt(outv[0]), it, ctl, true, &s_vs);
}

// End of a cycle: every block solves R y = gam (m x m upper triangular, staged in
// LDS) and adds x += sum_l y_l v_l for its rows.
template <typename TV, int RB>
__global__ __launch_bounds__(KTPB) void k_gm_update(TV *x, const TV *V, int64_t n, int64_t ld, const Ctl *ctl) {
  const int LD = MAXR + 1;
  __shared__ double coef[RB];
  __shared__ double Rs[RB * RB];
  __shared__ double gs[RB];
  __shared__ int s_m;
  if (threadIdx.x == 0) s_m = (ctl->state == ST_RUN) ? ctl->jend : -1;
  __syncthreads();
  const int m = s_m;
  if (m < 0) return;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int i = e % m, l = e / m;
    Rs[i + l * RB] = (i <= l) ? ctl->R[i + l * LD] : 0.0;
  }
  for (int l = threadIdx.x; l < RB; l += blockDim.x) gs[l] = (l < m) ? ctl->gam[l] : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = m - 1; i >= 0; --i) {
      double acc = gs[i];
      for (int l = i + 1; l < m; ++l) acc -= Rs[i + l * RB] * coef[l];
      coef[i] = acc / Rs[i + i * RB];
    }
    for (int i = 0; i < m; ++i) coef[i] *= ctl->vs[i];
    for (int i = m; i < RB; ++i) coef[i] = 0.0;
  }
  __syncthreads();
  KROWS(i, n) {
    double s = (double)x[i];
#pragma unroll
    for (int l = 0; l < RB; ++l)
      if (l < m) s += coef[l] * (double)V[(size_t)l * ld + i];
    x[i] = (TV)s;
  }
}

template <typename TV>
hipError_t launch_gm_start(const CsrView &A, const TV *b, const TV *x, TV *V, int restart_mode, double *partials,
                           Ctl *ctl, hipStream_t st) {
  const int nb = kblocks(A.n);
  if (A.fp32)
    hipLaunchKernelGGL((k_gm_start<float, TV>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const float *)A.val, b, x, V, A.n, restart_mode, PA(partials), ctl);
  else
    hipLaunchKernelGGL((k_gm_start<double, TV>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const double *)A.val, b, x, V, A.n, restart_mode, PA(partials), ctl);
  hipLaunchKernelGGL(k_gm_start_close, dim3(1), dim3(KTPB), 0, st, PA(partials), nb, restart_mode, ctl);
  return hipGetLastError();
}

template <typename TV, int RB>
static void gm_step_rb(const CsrView &A, TV *V, int64_t ld, int j, int it, int fresh, double *partials, Ctl *ctl,
                       hipStream_t st) {
  const int nb = kblocks(A.n);
  if (A.fp32)
    hipLaunchKernelGGL((k_gm_a1<float, TV, RB>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const float *)A.val, V, A.n, ld, j, it, fresh, PC(partials), nb, PA(partials), ctl);
  else
    hipLaunchKernelGGL((k_gm_a1<double, TV, RB>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const double *)A.val, V, A.n, ld, j, it, fresh, PC(partials), nb, PA(partials), ctl);
  hipLaunchKernelGGL((k_gm_a2<TV, RB>), dim3(nb), dim3(KTPB), 0, st, V, A.n, ld, j, PA(partials), nb,
                     PB(partials), ctl);
  hipLaunchKernelGGL((k_gm_a3<TV, RB>), dim3(nb), dim3(KTPB), 0, st, V, A.n, ld, j, PB(partials), nb,
                     PC(partials), ctl);
}

// it = global iteration number of step j (1-based)
template <typename TV>
hipError_t launch_gm_step_it(const CsrView &A, TV *V, int64_t ld, int j, int it, int fresh, double *partials,
                             Ctl *ctl, hipStream_t st) {
  if (j < 16)
    gm_step_rb<TV, 16>(A, V, ld, j, it, fresh, partials, ctl, st);
  else if (j < 32)
    gm_step_rb<TV, 32>(A, V, ld, j, it, fresh, partials, ctl, st);
  else
    gm_step_rb<TV, 64>(A, V, ld, j, it, fresh, partials, ctl, st);
  return hipGetLastError();
}

hipError_t launch_gm_close_it(double *partials, int64_t n, int j, int it, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_close, dim3(1), dim3(KTPB), 0, st, PC(partials), kblocks(n), j, it, ctl);
  return hipGetLastError();
}

template <typename TV>
hipError_t launch_gm_update(TV *x, const TV *V, int64_t n, int64_t ld, int restart, Ctl *ctl, hipStream_t st) {
  const int nb = kblocks(n);
  if (restart <= 16)
    hipLaunchKernelGGL((k_gm_update<TV, 16>), dim3(nb), dim3(KTPB), 0, st, x, V, n, ld, ctl);
  else if (restart <= 32)
    hipLaunchKernelGGL((k_gm_update<TV, 32>), dim3(nb), dim3(KTPB), 0, st, x, V, n, ld, ctl);
  else
    hipLaunchKernelGGL((k_gm_update<TV, 64>), dim3(nb), dim3(KTPB), 0, st, x, V, n, ld, ctl);
  return hipGetLastError();
}

#define SACC_INSTANTIATE_KRYLOV(TV)                                                                              \
  template hipError_t launch_cg_start_k<TV>(const CsrView &, const TV *, const TV *, TV *, TV *, int, int,       \
                                            double *, Ctl *, hipStream_t);                                       \
  template hipError_t launch_cg_iter_k<TV>(const CsrView &, TV *, TV *, TV *, TV *, int, int, int, double *,     \
                                           Ctl *, hipStream_t);                                                  \
  template hipError_t launch_gm_start<TV>(const CsrView &, const TV *, const TV *, TV *, int, double *, Ctl *,   \
                                          hipStream_t);                                                          \
  template hipError_t launch_gm_step_it<TV>(const CsrView &, TV *, int64_t, int, int, int, double *, Ctl *,      \
                                            hipStream_t);                                                        \
  template hipError_t launch_gm_update<TV>(TV *, const TV *, int64_t, int64_t, int, Ctl *, hipStream_t);

SACC_INSTANTIATE_KRYLOV(double)
SACC_INSTANTIATE_KRYLOV(float)

// leading dimension of column-major n-row blocks: rounded to 512 rows plus 576, so
// consecutive columns start 4.5 KB apart modulo any power of two (columns exactly a
// power of two apart map onto the same memory channels)
int64_t padded_ld(int64_t n) { return (n + 511) / 512 * 512 + 576; }

size_t krylov_partials_doubles() { return (size_t)3 * KMAXBLK * KW; }

}  // namespace sacc
