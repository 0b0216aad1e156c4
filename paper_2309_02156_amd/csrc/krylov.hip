// Krylov kernels: CG (Hestenes-Stiefel) and GMRES(m) with classical Gram-Schmidt
// applied twice (Alg. 1 (Krylov solve) of arXiv 2309.02156; stopping rule ||b - A x|| <=
// tol ||b||, tested before the first iteration and confirmed with the true residual).
//
// Vectors are stored as TV (double, or float for the inner solves of the mixed
// mode); every arithmetic operation is carried out in double from the stored
// operands and rounded to TV only when a vector is stored.
//
// The iteration is driven from the device: every kernel reads the solver state from
// the control block and returns at once when there is nothing left to do, so the
// host can enqueue whole batches (and a batch ahead) without waiting for a poll.
//
// No block waits on another block inside a kernel.  Each streaming kernel writes one
// row of per-block partial sums; the next kernel reduces those rows in a fixed order
// in every block and derives the same scalars everywhere.  Two partial buffers
// alternate so a kernel never overwrites rows that blocks of the same kernel still
// read.  Within a kernel, block 0 persists scalars only into fields that no block of
// that kernel reads.
#include <hip/hip_ext.h>
#include <math.h>

#include <stdlib.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace sacc {

constexpr int KTPB = 512;
constexpr int KNW = KTPB / WAVE;
constexpr int KMAXBLK = 256;
constexpr int KW = 64;  // stride of a partial row
// CG kernels: wave tiles, up to four blocks of KTPB threads per compute unit (each
// block's LDS is its waves' product slices), so up to 1024 partial rows
constexpr int CG_MAXBLK = 1024;
constexpr int PROWS = CG_MAXBLK > KMAXBLK ? CG_MAXBLK : KMAXBLK;  // rows of each partial buffer

static inline int kblocks(int64_t n) {
  int64_t b = (n + KTPB - 1) / KTPB;
  if (b < 1) b = 1;
  return (int)(b > KMAXBLK ? KMAXBLK : b);
}
static inline int cgblocks(int64_t n) { return wave_tile_blocks(n, KTPB, CG_MAXBLK); }
static inline double *PA(double *P) { return P; }
static inline double *PB(double *P) { return P + (size_t)PROWS * KW; }

#define KROWS(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// Row tiles of KTPB rows; every thread of a block runs the same number of tiles, so
// the tile SpMV may synchronise the block.
#define KTILES(r0, n) \
  for (int64_t r0 = (int64_t)blockIdx.x * KTPB; r0 < (n); r0 += (int64_t)gridDim.x * KTPB)

// block sums of K per-thread values -> out[0..kc) (K a power of two)
template <int K>
__device__ inline void kstore(double (&v)[K], int kc, double *red, double *out) {
  block_sum_store<K>(v, kc, red, out);
}

// block sums of two values and RB dots -> out[0], out[1], out[2 + k] (first kc entries)
template <int RB>
__device__ inline void kstore2(double (&ex)[2], double (&dots)[RB], int kc, double *red, double *out) {
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  constexpr int STEP = WAVE / RB;
  wave_sum_multi<2>(ex);
  wave_sum_multi<RB>(dots);
  double *rw = red + wid * (RB + 2);
  if (lane % 32 == 0) rw[lane / 32] = ex[0];
  if (lane % STEP == 0) rw[2 + lane / STEP] = dots[0];
  __syncthreads();
  for (int e = threadIdx.x; e < kc; e += blockDim.x) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < KNW; ++w) s += red[w * (RB + 2) + e];
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

// Stopping test on a true residual ||r||^2 = rho (and ||b||^2 = bb when first): the
// state after a start (mode 0), after a confirmation (mode 1, runs only in state
// CHECK) or the final residual (mode 2, norms only).  k = iterations done.
// accept: the recursive estimate already met the tolerance and the control block
// trusts it (inner solves of the mixed mode), so the solve ends converged.  Returns
// the new state; `persist` writes it (one thread of one block).
// The control-block fields the decision reads, loaded by the caller (with its other
// first-trip loads, or by decide_in).
struct DecideIn {
  double bnorm, tol;
  int iters, maxit, restarts;
};

__device__ inline DecideIn decide_in(const Ctl *ctl, int z) {
  return DecideIn{vread(&ctl->bnorm, z), vread(&ctl->tol, z), vread(&ctl->iters, z), vread(&ctl->maxit, z),
                  vread(&ctl->restarts, z)};
}

__device__ inline int residual_decide(double rho, double bb, int mode, const DecideIn &in, Ctl *ctl, bool persist,
                                      bool accept = false) {
  const int k = mode == 0 ? 0 : in.iters;
  const double bn = mode == 0 ? sqrt(bb) : in.bnorm;
  const double nr = sqrt(rho);
  const double rel = bn > 0.0 ? nr / bn : 0.0;
  int st;
  if (bn == 0.0)
    st = ST_ZERO_RHS;
  else if (nr <= in.tol * bn)
    st = ST_CONV;
  else if (!isfinite(nr))
    st = ST_BREAK;
  else
    st = (k >= in.maxit) ? ST_MAXIT : ST_RUN;
  if (accept && mode == 1 && (st == ST_RUN || st == ST_MAXIT)) st = ST_CONV;
  if (persist) {
    if (mode == 0) {
      ctl->bnorm = bn;
      ctl->relres0 = rel;
      ctl->iters = 0;
      ctl->restarts = 0;
    }
    ctl->relres = rel;
    if (mode != 2) ctl->state = st;
    if (mode == 1 && st == ST_RUN) ctl->restarts = in.restarts + 1;
  }
  return st;
}

__device__ inline int residual_decide(double rho, double bb, int mode, Ctl *ctl, bool persist, bool accept = false) {
  return residual_decide(rho, bb, mode, decide_in(ctl, vzero()), ctl, persist, accept);
}

// entry e (0..3) of a 4-entry register array without dynamic indexing
__device__ inline double pick4(const double (&r)[4], int e) {
  return e == 0 ? r[0] : (e == 1 ? r[1] : (e == 2 ? r[2] : r[3]));
}

// ============================================================================ CG
// Two streaming kernels per iteration k (1-based, numbered on the device):
//   cg_p(k):  r_{k-1}^T r_{k-1} from the previous partials -> stopping test, beta;
//             p_k = r + beta p_{k-1} (p double-buffered by the parity of k) and
//             q = A p_k, the SpMV gathering r + beta p_{k-1} for the neighbours;
//             partial p_k^T q.
//   cg_xr(k): alpha = r^T r / p^T q; x += alpha p; r -= alpha q; partial r^T r.
// start: r = b - A x with partial ||r||^2, ||b||^2; a one-block close decides.  After a
// recursive-residual stop (state CHECK) the host's batch-end confirmation recomputes
// the true residual; if it fails the direction restarts (p = r).

template <typename VT, typename TV, int C, bool PC, typename IT>
__global__ __launch_bounds__(KTPB) void k_cg_start(const int *rowptr, const IT *col, const VT *val,
                                                   const TV *b, const TV *x, TV *r, int64_t n, int mode,
                                                   double *Pout, Ctl *ctl, const TV *dinv) {
  __shared__ double red[KNW * 4];
  __shared__ int lcol[KNW * WT_CAP];
  __shared__ VT lval[KNW * WT_CAP];
  __shared__ int s_go;
  if (threadIdx.x == 0) {
    s_go = (mode != 1) || (ctl->state == ST_CHECK);
    // modes 1 and 2 follow the fix-up kernel: the pending x update is in x now (no other
    // block of this launch reads the mark)
    if (blockIdx.x == 0 && mode != 0) ctl->cg_xdone = ctl->cg_xk;
  }
  __syncthreads();
  if (!s_go) return;
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  int *lc = lcol + (size_t)wid * WT_CAP;
  VT *lv = lval + (size_t)wid * WT_CAP;
  (void)lane;
  const Gather1<TV> gx{x};
  // ||r||^2, ||b||^2 and (preconditioned) r^T z with z = D^-1 r
  constexpr int K = PC ? 4 : 2;
  double acc[K] = {};
  const WaveTiles wt = wave_tiles(n);
  wave_tiles_spmv<C>(
      rowptr, col, val, gx, n, wt.t, wt.end, wt.step, lc, lv,
      [&](int64_t i) { return (double)b[i]; },
      [&](int64_t i, double bi, double ax) {
        const TV rs = (TV)(bi - ax);
        if (mode != 2) r[i] = rs;
        const double ri = (double)rs;
        acc[0] += ri * ri;
        acc[1] += bi * bi;
        if constexpr (PC) acc[K - 2] += ri * ((double)dinv[i] * ri);
      });
  kstore<K>(acc, PC ? 3 : 2, red, Pout + (size_t)blockIdx.x * KW);
}

__global__ __launch_bounds__(KTPB) void k_cg_start_close(const double *Pin, int nblk, int mode, Ctl *ctl,
                                                         int serial, int pc) {
  __shared__ double outv[3];
  __shared__ double scratch[KTPB];
  __shared__ int s_go, s_st;
  if (threadIdx.x == 0) {
    s_st = ctl->state;
    s_go = (mode != 1) || (s_st == ST_CHECK);
  }
  __syncthreads();
  if (!s_go) {
    if (threadIdx.x == 0) mirror_report(ctl->mirror, serial, s_st == ST_RUN ? 0u : MIR_STOPPED);
    return;
  }
  final_sum(Pin, nblk, KW, pc ? 3 : 2, outv, scratch);
  if (threadIdx.x != 0) return;
  const int st = residual_decide(outv[0], outv[1], mode, ctl, true, ctl->trust_est != 0);
  if (mode == 0) ctl->cg_xk = ctl->cg_xdone = 0;  // a new solve: no x update pending
  if (mode != 2 && st == ST_RUN) {
    const int k = ctl->iters;
    ctl->rho[k & 3] = pc ? outv[2] : outv[0];  // r^T z (z = r without the preconditioner)
    ctl->fresh_at = k + 1;
  }
  if (mode != 2) mirror_report(ctl->mirror, serial, st == ST_RUN ? 0u : MIR_STOPPED);
}

template <typename TV, bool PC>
struct GatherDir {
  const TV *__restrict__ r;
  const TV *__restrict__ p;
  const TV *__restrict__ dinv;  // Jacobi: z = D^-1 r (PC)
  double beta;
  int fresh;
  // the direction entry as it is stored (rounded to TV), so q = A p uses the same p:
  // p = z + beta p_old, or p = z when the direction restarts.  Every entry is loaded
  // unconditionally: with the load of p[c] under the branch on `fresh` the compiler
  // waited for each gather before issuing the next one.
  // (returned in TV: the value is a TV in any case)
  __device__ TV operator()(int c) const {
    const unsigned u = (unsigned)c;
    const double rv = (double)r[u];
    const double pv = (double)p[u];
    double zv = rv;
    if constexpr (PC) zv = (double)dinv[u] * rv;
    const TV d = (TV)(zv + beta * pv);
    return fresh ? (TV)zv : d;
  }
};

// C = gathers per lane and round of a wave tile
// Also applies the x update of the previous iteration, x += alpha_{k-1} p_{k-1}, for its
// own rows (the x / r kernel leaves it pending: p_{k-1} is this kernel's input direction).
template <typename VT, typename TV, int C, bool PC, typename IT>
__global__ __launch_bounds__(KTPB) void k_cg_p(const int *rowptr, const IT *col, const VT *val, const TV *r,
                                               TV *P0, TV *P1, TV *q, int64_t n, const double *Pin, int nblk,
                                               double *Pout, Ctl *ctl, int lidx, const TV *dinv, TV *x) {
  __shared__ double red[KNW];
  __shared__ double outv[2];
  __shared__ double scratch[KTPB];
  __shared__ int lcol[KNW * WT_CAP];
  __shared__ VT lval[KNW * WT_CAP];
  __shared__ int s_k, s_fresh, s_go, s_cont, s_maxit, s_xpend;
  __shared__ double s_beta, s_tolb, s_rho2, s_alpha;
  // r^T r (and r^T z) of the previous iteration (unused when the direction restarts),
  // loaded together with the control block, and the row pointers of this wave's first
  // tile (they arrive during the prologue)
  const double part = final_part<2>(Pin, nblk, KW, PC ? 2 : 1);
  const WaveTiles wt = wave_tiles(n);
  const TileRows0 first = wave_tile_first_rows(rowptr, n, wt.t < wt.end ? wt.t : 0);
  if (threadIdx.x == 0) {
    // every control-block read of the kernel, issued together
    const int st = ctl->state, it = ctl->iters, fa = ctl->fresh_at, mx = ctl->maxit;
    const int xk = ctl->cg_xk, xd = ctl->cg_xdone;
    const double tol = ctl->tol, bn = ctl->bnorm, al = ctl->cg_alpha;
    s_xpend = xk == it && xk > xd;  // the previous iteration's x update, not yet applied
    s_alpha = al;
    double r4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) r4[e] = ctl->rho[e];
    s_go = st == ST_RUN;
    s_k = it + 1;
    s_fresh = (it + 1 == fa);
    s_maxit = mx;
    s_tolb = tol * bn;
    s_rho2 = pick4(r4, (it + 3) & 3);  // rho of iteration k - 2 = it - 1
  }
  __syncthreads();
  if (!s_go) return;
  const int k = s_k, fresh = s_fresh;
  if (!fresh) final_tree(part, PC ? 2 : 1, outv, scratch);
  if (threadIdx.x == 0) {
    int st = ST_RUN;
    double beta = 0.0;
    if (!fresh) {
      const double rr = outv[0], rho = PC ? outv[1] : outv[0];  // ||r||^2 decides; r^T z gives beta
      if (sqrt(rr) <= s_tolb)
        st = ST_CHECK;
      else if (!isfinite(rr) || !isfinite(rho))
        st = ST_BREAK;
      else
        beta = rho / s_rho2;
      if (blockIdx.x == 0) ctl->rho[(k - 1) & 3] = rho;
    }
    if (st == ST_RUN && k - 1 >= s_maxit) st = ST_MAXIT;
    if (blockIdx.x == 0) {
      if (st != ST_RUN) ctl->state = st;
      ctl->kcur = k;
    }
    s_cont = st == ST_RUN;
    s_beta = beta;
  }
  __syncthreads();
  if (!s_cont) return;
  if (lidx >= 0 && blockIdx.x == 0 && threadIdx.x == 0) ctl->work_log[lidx] = 1;
  const double beta = s_beta, alpha = s_alpha;
  const int xpend = s_xpend;
  const TV *pin = (k & 1) ? P0 : P1;
  TV *pout = (k & 1) ? P1 : P0;
  const GatherDir<TV, PC> gx{r, pin, dinv, beta, fresh};
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  int *lc = lcol + (size_t)wid * WT_CAP;
  VT *lv = lval + (size_t)wid * WT_CAP;
  (void)lane;
  double acc[1] = {0.0};
  // the row's own direction entry is requested with the tile's gathers (exact: gx rounds
  // to TV); the next tile's index loads overlap this tile's gathers
  wave_tiles_spmv<C>(
      rowptr, col, val, gx, n, wt.t, wt.end, wt.step, lc, lv, [&](int64_t i) { return gx((int)i); },
      [&](int64_t i, double pv, double qi) {
        const TV ps = (TV)pv;
        pout[i] = ps;
        const TV qs = (TV)qi;
        q[i] = qs;
        acc[0] += (double)ps * (double)qs;
        if (xpend) x[i] = (TV)((double)x[i] + alpha * (double)pin[i]);
      },
      &first);
  kstore<1>(acc, 1, red, Pout + (size_t)blockIdx.x * KW);
}

// The pending x update, applied on its own (before a true-residual check and at the end
// of a solve): x += alpha p of iteration cg_xk unless that was applied already.  The
// start kernel that follows (modes 1 and 2) marks it applied: a mark written here could
// reach blocks of this same launch that have not read the state yet.
template <typename TV>
__global__ __launch_bounds__(KTPB) void k_cg_xfix(TV *x, const TV *P0, const TV *P1, int64_t n, const Ctl *ctl) {
  __shared__ int s_go, s_k;
  __shared__ double s_alpha;
  if (threadIdx.x == 0) {
    const int xk = ctl->cg_xk, xd = ctl->cg_xdone;
    s_go = xk > xd;
    s_k = xk;
    s_alpha = ctl->cg_alpha;
  }
  __syncthreads();
  if (!s_go) return;
  const TV *p = (s_k & 1) ? P1 : P0;
  const double alpha = s_alpha;
  GRID_ROWS(i, n) x[i] = (TV)((double)x[i] + alpha * (double)p[i]);
}

// U = rows each thread takes per pass (all their loads issued before the first use)
template <typename TV, int U, bool PC>
__global__ __launch_bounds__(KTPB) void k_cg_xr(TV *x, TV *r, const TV *P0, const TV *P1, const TV *q, int64_t n,
                                                const double *Pin, int nblk, double *Pout, Ctl *ctl, int serial,
                                                const TV *dinv) {
  __shared__ double red[KNW * 2];
  __shared__ double outv[1];
  __shared__ double scratch[KTPB];
  __shared__ int s_k, s_go, s_st;
  __shared__ double s_rho;
  const double part = final_part<2>(Pin, nblk, KW, 1);  // p^T q, loaded with the control block
  // the first pass's r and q (they do not depend on alpha) go out before the reduction
  // (loads at clamped indices, unconditional; unused when the solve has stopped)
  TV r1[U], q1[U], d1[U];
  const int64_t rfirst = (int64_t)blockIdx.x * (U * KTPB);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = rfirst + (int64_t)u * KTPB + threadIdx.x;
    const int64_t ic = i < n ? i : n - 1;
    r1[u] = r[ic];
    q1[u] = q[ic];
    if constexpr (PC) d1[u] = dinv[ic];
  }
  if (threadIdx.x == 0) {
    const int st = ctl->state, k = ctl->kcur;
    double r4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) r4[e] = ctl->rho[e];
    s_go = st == ST_RUN;
    s_st = st;
    s_k = k;
    s_rho = pick4(r4, (k - 1) & 3);
  }
  __syncthreads();
  if (!s_go) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
      mirror_report(ctl->mirror, serial, s_st == ST_CHECK ? MIR_CHECK : MIR_STOPPED);
    return;
  }
  final_tree(part, 1, outv, scratch);
  const int k = s_k;
  const double pq = outv[0];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->state = ST_BREAK;
      // the p / q kernel of this iteration applied the previous x update
      ctl->cg_xdone = ctl->cg_xk;
      mirror_report(ctl->mirror, serial, MIR_STOPPED);
    }
    return;
  }
  const double alpha = s_rho / pq;
  (void)x;
  (void)P0;
  (void)P1;
  // ||r||^2 and (preconditioned) r^T z of the new residual; x += alpha p is left to the
  // next p / q kernel (or the fix-up kernel)
  constexpr int K = PC ? 2 : 1;
  double acc[K] = {};
  for (int64_t r0 = rfirst; r0 < n; r0 += (int64_t)gridDim.x * (U * KTPB)) {
    double rv[U], qv[U], dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = r0 + (int64_t)u * KTPB + threadIdx.x;
      const int64_t ic = i < n ? i : n - 1;
      const bool pre = r0 == rfirst;
      rv[u] = (double)(pre ? r1[u] : r[ic]);
      qv[u] = (double)(pre ? q1[u] : q[ic]);
      if constexpr (PC) dv[u] = (double)(pre ? d1[u] : dinv[ic]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = r0 + (int64_t)u * KTPB + threadIdx.x;
      if (i < n) {
        const TV rs = (TV)(rv[u] - alpha * qv[u]);
        r[i] = rs;
        const double ri = (double)rs;
        acc[0] += ri * ri;
        if constexpr (PC) acc[K - 1] += ri * (dv[u] * ri);
      }
    }
  }
  kstore<K>(acc, K, red, Pout + (size_t)blockIdx.x * KW);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->iters = k;
    ctl->cg_alpha = alpha;
    ctl->cg_xk = k;
    mirror_report(ctl->mirror, serial, 0u);
  }
}

// Grid of the CG iteration kernels: one wave tile per wave, at most the blocks the device
// holds at once (every block of the grid-stride loop resident, so no tail of late
// blocks), a multiple of NXCD.  The p / q kernel's registers decide the occupancy.
// the column array of the CG kernels: the packed 16-bit offsets or the columns; without
// nonzeros a stand-in (the SpMV reads one entry; never used in a product)
template <typename IT>
static inline const IT *cg_cols(const CsrView &A, const void *standin) {
  if (A.nnz == 0) return (const IT *)standin;
  if constexpr (sizeof(IT) == 2)
    return A.col16;
  else
    return A.col;
}

template <typename VT, typename TV, int C, bool PC, typename IT>
static int cg_grid(int64_t n) {
  static int resident = 0;  // blocks of k_cg_p<VT, TV, C, PC, IT> the device holds at once
  if (resident == 0) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cg_p<VT, TV, C, PC, IT>, KTPB, 0) != hipSuccess ||
        per < 1)
      return cgblocks(n);
    const int r = per * ncu / NXCD * NXCD;
    resident = r < NXCD ? NXCD : (r > CG_MAXBLK ? CG_MAXBLK : r);
  }
  const int nb = cgblocks(n);
  return nb < resident ? nb : resident;
}

// rows each thread of the x / r kernel takes per pass (all its loads issued first)
static inline int cg_rows(int64_t n, int nb) {
  const int64_t threads = (int64_t)KTPB * nb;
  const int64_t per = (n + threads - 1) / threads;
  return per >= 4 ? 4 : (per >= 2 ? 2 : 1);
}

template <typename VT, typename TV, int C, int U, bool PC, typename IT>
static void cg_iter_launch(const CsrView &A, TV *x, TV *r, TV *P0, TV *P1, TV *q, double *partials, Ctl *ctl,
                           hipStream_t st, const KTiming *tm, int serial, int nb, const TV *dinv) {
  // timed launches record their start/stop events in the kernel's own dispatch
  hipEvent_t e0 = tm ? tm->e0 : nullptr, e1 = tm ? tm->e1 : nullptr;
  const int lidx = tm ? tm->lidx : -1;
  // the SpMV reads one column / value entry even without nonzeros: stand-in arrays then
  // (the row pointers and the workspace's residual, never used in a product)
  const IT *colp = cg_cols<IT>(A, r);
  const VT *valp = A.nnz > 0 ? (const VT *)A.val : (const VT *)r;
  hipExtLaunchKernelGGL((k_cg_p<VT, TV, C, PC, IT>), dim3(nb), dim3(KTPB), 0, st, e0, e1, 0, A.rowptr, colp, valp, r,
                        P0, P1, q, A.n, PA(partials), nb, PB(partials), ctl, lidx, dinv, x);
  hipLaunchKernelGGL((k_cg_xr<TV, U, PC>), dim3(nb), dim3(KTPB), 0, st, x, r, P0, P1, q, A.n, PB(partials), nb,
                     PA(partials), ctl, serial, dinv);
}

template <typename VT, typename TV, int C, bool PC, typename IT>
static void cg_iter_u(const CsrView &A, TV *x, TV *r, TV *P0, TV *P1, TV *q, double *partials, Ctl *ctl,
                      hipStream_t st, const KTiming *tm, int serial, const TV *dinv) {
  const int nb = cg_grid<VT, TV, C, PC, IT>(A.n);
  const int U = cg_rows(A.n, nb);
  if (U == 4)
    cg_iter_launch<VT, TV, C, 4, PC, IT>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, nb, dinv);
  else if (U == 2)
    cg_iter_launch<VT, TV, C, 2, PC, IT>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, nb, dinv);
  else
    cg_iter_launch<VT, TV, C, 1, PC, IT>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, nb, dinv);
}

template <typename VT, typename TV, int C, bool PC, typename IT>
static int cg_start_c(const CsrView &A, const TV *b, const TV *x, TV *r, int mode, double *partials, Ctl *ctl,
                      hipStream_t st, const TV *dinv) {
  const int nb = cg_grid<VT, TV, C, PC, IT>(A.n);
  const IT *colp = cg_cols<IT>(A, r);
  const VT *valp = A.nnz > 0 ? (const VT *)A.val : (const VT *)r;
  hipLaunchKernelGGL((k_cg_start<VT, TV, C, PC, IT>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, colp, valp, b, x, r,
                     A.n, mode, PA(partials), ctl, dinv);
  return nb;
}

template <typename VT, typename TV, bool PC, typename IT>
static int cg_start_it(const CsrView &A, const TV *b, const TV *x, TV *r, int mode, double *partials, Ctl *ctl,
                       hipStream_t st, const TV *dinv, int chunk) {
  const int C = chunk > 0 ? chunk : wave_tile_chunk(A.n, A.nnz);
  if (C <= 5) return cg_start_c<VT, TV, 5, PC, IT>(A, b, x, r, mode, partials, ctl, st, dinv);
  if (C <= 7) return cg_start_c<VT, TV, 7, PC, IT>(A, b, x, r, mode, partials, ctl, st, dinv);
  return cg_start_c<VT, TV, 9, PC, IT>(A, b, x, r, mode, partials, ctl, st, dinv);
}

template <typename VT, typename TV, bool PC>
static int cg_start_launch(const CsrView &A, const TV *b, const TV *x, TV *r, int mode, double *partials,
                           Ctl *ctl, hipStream_t st, const TV *dinv, int chunk) {
  return A.col16 && A.nnz > 0 ? cg_start_it<VT, TV, PC, short>(A, b, x, r, mode, partials, ctl, st, dinv, chunk)
                              : cg_start_it<VT, TV, PC, int>(A, b, x, r, mode, partials, ctl, st, dinv, chunk);
}

template <typename TV>
hipError_t launch_cg_start_k(const CsrView &A, const TV *b, const TV *x, TV *r, int mode, double *partials, Ctl *ctl,
                             hipStream_t st, int serial, const TV *dinv, int chunk) {
  int nb;
  if (dinv)
    nb = A.fp32 ? cg_start_launch<float, TV, true>(A, b, x, r, mode, partials, ctl, st, dinv, chunk)
                : cg_start_launch<double, TV, true>(A, b, x, r, mode, partials, ctl, st, dinv, chunk);
  else
    nb = A.fp32 ? cg_start_launch<float, TV, false>(A, b, x, r, mode, partials, ctl, st, dinv, chunk)
                : cg_start_launch<double, TV, false>(A, b, x, r, mode, partials, ctl, st, dinv, chunk);
  hipLaunchKernelGGL(k_cg_start_close, dim3(1), dim3(KTPB), 0, st, PA(partials), nb, mode, ctl, serial,
                     dinv ? 1 : 0);
  return hipGetLastError();
}

template <typename VT, typename TV, bool PC, typename IT>
static void cg_iter_it(const CsrView &A, TV *x, TV *r, TV *P0, TV *P1, TV *q, double *partials, Ctl *ctl,
                       hipStream_t st, const KTiming *tm, int serial, const TV *dinv, int chunk) {
  const int C = chunk > 0 ? chunk : wave_tile_chunk(A.n, A.nnz);
  if (C <= 5)
    cg_iter_u<VT, TV, 5, PC, IT>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, dinv);
  else if (C <= 7)
    cg_iter_u<VT, TV, 7, PC, IT>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, dinv);
  else
    cg_iter_u<VT, TV, 9, PC, IT>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, dinv);
}

template <typename VT, typename TV, bool PC>
static void cg_iter_vt(const CsrView &A, TV *x, TV *r, TV *P0, TV *P1, TV *q, double *partials, Ctl *ctl,
                       hipStream_t st, const KTiming *tm, int serial, const TV *dinv, int chunk) {
  if (A.col16 && A.nnz > 0)
    cg_iter_it<VT, TV, PC, short>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, dinv, chunk);
  else
    cg_iter_it<VT, TV, PC, int>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, dinv, chunk);
}

template <typename TV>
hipError_t launch_cg_iter(const CsrView &A, TV *x, TV *r, TV *p2, TV *q, double *partials, Ctl *ctl,
                          hipStream_t st, const KTiming *tm, int serial, const TV *dinv, int chunk) {
  const int64_t ld = padded_ld(A.n);
  TV *P0 = p2, *P1 = p2 + ld;
  if (dinv) {
    if (A.fp32)
      cg_iter_vt<float, TV, true>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, dinv, chunk);
    else
      cg_iter_vt<double, TV, true>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, dinv, chunk);
  } else {
    if (A.fp32)
      cg_iter_vt<float, TV, false>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, dinv, chunk);
    else
      cg_iter_vt<double, TV, false>(A, x, r, P0, P1, q, partials, ctl, st, tm, serial, dinv, chunk);
  }
  return hipGetLastError();
}

template <typename TV>
hipError_t launch_cg_xfix(const CsrView &A, TV *x, TV *p2, Ctl *ctl, hipStream_t st) {
  const int64_t ld = padded_ld(A.n);
  hipLaunchKernelGGL((k_cg_xfix<TV>), dim3(kblocks(A.n)), dim3(KTPB), 0, st, x, p2, p2 + ld, A.n, ctl);
  return hipGetLastError();
}

// Tile autotuner of the CG kernels: the gathers per lane and step (C = 5, 7 or 9) of
// their wave tiles, chosen by timing the start kernel's SpMV (mode 2: it writes only its
// partial rows) for each C on the operator at hand: three timed runs of four back-to-back
// launches each (after one untimed launch), the fastest run kept.  The average row
// length's C (the heuristic) stays unless another is at least 3 % faster, so timing
// noise does not flip the choice.  Cached per (n, nnz, value type, vector type) for the
// process; the first solve of a new shape pays about 40 launches and three waits.
template <typename TV>
int cg_tile_tune(const CsrView &A, const TV *b, const TV *x, TV *r, double *partials, Ctl *ctl, hipStream_t st) {
  using Key = std::tuple<int64_t, int64_t, int, int, int>;
  static std::map<Key, int> cache;
  static std::mutex mu;
  const Key key{A.n, A.nnz, A.fp32, (int)sizeof(TV), A.col16 ? 1 : 0};
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const int heuristic = wave_tile_chunk(A.n, A.nnz);
  if (A.nnz == 0) return heuristic;
  // SACC_CG_CHUNK = 5, 7 or 9 pins the choice (reproducible measurements: a profiler's
  // per-launch overhead distorts the timing)
  static const int pinned = [] {
    const char *e = getenv("SACC_CG_CHUNK");
    const int v = e ? atoi(e) : 0;
    return (v == 5 || v == 7 || v == 9) ? v : 0;
  }();
  if (pinned) return pinned;
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess) return heuristic;
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return heuristic;
  }
  const int cands[3] = {5, 7, 9};
  float tmin[3] = {0.0f, 0.0f, 0.0f};
  bool ok = true;
  for (int ci = 0; ci < 3 && ok; ++ci) {
    const int C = cands[ci];
    ok = launch_cg_start_k<TV>(A, b, x, r, 2, partials, ctl, st, 0, nullptr, C) == hipSuccess;
    for (int rep = 0; rep < 3 && ok; ++rep) {
      ok = hipEventRecord(ev[0], st) == hipSuccess;
      for (int l = 0; l < 4 && ok; ++l)
        ok = launch_cg_start_k<TV>(A, b, x, r, 2, partials, ctl, st, 0, nullptr, C) == hipSuccess;
      float t = 0.0f;
      ok = ok && hipEventRecord(ev[1], st) == hipSuccess && hipEventSynchronize(ev[1]) == hipSuccess &&
           hipEventElapsedTime(&t, ev[0], ev[1]) == hipSuccess;
      if (ok && (rep == 0 || t < tmin[ci])) tmin[ci] = t;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (!ok) return heuristic;
  const int hi = heuristic == 5 ? 0 : (heuristic == 7 ? 1 : 2);
  int pick = heuristic;
  float best = tmin[hi];
  for (int ci = 0; ci < 3; ++ci)
    if (tmin[ci] < 0.97f * tmin[hi] && tmin[ci] < best) {
      best = tmin[ci];
      pick = cands[ci];
    }
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = pick;
  return pick;
}

// ============================================================================ GMRES
// One cycle of GMRES(m), CGS2, two streaming kernels per Arnoldi step.  Columns of V
// are kept raw with a scale: v_l = vs[l] V[:, l].  T is a scratch column.
//
//   F(j): finalise column j, w''_j = w'_j - sum_{l<j} g_l v_l, where w'_j (in T) is the
//         once-orthogonalised vector of step j-1 and g its second-pass coefficients
//         (reduced from G(j-1)'s partials; column j-1 of H is h1 + g); ||w''_j||^2;
//         y = A w''_j evaluated as A w'_j - sum_{l<j} g_l A v_l with the Arnoldi
//         relation A v_l = sum_{k<=l} H_kl v_k + w''_{l+1}, so the SpMV reads the
//         complete w'_j; y (raw) into V[:, j+1]; partial dots V[:, k]^T y, k <= j.
//   G(j): beta_j = ||w''_j|| closes step j-1 (Givens rotation, residual estimate,
//         end-of-cycle test); h1 = V_j^T A v_j; w'_{j+1} = A v_j - V h1 into T;
//         partial dots V[:, k]^T w'_{j+1} (the second pass of step j).
// F(0) instead reduces the start kernel's partials (||r||^2, ||b||^2) and opens the
// cycle.  After G(m-1) of a full cycle: the update x += V y, whose blocks first close
// step m - 1 themselves from G(m-1)'s partial rows (with F(m) in finalise-only mode
// before it where m fills its column tier: 8, 16, 32); a cycle cut short by its close
// in G goes to the update directly; the one-block close kernel k_gm_close remains for
// callers of launch_gm_finish with close.  The pair (F, G) reads V twice per step, the same as
// CGS2 needs for its two projections, and the second projection of step j shares
// the pass of the SpMV of step j + 1.
//
// Partial rows: start [||r||^2, ||b||^2] -> PA; F: [||w''_j||^2, V_j^T y, V_{0..j-1}^T y]
// -> PB; G: [V_{0..j}^T w' (, ||w'||^2 at the last step of a full cycle)] -> PA.

template <typename VT, typename TV>
__global__ __launch_bounds__(KTPB) void k_gm_start(const int *rowptr, const int *col, const VT *val,
                                                   const TV *b, const TV *x, TV *V, int64_t n, int restart_mode,
                                                   double *Pout, const Ctl *ctl) {
  // two row tiles per pass (one pass over n = 2^18 rows with the full grid): their
  // row-pointer, column / value and gather trips are shared
  constexpr int R = 2;
  __shared__ double red[KNW * 2];
  __shared__ double prod[SPMV_CAP * R];
  const int t = threadIdx.x;
  // the run state is read with the first loads; a stopped solve returns after the
  // stage (block-uniform)
  const int z = vzero();
  const int st = vread(&ctl->state, z);
  const Gather1<TV> gx{x};
  double acc[2] = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * (R * KTPB);
  for (int64_t r0 = (int64_t)blockIdx.x * (R * KTPB); r0 < n; r0 += stride) {
    TV bv[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = r0 + (int64_t)u * KTPB + t;
      bv[u] = b[i < n ? i : n - 1];
    }
    const TileRowsR<R> tr = tile_spmv_stage_r<KTPB, R, SPMV_CAP * R>(rowptr, col, val, gx, n, r0, prod);
    __syncthreads();
    double ax[R];
    tile_spmv_sum_r(tr, col, val, gx, prod, ax);
    __syncthreads();
    if (restart_mode && st != ST_RUN) return;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = r0 + (int64_t)u * KTPB + t;
      if (i < n) {
        const double bi = (double)bv[u];
        const TV rs = (TV)(bi - ax[u]);
        V[i] = rs;
        const double ri = (double)rs;
        acc[0] += ri * ri;
        acc[1] += bi * bi;
      }
    }
  }
  if (restart_mode && st != ST_RUN) return;
  kstore<2>(acc, 2, red, Pout + (size_t)blockIdx.x * KW);
}

// Inputs of the close of step j, staged into LDS by all threads at once (the control
// block was written by earlier kernels, so each read is a trip to memory; issuing
// them together costs one).
struct CloseIn {
  double col[MAXR + 1], cs[MAXR], sn[MAXR];
  double gj, tolb;
  int maxit, restart, trust;
};

__device__ inline void close_stage(int j, const Ctl *ctl, CloseIn *ci) {
  const int LD = MAXR + 1;
  const int t = threadIdx.x;
  if (t <= j) ci->col[t] = ctl->Hraw[t + j * LD];
  if (t < j) {
    ci->cs[t] = ctl->cs[t];
    ci->sn[t] = ctl->sn[t];
  }
  const int z = vzero();
  const double gj = vread(&ctl->gnext[j], z), tol = vread(&ctl->tol, z), bn = vread(&ctl->bnorm, z);
  const int maxit = vread(&ctl->maxit, z), restart = vread(&ctl->restart, z), trust = vread(&ctl->trust_est, z);
  if (t == WAVE) {
    ci->gj = gj;
    ci->tolb = tol * bn;
    ci->maxit = maxit;
    ci->restart = restart;
    ci->trust = trust;
  }
}

// Close Arnoldi step j given hn = ||w''_{j+1}|| from the staged inputs: rotate the raw
// column j, new Givens rotation, rotated right-hand side, cycle-end test.  `it` =
// global iteration number of step j (1-based).  Run by a whole wave, every lane
// computing the same scalars: lane l holds entry l of the column and rotation l, and
// the scalar recurrence reads them with v_readlane (no LDS round trip per rotation).
// Every block computes the same result; only `persist` (block 0) writes the control
// block, the rotated column included (lanes 0..j; j < 64).  Returns CLOSE_END when the
// cycle ends, with CLOSE_EST when it ends on the residual estimate.
enum : int { CLOSE_END = 1, CLOSE_EST = 2 };
// With col_out / gam_out the rotated column (rows 0..j) and gam_j also go to those (LDS)
// locations in every block; keep_active leaves ctl->active as it is (for a kernel whose
// other blocks read it).
__device__ inline int gm_close_wave(int j, double hn, int it, const CloseIn *ci, Ctl *ctl, bool persist,
                                   double *col_out = nullptr, double *gam_out = nullptr, bool keep_active = false) {
  const int LD = MAXR + 1;
  const int lane = threadIdx.x % WAVE;
  double cv = ci->col[lane <= j ? lane : 0];
  const double cl = ci->cs[lane < j ? lane : 0], sl = ci->sn[lane < j ? lane : 0];
  double cur = lane_bcast(cv, 0);
  for (int l = 0; l < j; ++l) {
    const double nxt = lane_bcast(cv, l + 1), c = lane_bcast(cl, l), s = lane_bcast(sl, l);
    const double nl = c * cur + s * nxt;
    cur = -s * cur + c * nxt;
    cv = lane == l ? nl : cv;
  }
  const double a = cur;
  const double rr = hypot(a, hn);
  double c = 1.0, s = 0.0;
  if (rr != 0.0) {
    c = a / rr;
    s = hn / rr;
  }
  cv = lane == j ? rr : cv;
  const double gj = ci->gj;
  const double gam_j = c * gj, gnext = -s * gj;
  const bool est_conv = fabs(gnext) <= ci->tolb;
  const bool end = est_conv || hn == 0.0 || it >= ci->maxit || j + 1 >= ci->restart || !isfinite(gnext);
  if (persist) {
    if (lane <= j) ctl->R[lane + j * LD] = cv;
    if (lane == 0) {
      ctl->cs[j] = c;
      ctl->sn[j] = s;
      ctl->gam[j] = gam_j;
      ctl->gnext[j + 1] = gnext;
      ctl->vs[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
      ctl->iters = it;
      ctl->jend = j + 1;
      if (end && !keep_active) ctl->active = 0;
      if (est_conv && ci->trust) ctl->conv_pending = 1;
    }
  }
  if (col_out && lane <= j) col_out[lane] = cv;
  if (gam_out && lane == 0) *gam_out = gam_j;
  return end ? (CLOSE_END | (est_conv ? CLOSE_EST : 0)) : 0;
}

// gm_close_wave for a whole block (after close_stage and a barrier): wave 0 runs it and
// persists the rotated column.  Returns the cycle-end flag to every thread.
__device__ inline bool gm_close_block(int j, double hn, int it, CloseIn *ci, Ctl *ctl, bool persist) {
  __shared__ int s_endf;
  if (threadIdx.x < WAVE) {
    const int cl = gm_close_wave(j, hn, it, ci, ctl, persist);
    if (threadIdx.x == 0) s_endf = cl & CLOSE_END;
  }
  __syncthreads();
  return s_endf != 0;
}

// Row pointers of a pass of R KTPB rows from r0: the pass's nonzero range [p0, p1) and
// this thread's rows (empty past n).  Loads stay in bounds for any r0.
template <int R>
struct PassRows {
  int a[R], b[R];
  int p0, p1;
};

template <int R>
__device__ inline PassRows<R> pass_rows(const int *__restrict__ rowptr, int64_t n, int64_t r0, int z) {
  const int64_t rs = r0 < n ? r0 : n;
  const int64_t re = r0 + (int64_t)R * KTPB < n ? r0 + (int64_t)R * KTPB : n;
  PassRows<R> pr;
  // vector loads (z = vzero()): see vread; made uniform where the pass uses them
  pr.p0 = rowptr[rs + z];
  pr.p1 = rowptr[re + z];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int64_t i = r0 + (int64_t)u * KTPB + threadIdx.x;
    const int64_t ic = i < n ? i : n - 1;
    const int a = rowptr[ic], b = rowptr[ic + 1];
    pr.a[u] = i < n ? a : 0;
    pr.b[u] = i < n ? b : 0;
  }
  return pr;
}

// One staging round of a pass's SpMV (the scheme of tile_spmv_stage_r): C nonzeros per
// thread from `base`, split into the column / value loads, the gathers and the LDS
// writes, so that a kernel can issue other loads between them.  stage_load reads
// in bounds for any range (col / val hold at least one entry).
template <int C>
struct StageRound {
  int cc[C];
  double vv[C], xx[C];
};

template <int C, typename VT>
__device__ inline void stage_load(StageRound<C> &sr, const int *__restrict__ col, const VT *__restrict__ val, int base,
                                  int p1) {
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const int p = base + threadIdx.x + u * KTPB;
    const int pc = p < p1 ? p : (p1 > 0 ? p1 - 1 : 0);
    sr.cc[u] = col[pc];
    sr.vv[u] = (double)val[pc];
  }
}

template <int C, typename G>
__device__ inline void stage_gather(StageRound<C> &sr, const G &gx) {
#pragma unroll
  for (int u = 0; u < C; ++u) sr.xx[u] = gx(sr.cc[u]);
}

template <int C>
__device__ inline void stage_write(const StageRound<C> &sr, int base, int p0, int p1, double *prod) {
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const int p = base + threadIdx.x + u * KTPB;
    if (p < p1) prod[p - p0] = sr.vv[u] * sr.xx[u];
  }
}

// Column value of slot k when the live columns are 0..live-1 (live >= 0), zero past
// them.  Double: a uniform branch skips the load.  Float: the compiler makes every
// guarded 32-bit load wait for its data before the next one is issued, so every load
// is issued instead (slots past the live columns re-read column max(live - 1, 0)) and
// masked.
template <typename TV>
__device__ inline TV slot_load(const TV *V, int64_t ld, int64_t i, int k, int live) {
  if constexpr (sizeof(TV) == 8) {
    return k < live ? V[(size_t)k * ld + i] : (TV)0;
  } else {
    const int kc = k < live ? k : (live > 0 ? live - 1 : 0);
    const TV v = V[(size_t)kc * ld + i];
    return k < live ? v : (TV)0;
  }
}

// Right-preconditioned operand of the Arnoldi product: A (D^-1 v) gathers d_c^-1 v_c
template <typename TV>
struct GatherScaled {
  const TV *__restrict__ x;
  const TV *__restrict__ dinv;
  __device__ double operator()(int c) const { return (double)dinv[c] * (double)x[c]; }
};

// F(j); mode 0: first cycle, 1: restart cycle (both only matter for j = 0), 2: the
// finalise-only step j = m.  PC: Jacobi right preconditioning, w = A D^-1 v.  R = row tiles of KTPB rows each block takes per pass.
//
// Order of the memory traffic (the first pass): one trip for the control block, the
// previous kernel's partial rows and the pass's row pointers; then the SpMV's column /
// value loads, the pass's column values and the gathers (from 16 slots on the gathers
// before the column values), so the column stream overlaps the SpMV's dependent trips
// and the LDS work of the prologue.  The gathers read in bounds for any pass: column
// indices come from clamped in-range loads.
template <typename VT, typename TV, int RB, int R, bool PC>
__global__ __launch_bounds__(KTPB) void k_gm_f(const int *rowptr, const int *col, const VT *val, TV *V, TV *T,
                                               int64_t n, int64_t ld, int j, int mode, const double *Pin, int nblk,
                                               double *Pout, Ctl *ctl, int lidx, const TV *dinv) {
  const int LD = MAXR + 1;
  constexpr int NR = R * KTPB;
  constexpr int CAP = SPMV_CAP * R;
  constexpr int C = 6 * R;
  constexpr int HPT = ((MAXR + 1) * MAXR + KTPB - 1) / KTPB;  // raw Hessenberg entries staged per thread
  static_assert(RB + 2 <= WAVE, "partial rows are reduced in one group");
  __shared__ double red[KNW * (RB + 2)];
  __shared__ double outv[RB + 2];
  __shared__ double scratch[KTPB];
  __shared__ double prod[CAP];
  __shared__ double gsh[RB], fco[RB], cco[RB + 1];
  __shared__ double Hs[(MAXR + 1) * MAXR], vsh[MAXR + 1], h1s[MAXR + 1];
  __shared__ int s_go, s_open;
  const int t = threadIdx.x;
  const TV *src = (j == 0) ? V : T;
  TV *wcol = V + (size_t)j * ld;
  TV *ycol = V + (size_t)(j + 1) * ld;
  using Gx = std::conditional_t<PC, GatherScaled<TV>, Gather1<TV>>;
  Gx gx;
  if constexpr (PC)
    gx = Gx{src, dinv};
  else
    gx = Gx{src};
  const int64_t stride = (int64_t)gridDim.x * NR;
  int64_t r0 = (int64_t)blockIdx.x * NR;

  // ---- one trip: first pass's row pointers, control block, partial rows
  const int z = vzero();
  PassRows<R> pr = pass_rows<R>(rowptr, n, r0, z);
  const int st = vread(&ctl->state, z), act = vread(&ctl->active, z);
  const DecideIn din = decide_in(ctl, z);
  const int trust = vread(&ctl->trust_est, z), pend = vread(&ctl->conv_pending, z);
  const int hcnt = j > 1 ? (j - 1) * LD : 0;
  const int jm = j > 0 ? j - 1 : 0;
  double hreg[HPT];
#pragma unroll
  for (int u = 0; u < HPT; ++u) {
    const int e = t + u * KTPB;
    hreg[u] = ctl->Hraw[e < hcnt ? e : 0];
  }
  const double vs_t = ctl->vs[t < jm ? t : jm], h1_t = ctl->h1[t < jm ? t : jm];
  const int kp = j == 0 ? 2 : j;
  // partial rows a thread needs: nblk <= KMAXBLK rows of kp <= RB entries
  double pt[RB / 2 > 0 ? RB / 2 : 1];
  final_part_load(Pin, nblk, KW, kp, pt);
  if (t == 0) s_go = j == 0 ? ((mode == 0) || st == ST_RUN) : ((st == ST_RUN) && act);
#pragma unroll
  for (int u = 0; u < HPT; ++u) {
    const int e = t + u * KTPB;
    if (e < hcnt) Hs[e] = hreg[u];
  }
  if (t < j) {
    vsh[t] = vs_t;
    h1s[t] = h1_t;
  }
  __syncthreads();
  if (!s_go) return;
  // (summed here: holding the loaded rows past the column loads below would spill)
  const double part = final_part_sum(Pin, nblk, KW, kp, pt);
  if (j == 0) {
    // open the cycle from the start kernel's partials
    final_tree(part, 2, outv, scratch);
    if (t == 0) {
      const bool persist = blockIdx.x == 0;
      const bool accept = mode != 0 && trust && pend;
      const int sd = residual_decide(outv[0], outv[1], mode == 0 ? 0 : 1, din, ctl, persist, accept);
      if (persist && sd == ST_RUN) {
        ctl->conv_pending = 0;
        const double beta = sqrt(outv[0]);
        ctl->active = 1;
        ctl->jend = 0;
        ctl->ibase = mode == 0 ? 0 : din.iters;
        ctl->gnext[0] = beta;
        ctl->vs[0] = 1.0 / beta;
      }
      s_open = sd == ST_RUN;
    }
    __syncthreads();
    if (!s_open) return;
    for (int l = t; l <= RB; l += blockDim.x) {
      if (l < RB) fco[l] = 0.0;
      cco[l] = 0.0;
    }
  }
  if (lidx >= 0 && blockIdx.x == 0 && t == 0) ctl->work_log[lidx] = 1;

  double ex[2] = {0.0, 0.0};  // ||w''_j||^2, V[:, j]^T y
  double acc[RB];             // V[:, k]^T y, k < j
#pragma unroll
  for (int l = 0; l < RB; ++l) acc[l] = 0.0;
  bool first = true;
  // SpMV round 1 of a pass: columns and values (issued unconditionally: a branch around
  // them would make the column loads below wait for them).  With one row tile per pass
  // the next pass's round 1 is requested before this pass's arithmetic (its row pointers
  // with this pass's first loads), so a later pass starts with its gathers.
  StageRound<C> sr;
  if constexpr (R == 1)
    stage_load<C>(sr, col, val, __builtin_amdgcn_readfirstlane(pr.p0), __builtin_amdgcn_readfirstlane(pr.p1));
  for (; r0 < n; r0 += stride) {
    const bool spmv = mode != 2;
    const int p0 = __builtin_amdgcn_readfirstlane(pr.p0), p1 = __builtin_amdgcn_readfirstlane(pr.p1);
    const bool staged = spmv && p1 > p0 && p1 - p0 <= CAP;
    PassRows<R> prn;
    if constexpr (R == 1)
      prn = pass_rows<R>(rowptr, n, r0 + stride, z);  // in bounds past the last pass
    else
      stage_load<C>(sr, col, val, p0, p1);
    // with 16 or more slots the gathers go out before the column stream too (their LDS
    // write and the row sums then overlap the stream; measured faster there, slower at 8)
    constexpr bool gathers_first = RB >= 16;
    if constexpr (gathers_first) stage_gather<C>(sr, gx);
    // the pass's column values (slots past the live columns are skipped by a uniform
    // branch and hold zero)
    // (kept in the stored type and widened where used)
    TV vl[R][RB];
    double s0[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = r0 + (int64_t)u * KTPB + t;
      const int64_t ic = i < n ? i : n - 1;
#pragma unroll
      for (int k = 0; k < RB; ++k) vl[u][k] = slot_load(V, ld, ic, k, j);
      s0[u] = (double)src[ic];
    }
    if (first && j > 0) {
      // prologue, while the loads above are in flight: second-pass coefficients of
      // w'_j, the completed column j - 1 of H, and the coefficients of
      // A (sum_{l<j} g_l v_l) on the raw columns 0..j
      final_tree(part, j, outv, scratch);
      for (int l = t; l < RB; l += blockDim.x) {
        const double g = (l < j) ? outv[l] * vsh[l] : 0.0;
        gsh[l] = g;
        fco[l] = (l < j) ? g * vsh[l] : 0.0;
        if (l < j) {
          Hs[l + (j - 1) * LD] = h1s[l] + g;
          if (blockIdx.x == 0) ctl->Hraw[l + (j - 1) * LD] = h1s[l] + g;
        }
      }
      __syncthreads();
      if (mode != 2) {
        for (int k = t; k <= RB; k += blockDim.x) {
          double c = 0.0;
          if (k < j) {
            double sacc = 0.0;
#pragma unroll 4
            for (int l = k; l < j; ++l) sacc += gsh[l] * Hs[k + l * LD];
            c = sacc * vsh[k];
          }
          if (k >= 1 && k <= j) c += gsh[k - 1];
          cco[k] = c;
        }
      }
    }
    first = false;
    double ax[R];
#pragma unroll
    for (int u = 0; u < R; ++u) ax[u] = 0.0;
    if (spmv) {
      if (staged) {
        if constexpr (!gathers_first) stage_gather<C>(sr, gx);
        stage_write<C>(sr, p0, p0, p1, prod);
        for (int base = p0 + C * KTPB; base < p1; base += C * KTPB) {
          stage_load<C>(sr, col, val, base, p1);
          stage_gather<C>(sr, gx);
          stage_write<C>(sr, base, p0, p1, prod);
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < R; ++u) {
        double a = 0.0;
        if (staged) {
          for (int p = pr.a[u]; p < pr.b[u]; ++p) a += prod[p - p0];
        } else {
          for (int p = pr.a[u]; p < pr.b[u]; ++p) a += (double)val[p] * gx(col[p]);
        }
        ax[u] = a;
      }
    }
    __syncthreads();  // fco / cco visible; prod free for the next pass
    if constexpr (R == 1) {
      // the next pass's round 1 (past the last pass: in-bounds loads nobody uses)
      pr = prn;
      stage_load<C>(sr, col, val, __builtin_amdgcn_readfirstlane(pr.p0), __builtin_amdgcn_readfirstlane(pr.p1));
    } else {
      // the next pass's row pointers, requested before this pass's arithmetic
      if (r0 + stride < n) pr = pass_rows<R>(rowptr, n, r0 + stride, z);
    }
    const double cj = cco[j < RB ? j : RB];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = r0 + (int64_t)u * KTPB + t;
      if (i < n) {
        double w = s0[u];
#pragma unroll
        for (int k = 0; k < RB; ++k) w -= fco[k] * (double)vl[u][k];
        const TV ws = (TV)w;
        if (j > 0 && mode != 2) wcol[i] = ws;
        const double wd = (double)ws;
        ex[0] += wd * wd;
        if (mode != 2) {
          double y = ax[u] - cj * wd;
#pragma unroll
          for (int k = 0; k < RB; ++k) y -= cco[k] * (double)vl[u][k];
          const TV ys = (TV)y;
          ycol[i] = ys;
          const double yd = (double)ys;
          ex[1] += wd * yd;
#pragma unroll
          for (int k = 0; k < RB; ++k) acc[k] += (double)vl[u][k] * yd;
        }
      }
    }
  }
  if (first && j > 0) {
    // a block without rows still completes the prologue (block 0 persists column j - 1)
    final_tree(part, j, outv, scratch);
    for (int l = t; l < RB && l < j; l += blockDim.x)
      if (blockIdx.x == 0) ctl->Hraw[l + (j - 1) * LD] = h1s[l] + outv[l] * vsh[l];
  }
  kstore2<RB>(ex, acc, mode == 2 ? 1 : j + 2, red, Pout + (size_t)blockIdx.x * KW);
}

// G(j); R = row tiles of KTPB rows each block takes per pass.  One trip for the
// control block and F(j)'s partial rows; then the first pass's columns are requested
// before the reduction and the close of step j - 1 run, which they overlap.  NW (the
// last step of a full cycle, j + 1 < RB): ||w'||^2 also goes to the partial rows, in
// slot j + 1, for the close of step j at the cycle end.
template <typename TV, int RB, int R, bool NW>
__global__ __launch_bounds__(KTPB) void k_gm_g(const TV *V, TV *T, int64_t n, int64_t ld, int j, const double *Pin,
                                               int nblk, double *Pout, Ctl *ctl, int serial) {
  const int LD = MAXR + 1;
  static_assert(RB + 2 <= WAVE, "partial rows are reduced in one group");
  __shared__ double red[KNW * RB];
  __shared__ double outv[RB + 2];
  __shared__ double scratch[KTPB];
  __shared__ double coef[RB];
  __shared__ double vsh[MAXR + 1];
  __shared__ int s_ibase, s_go;
  __shared__ CloseIn ci;
  const int t = threadIdx.x;
  // ---- one trip: control block (run flag, close inputs, column scales), partial rows
  const int z = vzero();
  const int st = vread(&ctl->state, z), act = vread(&ctl->active, z), ib = vread(&ctl->ibase, z);
  unsigned long long *const mir = vread(&ctl->mirror, z);
  const int jc = j > 0 ? j - 1 : 0;  // step closed here
  const double col_t = ctl->Hraw[(t <= jc ? t : jc) + jc * LD];
  const double cs_t = ctl->cs[t < jc ? t : 0], sn_t = ctl->sn[t < jc ? t : 0];
  const double gj = vread(&ctl->gnext[jc], z), tol = vread(&ctl->tol, z), bn = vread(&ctl->bnorm, z);
  const int maxit = vread(&ctl->maxit, z), restart = vread(&ctl->restart, z), trust = vread(&ctl->trust_est, z);
  const double vs_t = ctl->vs[t <= j ? t : j];
  // partial rows a thread needs: nblk <= KMAXBLK rows of j + 2 <= 32 entries (more are
  // summed by final_part_sum)
  double pt[RB < 16 ? RB : 16];
  final_part_load(Pin, nblk, KW, j + 2, pt);
  if (t == 0) {
    s_go = (st == ST_RUN) && act;
    s_ibase = ib;
  }
  if (j > 0) {
    if (t <= jc) ci.col[t] = col_t;
    if (t < jc) {
      ci.cs[t] = cs_t;
      ci.sn[t] = sn_t;
    }
    if (t == WAVE) {
      ci.gj = gj;
      ci.tolb = tol * bn;
      ci.maxit = maxit;
      ci.restart = restart;
      ci.trust = trust;
    }
  }
  if (t <= j) vsh[t] = vs_t;
  __syncthreads();
  if (!s_go) {
    if (blockIdx.x == 0 && t == 0) mirror_report(mir, serial, st != ST_RUN ? MIR_STOPPED : MIR_CYCLE_END);
    return;
  }
  // ---- the first pass's columns, requested before the LDS work below
  const TV *ycol = V + (size_t)(j + 1) * ld;
  const int64_t stride = (int64_t)gridDim.x * (R * KTPB);
  int64_t r0 = (int64_t)blockIdx.x * (R * KTPB);
  // column values kept in the stored type and widened where used
  TV vl[R][RB], yv[R];
  auto load_pass = [&](int64_t rb) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = rb + (int64_t)u * KTPB + t;
      const int64_t ic = i < n ? i : n - 1;
#pragma unroll
      for (int k = 0; k < RB; ++k) vl[u][k] = slot_load(V, ld, ic, k, j + 1);
      yv[u] = ycol[ic];
    }
  };
  // the partial rows came with the control block; summed before the column loads go
  // out (a wait for them behind the column loads, which sit in uniform branches, would
  // be counted as a wait for those too)
  const double part = final_part_sum(Pin, nblk, KW, j + 2, pt);
  load_pass(r0);
  final_tree(part, j + 2, outv, scratch);
  // scale of v_j: 1 / ||w''_j|| (the close of step j - 1 records the same), or vs[0]
  // as F(0) opened the cycle
  const double hn = sqrt(outv[0]);
  const double vsj = j > 0 ? (hn > 0.0 ? 1.0 / hn : 0.0) : vsh[0];
  // h1_k = v_k^T A v_j = vs[k] vs[j] V[:, k]^T y
  for (int k = t; k < RB; k += blockDim.x) {
    double c = 0.0;
    if (k <= j) {
      const double vk = (k == j) ? vsj : vsh[k];
      const double dk = (k == j) ? outv[1] : outv[2 + k];
      const double h1 = vk * dk * vsj;
      if (blockIdx.x == 0) ctl->h1[k] = h1;
      c = h1 * vk;
    }
    coef[k] = c;
  }
  __syncthreads();
  // close of step j - 1 (Givens rotation, residual estimate, cycle-end test) on wave 0
  // while the other waves stream: when it ends the cycle, nothing reads this kernel's
  // outputs (every later kernel of the cycle checks `active`)
  if (j > 0 && t < WAVE) {
    const bool persist = blockIdx.x == 0;
    const int cl = gm_close_wave(j - 1, hn, s_ibase + j, &ci, ctl, persist);
    if (persist && t == 0)
      mirror_report(mir, serial, (cl & CLOSE_END) ? (MIR_CYCLE_END | ((cl & CLOSE_EST) ? MIR_EST_CONV : 0u)) : 0u);
  } else if (j == 0 && blockIdx.x == 0 && t == 0) {
    mirror_report(mir, serial, 0u);
  }
  double acc[RB], ww = 0.0;
#pragma unroll
  for (int l = 0; l < RB; ++l) acc[l] = 0.0;
#pragma unroll 1
  for (; r0 < n;) {
    // compiler barrier: re-read the LDS coefficients per row instead of holding all of
    // them in registers next to the column values and the partial dots
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = r0 + (int64_t)u * KTPB + t;
      if (i < n) {
        double w = vsj * (double)yv[u];
#pragma unroll
        for (int k = 0; k < RB; ++k) w -= coef[k] * (double)vl[u][k];
        const TV ws = (TV)w;
        T[i] = ws;
        const double wd = (double)ws;
#pragma unroll
        for (int k = 0; k < RB; ++k) acc[k] += (double)vl[u][k] * wd;
        if constexpr (NW) ww += wd * wd;
      }
    }
    r0 += stride;
    if (r0 >= n) break;
    load_pass(r0);
  }
  if constexpr (NW) {
    // ||w'||^2 in slot j + 1 (a column past the live ones)
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (k == j + 1) acc[k] = ww;
  }
  kstore<RB>(acc, NW ? j + 2 : j + 1, red, Pout + (size_t)blockIdx.x * KW);
}

// close of the last step of a cycle (after the finalise-only F(m))
__global__ __launch_bounds__(KTPB) void k_gm_close(const double *Pin, int nblk, int j, Ctl *ctl) {
  __shared__ double outv[1];
  __shared__ double scratch[KTPB];
  __shared__ int s_go, s_ibase;
  __shared__ CloseIn ci;
  // one trip: control block and F(m)'s partial rows
  const int z = vzero();
  const int st = vread(&ctl->state, z), act = vread(&ctl->active, z), ib = vread(&ctl->ibase, z);
  close_stage(j, ctl, &ci);
  double pt[1];
  final_part_load(Pin, nblk, KW, 1, pt);
  if (threadIdx.x == 0) {
    s_go = (st == ST_RUN) && act;
    s_ibase = ib;
  }
  __syncthreads();
  if (!s_go) return;
  final_tree(final_part_sum(Pin, nblk, KW, 1, pt), 1, outv, scratch);
  gm_close_block(j, sqrt(outv[0]), s_ibase + j + 1, &ci, ctl, true);
}

// End of a cycle: every block solves R y = gam (m x m upper triangular, staged in
// LDS) and adds x += sum_l y_l v_l for its rows.  The block's column values are
// requested before the triangular solve, which runs while they arrive; R = row tiles
// per pass.  jclose >= 0 (a cycle that ran all its steps): every block first closes step
// jclose = m - 1 itself, the work of k_gm_close, and takes the rotated column and gam
// from that close; block 0 persists it (not `active`, which the other blocks read here;
// the restart sets it).  The close's inputs come from the finalise-only F(m)'s partial
// rows (Pin = ||w''_m||^2), or with pyth from G(m - 1)'s (Pin = V^T w'_m and ||w'_m||^2):
// the second-pass coefficients g, column m - 1 of H = h1 + g, and ||w''_m||^2 =
// ||w'_m||^2 - ||g||^2 (w''_m = w'_m - V g with V orthonormal; g is the small second
// correction, so there is no cancellation), which saves F(m).  When the cycle had
// already ended (active = 0: its last close ran in G) the staged values serve.
template <typename TV, int RB, int R, bool PC>
__global__ __launch_bounds__(KTPB) void k_gm_update(TV *x, const TV *V, int64_t n, int64_t ld, Ctl *ctl,
                                                    const double *Pin, int nblk, int jclose, int pyth,
                                                    const TV *dinv) {
  const int LD = MAXR + 1;
  __shared__ double coef[RB];
  __shared__ double Rs[RB * RB];
  __shared__ double gs[RB];
  __shared__ int s_m, s_close, s_ibase;
  __shared__ double vsh[RB];
  __shared__ double outv[RB + 2];
  __shared__ double scratch[KTPB];
  __shared__ double gsq[RB];
  __shared__ CloseIn ci;
  const int t = threadIdx.x;
  // ---- one trip: every input of the prologue is requested before any is used (loads
  // at clamped indices, outside branches: a load whose value is stored under a branch
  // waits before the next one goes out)
  const int z = vzero();
  const int st = vread(&ctl->state, z), je = vread(&ctl->jend, z), act = vread(&ctl->active, z);
  const int ib = vread(&ctl->ibase, z);
  const int jc = jclose >= 0 ? jclose : 0;
  // partial entries: 1 (F(m)'s ||w''||^2) or m + 1 (G(m - 1)'s dots and ||w'||^2)
  const int kc = pyth ? jclose + 2 : 1;
  const double h1_t = ctl->h1[t <= jc ? t : 0];
  // inputs of the close of step jclose (as close_stage stages them)
  const double col_t = ctl->Hraw[(t <= jc ? t : jc) + jc * LD];
  const double cs_t = ctl->cs[t < jc ? t : 0], sn_t = ctl->sn[t < jc ? t : 0];
  const double gj = vread(&ctl->gnext[jc], z), tol = vread(&ctl->tol, z), bn = vread(&ctl->bnorm, z);
  const int maxit = vread(&ctl->maxit, z), restart = vread(&ctl->restart, z), trust = vread(&ctl->trust_est, z);
  // the triangle, right-hand side and scales
  constexpr int RPT = (RB * RB + KTPB - 1) / KTPB;
  double rv[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int e = t + u * KTPB;
    const int ec = e < RB * RB ? e : 0;
    rv[u] = ctl->R[ec % RB + (ec / RB) * LD];
  }
  const double gs_t = ctl->gam[t < RB ? t : 0], vs_t = ctl->vs[t < RB ? t : 0];
  double pt[RB / 2];
  if (jclose >= 0) final_part_load(Pin, nblk, KW, kc, pt);
  if (t == 0) {
    const bool close = jclose >= 0 && st == ST_RUN && act;
    s_close = close ? 1 : 0;
    s_m = (st == ST_RUN) ? (close ? jclose + 1 : je) : -1;
    s_ibase = ib;
  }
  if (jclose >= 0) {
    if (t <= jclose) ci.col[t] = col_t;
    if (t < jclose) {
      ci.cs[t] = cs_t;
      ci.sn[t] = sn_t;
    }
    if (t == WAVE) {
      ci.gj = gj;
      ci.tolb = tol * bn;
      ci.maxit = maxit;
      ci.restart = restart;
      ci.trust = trust;
    }
  }
  // (unused entries are never read)
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int e = t + u * KTPB;
    if (e < RB * RB) {
      const int i = e % RB, l = e / RB;
      Rs[i + l * RB] = (i <= l) ? rv[u] : 0.0;
    }
  }
  if (t < RB) {
    gs[t] = gs_t;
    vsh[t] = vs_t;
  }
  __syncthreads();
  const int m = s_m;
  if (m <= 0) return;
  const int64_t stride = (int64_t)gridDim.x * (R * KTPB);
  int64_t r0 = (int64_t)blockIdx.x * (R * KTPB);
  TV vl[R][RB], xv[R], dv[R];
  auto load_pass = [&](int64_t rb) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = rb + (int64_t)u * KTPB + t;
      const int64_t ic = i < n ? i : n - 1;
#pragma unroll
      for (int l = 0; l < RB; ++l) vl[u][l] = slot_load(V, ld, ic, l, m);
      xv[u] = x[ic];
      if constexpr (PC) dv[u] = dinv[ic];
    }
  };
  // the partial rows are summed before the column loads go out (a wait for them behind
  // loads in uniform branches would wait for those too); the columns then arrive while
  // the close and the triangular solve run
  const double part = s_close ? final_part_sum(Pin, nblk, KW, kc, pt) : 0.0;
  load_pass(r0);
  if (s_close) {
    // hn = ||w''_m||; the close of step m - 1 on wave 0
    final_tree(part, kc, outv, scratch);
    double hn;
    if (pyth) {
      // column m - 1 of H and ||g||^2 (every block, the same fixed order)
      if (t <= jclose) {
        const double g = outv[t] * vsh[t];
        ci.col[t] = h1_t + g;
        gsq[t] = g * g;
        if (blockIdx.x == 0) ctl->Hraw[t + jclose * LD] = h1_t + g;
      }
      __syncthreads();
      double gg = 0.0;
      for (int l = 0; l <= jclose; ++l) gg += gsq[l];
      const double hh = outv[jclose + 1] - gg;
      hn = hh > 0.0 ? sqrt(hh) : 0.0;
    } else {
      hn = sqrt(outv[0]);
    }
    if (t < WAVE)
      gm_close_wave(jclose, hn, s_ibase + jclose + 1, &ci, ctl, blockIdx.x == 0, Rs + jclose * RB, gs + jclose,
                    true);
    __syncthreads();
  }
  // R y = gam by columns on one wave: lane l keeps the right-hand side entry l
  if (t < WAVE) {
    const int l = t;
    double g = (l < m) ? gs[l] : 0.0;
    for (int i = m - 1; i >= 0; --i) {
      const double yi = lane_bcast(g, i) / Rs[i + i * RB];
      if (l < i) g -= Rs[l + i * RB] * yi;
      if (l == i) coef[i] = yi * vsh[i];
    }
    if (l >= m && l < RB) coef[l] = 0.0;
  }
  __syncthreads();
#pragma unroll 1
  for (; r0 < n;) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = r0 + (int64_t)u * KTPB + t;
      if (i < n) {
        if constexpr (PC) {
          // right preconditioning: x += D^-1 (V y)
          double s = 0.0;
#pragma unroll
          for (int l = 0; l < RB; ++l) s += coef[l] * (double)vl[u][l];
          x[i] = (TV)((double)xv[u] + (double)dv[u] * s);
        } else {
          double s = (double)xv[u];
#pragma unroll
          for (int l = 0; l < RB; ++l) s += coef[l] * (double)vl[u][l];
          x[i] = (TV)s;
        }
      }
    }
    r0 += stride;
    if (r0 >= n) break;
    load_pass(r0);
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
  return hipGetLastError();
}

// rows per thread of the GMRES step kernels: two row tiles at once when every block
// has at least two (the grid is capped at KMAXBLK blocks)
static inline bool gm_two_rows(int64_t n) { return n >= (int64_t)2 * KTPB * KMAXBLK; }

template <typename TV, int RB, int R, bool PC>
static void gm_f_launch_pc(const CsrView &A, TV *V, TV *T, int64_t ld, int j, int mode, double *partials, Ctl *ctl,
                           hipStream_t st, const KTiming *tm, const TV *dinv) {
  const int nb = kblocks(A.n);
  // timed launches record their start/stop events in the kernel's own dispatch
  hipEvent_t e0 = tm ? tm->e0 : nullptr, e1 = tm ? tm->e1 : nullptr;
  const int lidx = tm ? tm->lidx : -1;
  // F reads one column / value entry even for an empty pass: a matrix without nonzeros
  // gets stand-in arrays (never used in a product)
  const int *colp = A.nnz > 0 ? A.col : A.rowptr;
  const void *valp = A.nnz > 0 ? A.val : (const void *)V;
  if (A.fp32)
    hipExtLaunchKernelGGL((k_gm_f<float, TV, RB, R, PC>), dim3(nb), dim3(KTPB), 0, st, e0, e1, 0, A.rowptr, colp,
                          (const float *)valp, V, T, A.n, ld, j, mode, PA(partials), nb, PB(partials), ctl, lidx,
                          dinv);
  else
    hipExtLaunchKernelGGL((k_gm_f<double, TV, RB, R, PC>), dim3(nb), dim3(KTPB), 0, st, e0, e1, 0, A.rowptr,
                          colp, (const double *)valp, V, T, A.n, ld, j, mode, PA(partials), nb, PB(partials), ctl,
                          lidx, dinv);
}

template <typename TV, int RB, int R>
static void gm_f_launch(const CsrView &A, TV *V, TV *T, int64_t ld, int j, int mode, double *partials, Ctl *ctl,
                        hipStream_t st, const KTiming *tm, const TV *dinv) {
  if (dinv)
    gm_f_launch_pc<TV, RB, R, true>(A, V, T, ld, j, mode, partials, ctl, st, tm, dinv);
  else
    gm_f_launch_pc<TV, RB, R, false>(A, V, T, ld, j, mode, partials, ctl, st, tm, dinv);
}

// F takes two row tiles per pass only at 8 slots on grids with two tiles per block
// (measured 9.5 against 9.8 us); from 16 slots one tile per pass with the next pass's
// SpMV round requested ahead is faster (12.9 against 13.8 us at j = 12), and at 32 two
// tiles would not fit in the registers of two waves per SIMD
template <typename TV, int RB>
static void gm_f_rb(const CsrView &A, TV *V, TV *T, int64_t ld, int j, int mode, double *partials, Ctl *ctl,
                    hipStream_t st, const KTiming *tm, const TV *dinv) {
  if constexpr (RB <= 8) {
    if (gm_two_rows(A.n)) {
      gm_f_launch<TV, RB, 2>(A, V, T, ld, j, mode, partials, ctl, st, tm, dinv);
      return;
    }
  }
  gm_f_launch<TV, RB, 1>(A, V, T, ld, j, mode, partials, ctl, st, tm, dinv);
}

// G takes two row tiles per pass up to 8 columns on grids with two tiles per block, one
// tile otherwise (measured: two tiles 6.2 against 6.4 us at 8 slots, equal at 16, slower
// at 32 where the column values of two tiles take most of the registers)
template <typename TV, int RB, bool NW>
static void gm_g_rb_nw(const CsrView &A, TV *V, TV *T, int64_t ld, int j, double *partials, Ctl *ctl, hipStream_t st,
                       int serial) {
  const int nb = kblocks(A.n);
  if constexpr (RB <= 8) {
    if (gm_two_rows(A.n)) {
      hipLaunchKernelGGL((k_gm_g<TV, RB, 2, NW>), dim3(nb), dim3(KTPB), 0, st, V, T, A.n, ld, j, PB(partials), nb,
                         PA(partials), ctl, serial);
      return;
    }
  }
  hipLaunchKernelGGL((k_gm_g<TV, RB, 1, NW>), dim3(nb), dim3(KTPB), 0, st, V, T, A.n, ld, j, PB(partials), nb,
                     PA(partials), ctl, serial);
}

template <typename TV, int RB>
static void gm_g_rb(const CsrView &A, TV *V, TV *T, int64_t ld, int j, double *partials, Ctl *ctl, hipStream_t st,
                    int serial, bool nw) {
  if (nw && j + 1 < RB)
    gm_g_rb_nw<TV, RB, true>(A, V, T, ld, j, partials, ctl, st, serial);
  else
    gm_g_rb_nw<TV, RB, false>(A, V, T, ld, j, partials, ctl, st, serial);
}

// Arnoldi step j of a cycle: F(j), G(j).  first_mode: 0 first cycle, 1 restart
// (used at j = 0); norm_w: G(j) also records ||w'||^2 (see k_gm_g).
template <typename TV>
hipError_t launch_gm_step(const CsrView &A, TV *V, TV *T, int64_t ld, int j, int first_mode, double *partials,
                          Ctl *ctl, hipStream_t st, const KTiming *tm, int serial, bool norm_w, const TV *dinv) {
  const int mode = j == 0 ? first_mode : 0;
  if (j <= 8)
    gm_f_rb<TV, 8>(A, V, T, ld, j, mode, partials, ctl, st, tm, dinv);
  else if (j <= 16)
    gm_f_rb<TV, 16>(A, V, T, ld, j, mode, partials, ctl, st, tm, dinv);
  else
    gm_f_rb<TV, 32>(A, V, T, ld, j, mode, partials, ctl, st, tm, dinv);
  if (j < 8)
    gm_g_rb<TV, 8>(A, V, T, ld, j, partials, ctl, st, serial, norm_w);
  else if (j < 16)
    gm_g_rb<TV, 16>(A, V, T, ld, j, partials, ctl, st, serial, norm_w);
  else
    gm_g_rb<TV, 32>(A, V, T, ld, j, partials, ctl, st, serial, norm_w);
  return hipGetLastError();
}

// end of a cycle of m steps: F(m) finalise-only, then (close) the close of step m - 1
template <typename TV>
hipError_t launch_gm_finish(const CsrView &A, TV *V, TV *T, int64_t ld, int m, double *partials, Ctl *ctl,
                            hipStream_t st, bool close) {
  // the finalise-only step F(m) forms no product: the operand scaling does not matter
  const int nb = kblocks(A.n);
  if (m <= 8)
    gm_f_rb<TV, 8>(A, V, T, ld, m, 2, partials, ctl, st, nullptr, nullptr);
  else if (m <= 16)
    gm_f_rb<TV, 16>(A, V, T, ld, m, 2, partials, ctl, st, nullptr, nullptr);
  else
    gm_f_rb<TV, 32>(A, V, T, ld, m, 2, partials, ctl, st, nullptr, nullptr);
  if (close) hipLaunchKernelGGL(k_gm_close, dim3(1), dim3(KTPB), 0, st, PB(partials), nb, m - 1, ctl);
  return hipGetLastError();
}

template <typename TV, int RB, bool PC>
static void gm_update_pc(TV *x, const TV *V, int64_t n, int64_t ld, Ctl *ctl, const double *Pin, int jclose,
                         int pyth, hipStream_t st, const TV *dinv) {
  const int nb = kblocks(n);
  if (gm_two_rows(n))
    hipLaunchKernelGGL((k_gm_update<TV, RB, 2, PC>), dim3(nb), dim3(KTPB), 0, st, x, V, n, ld, ctl, Pin, nb,
                       jclose, pyth, dinv);
  else
    hipLaunchKernelGGL((k_gm_update<TV, RB, 1, PC>), dim3(nb), dim3(KTPB), 0, st, x, V, n, ld, ctl, Pin, nb,
                       jclose, pyth, dinv);
}

template <typename TV, int RB>
static void gm_update_rb(TV *x, const TV *V, int64_t n, int64_t ld, Ctl *ctl, const double *Pin, int jclose,
                         int pyth, hipStream_t st, const TV *dinv) {
  if (dinv)
    gm_update_pc<TV, RB, true>(x, V, n, ld, ctl, Pin, jclose, pyth, st, dinv);
  else
    gm_update_pc<TV, RB, false>(x, V, n, ld, ctl, Pin, jclose, pyth, st, dinv);
}

// whether G(m - 1) stores ||w'_m||^2 (a spare slot past its live columns): then a full
// cycle of m steps needs no finalise step F(m)
bool gm_norm_in_g(int m) { return m >= 1 && m < 32 && m != 8 && m != 16; }

template <typename TV>
hipError_t launch_gm_update(TV *x, const TV *V, int64_t n, int64_t ld, int restart, Ctl *ctl, hipStream_t st,
                            double *partials, bool close_last, bool from_g, const TV *dinv) {
  const int pyth = close_last && from_g ? 1 : 0;
  const double *Pin = partials ? (pyth ? PA(partials) : PB(partials)) : nullptr;
  const int jclose = close_last ? restart - 1 : -1;
  if (restart <= 8)
    gm_update_rb<TV, 8>(x, V, n, ld, ctl, Pin, jclose, pyth, st, dinv);
  else if (restart <= 16)
    gm_update_rb<TV, 16>(x, V, n, ld, ctl, Pin, jclose, pyth, st, dinv);
  else
    gm_update_rb<TV, 32>(x, V, n, ld, ctl, Pin, jclose, pyth, st, dinv);
  return hipGetLastError();
}

// Jacobi: one thread per row sums the row's entries in the diagonal column
template <typename VT, typename TV>
__global__ __launch_bounds__(KTPB) void k_jacobi_dinv(const int *rowptr, const int *col, const VT *val, TV *dinv,
                                                      int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * KTPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KTPB) {
    double d = 0.0;
    for (int k = rowptr[i], e = rowptr[i + 1]; k < e; ++k)
      if (col[k] == (int)i) d += (double)val[k];
    dinv[i] = (TV)(d != 0.0 ? 1.0 / d : 1.0);
  }
}

template <typename TV>
hipError_t launch_jacobi_dinv(const CsrView &A, TV *dinv, hipStream_t st) {
  const int nb = kblocks(A.n);
  if (A.fp32)
    hipLaunchKernelGGL((k_jacobi_dinv<float, TV>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const float *)A.val, dinv, A.n);
  else
    hipLaunchKernelGGL((k_jacobi_dinv<double, TV>), dim3(nb), dim3(KTPB), 0, st, A.rowptr, A.col,
                       (const double *)A.val, dinv, A.n);
  return hipGetLastError();
}

// Packed 16-bit column offsets: out[p] = col[p] - row for every entry; *ok = 0 when an
// offset does not fit (the caller sets *ok = 1 first; every failing row writes 0).
__global__ __launch_bounds__(KTPB) void k_col_rel16(const int *rowptr, const int *col, int64_t n, short *out,
                                                    int *ok) {
  bool fits = true;
  GRID_ROWS(i, n) {
    const int a = rowptr[i], b = rowptr[i + 1];
    for (int p = a; p < b; ++p) {
      const int64_t d = (int64_t)col[p] - i;
      fits = fits && d >= -32768 && d <= 32767;
      out[p] = (short)d;
    }
  }
  if (!fits) *ok = 0;
}

hipError_t launch_col_rel16(const CsrView &A, short *out, int *ok, hipStream_t st) {
  if (A.nnz > 0)
    hipLaunchKernelGGL(k_col_rel16, dim3(kblocks(A.n)), dim3(KTPB), 0, st, A.rowptr, A.col, A.n, out, ok);
  return hipGetLastError();
}

#define SACC_INSTANTIATE_KRYLOV(TV)                                                                              \
  template hipError_t launch_cg_start_k<TV>(const CsrView &, const TV *, const TV *, TV *, int, double *, Ctl *, \
                                            hipStream_t, int, const TV *, int);                                  \
  template hipError_t launch_cg_iter<TV>(const CsrView &, TV *, TV *, TV *, TV *, double *, Ctl *, hipStream_t,  \
                                         const KTiming *, int, const TV *, int);                                 \
  template int cg_tile_tune<TV>(const CsrView &, const TV *, const TV *, TV *, double *, Ctl *, hipStream_t);    \
  template hipError_t launch_cg_xfix<TV>(const CsrView &, TV *, TV *, Ctl *, hipStream_t);                       \
  template hipError_t launch_gm_start<TV>(const CsrView &, const TV *, const TV *, TV *, int, double *, Ctl *,   \
                                          hipStream_t);                                                          \
  template hipError_t launch_gm_step<TV>(const CsrView &, TV *, TV *, int64_t, int, int, double *, Ctl *,        \
                                         hipStream_t, const KTiming *, int, bool, const TV *);                   \
  template hipError_t launch_gm_finish<TV>(const CsrView &, TV *, TV *, int64_t, int, double *, Ctl *,           \
                                           hipStream_t, bool);                                                   \
  template hipError_t launch_gm_update<TV>(TV *, const TV *, int64_t, int64_t, int, Ctl *, hipStream_t, double *, \
                                           bool, bool, const TV *);                                              \
  template hipError_t launch_jacobi_dinv<TV>(const CsrView &, TV *, hipStream_t);

SACC_INSTANTIATE_KRYLOV(double)
SACC_INSTANTIATE_KRYLOV(float)

// leading dimension of column-major n-row blocks: rounded to 512 rows plus 576, so
// consecutive columns start 4.5 KB apart modulo any power of two (columns exactly a
// power of two apart map onto the same memory channels)
int64_t padded_ld(int64_t n) { return (n + 511) / 512 * 512 + 576; }

size_t krylov_partials_doubles() { return (size_t)2 * PROWS * KW; }

int gm_f_rows_per_thread(int64_t n, int rb) { return rb <= 8 && gm_two_rows(n) ? 2 : 1; }

int cg_tile_chunk(int64_t n, int64_t nnz) { return wave_tile_chunk(n, nnz); }

}  // namespace sacc
