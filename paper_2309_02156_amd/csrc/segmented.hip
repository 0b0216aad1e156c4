// Segmented solve of many independent systems at once (the batched step of Section 5's
// independent plane sequences): FP64 iterative refinement around float32 CG or
// GMRES(m) inner solves, the same method as one sequence's mixed-mode solve, for every
// system of a batch in lockstep.
//
// The systems are segments of one launch.  Each segment owns a contiguous range of work
// items (1024 rows each: four waves of four 64-row tiles) and a state record in device
// memory that holds its phase and scalars.  A step of the engine is two launches over
// all segments: the data kernel (a resident grid striding over the items) does the row
// work of every item's segment in its current phase (items of finished segments are
// skipped) and leaves one partial row per item; the close kernel (one block per
// segment) reduces those rows in a fixed order and runs the segment's scalar logic,
// which picks its next phase.  No cross-block atomics or device-scope fences:
// the launch boundary orders the partial rows, as in the single-sequence kernels.  The
// host enqueues steps in chunks (a captured hipGraph of the chunk, or eager launches)
// and stops once every segment reports its end through a word in pinned host memory.
//
// Per segment (Alg. 1's Krylov stage; the refinement is this build's mixed mode):
//   RES   r = b - A x (FP64), r32 = fl32(r), d = 0; ||r||, ||r32||, ||b|| -> stop
//         (converged, breakdown, sweeps or iterations spent) or start an inner solve
//   CG:   CGQ  p = fl32(r + beta p) (p = r first), q = fl32(A p), p^T q -> alpha
//         CGU  d = fl32(d + alpha p), r = fl32(r - alpha q), r^T r -> stop or beta
//   GMRES (classical Gram-Schmidt twice, two passes over V per Arnoldi step):
//         F(j) v_j = fl32((u - V_{<j} h2) / s), with u the once-orthogonalised vector of
//              step j - 1 (the residual and s = beta at j = 0) and s = ||w''_{j-1}||;
//              w_j = A v_j = fl32((fl32(A u) - sum_{l<j} h2_l A v_l) / s), the SpMV taken
//              of the stored u and each A v_l = V H[:, l] by the Arnoldi relation, so the
//              correction is a combination sum_k c_k v_k of the columns the pass reads
//              anyway; h = V_{<=j}^T w_j
//         G(j) w' = fl32(w_j - V h), h2 = V_{<=j}^T w', ||w'||^2 -> column j of H =
//              h + h2, ||w''_j|| = sqrt(||w'||^2 - ||h2||^2), Givens rotation, residual
//              estimate, end of cycle or F(j + 1)
//         UPD  d = fl32(d + V y)          (end of a cycle)
//         GRES u = fl32(r32 - A d), ||u|| -> restart or stop
//   XUPD  x += d (FP64), next sweep
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/sacc.h"
#include "kernels.h"

namespace sacc {

namespace {

constexpr int SG_TPB = 256;                    // threads per block
constexpr int SG_NW = SG_TPB / WAVE;           // waves per block
// A work item is TW 64-row tiles per wave: SG_NW TW 64 rows, TW rows per thread in the
// element-wise phases.  TW = 4 (1024 rows) or 2 (512 rows), chosen per batch: larger
// items leave fewer partial rows, smaller ones shorten a block's chain of tiles, which
// sets the step time when every system is small.
constexpr int SG_TW_MAX = 4;
__host__ __device__ constexpr int item_rows(int tw) { return SG_NW * tw * WAVE; }
constexpr int SG_R = MAXR;                     // longest GMRES cycle
constexpr int SG_PW = SG_R + 2;                // doubles per partial row

enum SegPhase : int { SP_RES, SP_XUPD, SP_CGQ, SP_CGU, SP_F, SP_G, SP_UPD, SP_GRES, SP_DONE };

// State of one segment.  The summary (ints and the norms) comes first: the host copies
// only that part back.
struct SegState {
  int phase, status, sweep, sweeps, iters, restarts;
  int inner_it, icap_cur, j, jend, cycles, par, first, pad;
  double bnorm, relres0, relres;
  double bytes;  // algorithmic bytes of the row work done so far in this solve
  double ith, rho, alpha, beta, hn;
  double h[SG_R + 1], h2[SG_R + 1], c[SG_R + 1], g[SG_R + 1], cs[SG_R], sn[SG_R], y[SG_R];
  double Hraw[SG_R * (SG_R + 1)];  // Hessenberg columns as built: column j at Hraw[j * (SG_R + 1)]
  double H[SG_R * (SG_R + 1)];     // the same after the Givens rotations
};
constexpr size_t SG_SUMMARY = offsetof(SegState, ith);

// partial-row entries a phase leaves (j: the Arnoldi step)
__host__ __device__ inline int phase_cols(int phase, int j) {
  switch (phase) {
    case SP_RES: return 3;
    case SP_CGQ: case SP_CGU: case SP_GRES: return 1;
    case SP_F: return j + 1;
    case SP_G: return j + 2;
    default: return 0;
  }
}

__device__ inline float *kcol(const SegDesc &d, int c) { return d.kry + (size_t)c * (size_t)d.ld; }
// GMRES work columns: F(j) reads xcol(d, j + 1) and writes xcol(d, j), which G(j)
// rewrites in place (columns m and m + 1: V_m itself is never formed)
__device__ inline float *xcol(const SegDesc &d, int j) { return kcol(d, d.m + (j & 1)); }

// ---------------------------------------------------------------------------- data kernel
// Column dots of a wave's tile through LDS: the tile's rows of V[:, 0..jc) are staged
// column by column (lane = row, loads coalesced), then lane L sums column L % 32 over
// half L / 32 of the tile's rows, so a lane keeps one running sum however many columns
// there are.  sV: the wave's LDS slice of SG_R + 1 columns of 65 floats (stride 65: the
// 32 lanes of a half read 32 different banks); sy: the tile's y values (64 floats).
constexpr int SG_LDV = WAVE + 1;

__device__ inline double tile_col_dots(const float *sV, const float *sy, int jc) {
  const int lane = threadIdx.x % WAVE, c = lane & 31, r0 = (lane >> 5) * 32;
  double s = 0.0;
  if (c < jc) {
#pragma unroll 8
    for (int r = 0; r < 32; ++r) s += (double)sV[c * SG_LDV + r0 + r] * (double)sy[r0 + r];
  }
  return s;
}

// Row ic of V's columns 0..NV-1 into v, all loads issued before any use (columns past
// `last` re-read column `last`; callers ignore them)
template <int NV>
__device__ inline void load_cols(const float *__restrict__ V, size_t ld, int64_t ic, int last, float (&v)[NV]) {
#pragma unroll
  for (int l = 0; l < NV; ++l) v[l] = V[(size_t)(l <= last ? l : last) * ld + ic];
}

// fn(Nch<k>) for k = nch clamped to 0..4: the number of 8-column chunks a phase touches
// as a compile-time constant
template <int N>
struct Nch {
  static constexpr int value = N;
};
template <typename Fn>
__device__ inline void with_nch(int nch, const Fn &fn) {
  switch (nch) {
    case 0: fn(Nch<0>{}); break;
    case 1: fn(Nch<1>{}); break;
    case 2: fn(Nch<2>{}); break;
    case 3: fn(Nch<3>{}); break;
    default: fn(Nch<4>{}); break;
  }
}

// the block's column sums (columns < kc <= 32) of per-lane sums laid out as in
// tile_col_dots, into out[0..kc)
__device__ inline void col_sums_store(double acc, int kc, double *red, double *out) {
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  const double other = __shfl_down(acc, 32);
  if (lane < 32) red[wid * 32 + lane] = acc + other;
  __syncthreads();
  if ((int)threadIdx.x < kc) {
    double s = 0.0;
    for (int w = 0; w < SG_NW; ++w) s += red[w * 32 + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// The row work of one work item (a segment's block of item_rows(TW) rows) in the
// segment's current phase; leaves the item's partial row.
template <int C, int TW>
__device__ inline void seg_item(const SegDesc &d, const SegState &st, int phase, int lb, char *lds, double *red,
                                double *red1, double *coef, double *coef2) {
  int(*lcol)[WT_CAP] = (int(*)[WT_CAP])lds;
  float(*lval)[WT_CAP] = (float(*)[WT_CAP])(lds + SG_NW * WT_CAP * sizeof(int));
  float *sV = (float *)lds + (threadIdx.x / WAVE) * ((SG_R + 1) * SG_LDV + WAVE);
  float *sy = sV + (SG_R + 1) * SG_LDV;
  const int tid = threadIdx.x, wid = tid / WAVE;
  const int64_t n = d.n;
  const int64_t T = (n + WAVE - 1) / WAVE;
  const int64_t t0 = (int64_t)lb * (SG_NW * TW);
  const int64_t tend = t0 + SG_NW * TW < T ? t0 + SG_NW * TW : T;
  const int64_t row0 = (int64_t)lb * item_rows(TW);
  double *out = d.part + (size_t)lb * SG_PW;
  const int gm = d.solver == SA_GMRES;
  const int m = d.m;

  switch (phase) {
    case SP_RES: {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      const double *__restrict__ x = d.x;
      const double *__restrict__ b = d.b;
      float *__restrict__ R = gm ? kcol(d, m + 1) : kcol(d, 0);
      float *__restrict__ r32 = d.r32;
      float *__restrict__ dd = d.d32;
      wave_tiles_spmv<C>(
          d.rowptr, d.col, d.val, [&](int c) { return x[c]; }, n, t0 + wid, tend, SG_NW, lcol[wid], lval[wid],
          [&](int64_t ic) { return b[ic]; },
          [&](int64_t i, double bi, double ax) {
            const double r = bi - ax;
            const float rf = (float)r;
            r32[i] = rf;
            R[i] = rf;
            dd[i] = 0.0f;
            acc[0] += r * r;
            acc[1] += (double)rf * (double)rf;
            acc[2] += bi * bi;
          });
      block_sum_store<4>(acc, 3, red, out);
      break;
    }
    case SP_XUPD: {
      double *__restrict__ x = d.x;
      const float *__restrict__ dd = d.d32;
#pragma unroll
      for (int k = 0; k < TW; ++k) {
        const int64_t i = row0 + k * SG_TPB + tid;
        if (i < n) x[i] = x[i] + (double)dd[i];
      }
      break;
    }
    case SP_CGQ: {
      const int par = st.par;
      const bool first = st.first != 0;
      const double beta = st.beta;
      const float *__restrict__ R = kcol(d, 0);
      const float *__restrict__ Po = kcol(d, 1 + par);
      float *__restrict__ Pn = kcol(d, 2 - par);
      float *__restrict__ Q = kcol(d, 3);
      // p at any row, from r and the previous p (the same rounding wherever it is formed)
      auto pv = [&](int64_t c) -> float {
        return first ? R[c] : (float)__dadd_rn((double)R[c], __dmul_rn(beta, (double)Po[c]));
      };
      double acc[1] = {0.0};
      wave_tiles_spmv<C>(
          d.rowptr, d.col, d.val, [&](int c) { return pv(c); }, n, t0 + wid, tend, SG_NW, lcol[wid], lval[wid],
          [&](int64_t ic) { return (double)pv(ic); },
          [&](int64_t i, double p, double ap) {
            const float q = (float)ap;
            Q[i] = q;
            Pn[i] = (float)p;
            acc[0] += p * (double)q;
          });
      block_sum_store<1>(acc, 1, red, out);
      break;
    }
    case SP_CGU: {
      const double alpha = st.alpha;
      const float *__restrict__ P = kcol(d, 2 - st.par);
      float *__restrict__ R = kcol(d, 0);
      const float *__restrict__ Q = kcol(d, 3);
      float *__restrict__ dd = d.d32;
      double acc[1] = {0.0};
#pragma unroll
      for (int k = 0; k < TW; ++k) {
        const int64_t i = row0 + k * SG_TPB + tid;
        if (i < n) {
          const float dn = (float)__dadd_rn((double)dd[i], __dmul_rn(alpha, (double)P[i]));
          const float rn = (float)__dadd_rn((double)R[i], -__dmul_rn(alpha, (double)Q[i]));
          dd[i] = dn;
          R[i] = rn;
          acc[0] += (double)rn * (double)rn;
        }
      }
      block_sum_store<1>(acc, 1, red, out);
      break;
    }
    case SP_F: {
      const int j = st.j;
      const double sc = st.hn;
      if (tid < j) coef[tid] = st.h2[tid];
      if (tid <= j) coef2[tid] = st.c[tid];
      const float *__restrict__ U = xcol(d, j + 1);
      float *__restrict__ Wn = xcol(d, j);
      float *__restrict__ Vj = kcol(d, j);
      const float *__restrict__ V = d.kry;
      const size_t ld = (size_t)d.ld;
      // y = A u (stored in float32 where w_j goes), then per tile: v_j, w_j and the dots
      wave_tiles_spmv<C>(
          d.rowptr, d.col, d.val, [&](int c) { return U[c]; }, n, t0 + wid, tend, SG_NW, lcol[wid], lval[wid],
          [&](int64_t) { return 0.0; }, [&](int64_t i, double, double au) { Wn[i] = (float)au; });
      __syncthreads();  // coefficients in; the LDS slices become the staged columns
      double acc = 0.0;
      const int lane = tid % WAVE;
      with_nch((j + 8) / 8, [&](auto kk) {
        constexpr int NV = (decltype(kk)::value > 0 ? decltype(kk)::value : 1) * 8;  // columns l <= j
        for (int64_t t = t0 + wid; t < tend; t += SG_NW) {
          const int64_t i = t * WAVE + lane;
          const bool ok = i < n;
          const int64_t ic = ok ? i : n - 1;
          float vv[NV];
          load_cols<NV>(V, ld, ic, j > 0 ? j - 1 : 0, vv);
          // coefficients read from LDS at each use (z: an offset the compiler cannot
          // hoist; kept in registers they would take 128 per lane and halve occupancy)
          const int z = vzero();
          double v = (double)U[ic], a = (double)Wn[ic];
#pragma unroll
          for (int l = 0; l < NV; ++l)
            if (l < j) {
              v = __dadd_rn(v, -__dmul_rn(coef[l + z], (double)vv[l]));
              a = __dadd_rn(a, -__dmul_rn(coef2[l + z], (double)vv[l]));
              sV[l * SG_LDV + lane] = ok ? vv[l] : 0.0f;
            }
          const float vj = (float)(v / sc);
          a = __dadd_rn(a, -__dmul_rn(coef2[j], (double)vj));
          const float wf = (float)(a / sc);
          if (ok) {
            Vj[i] = vj;
            Wn[i] = wf;
          }
          sV[j * SG_LDV + lane] = ok ? vj : 0.0f;
          sy[lane] = ok ? wf : 0.0f;
          wave_lds_sync();
          acc += tile_col_dots(sV, sy, j + 1);
          wave_lds_sync();
        }
      });
      col_sums_store(acc, j + 1, red, out);
      break;
    }
    case SP_G: {
      const int j = st.j;
      if (tid <= j) coef[tid] = st.h[tid];
      __syncthreads();
      float *__restrict__ W = xcol(d, j);
      const float *__restrict__ V = d.kry;
      const size_t ld = (size_t)d.ld;
      const int lane = tid % WAVE;
      double acc = 0.0, ww[1] = {0.0};
      with_nch((j + 8) / 8, [&](auto kk) {
        constexpr int NV = (decltype(kk)::value > 0 ? decltype(kk)::value : 1) * 8;  // columns l <= j
        for (int64_t t = t0 + wid; t < tend; t += SG_NW) {
          const int64_t i = t * WAVE + lane;
          const bool ok = i < n;
          const int64_t ic = ok ? i : n - 1;
          float vv[NV];
          load_cols<NV>(V, ld, ic, j, vv);
          const int z = vzero();
          double w = (double)W[ic];
#pragma unroll
          for (int l = 0; l < NV; ++l)
            if (l <= j) {
              sV[l * SG_LDV + lane] = ok ? vv[l] : 0.0f;
              w = __dadd_rn(w, -__dmul_rn(coef[l + z], (double)vv[l]));
            }
          const float wf = (float)w;
          if (ok) W[i] = wf;
          sy[lane] = ok ? wf : 0.0f;
          if (ok) ww[0] += (double)wf * (double)wf;
          wave_lds_sync();
          acc += tile_col_dots(sV, sy, j + 1);
          wave_lds_sync();
        }
      });
      col_sums_store(acc, j + 1, red, out);
      __syncthreads();
      block_sum_store<1>(ww, 1, red1, out + j + 1);
      break;
    }
    case SP_UPD: {
      const int jend = st.jend;
      if (tid < jend) coef[tid] = st.y[tid];
      __syncthreads();
      const float *__restrict__ V = d.kry;
      float *__restrict__ dd = d.d32;
      const size_t ld = (size_t)d.ld;
      with_nch((jend + 7) / 8, [&](auto kk) {
        constexpr int NV = decltype(kk)::value * 8;  // columns l < jend
        if constexpr (NV > 0) {
          for (int k = 0; k < TW; ++k) {
            const int64_t i = row0 + k * SG_TPB + tid;
            if (i < n) {
              float vv[NV];
              load_cols<NV>(V, ld, i, jend - 1, vv);
              const int z = vzero();
              double u = 0.0;
#pragma unroll
              for (int l = 0; l < NV; ++l)
                if (l < jend) u = __dadd_rn(u, __dmul_rn((double)vv[l], coef[l + z]));
              dd[i] = (float)((double)dd[i] + u);
            }
          }
        }
      });
      break;
    }
    case SP_GRES: {
      const float *__restrict__ dd = d.d32;
      const float *__restrict__ r32 = d.r32;
      float *__restrict__ W = kcol(d, m + 1);
      double acc[1] = {0.0};
      wave_tiles_spmv<C>(
          d.rowptr, d.col, d.val, [&](int c) { return dd[c]; }, n, t0 + wid, tend, SG_NW, lcol[wid], lval[wid],
          [&](int64_t ic) { return (double)r32[ic]; },
          [&](int64_t i, double bi, double ad) {
            const float r = (float)(bi - ad);
            W[i] = r;
            acc[0] += (double)r * (double)r;
          });
      block_sum_store<1>(acc, 1, red, out);
      break;
    }
    default:
      break;
  }
}

// A resident grid that strides over the work items (item i: block i - blk0[s] of the
// segment s owning it).  Each block first reads, with one load per item, which of its
// items belong to a segment still running, so finished segments cost no memory trips.
constexpr int SG_MAXIT = 64;  // work items per block at most (the grid is sized for it)

template <int C, int TW>
__global__ __launch_bounds__(SG_TPB, 4) void k_seg_data(const SegDesc *__restrict__ D, const SegState *__restrict__ S,
                                                    const int *__restrict__ blkseg, const int *__restrict__ blk0,
                                                    int nitems) {
  // LDS: the SpMV tiles' column / value slices, or the staged V columns of the dots
  constexpr int SPMV_B = SG_NW * WT_CAP * (int)(sizeof(int) + sizeof(float));
  constexpr int DOTS_B = SG_NW * ((SG_R + 1) * SG_LDV + WAVE) * (int)sizeof(float);
  __shared__ __align__(16) char lds[SPMV_B > DOTS_B ? SPMV_B : DOTS_B];
  __shared__ double red[SG_NW * 32];
  __shared__ double red1[SG_NW];
  __shared__ double coef[SG_R + 1], coef2[SG_R + 1];
  __shared__ int iseg[SG_MAXIT], iph[SG_MAXIT];
  const int G = gridDim.x;
  const int mine = (nitems - (int)blockIdx.x + G - 1) / G;
  for (int k = threadIdx.x; k < mine && k < SG_MAXIT; k += blockDim.x) {
    const int s = blkseg[blockIdx.x + k * G];
    iseg[k] = s;
    iph[k] = S[s].phase;
  }
  __syncthreads();
  for (int k = 0; k < mine && k < SG_MAXIT; ++k) {
    const int phase = iph[k];
    if (phase == SP_DONE) continue;
    const int s = iseg[k];
    const SegDesc d = D[s];
    seg_item<C, TW>(d, S[s], phase, (int)blockIdx.x + k * G - blk0[s], lds, red, red1, coef, coef2);
    __syncthreads();  // LDS reuse by the next item
  }
}

// ---------------------------------------------------------------------------- close kernel
// Givens rotation [c s; -s c] [a; b] = [rho; 0] (c = 1, s = 0 when a = b = 0)
__device__ inline void givens(double a, double b, double &c, double &s, double &rho) {
  rho = hypot(a, b);
  if (rho == 0.0) {
    c = 1.0;
    s = 0.0;
  } else {
    c = a / rho;
    s = b / rho;
  }
}

__device__ inline void seg_finish(SegState &st, int status, int s, volatile int *done) {
  st.status = status;
  st.phase = SP_DONE;
  done[s] = 1;
}

// the end of an inner solve (not a breakdown): the correction goes into x
__device__ inline void inner_end(SegState &st) {
  st.restarts += st.cycles > 1 ? st.cycles - 1 : 0;
  st.phase = SP_XUPD;
}

// a GMRES cycle from the residual in xcol(d, 1) with norm beta: F(0) forms v_0 = r / beta
__device__ inline void cycle_start(SegState &st, double beta) {
  st.beta = beta;
  st.g[0] = beta;
  st.hn = beta;
  st.c[0] = 0.0;
  st.j = 0;
  st.phase = SP_F;
}

// Algorithmic bytes of one phase's row work (float32 operator values and Krylov
// columns, FP64 x and b): the CSR arrays once, each vector read or written once.
__device__ inline double phase_bytes(int phase, int j, int jend, int64_t n, int64_t nnz) {
  const double csr = 4.0 * (double)(n + 1) + 8.0 * (double)nnz, N = (double)n;
  switch (phase) {
    case SP_RES: return csr + 28.0 * N;             // x, b; r32, r, d
    case SP_XUPD: return 20.0 * N;                  // x read and written, d
    case SP_CGQ: return csr + 16.0 * N;             // r, p; p', q
    case SP_CGU: return 24.0 * N;                   // p, q, d, r; d, r
    case SP_F: return csr + (12.0 + 4.0 * j) * N;   // u, V_{<j}; v_j, w_j
    case SP_G: return (12.0 + 4.0 * j) * N;         // w, V_{<=j}; w'
    case SP_UPD: return (8.0 + 4.0 * jend) * N;     // V_{<jend}, d; d
    case SP_GRES: return csr + 12.0 * N;            // d, r32; u
    default: return 0.0;
  }
}

__device__ void seg_logic(const SegDesc &d, SegState &st, const double *tot, int s, volatile int *done) {
  const bool gm = d.solver == SA_GMRES;
  st.bytes += phase_bytes(st.phase, st.j, st.jend, d.n, d.nnz);
  switch (st.phase) {
    case SP_RES: {
      const double nr = sqrt(tot[0]);
      if (st.sweep == 0) st.bnorm = sqrt(tot[2]);
      const double bn = st.bnorm;
      if (bn == 0.0) {
        st.relres0 = st.relres = 0.0;
        seg_finish(st, ST_ZERO_RHS, s, done);
        return;
      }
      st.relres = nr / bn;
      if (st.sweep == 0) st.relres0 = st.relres;
      if (nr <= d.tol * bn) {
        seg_finish(st, ST_CONV, s, done);
      } else if (!isfinite(nr)) {
        seg_finish(st, ST_BREAK, s, done);
      } else if (st.sweep == d.max_refine || st.iters >= d.maxit) {
        seg_finish(st, ST_MAXIT, s, done);
      } else {
        const double ibn = sqrt(tot[1]);
        st.ith = d.itol * ibn;
        st.icap_cur = d.maxit - st.iters < d.icap ? d.maxit - st.iters : d.icap;
        st.inner_it = 0;
        st.cycles = 0;
        if (!gm) {
          st.rho = tot[1];
          st.first = 1;
          st.par = 0;
          st.phase = ibn <= st.ith ? SP_XUPD : SP_CGQ;
        } else if (ibn > st.ith) {
          cycle_start(st, ibn);
        } else {
          st.phase = SP_XUPD;
        }
      }
      return;
    }
    case SP_XUPD:
      st.sweeps = st.sweep + 1;
      st.sweep += 1;
      st.phase = SP_RES;
      return;
    case SP_CGQ: {
      const double pq = tot[0];
      if (!(pq > 0.0) || !isfinite(pq)) {
        seg_finish(st, ST_BREAK, s, done);
        return;
      }
      st.alpha = st.rho / pq;
      st.phase = SP_CGU;
      return;
    }
    case SP_CGU: {
      const double rr = tot[0];
      st.inner_it += 1;
      st.iters += 1;
      if (sqrt(rr) <= st.ith || st.inner_it >= st.icap_cur) {
        inner_end(st);
      } else {
        st.beta = rr / st.rho;
        st.rho = rr;
        st.par ^= 1;
        st.first = 0;
        st.phase = SP_CGQ;
      }
      return;
    }
    case SP_F:
      for (int l = 0; l <= st.j; ++l) st.h[l] = tot[l];
      st.phase = SP_G;
      return;
    case SP_G: {
      const int j = st.j;
      double *Hr = st.Hraw + j * (SG_R + 1);
      double *Hc = st.H + j * (SG_R + 1);
      double h2sq = 0.0;
      for (int l = 0; l <= j; ++l) {
        st.h2[l] = tot[l];
        Hr[l] = Hc[l] = st.h[l] + tot[l];
        h2sq += tot[l] * tot[l];
      }
      const double wsq = tot[j + 1] - h2sq;
      const double hnext = wsq > 0.0 ? sqrt(wsq) : 0.0;
      Hr[j + 1] = hnext;
      for (int l = 0; l < j; ++l) {
        const double t = st.cs[l] * Hc[l] + st.sn[l] * Hc[l + 1];
        Hc[l + 1] = -st.sn[l] * Hc[l] + st.cs[l] * Hc[l + 1];
        Hc[l] = t;
      }
      double c, sn, rho;
      givens(Hc[j], hnext, c, sn, rho);
      st.cs[j] = c;
      st.sn[j] = sn;
      Hc[j] = rho;
      st.g[j + 1] = -sn * st.g[j];
      st.g[j] = c * st.g[j];
      st.inner_it += 1;
      st.iters += 1;
      st.jend = j + 1;
      if (fabs(st.g[j + 1]) <= st.ith || hnext == 0.0 || st.inner_it >= st.icap_cur || j + 1 == d.m) {
        // the cycle ends: y from the rotated triangle
        const int je = j + 1;
        for (int i = je - 1; i >= 0; --i) {
          double t = st.g[i];
          for (int k = i + 1; k < je; ++k) t -= st.H[k * (SG_R + 1) + i] * st.y[k];
          st.y[i] = t / st.H[i * (SG_R + 1) + i];
        }
        st.phase = SP_UPD;
      } else {
        // F(j + 1) next; its coefficients c (seg_coefs) are formed by the whole block
        st.hn = hnext;
        st.j = j + 1;
        st.phase = SP_F;
      }
      return;
    }
    case SP_UPD:
      st.phase = SP_GRES;
      return;
    case SP_GRES: {
      const double beta = sqrt(tot[0]);
      st.cycles += 1;
      const bool est = fabs(st.g[st.jend]) <= st.ith;
      if (beta <= st.ith || (est && isfinite(beta))) {
        inner_end(st);
      } else if (!isfinite(beta)) {
        st.restarts += st.cycles > 1 ? st.cycles - 1 : 0;
        seg_finish(st, ST_BREAK, s, done);
      } else if (st.inner_it >= st.icap_cur) {
        inner_end(st);
      } else {
        cycle_start(st, beta);
      }
      return;
    }
    default:
      return;
  }
}

// F(j)'s coefficients after G(j - 1): sum_{l<j} h2_l A v_l = sum_{k<=j} c_k v_k with
// A v_l = V Hraw[:, l] (the Arnoldi relation); thread k forms c_k.
__device__ inline void seg_coefs(SegState &st) {
  const int j = st.j, k = threadIdx.x;
  if (k <= j) {
    double t = 0.0;
    for (int l = k > 0 ? k - 1 : 0; l < j; ++l) t += st.h2[l] * st.Hraw[l * (SG_R + 1) + k];
    st.c[k] = t;
  }
}

constexpr int SC_TPB = 1024;  // threads of a close block

// The close kernel's sum of a segment's partial rows: final_sum with U rows per thread
// and round.  The rows and their order are the same whatever U, so are the sums; U is
// picked from the segment's item count so that a system of few work items does not
// issue 32 clamped loads per thread.
template <int U>
__device__ inline void close_sum_u(const double *partials, int nblk, int W, int kc, double *out, double *scratch) {
  for (int e0 = 0; e0 < kc; e0 += WAVE) {
    const int ec = kc - e0 < WAVE ? kc - e0 : WAVE;
    final_tree(final_part<U>(partials + e0, nblk, W, ec), ec, out + e0, scratch);
  }
}

__device__ inline void close_sum(const double *partials, int nblk, int W, int kc, double *out, double *scratch) {
  int ep = 1;
  while (ep < (kc < WAVE ? kc : WAVE)) ep <<= 1;
  const int ngrp = SC_TPB / ep;
  const int rows = (nblk + ngrp - 1) / ngrp;  // rows per thread
  if (rows <= 1)
    close_sum_u<1>(partials, nblk, W, kc, out, scratch);
  else if (rows <= 4)
    close_sum_u<4>(partials, nblk, W, kc, out, scratch);
  else
    close_sum_u<32>(partials, nblk, W, kc, out, scratch);
}

// One block per segment: the partial rows' sums in a fixed order, then the scalar logic
// on a copy of the state in LDS (one thread; the coefficients of the next F step by
// the block), copied back by the whole block.
static_assert(sizeof(SegState) % sizeof(double) == 0 && offsetof(SegState, Hraw) % sizeof(double) == 0 &&
                  offsetof(SegState, H) > offsetof(SegState, Hraw),
              "state copied as 8-byte words, the Hessenberg arrays last");

__global__ __launch_bounds__(SC_TPB) void k_seg_close(const SegDesc *__restrict__ D, SegState *__restrict__ S,
                                                     int *done) {
  __shared__ double tot[SG_PW];
  __shared__ double scratch[SC_TPB];
  __shared__ SegState ls;
  const int s = blockIdx.x;
  SegState &gs = S[s];
  const int phase = gs.phase;
  if (phase == SP_DONE) return;
  // the Hessenberg arrays (most of the state) are read and written only by a G close
  constexpr int NW8 = (int)(sizeof(SegState) / sizeof(double));
  constexpr int NSMALL = (int)(offsetof(SegState, Hraw) / sizeof(double));
  const int ncopy = phase == SP_G ? NW8 : NSMALL;
  for (int k = threadIdx.x; k < ncopy; k += SC_TPB) ((double *)&ls)[k] = ((const double *)&gs)[k];
  const SegDesc &d = D[s];
  const int kc = phase_cols(phase, gs.j);
  if (kc > 0) close_sum(d.part, d.nblk, SG_PW, kc, tot, scratch);
  __syncthreads();
  if (threadIdx.x == 0) seg_logic(d, ls, tot, s, (volatile int *)done);
  __syncthreads();
  if (phase == SP_G && ls.phase == SP_F) {
    seg_coefs(ls);
    __syncthreads();
  }
  for (int k = threadIdx.x; k < ncopy; k += SC_TPB) ((double *)&gs)[k] = ((const double *)&ls)[k];
}

__global__ void k_seg_init(SegState *S, int nseg) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  SegState &st = S[s];
  st.phase = SP_RES;
  st.status = ST_RUN;
  st.sweep = st.sweeps = st.iters = st.restarts = 0;
  st.inner_it = st.icap_cur = st.j = st.jend = st.cycles = st.par = st.first = 0;
  st.bnorm = st.relres0 = st.relres = 0.0;
  st.bytes = 0.0;
  st.ith = st.rho = st.alpha = st.beta = st.hn = 0.0;
}

template <int C, int TW>
hipError_t seg_step_launch(SegEngine *e, hipStream_t st);

}  // namespace

// ---------------------------------------------------------------------------- host engine
struct SegEngine {
  int nseg = 0, nblk = 0, chunk = 5;
  int tw = SG_TW_MAX;         // tiles per wave of a work item (the items below are for it)
  int oversub = 8;            // data-kernel grid: this many times the resident blocks
  std::vector<int64_t> n;
  std::vector<int> blk0h;
  SegDesc *ddesc = nullptr;   // device descriptors
  SegDesc *hdesc = nullptr;   // pinned staging of the descriptors
  SegState *dstate = nullptr;
  char *hsum = nullptr;       // pinned copy of the state summaries
  int *dblkseg = nullptr, *dblk0 = nullptr;
  double *dpart = nullptr;
  int *done = nullptr;        // pinned host flags (device-visible)
  int *done_dev = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t gstream = nullptr;  // stream the graph was captured on
  hipEvent_t ev[2] = {nullptr, nullptr};
};

namespace {

template <int C, int TW>
hipError_t seg_step_launch(SegEngine *e, hipStream_t st) {
  static int resident = 0;
  int grid = resident_blocks((const void *)k_seg_data<C, TW>, SG_TPB, resident) * e->oversub;
  if (grid < 8) grid = 8;
  grid = grid / 8 * 8;
  const int need = (e->nblk + SG_MAXIT - 1) / SG_MAXIT;
  if (grid < need) grid = need;
  if (grid > e->nblk) grid = e->nblk;
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_seg_data<C, TW>), dim3(grid), dim3(SG_TPB), 0, st, e->ddesc,
                     (const SegState *)e->dstate, (const int *)e->dblkseg, (const int *)e->dblk0, e->nblk);
  hipLaunchKernelGGL(k_seg_close, dim3(e->nseg), dim3(SC_TPB), 0, st, (const SegDesc *)e->ddesc, e->dstate,
                     e->done_dev);
  return hipGetLastError();
}

template <int TW>
hipError_t seg_step_tw(SegEngine *e, hipStream_t st) {
  switch (e->chunk) {
    case 7: return seg_step_launch<7, TW>(e, st);
    case 9: return seg_step_launch<9, TW>(e, st);
    default: return seg_step_launch<5, TW>(e, st);
  }
}

hipError_t seg_step(SegEngine *e, hipStream_t st) {
  return e->tw == 2 ? seg_step_tw<2>(e, st) : seg_step_tw<SG_TW_MAX>(e, st);
}

// the item tables (segment of each item, first item of each segment) for e->tw; the
// device arrays are sized for the smallest items
hipError_t seg_items_build(SegEngine *e) {
  std::vector<int> blkseg;
  e->blk0h.clear();
  const int rows = item_rows(e->tw);
  for (int s = 0; s < e->nseg; ++s) {
    const int nb = (int)((e->n[s] + rows - 1) / rows);
    e->blk0h.push_back((int)blkseg.size());
    for (int k = 0; k < (nb > 0 ? nb : 1); ++k) blkseg.push_back(s);
  }
  e->nblk = (int)blkseg.size();
  hipError_t r = hipMemcpy(e->dblkseg, blkseg.data(), e->nblk * sizeof(int), hipMemcpyHostToDevice);
  if (r == hipSuccess) r = hipMemcpy(e->dblk0, e->blk0h.data(), e->nseg * sizeof(int), hipMemcpyHostToDevice);
  return r;
}

constexpr int SG_CHUNK = 16;  // engine steps per chunk (one graph launch)

hipError_t seg_chunk(SegEngine *e, bool graph, hipStream_t st) {
  if (!graph) {
    for (int k = 0; k < SG_CHUNK; ++k) {
      const hipError_t r = seg_step(e, st);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  }
  if (e->gexec && e->gstream != st) {
    (void)hipGraphExecDestroy(e->gexec);
    (void)hipGraphDestroy(e->graph);
    e->gexec = nullptr;
    e->graph = nullptr;
  }
  if (!e->gexec) {
    hipError_t r = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (r != hipSuccess) return r;
    for (int k = 0; k < SG_CHUNK && r == hipSuccess; ++k) r = seg_step(e, st);
    hipGraph_t g = nullptr;
    const hipError_t r2 = hipStreamEndCapture(st, &g);
    if (r != hipSuccess || r2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return r != hipSuccess ? r : r2;
    }
    r = hipGraphInstantiate(&e->gexec, g, nullptr, nullptr, 0);
    if (r != hipSuccess) {
      (void)hipGraphDestroy(g);
      e->gexec = nullptr;
      return r;
    }
    e->graph = g;
    e->gstream = st;
  }
  return hipGraphLaunch(e->gexec, st);
}

}  // namespace

int seg_engine_create(const int64_t *n, int nseg, SegEngine **out) {
  *out = nullptr;
  if (nseg < 1) return -1;
  SegEngine *e = new (std::nothrow) SegEngine();
  if (!e) return -1;
  e->nseg = nseg;
  e->chunk = 5;
  e->tw = SG_TW_MAX;
  e->n.assign(n, n + nseg);
  int64_t maxitems = 0;  // items with the smallest work items
  for (int s = 0; s < nseg; ++s) maxitems += std::max<int64_t>(1, (n[s] + item_rows(2) - 1) / item_rows(2));
  if (maxitems > (int64_t)1 << 30) {
    delete e;
    return -1;
  }
  const int mi = (int)maxitems;
  bool ok = hipMalloc((void **)&e->ddesc, nseg * sizeof(SegDesc)) == hipSuccess &&
            hipHostMalloc((void **)&e->hdesc, nseg * sizeof(SegDesc), hipHostMallocDefault) == hipSuccess &&
            hipMalloc((void **)&e->dstate, nseg * sizeof(SegState)) == hipSuccess &&
            hipHostMalloc((void **)&e->hsum, nseg * SG_SUMMARY, hipHostMallocDefault) == hipSuccess &&
            hipMalloc((void **)&e->dblkseg, mi * sizeof(int)) == hipSuccess &&
            hipMalloc((void **)&e->dblk0, nseg * sizeof(int)) == hipSuccess &&
            hipMalloc((void **)&e->dpart, (size_t)mi * SG_PW * sizeof(double)) == hipSuccess &&
            hipHostMalloc((void **)&e->done, nseg * sizeof(int), hipHostMallocDefault) == hipSuccess &&
            hipHostGetDevicePointer((void **)&e->done_dev, e->done, 0) == hipSuccess &&
            hipEventCreateWithFlags(&e->ev[0], hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&e->ev[1], hipEventDisableTiming) == hipSuccess;
  ok = ok && seg_items_build(e) == hipSuccess;
  if (!ok) {
    seg_engine_destroy(e);
    return -1;
  }
  *out = e;
  return 0;
}

void seg_engine_destroy(SegEngine *e) {
  if (!e) return;
  if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  for (auto &v : e->ev)
    if (v) (void)hipEventDestroy(v);
  if (e->ddesc) (void)hipFree(e->ddesc);
  if (e->hdesc) (void)hipHostFree(e->hdesc);
  if (e->dstate) (void)hipFree(e->dstate);
  if (e->hsum) (void)hipHostFree(e->hsum);
  if (e->dblkseg) (void)hipFree(e->dblkseg);
  if (e->dblk0) (void)hipFree(e->dblk0);
  if (e->dpart) (void)hipFree(e->dpart);
  if (e->done) (void)hipHostFree(e->done);
  delete e;
}

// Upper bound on engine steps for a segment: every step advances it by one phase; a
// sweep takes RES and XUPD, every inner iteration two phases (F, G or CGQ, CGU) and every
// GMRES cycle (at least one iteration) two more (UPD, GRES).
static long long seg_step_bound(const SegDesc &d) {
  const long long it = d.maxit, sw = (long long)d.max_refine + 1;
  return 2 * sw + 6 * it + 16;
}

hipError_t seg_engine_solve(SegEngine *e, const SegDesc *desc, bool graph, int oversub, int chunk, int rows,
                            hipStream_t st, SegResult *res) {
  const int nseg = e->nseg;
  // work-item size: 512 or 1024 rows (anything else: 1024), pinned by SACC_SEG_ROWS when
  // that is set to one of them; a change rebuilds the item tables and re-captures the graph
  {
    const char *ev = getenv("SACC_SEG_ROWS");
    const int v = ev ? atoi(ev) : 0;
    if (v == item_rows(2) || v == item_rows(SG_TW_MAX)) rows = v;
    const int tw = rows == item_rows(2) ? 2 : SG_TW_MAX;
    if (tw != e->tw) {
      if (e->gexec) {
        (void)hipGraphExecDestroy(e->gexec);
        (void)hipGraphDestroy(e->graph);
        e->gexec = nullptr;
        e->graph = nullptr;
      }
      hipError_t r = hipStreamSynchronize(st);  // no step of the previous layout still queued
      e->tw = tw;
      if (r == hipSuccess) r = seg_items_build(e);
      if (r != hipSuccess) return r;
    }
  }
  // the SpMV tile shape of this solve's matrices (a change re-captures the graph)
  {
    const int c = chunk == 7 || chunk == 9 ? chunk : 5;
    if (c != e->chunk && e->gexec) {
      (void)hipGraphExecDestroy(e->gexec);
      (void)hipGraphDestroy(e->graph);
      e->gexec = nullptr;
      e->graph = nullptr;
    }
    e->chunk = c;
  }
  // the data kernel's grid multiple: the caller's (the batch tuner's), 8 by default;
  // SACC_SEG_OVERSUB (1..64) pins it (reproducible measurements)
  {
    const char *ev = getenv("SACC_SEG_OVERSUB");
    const int v = ev ? atoi(ev) : 0;
    const int want = v >= 1 && v <= 64 ? v : (oversub >= 1 && oversub <= 64 ? oversub : 8);
    if (want != e->oversub && e->gexec) {
      (void)hipGraphExecDestroy(e->gexec);
      (void)hipGraphDestroy(e->graph);
      e->gexec = nullptr;
      e->graph = nullptr;
    }
    e->oversub = want;
  }
  long long bound = 0;
  for (int s = 0; s < nseg; ++s) {
    e->hdesc[s] = desc[s];
    e->hdesc[s].part = e->dpart + (size_t)e->blk0h[s] * SG_PW;
    e->hdesc[s].nblk = (int)((e->n[s] + item_rows(e->tw) - 1) / item_rows(e->tw));
    e->done[s] = 0;
    bound = std::max(bound, seg_step_bound(desc[s]));
  }
  hipError_t r = hipMemcpyAsync(e->ddesc, e->hdesc, nseg * sizeof(SegDesc), hipMemcpyHostToDevice, st);
  if (r != hipSuccess) return r;
  hipLaunchKernelGGL(k_seg_init, dim3((nseg + 63) / 64), dim3(64), 0, st, e->dstate, nseg);
  if ((r = hipGetLastError()) != hipSuccess) return r;
  // chunks of engine steps; the host waits for the chunk before the one just enqueued,
  // so the device always has one chunk queued, and stops once every segment has ended
  long long steps = 0;
  for (int c = 0;; ++c) {
    if (steps > bound) return hipErrorUnknown;
    if ((r = seg_chunk(e, graph, st)) != hipSuccess) return r;
    steps += SG_CHUNK;
    if ((r = hipEventRecord(e->ev[c & 1], st)) != hipSuccess) return r;
    if (c == 0) continue;
    if ((r = hipEventSynchronize(e->ev[(c - 1) & 1])) != hipSuccess) return r;
    bool all = true;
    for (int s = 0; s < nseg && all; ++s) all = ((volatile int *)e->done)[s] != 0;
    if (all) break;
  }
  r = hipMemcpy2DAsync(e->hsum, SG_SUMMARY, e->dstate, sizeof(SegState), SG_SUMMARY, nseg, hipMemcpyDeviceToHost, st);
  if (r == hipSuccess) r = hipStreamSynchronize(st);
  if (r != hipSuccess) return r;
  for (int s = 0; s < nseg; ++s) {
    SegState sm;
    memcpy(&sm, e->hsum + (size_t)s * SG_SUMMARY, SG_SUMMARY);
    if (sm.phase != SP_DONE) return hipErrorUnknown;
    res[s].state = sm.status;
    res[s].iters = sm.iters;
    res[s].restarts = sm.restarts;
    res[s].sweeps = sm.sweeps;
    res[s].relres0 = sm.relres0;
    res[s].relres = sm.relres;
    res[s].bytes = sm.bytes;
  }
  return hipSuccess;
}

}  // namespace sacc
