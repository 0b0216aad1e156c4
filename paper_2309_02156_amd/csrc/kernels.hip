// Device kernels of one time step for FP64 vectors (A may hold FP32 values).
//
// Step layout (Alg. 1 of arXiv 2309.02156, Section 2):
//   push      X[:, slot] = x(t_{i-1});  SX[:, slot] = S x(t_{i-1})     (history window)
//   qrcp      QR with column pivoting of SX -> rank k, T1 = P R11^-1    (sketched QR)
//   basis     Q1 = X T1                                                 (n x k)
//   spmm_gram per row tile: W = A Q1 in registers, MFMA-accumulated Q1^T [Q1 | W | b]
//   small     pivoted Cholesky of G = Q1^T Q1 (Cholesky-QR finish), reduced Galerkin
//             system R2^-T (Q1^T A Q1) R2^-1 y = R2^-T Q1^T b, c = R2^-1 y
//   x0        x0 = Q1 c
//   Krylov    CG (2 kernels / iteration) or GMRES with classical Gram-Schmidt applied
//             twice (2 kernels / Arnoldi step), device-side scalars and stopping tests
//             (krylov.hip).
//
// Reductions are deterministic: per-block partial sums in fixed order, reduced in a
// fixed order by the kernel that follows (or a column-sum kernel), never by
// floating-point atomics.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace sacc {

typedef double d4 __attribute__((ext_vector_type(4)));

template <typename VT>
__device__ inline double row_dot(const int *__restrict__ rowptr, const int *__restrict__ col,
                                 const VT *__restrict__ val, const double *__restrict__ x, int64_t i) {
  const int p0 = rowptr[i], p1 = rowptr[i + 1];
  double s = 0.0;
  for (int p = p0; p < p1; ++p) s += (double)val[p] * x[col[p]];
  return s;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// ============================================================================ SpMV
// Wave tiles of 64 rows (the CG kernels' scheme): columns / values staged coalesced in
// LDS, each lane gathers along its own row.  C: gathers per lane and step.
template <typename VT, int C>
__global__ __launch_bounds__(TPB) void k_spmv(const int *rowptr, const int *col, const VT *val,
                                              const double *x, double *y, int64_t n) {
  __shared__ int lcol[NWAVE * WT_CAP];
  __shared__ VT lval[NWAVE * WT_CAP];
  const int wid = threadIdx.x / WAVE;
  const WaveTiles wt = wave_tiles(n);
  wave_tiles_spmv<C>(
      rowptr, col, val, Gather1<double>{x}, n, wt.t, wt.end, wt.step, lcol + wid * WT_CAP, lval + wid * WT_CAP,
      [&](int64_t) { return 0.0; }, [&](int64_t i, double, double s) { y[i] = s; });
}

// grid of a wave-tile streaming kernel: one tile per wave up to what the device holds
// at once, at most cap blocks (MAXBLK when the runtime cannot say)
static int wave_grid(const void *kernel, int64_t n, int &cache, int cap) {
  const int res = resident_blocks(kernel, TPB, cache);
  return wave_tile_blocks(n, TPB, res > 0 ? (res < cap ? res : cap) : MAXBLK);
}

// partial rows of 2 entries the mixed-mode residual may leave (the Krylov partials
// buffer holds far more)
constexpr int IR_MAXBLK = 4096;

template <typename VT, int C>
static void spmv_c(const CsrView &A, const double *x, double *y, hipStream_t st) {
  static int cache = 0;
  const int nb = wave_grid((const void *)k_spmv<VT, C>, A.n, cache, 1 << 16);
  // stand-ins for a matrix without nonzeros (one entry is read, never used)
  const int *colp = A.nnz > 0 ? A.col : A.rowptr;
  const VT *valp = A.nnz > 0 ? (const VT *)A.val : (const VT *)x;
  hipLaunchKernelGGL((k_spmv<VT, C>), dim3(nb), dim3(TPB), 0, st, A.rowptr, colp, valp, x, y, A.n);
}

template <typename VT>
static void spmv_vt(const CsrView &A, const double *x, double *y, hipStream_t st) {
  const int C = wave_tile_chunk(A.n, A.nnz);
  if (C <= 5)
    spmv_c<VT, 5>(A, x, y, st);
  else if (C <= 7)
    spmv_c<VT, 7>(A, x, y, st);
  else
    spmv_c<VT, 9>(A, x, y, st);
}

hipError_t launch_spmv(const CsrView &A, const double *x, double *y, hipStream_t st) {
  if (A.fp32)
    spmv_vt<float>(A, x, y, st);
  else
    spmv_vt<double>(A, x, y, st);
  return hipGetLastError();
}

// ============================================================================ push + sketch
// Grid (nbx, ceil(s / SKETCH_RG)): block row-group g accumulates rows [16 g, 16 g + 16)
// of S x; group 0 also copies x into the history slot.  The next kernel reduces.
// zero_rhs: the pushed column is zero when the solve just ended in the zero right-hand
// side state (its solution is x = 0, written after the push was enqueued).
template <int SK, typename TX>
__global__ __launch_bounds__(TPB) void k_push(const double *x, TX *X, double *SX, int64_t n, int64_t ld, int slot,
                                              int s, uint64_t seed, const long long *rows,
                                              const unsigned long long *signs, double *partials,
                                              const Ctl *ctl, int zero_rhs) {
  __shared__ double red[NWAVE * SKETCH_RG];
  __shared__ double outv[MAXS];
  __shared__ double scratch[TPB];
  const int g = blockIdx.y, r0 = g * SKETCH_RG;
  const int rc = (s - r0) < SKETCH_RG ? (s - r0) : SKETCH_RG;
  double acc[SKETCH_RG];
#pragma unroll
  for (int r = 0; r < SKETCH_RG; ++r) acc[r] = 0.0;
  long long myrows[SKETCH_RG];
  if (SK == 1) {
#pragma unroll
    for (int r = 0; r < SKETCH_RG; ++r) myrows[r] = (r < rc) ? rows[r0 + r] : 0;
  }
  const bool zero = zero_rhs && ctl->state == ST_ZERO_RHS;
  GRID_ROWS(j, n) {
    // the stored (possibly FP32-rounded) column is what gets sketched
    const TX xs = zero ? (TX)0 : (TX)x[j];
    const double xj = (double)xs;
    if (g == 0) X[(size_t)slot * ld + j] = xs;
    if (SK == 0) {
#pragma unroll
      for (int q = 0; q < SKETCH_RG / 4; ++q) {
        if (4 * q < rc) {
          double gq[4];
          normals4((uint64_t)j, (uint64_t)((r0 >> 2) + q), STREAM_GAUSS_SKETCH, seed, gq);
#pragma unroll
          for (int l = 0; l < 4; ++l) acc[4 * q + l] += gq[l] * xj;
        }
      }
    } else {
      const double d = srht_negative(signs, (uint64_t)j) ? -xj : xj;
#pragma unroll
      for (int r = 0; r < SKETCH_RG; ++r)
        acc[r] += (__popcll((unsigned long long)myrows[r] & (unsigned long long)j) & 1) ? -d : d;
    }
  }
  const int blk = blockIdx.y * gridDim.x + blockIdx.x;
  (void)outv;
  (void)scratch;
  (void)SX;
  // per-block partial sums; the QRCP kernel that follows reduces them into SX[:, slot]
  block_sum_store<SKETCH_RG>(acc, rc, red, partials + (size_t)blk * SKETCH_RG);
}

__global__ __launch_bounds__(TPB) void k_srht_signs(unsigned long long *words, int64_t nw, uint64_t seed) {
  GRID_ROWS(w, nw) words[w] = srht_sign_word((uint64_t)w, seed);
}

hipError_t launch_srht_signs(unsigned long long *words, int64_t n, uint64_t seed, hipStream_t st) {
  const int64_t nw = (n + 63) / 64;
  hipLaunchKernelGGL(k_srht_signs, dim3(stream_blocks(nw)), dim3(TPB), 0, st, words, nw, seed);
  return hipGetLastError();
}

int push_blocks_x(int64_t n, int s) {
  const int ng = (s + SKETCH_RG - 1) / SKETCH_RG;
  int nbx = stream_blocks(n);
  if (nbx * ng > MAXBLK) nbx = MAXBLK / ng > 0 ? MAXBLK / ng : 1;
  return nbx;
}

template <typename TX>
hipError_t launch_push(const double *x, TX *X, double *SX, int64_t n, int64_t ld, int slot, int s, int sketch,
                       uint64_t seed, const long long *srht_rows, const unsigned long long *srht_signs,
                       double *partials, const Ctl *ctl, int zero_rhs, hipStream_t st) {
  const int ng = (s + SKETCH_RG - 1) / SKETCH_RG;
  const int nbx = push_blocks_x(n, s);
  if (sketch == 0)
    hipLaunchKernelGGL((k_push<0, TX>), dim3(nbx, ng), dim3(TPB), 0, st, x, X, SX, n, ld, slot, s, seed,
                       srht_rows, srht_signs, partials, ctl, zero_rhs);
  else
    hipLaunchKernelGGL((k_push<1, TX>), dim3(nbx, ng), dim3(TPB), 0, st, x, X, SX, n, ld, slot, s, seed,
                       srht_rows, srht_signs, partials, ctl, zero_rhs);
  return hipGetLastError();
}

// ============================================================================ BF16 sketch (MFMA)
// The mixed mode's Gaussian sketch is applied in BF16 on the matrix cores: the normals
// G (s x n, the same Philox / Box-Muller entries as the FP64 sketch) are generated once
// per sequence, rounded FP64 -> FP32 -> BF16 (nearest even) and kept in HBM, rows padded
// to a multiple of 16 and columns to a multiple of 64 with zeros; a push streams them.
// S = BF16(G) / sqrt(s): the scale is applied where the push partials are reduced.
__device__ inline unsigned short bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even (finite values)
  return (unsigned short)(u >> 16);
}

__global__ __launch_bounds__(TPB) void k_gen_sketch_bf16(unsigned short *G, int64_t n, int64_t lds, int s, int spad,
                                                         uint64_t seed) {
  const int nq = spad / 4;
  GRID_ROWS(e, lds * nq) {
    const int64_t j = e % lds;
    const int q = (int)(e / lds);
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (j < n && 4 * q < s) normals4((uint64_t)j, (uint64_t)q, STREAM_GAUSS_SKETCH, seed, g);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int r = 4 * q + l;
      G[(size_t)r * lds + j] = (r < s && j < n) ? bf16_bits((float)g[l]) : (unsigned short)0;
    }
  }
}

int64_t sketch_bf16_ld(int64_t n) { return (n + 63) / 64 * 64; }
int sketch_bf16_rows(int s) { return (s + SKETCH_RG - 1) / SKETCH_RG * SKETCH_RG; }

hipError_t launch_gen_sketch_bf16(unsigned short *G, int64_t n, int s, uint64_t seed, hipStream_t st) {
  const int64_t lds = sketch_bf16_ld(n);
  const int spad = sketch_bf16_rows(s);
  hipLaunchKernelGGL(k_gen_sketch_bf16, dim3(stream_blocks(lds * (spad / 4))), dim3(TPB), 0, st, G, n, lds, s, spad,
                     seed);
  return hipGetLastError();
}

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int PUSH_TPB = 512;  // eight waves per block: four per SIMD with the push grid's block count
constexpr int PUSH_NW = PUSH_TPB / WAVE;

// Push with the BF16 sketch.  Grid (nbx, ceil(s / 16)) as k_push, the same partial rows.
// A wave takes chunks of 64 entries, PU of them per round (their loads issued together);
// per chunk four v_mfma_f32_16x16x16bf16_1k with A = G[16 rows of the group][16 entries]
// and B = the chunk's FP32 column split exactly into three BF16 terms, hi, mid and lo
// (each the BF16 rounding of what the previous ones leave), in B's columns 0, 1 and 2
// (columns 3..15 zero): D[:, 0..2] hold the 16 rows' sums of the three terms.  Operand
// layout: A[i][4 kq + e] from lane i + 16 kq, B[4 kq + e][j] from lane j + 16 kq
// (e = 0..3, the four 16-bit halves of the operand), D[4 kq + v][j] in lane j + 16 kq,
// element v.  In MFMA m of a chunk, k slot 4 kq + e is the chunk's entry 16 kq + 4 m + e.
// D is added into FP64 after every chunk (64 exact products per FP32 sum), the three
// columns when the block's partial row is formed.  The stored column X[:, slot] = TX(x)
// is written by row group 0; the FP32 values reach the B lanes through the wave's LDS.
template <typename TX>
__global__ __launch_bounds__(PUSH_TPB) void k_push_bf16(const double *x, TX *X, const unsigned short *G, int64_t n,
                                                   int64_t ld, int64_t lds, int slot, int s, double *partials,
                                                   const Ctl *ctl, int zero_rhs) {
  constexpr int PU = 8;
  __shared__ __align__(16) float xf[PUSH_NW * PU * WAVE];
  __shared__ double red[PUSH_NW * 3 * SKETCH_RG];
  const int g = blockIdx.y, r0 = g * SKETCH_RG;
  const int rc = (s - r0) < SKETCH_RG ? (s - r0) : SKETCH_RG;
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  const int i16 = lane % 16, kq = lane / 16;
  float *xw = xf + wid * PU * WAVE;
  const bool zero = zero_rhs && ctl->state == ST_ZERO_RHS;
  double accd[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t nch = (n + WAVE - 1) / WAVE;  // chunks of 64 entries
  const int64_t wstep = (int64_t)gridDim.x * PUSH_NW * PU;
  const unsigned short *grow = G + (size_t)(r0 + i16) * lds + 16 * kq;
  for (int64_t c0 = ((int64_t)blockIdx.x * PUSH_NW + wid) * PU; c0 < nch; c0 += wstep) {
    uint4 av[PU][2];
    double xv[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      // chunks past the end re-read the last one (their B operand is zero)
      const int64_t ch = c0 + u < nch ? c0 + u : nch - 1;
      const uint4 *ap = (const uint4 *)(grow + ch * WAVE);
      av[u][0] = ap[0];
      av[u][1] = ap[1];
      const int64_t j = (c0 + u) * WAVE + lane;
      xv[u] = x[j < n ? j : n - 1];
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int64_t j = (c0 + u) * WAVE + lane;
      const bool in = j < n;
      const TX xs = (zero || !in) ? (TX)0 : (TX)xv[u];
      if (g == 0 && in) X[(size_t)slot * ld + j] = xs;
      xw[u * WAVE + lane] = (float)xs;
    }
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      // this lane's B operand: term i16 (< 3) of 16 entries from 16 kq on
      unsigned bw[8];
      const float4 *bp = (const float4 *)(xw + u * WAVE + 16 * kq);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const float4 f = bp[h];
        const float fv[4] = {f.x, f.y, f.z, f.w};
        unsigned short t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const unsigned short hi = bf16_bits(fv[e]);
          const float r1 = fv[e] - __uint_as_float((unsigned)hi << 16);
          const unsigned short mid = bf16_bits(r1);
          const float r2 = r1 - __uint_as_float((unsigned)mid << 16);
          const unsigned short lo = bf16_bits(r2);  // exact: r2 has at most 8 significant bits
          t[e] = i16 == 0 ? hi : (i16 == 1 ? mid : (i16 == 2 ? lo : (unsigned short)0));
        }
        bw[2 * h] = (unsigned)t[0] | ((unsigned)t[1] << 16);
        bw[2 * h + 1] = (unsigned)t[2] | ((unsigned)t[3] << 16);
      }
      f4v d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const uint4 &aw = av[u][m / 2];
        const unsigned a0 = (m & 1) ? aw.z : aw.x, a1 = (m & 1) ? aw.w : aw.y;
        const unsigned b0 = bw[2 * m], b1 = bw[2 * m + 1];
        const s4v a = {(short)(a0 & 0xFFFFu), (short)(a0 >> 16), (short)(a1 & 0xFFFFu), (short)(a1 >> 16)};
        const s4v b = {(short)(b0 & 0xFFFFu), (short)(b0 >> 16), (short)(b1 & 0xFFFFu), (short)(b1 >> 16)};
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, d, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) accd[v] += (double)d[v];
    }
    wave_lds_sync();  // the slice is rewritten in the next round
  }
  // lanes j + 16 kq (j < 3: column j of D) hold rows 4 kq .. 4 kq + 3 of term j; the block
  // adds the waves' rows in wave order, the three terms of a wave in order
  if (i16 < 3) {
#pragma unroll
    for (int v = 0; v < 4; ++v) red[(wid * 3 + i16) * SKETCH_RG + 4 * kq + v] = accd[v];
  }
  __syncthreads();
  const int blk = blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x < rc) {
    double a = 0.0;
    for (int w = 0; w < PUSH_NW; ++w)
      for (int j = 0; j < 3; ++j) a += red[(w * 3 + j) * SKETCH_RG + threadIdx.x];
    partials[(size_t)blk * SKETCH_RG + threadIdx.x] = a;
  }
}

template <typename TX>
hipError_t launch_push_bf16(const double *x, TX *X, const unsigned short *G, double *SX, int64_t n, int64_t ld,
                            int slot, int s, double *partials, const Ctl *ctl, int zero_rhs, hipStream_t st) {
  (void)SX;
  const int ng = (s + SKETCH_RG - 1) / SKETCH_RG;
  const int nbx = push_blocks_x(n, s);
  hipLaunchKernelGGL((k_push_bf16<TX>), dim3(nbx, ng), dim3(PUSH_TPB), 0, st, x, X, G, n, ld, sketch_bf16_ld(n), slot, s,
                     partials, ctl, zero_rhs);
  return hipGetLastError();
}

// ============================================================================ sketched QRCP
// One workgroup.  Householder QR with column pivoting (largest remaining column norm,
// recomputed exactly at every step; ties pick the lowest index) of Y = SX[:, 0:cnt],
// diag(R) >= 0, rank k = leading count of |R_jj| > tau |R_11|, T1 = P R11^-1.
//
// Wave w owns the columns c = w (mod NWAVE).  A pivot step: every wave forms the norms of
// its remaining columns (all their LDS reads issued together, one multi-value wave
// reduction: each norm is the same lane-order sum and tree as a one-column reduction),
// every wave finds the pivot on its own (no serial scan, no barrier for it), the columns
// swap, and every wave applies the reflector to its columns (the dots batched the same
// way).  Three barriers a step.  MC = columns a wave owns at most, RW = 64-row chunks.
template <int MC, int RW>
__device__ __forceinline__ void qrcp_body(double *SX, int s, int cnt, int newest, double tau,
                                          const double *partials, int nbx, Ctl *ctl, const ZRows &zr,
                                          uint64_t seed) {
  extern __shared__ double sh[];
  // zr.m > 0: the range finder's Z (cnt x m) multiplies S X first (Alg. 3: the sketch of
  // Omega = X Z), and the QR runs over the m columns of Y = (S X) Z
  const int nq = zr.m > 0 ? zr.m : cnt;  // columns of the factorised matrix
  double *Y = sh;                     // s x cnt, ld s (then s x nq)
  double *Ri = sh + (size_t)s * cnt;  // nq x nq inverse, ld nq
  double *Zm = Ri + (size_t)nq * nq;  // cnt x m, ld cnt
  double *Yz = Zm + (size_t)cnt * (zr.m > 0 ? zr.m : 0);  // s x m, ld s
  __shared__ double nrm[MAXM];
  __shared__ double v[MAXS];
  __shared__ double scratch[TPB];
  __shared__ int perm[MAXM], iperm[MAXM];
  __shared__ int s_bad, s_newest_bad;
  const int tid = threadIdx.x, lane = tid % WAVE, wid = tid / WAVE;
  if (tid == 0) {
    s_bad = 0;
    s_newest_bad = 0;
  }
  // finish the push: SX[:, newest] = (sum over push blocks of the sketch partials) / sqrt(s).
  // Sketch row r sits in row group r / SKETCH_RG, entry r % SKETCH_RG of each push block's
  // partial row; `parts` threads per sketch row sum every parts-th block, then one adds
  // the parts in order.
  {
    static_assert(MAXS <= TPB, "one thread at least per sketch row");
    const int parts = (int)blockDim.x / s;
    const int r = tid % s, part = tid / s;
    if (part < parts) {
      const double *pr = partials + ((size_t)(r / SKETCH_RG) * nbx) * SKETCH_RG + r % SKETCH_RG;
      double acc = 0.0;
      // (unrolled so that a thread's loads go out together: a loop over ~85 blocks with
      // 8 loads per round made 11 dependent trips to memory)
#pragma unroll 32
      for (int b = part; b < nbx; b += parts) acc += pr[(size_t)b * SKETCH_RG];
      scratch[tid] = acc;
    }
    __syncthreads();
    if (tid < s) {
      double a = 0.0;
      for (int q = 0; q < parts; ++q) a += scratch[q * s + tid];
      v[tid] = a;
    }
    __syncthreads();
  }
  const double inv = 1.0 / sqrt((double)s);
  for (int r = tid; r < s; r += blockDim.x) SX[(size_t)newest * s + r] = v[r] * inv;
  __syncthreads();
  // the stored sketch columns, 8 entries per thread and round requested together
  for (int e0 = 0; e0 < s * cnt; e0 += 8 * (int)blockDim.x) {
    double sv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * (int)blockDim.x + tid;
      sv[u] = SX[e < s * cnt ? e : s * cnt - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * (int)blockDim.x + tid;
      if (e < s * cnt) {
        const double y = (e / s == newest) ? v[e % s] * inv : sv[u];
        Y[e] = y;
        if (!isfinite(y)) {
          s_bad = 1;
          if (e / s == newest) s_newest_bad = 1;
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    ctl->newest = newest;
    ctl->newest_ok = s_newest_bad ? 0 : 1;
  }
  if (s_bad) {
    if (tid == 0) {
      ctl->k = 0;
      ctl->nonfinite = 1;
    }
    return;
  }
  if (zr.m > 0) {
    // Z[l][c] = Gaussian entry (row zr.row[l], column c) of the epoch's stream: normal
    // lane c & 3 of Philox block (row, (epoch << 16) | (c >> 2), STREAM_RANGE_Z)
    const int nq4 = (zr.m + 3) / 4;
    for (int e = tid; e < cnt * nq4; e += blockDim.x) {
      const int l = e % cnt, q4 = e / cnt;
      double g[4];
      normals4((uint64_t)zr.row[l], ((uint64_t)zr.epoch << 16) | (uint64_t)q4, STREAM_RANGE_Z, seed, g);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (4 * q4 + u < zr.m) Zm[l + (size_t)(4 * q4 + u) * cnt] = g[u];
    }
    __syncthreads();
    for (int e = tid; e < s * zr.m; e += blockDim.x) {
      const int r = e % s, c = e / s;
      double acc = 0.0;
      for (int l = 0; l < cnt; ++l) acc += Y[r + (size_t)l * s] * Zm[l + (size_t)c * cnt];
      Yz[e] = acc;
    }
    __syncthreads();
    Y = Yz;
  }
  for (int c = tid; c < nq; c += blockDim.x) perm[c] = c;
  __syncthreads();
  int jj = 0;
  for (; jj < nq; ++jj) {
    // exact column norms over rows jj..s-1 of this wave's remaining columns
    {
      double a[MC];
#pragma unroll
      for (int u = 0; u < MC; ++u) {
        const int c = jj + wid + NWAVE * u;
        const int cc = c < nq ? c : nq - 1;
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < RW; ++w) {
          const int r = jj + lane + WAVE * w;
          const double y = Y[(size_t)cc * s + (r < s ? r : s - 1)];
          if (r < s) acc += y * y;
        }
        a[u] = acc;
      }
      wave_sum_multi<MC>(a);
      constexpr int LPE = WAVE / MC;  // lanes per entry after the reduction
      const int c = jj + wid + NWAVE * (lane / LPE);
      if (lane % LPE == 0 && c < nq) nrm[c] = a[0];
    }
    __syncthreads();
    // pivot: largest norm, lowest index among equal ones (each wave, the same result)
    const int p = wave_argmax((jj + lane < nq) ? nrm[jj + lane] : -1.0, jj + lane);
    if (tid == 0) {
      const int t = perm[jj];
      perm[jj] = perm[p];
      perm[p] = t;
    }
    if (p != jj) {
      for (int r = tid; r < s; r += blockDim.x) {
        const double t = Y[(size_t)jj * s + r];
        Y[(size_t)jj * s + r] = Y[(size_t)p * s + r];
        Y[(size_t)p * s + r] = t;
      }
      __syncthreads();
    }
    const double alpha = sqrt(nrm[p]);
    const double x0 = Y[(size_t)jj * s + jj];
    if (alpha == 0.0) {
      // the rest is zero: R_jj = 0 onward
      for (int c = jj + tid; c < nq; c += blockDim.x) Y[(size_t)c * s + c] = 0.0;
      __syncthreads();
      break;
    }
    const double beta = x0 >= 0.0 ? -alpha : alpha;  // R_jj (sign fixed below)
    const double v0 = x0 - beta;
    const double tauh = 2.0 / (v0 * v0 + (alpha * alpha - x0 * x0));
    // reflector v = (v0, Y[jj+1.., jj]) applied to this wave's columns c > jj
    {
      double vr[RW];
#pragma unroll
      for (int w = 0; w < RW; ++w) {
        const int r = jj + lane + WAVE * w;
        const double y = Y[(size_t)jj * s + (r < s ? r : s - 1)];
        vr[w] = r == jj ? v0 : y;
      }
      double yc[MC][RW], d[MC];
#pragma unroll
      for (int u = 0; u < MC; ++u) {
        const int c = jj + 1 + wid + NWAVE * u;
        const int cc = c < nq ? c : nq - 1;
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < RW; ++w) {
          const int r = jj + lane + WAVE * w;
          yc[u][w] = Y[(size_t)cc * s + (r < s ? r : s - 1)];
          if (r < s) acc += vr[w] * yc[u][w];
        }
        d[u] = acc;
      }
      double dr[MC];
#pragma unroll
      for (int u = 0; u < MC; ++u) dr[u] = d[u];
      wave_sum_multi<MC>(dr);
      constexpr int LPE = WAVE / MC;
#pragma unroll
      for (int u = 0; u < MC; ++u) {
        const int c = jj + 1 + wid + NWAVE * u;
        const double du = lane_bcast(dr[0], u * LPE) * tauh;
        if (c < nq) {
#pragma unroll
          for (int w = 0; w < RW; ++w) {
            const int r = jj + lane + WAVE * w;
            if (r < s) Y[(size_t)c * s + r] = yc[u][w] - du * vr[w];
          }
        }
      }
    }
    if (tid == 0) Y[(size_t)jj * s + jj] = beta;
    __syncthreads();
  }
  // sign convention diag(R) >= 0: negate rows with a negative diagonal
  for (int r = wid; r < nq && r < s; r += NWAVE) {
    const bool neg = Y[(size_t)r * s + r] < 0.0;
    if (neg)
      for (int c = r + lane; c < nq; c += WAVE) Y[(size_t)c * s + r] = -Y[(size_t)c * s + r];
  }
  __syncthreads();
  // rank: leading count of |R_jj| > tau |R_11| (every thread, from LDS)
  const double r00 = fabs(Y[0]);
  int k = 0;
  if (r00 > 0.0)
    while (k < nq && k < s && fabs(Y[(size_t)k * s + k]) > tau * r00) ++k;
  // R11^-1 on wave 0, lane c = column c, row by row from the bottom (each entry the same
  // ascending sum as a per-column back substitution)
  if (wid == 0) {
    const int c = lane;
    if (c < k) {
      for (int i = 0; i < k; ++i) Ri[i + c * k] = 0.0;
      Ri[c + c * k] = 1.0 / Y[(size_t)c * s + c];
    }
    for (int i = k - 2; i >= 0; --i) {
      if (c > i && c < k) {
        double acc = 0.0;
#pragma unroll 4
        for (int l = i + 1; l <= c; ++l) acc += Y[(size_t)l * s + i] * Ri[l + c * k];
        Ri[i + c * k] = -acc / Y[(size_t)i * s + i];
      }
    }
  }
  for (int i = tid; i < nq; i += blockDim.x) iperm[perm[i]] = i;
  __syncthreads();
  // T1 = P R11^-1, or Z P R11^-1 with the range finder (zero elsewhere), every entry
  // written once
  for (int e = tid; e < MAXM * MAXM; e += blockDim.x) {
    const int row = e % MAXM, c = e / MAXM;
    double t = 0.0;
    if (c < k && row < cnt) {
      if (zr.m > 0) {
        for (int i = 0; i <= c; ++i) t += Zm[row + (size_t)perm[i] * cnt] * Ri[i + c * k];
      } else {
        const int i = iperm[row];
        if (i <= c) t = Ri[i + c * k];
      }
    }
    ctl->T1[e] = t;
  }
  if (tid == 0) {
    ctl->k = k;
    ctl->nonfinite = 0;
  }
}

template <int MC, int RW>
__global__ __launch_bounds__(TPB) void k_qrcp(double *SX, int s, int cnt, int newest, double tau,
                                              const double *partials, int nbx, Ctl *ctl, ZRows zr,
                                              uint64_t seed) {
  qrcp_body<MC, RW>(SX, s, cnt, newest, tau, partials, nbx, ctl, zr, seed);
}

// many sequences' QRCPs in one launch: block b runs job b (the same body as k_qrcp)
template <int MC, int RW>
__global__ __launch_bounds__(TPB) void k_qrcp_batch(const QrcpJob *__restrict__ jobs) {
  const QrcpJob &j = jobs[blockIdx.x];
  qrcp_body<MC, RW>(j.SX, j.s, j.cnt, j.newest, j.tau, j.partials, j.nbx, j.ctl, j.zr, j.seed);
}

// dynamic LDS bytes of a QRCP, and whether it takes the small instantiation
static size_t qrcp_lds(int s, int cnt, const ZRows &zr) {
  const int nq = zr.m > 0 ? zr.m : cnt;
  size_t lds = ((size_t)s * cnt + (size_t)nq * nq) * sizeof(double);
  if (zr.m > 0) lds += ((size_t)cnt * zr.m + (size_t)s * zr.m) * sizeof(double);
  return lds;
}
static bool qrcp_small(int s, int cnt, const ZRows &zr) {
  const int nq = zr.m > 0 ? zr.m : cnt;
  return nq <= 2 * NWAVE * 4 && s <= 2 * WAVE;
}

hipError_t launch_qrcp_batch(const QrcpJob *jobs_dev, const QrcpJob *jobs_host, int njobs, hipStream_t st) {
  // one launch per instantiation; the jobs are sorted by it (small ones first)
  int nsmall = 0;
  size_t lds_s = sizeof(double), lds_l = sizeof(double);
  for (int i = 0; i < njobs; ++i) {
    const QrcpJob &j = jobs_host[i];
    const size_t b = qrcp_lds(j.s, j.cnt, j.zr);
    if (qrcp_small(j.s, j.cnt, j.zr)) {
      if (i != nsmall) return hipErrorInvalidValue;  // not sorted
      ++nsmall;
      lds_s = std::max(lds_s, b);
    } else {
      lds_l = std::max(lds_l, b);
    }
  }
  if (nsmall > 0)
    hipLaunchKernelGGL((k_qrcp_batch<8, 2>), dim3(nsmall), dim3(TPB), lds_s, st, jobs_dev);
  if (njobs > nsmall)
    hipLaunchKernelGGL((k_qrcp_batch<MAXM / NWAVE, MAXS / WAVE>), dim3(njobs - nsmall), dim3(TPB), lds_l, st,
                       jobs_dev + nsmall);
  return hipGetLastError();
}

bool qrcp_job_small(const QrcpJob &j) { return qrcp_small(j.s, j.cnt, j.zr); }

hipError_t launch_qrcp(double *SX, int s, int cnt, int newest, double tau, const double *partials, int64_t n,
                       Ctl *ctl, const ZRows &zr, uint64_t seed, hipStream_t st) {
  const size_t lds = qrcp_lds(s, cnt, zr);
  if (qrcp_small(s, cnt, zr))
    hipLaunchKernelGGL((k_qrcp<8, 2>), dim3(1), dim3(TPB), lds, st, SX, s, cnt, newest, tau, partials,
                       push_blocks_x(n, s), ctl, zr, seed);
  else
    hipLaunchKernelGGL((k_qrcp<MAXM / NWAVE, MAXS / WAVE>), dim3(1), dim3(TPB), lds, st, SX, s, cnt, newest, tau,
                       partials, push_blocks_x(n, s), ctl, zr, seed);
  return hipGetLastError();
}

// ============================================================================ basis Q1 = X T1
// A tall-skinny dense product on the matrix cores, formed transposed so that the stores
// run along rows: Q1^T = T1^T X^T with v_mfma_f64_16x16x4f64, A = T1^T[16 basis columns]
// [4 history columns] (lane i + 16 kq: basis column i, history column kq of the chunk;
// read once per wave and kept in registers), B = X^T[4 history columns][16 rows]
// (lane j + 16 kq: row j), D[kq + 4 v][j] (basis column kq + 4 v, row j) in lane
// j + 16 kq: each store instruction writes 16 consecutive rows of four columns.
// A wave takes RB blocks of 16 rows per round, all their X loads issued together.
// Columns past cnt of X and past k of T1 are zero; Q1 is written for columns < k.
template <int MC, typename TX>
__global__ __launch_bounds__(TPB) void k_basis(const TX *X, TX *Q1, int64_t n, int64_t ld, int cnt,
                                               const Ctl *ctl) {
  constexpr int NL = MC / 4, NC = MC / 16, RB = 2;
  const int k = ctl->k;
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  const int i16 = lane % 16, kq = lane / 16;
  double bop[NL][NC];
#pragma unroll
  for (int lc = 0; lc < NL; ++lc)
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) {
      const int l = 4 * lc + kq, c = 16 * cb + i16;
      bop[lc][cb] = (l < cnt && c < k) ? ctl->T1[l + c * MAXM] : 0.0;
    }
  const int64_t nblk = (n + 15) / 16;
  const int64_t step = (int64_t)gridDim.x * NWAVE * RB;
  for (int64_t b0 = ((int64_t)blockIdx.x * NWAVE + wid) * RB; b0 < nblk; b0 += step) {
    double aop[RB][NL];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int64_t row = (b0 + r) * 16 + i16;
      const int64_t rc = row < n ? row : n - 1;
#pragma unroll
      for (int lc = 0; lc < NL; ++lc) {
        const int l = 4 * lc + kq;
        const double v = (double)X[(size_t)(l < cnt ? l : 0) * ld + rc];
        aop[r][lc] = (l < cnt && row < n) ? v : 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int lc = 0; lc < NL; ++lc) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bop[lc][cb], aop[r][lc], acc, 0, 0, 0);
        const int64_t row = (b0 + r) * 16 + i16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * cb + kq + 4 * v;
          if (c < k && row < n) Q1[(size_t)c * ld + row] = (TX)acc[v];
        }
      }
    }
  }
}

template <typename TX>
hipError_t launch_basis(const TX *X, TX *Q1, int64_t n, int64_t ld, int cnt, Ctl *ctl, hipStream_t st) {
  static int cache16 = 0, cache32 = 0;
  const int64_t waves = ((n + 15) / 16 + 1) / 2;  // rounds of 2 row blocks
  int64_t want = (waves + NWAVE - 1) / NWAVE;
  if (cnt <= 16) {
    const int res = resident_blocks((const void *)k_basis<16, TX>, TPB, cache16);
    if (res > 0 && want > res) want = res;
    hipLaunchKernelGGL((k_basis<16, TX>), dim3(want < 1 ? 1 : want), dim3(TPB), 0, st, X, Q1, n, ld, cnt, ctl);
  } else {
    const int res = resident_blocks((const void *)k_basis<32, TX>, TPB, cache32);
    if (res > 0 && want > res) want = res;
    hipLaunchKernelGGL((k_basis<32, TX>), dim3(want < 1 ? 1 : want), dim3(TPB), 0, st, X, Q1, n, ld, cnt, ctl);
  }
  return hipGetLastError();
}

// ============================================================================ SpMM + Gram (MFMA)
// A wave owns tiles of 16 rows (XCD-aware order); lane l works on row rr = l % 16 of the
// tile and on the basis columns [CPL q, CPL q + CPL) with q = l / 16, CPL = KB / 4.
// SpMM: w = (A Q1)_{row, cols} accumulated in registers; the row's nonzeros in rounds
// of NZ (their columns and values loaded together), the CPL gathers of every nonzero of
// a round issued together (consecutive rows of a column sit side by side, so each load
// instruction touches four short runs of a column).
// Gram: the tile's W, with b as column k, goes to the wave's LDS slice, and
// v_mfma_f64_16x16x4f64 accumulates over the tile's four row quads
//   G += Q1^T Q1 (blocks on and above the diagonal), H += Q1^T [W | b],
//   and for the minimum-residual problem K += W^T [W | b];
// the Q1 operands are read straight from memory (the tile's 16 rows of a column share
// one cache line), the W operands from LDS.  Operand layout of the instruction:
// A[i][kq] from lane i + 16 kq, B[kq][j] from lane j + 16 kq, D[lane / 16 + 4 v][lane % 16]
// in accumulator element v.  Columns >= k of Q1 and W are zero.
// The waves' accumulators are added in wave order in LDS and the block writes one row
// of partial sums: P[a + col cnt] for a < cnt, col < 2 cnt + 1 (Q1^T Q1 | Q1^T W | Q1^T b),
// then for the minimum residual K[a + col cnt], col < cnt + 1 (W^T W | W^T b).
constexpr int GRAM_TPB = 256;
constexpr int GRAM_NW = GRAM_TPB / WAVE;
constexpr int GRAM_ROWS = 16;
constexpr int GRAM_MAXBLK = 1024;
constexpr int GRAM_STAGE = 128;  // nonzeros of a 16-row tile staged in LDS (longer tiles read directly)


template <int KB, bool MR>
struct GramShape {
  static constexpr int NA = KB / 16;                       // 16-column blocks of Q1
  static constexpr int NWB = KB / 16 + 1;                  // 16-column blocks of [W | b]
  static constexpr int LDW = NWB * 16 + 1;                 // LDS row stride of the W tile
  static constexpr int NG = NA * (NA + 1) / 2;             // G blocks kept
  static constexpr int NBLK = NG + NA * NWB + (MR ? NA * NWB : 0);
  static constexpr int TILE = GRAM_NW * GRAM_ROWS * LDW;   // doubles of the W tiles
  static constexpr int COMB = NBLK * 256;                  // doubles of the combined blocks
  static constexpr int LDS = TILE > COMB ? TILE : COMB;
};

__device__ inline int gram_gidx(int a, int bq, int na) {  // index of G block (a <= bq)
  return a * na - a * (a - 1) / 2 + (bq - a);
}

template <typename VT, int KB, typename TX, bool MR>
__global__ __launch_bounds__(GRAM_TPB) void k_spmm_gram(const int *rowptr, const int *col, const VT *val,
                                                        const TX *Q1, const double *b, int64_t n, int64_t ld,
                                                        int cnt, double *partials, const Ctl *ctl) {
  using S = GramShape<KB, MR>;
  constexpr int CPL = KB / 4, NA = S::NA, NWB = S::NWB, LDW = S::LDW;
  constexpr int SU = GRAM_STAGE / WAVE;  // staged nonzeros per lane
  constexpr int GRAM_NZ = sizeof(TX) == 4 ? 4 : 2;  // nonzeros of a row whose gathers go out together
  __shared__ double lds[S::LDS];
  __shared__ int scol[GRAM_NW * GRAM_STAGE];
  __shared__ VT sval[GRAM_NW * GRAM_STAGE];
  const int k = ctl->k;
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  const int rr = lane % 16, q = lane / 16;
  const int na = (k + 15) / 16, nwb = (k + 1 + 15) / 16;
  double *Wl = lds + (size_t)wid * GRAM_ROWS * LDW;
  int *lc = scol + wid * GRAM_STAGE;
  VT *lv = sval + wid * GRAM_STAGE;
  d4 accG[S::NG], accH[NA][NWB], accK[MR ? NA : 1][MR ? NWB : 1];
#pragma unroll
  for (int e = 0; e < S::NG; ++e) accG[e] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int bw = 0; bw < NWB; ++bw) {
      accH[a][bw] = (d4){0.0, 0.0, 0.0, 0.0};
      if constexpr (MR) accK[a][bw] = (d4){0.0, 0.0, 0.0, 0.0};
    }
  const int64_t T = (n + GRAM_ROWS - 1) / GRAM_ROWS;
  const int groups = gridDim.x >= NXCD ? NXCD : 1;
  const int64_t per = (T + groups - 1) / groups;
  const int64_t tlo = (int64_t)(blockIdx.x % groups) * per;
  const int64_t thi = tlo + per < T ? tlo + per : T;
  const int64_t tstep = (int64_t)(gridDim.x / groups) * GRAM_NW;
  // Two-stage tile prefetch: a tile's row pointers are requested two tiles ahead and
  // its first GRAM_STAGE nonzeros (columns, values) one tile ahead, both with the current
  // tile's gathers, so a tile waits for one trip to memory.  Loads are unconditional and
  // in bounds (col / val hold at least one entry); past the last tile they re-read it.
  struct Rows {
    int pa, pb, p0, p1;
  };
  struct Nz {
    int c[SU];
    VT v[SU];
  };
  auto load_rows = [&](int64_t tt, Rows &f) {
    const int64_t r0 = tt * GRAM_ROWS, row = r0 + rr;
    const int64_t rc = row < n ? row : n - 1;
    const int64_t rl = r0 + GRAM_ROWS < n ? r0 + GRAM_ROWS : n;
    f.pa = rowptr[rc];
    f.pb = rowptr[rc + 1];
    f.p0 = rowptr[r0 < n ? r0 : n - 1];
    f.p1 = rowptr[rl];
  };
  auto load_nz = [&](const Rows &f, Nz &z) {
    const int p0 = __builtin_amdgcn_readfirstlane(f.p0), p1 = __builtin_amdgcn_readfirstlane(f.p1);
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int pp = p0 + u * WAVE + lane;
      const int pc = pp < p1 ? pp : (p1 > 0 ? p1 - 1 : 0);
      z.c[u] = col[(unsigned)pc];
      z.v[u] = val[(unsigned)pc];
    }
  };
  int64_t t = tlo + (int64_t)(blockIdx.x / groups) * GRAM_NW + wid;
  auto clampt = [&](int64_t tt) { return tt < thi ? tt : (t < thi ? thi - 1 : t); };
  Rows cur, nr;
  Nz cz;
  if (k > 0 && t < thi) {
    load_rows(t, cur);
    load_rows(clampt(t + tstep), nr);
    load_nz(cur, cz);
  }
  for (; k > 0 && t < thi; t += tstep) {
    const int64_t r0 = t * GRAM_ROWS, row = r0 + rr;
    const bool valid = row < n;
    const int p0 = __builtin_amdgcn_readfirstlane(cur.p0), p1 = __builtin_amdgcn_readfirstlane(cur.p1);
    const int pa = valid ? cur.pa : 0, len = valid ? cur.pb - cur.pa : 0;
    const bool staged = p1 - p0 <= GRAM_STAGE;
    // the next tile's nonzeros (its row pointers arrived during this tile's predecessor)
    // and the row pointers of the tile after it
    Nz nz;
    Rows nr2;
    load_nz(nr, nz);
    load_rows(clampt(t + 2 * tstep), nr2);
    __builtin_amdgcn_sched_barrier(0);
    const Nz &cc = cz;
    // this tile's nonzeros into the wave's staging slice
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int pp = p0 + u * WAVE + lane;
      if (pp < p1 && pp - p0 < GRAM_STAGE) {
        lc[pp - p0] = cc.c[u];
        lv[pp - p0] = cc.v[u];
      }
    }
    wave_lds_sync();
    // the Gram operands of the tile's rows and the row's b (independent of the SpMM):
    // requested first, so that their trips overlap the gathers'
    const double bv = b[valid ? row : n - 1];
    const int i16 = lane % 16, kq = lane / 16;
    TX aqr[GRAM_ROWS / 4][NA];
#pragma unroll
    for (int s4 = 0; s4 < GRAM_ROWS / 4; ++s4) {
      const int64_t rowk = r0 + 4 * s4 + kq;
      const int64_t rq = rowk < n ? rowk : n - 1;
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const int ca = a * 16 + i16;
        aqr[s4][a] = Q1[(size_t)(ca < k ? ca : k - 1) * ld + rq];
      }
    }
    // SpMM: w = (A Q1)_{row, cols}, the row's nonzeros NZ at a time from the staging
    // slice (the gathers of a round issued together)
    double w[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) w[u] = 0.0;
    const int off = pa - p0;
    for (int z0 = 0; __any(z0 < len); z0 += GRAM_NZ) {
      int cj[GRAM_NZ];
      double av[GRAM_NZ];
#pragma unroll
      for (int z = 0; z < GRAM_NZ; ++z) {
        const bool on = z0 + z < len;
        if (staged) {
          const int idx = on ? off + z0 + z : 0;
          cj[z] = on ? lc[idx] : (int)(valid ? row : n - 1);
          av[z] = on ? (double)lv[idx] : 0.0;
        } else {
          const int pp = on ? pa + z0 + z : 0;
          cj[z] = on ? col[(unsigned)pp] : (int)(valid ? row : n - 1);
          av[z] = on ? (double)val[(unsigned)pp] : 0.0;
        }
      }
      TX g[GRAM_NZ][CPL];
#pragma unroll
      for (int z = 0; z < GRAM_NZ; ++z)
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
          const int c = q * CPL + u;
          g[z][u] = Q1[(size_t)(c < k ? c : k - 1) * ld + (unsigned)cj[z]];
        }
#pragma unroll
      for (int u = 0; u < CPL; ++u) {
        double acc = 0.0;
#pragma unroll
        for (int z = 0; z < GRAM_NZ; ++z) acc += av[z] * (double)g[z][u];
        w[u] += acc;
      }
    }
    // the tile's [W | b] into the wave's slice: W, zero columns past k, then b in column k
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int c = q * CPL + u;
      Wl[rr * LDW + c] = (c < k && valid) ? w[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < (NWB * 16 - KB) / 4; ++u) Wl[rr * LDW + KB + q * ((NWB * 16 - KB) / 4) + u] = 0.0;
    wave_lds_sync();
    if (q == 0) Wl[rr * LDW + k] = valid ? bv : 0.0;
    wave_lds_sync();
#pragma unroll
    for (int s4 = 0; s4 < GRAM_ROWS / 4; ++s4) {
      const int lr = 4 * s4 + kq;
      const int64_t rowk = r0 + lr;
      double aq[NA], wv[NWB];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const int ca = a * 16 + i16;
        aq[a] = (ca < k && rowk < n) ? (double)aqr[s4][a] : 0.0;
      }
#pragma unroll
      for (int bw = 0; bw < NWB; ++bw) wv[bw] = Wl[lr * LDW + bw * 16 + i16];
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        if (a < na) {
#pragma unroll
          for (int bq = a; bq < NA; ++bq)
            if (bq < na)
              accG[gram_gidx(a, bq, NA)] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(aq[a], aq[bq], accG[gram_gidx(a, bq, NA)], 0, 0, 0);
#pragma unroll
          for (int bw = 0; bw < NWB; ++bw)
            if (bw < nwb) {
              accH[a][bw] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[a], wv[bw], accH[a][bw], 0, 0, 0);
              if constexpr (MR) accK[a][bw] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[a], wv[bw], accK[a][bw], 0, 0, 0);
            }
        }
      }
    }
    wave_lds_sync();  // the slices are rewritten by the wave's next tile
    cur = nr;
    nr = nr2;
    cz = nz;
  }
  // the waves' blocks added in wave order: D element v of a block sits at row
  // lane / 16 + 4 v, column lane % 16 (row-major 16 x 16)
  __syncthreads();
  for (int wv = 0; wv < GRAM_NW; ++wv) {
    if (wid == wv) {
      int blk = 0;
      auto put = [&](const d4 &acc) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double *dst = lds + (size_t)blk * 256 + (lane / 16 + 4 * v) * 16 + lane % 16;
          *dst = wv == 0 ? acc[v] : *dst + acc[v];
        }
        ++blk;
      };
#pragma unroll
      for (int e = 0; e < S::NG; ++e) put(accG[e]);
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int bw = 0; bw < NWB; ++bw) put(accH[a][bw]);
      if constexpr (MR) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int bw = 0; bw < NWB; ++bw) put(accK[a][bw]);
      }
    }
    __syncthreads();
  }
  const int Wg = cnt * (2 * cnt + 1), Wout = MR ? Wg + cnt * (cnt + 1) : Wg;
  double *out = partials + (size_t)blockIdx.x * Wout;
  const double *comb = lds;
  const int hbase = S::NG, kbase = S::NG + NA * NWB;
  for (int e = threadIdx.x; e < Wout; e += blockDim.x) {
    double v = 0.0;
    if (e < Wg) {
      const int a = e % cnt, cx = e / cnt;
      if (a < k) {
        if (cx < cnt) {  // G, from the block on or above the diagonal
          if (cx < k) {
            const int r = a <= cx ? a : cx, c = a <= cx ? cx : a;
            if (r / 16 == c / 16 || r / 16 < c / 16)
              v = comb[(size_t)gram_gidx(r / 16, c / 16, NA) * 256 + (r % 16) * 16 + c % 16];
          }
        } else if (cx < 2 * cnt) {  // Q1^T W
          const int c = cx - cnt;
          if (c < k) v = comb[(size_t)(hbase + (a / 16) * NWB + c / 16) * 256 + (a % 16) * 16 + c % 16];
        } else {  // Q1^T b (column k of the W tile)
          v = comb[(size_t)(hbase + (a / 16) * NWB + k / 16) * 256 + (a % 16) * 16 + k % 16];
        }
      }
    } else {
      const int e2 = e - Wg, a = e2 % cnt, cx = e2 / cnt;
      if (a < k) {
        const int c = cx < cnt ? cx : k;  // W^T W column, or W^T b (column k)
        if (cx == cnt || c < k) v = comb[(size_t)(kbase + (a / 16) * NWB + c / 16) * 256 + (a % 16) * 16 + c % 16];
      }
    }
    out[e] = v;
  }
}

template <typename VT, int KB, typename TX, bool MR>
static int gram_grid(int64_t n) {
  static int resident = 0;  // blocks of this instantiation the device holds at once
  const int64_t T = (n + GRAM_ROWS - 1) / GRAM_ROWS;
  int64_t want = (T + GRAM_NW - 1) / GRAM_NW;
  if (resident == 0) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_spmm_gram<VT, KB, TX, MR>, GRAM_TPB, 0) ==
            hipSuccess &&
        per >= 1) {
      const int r = per * ncu / NXCD * NXCD;
      resident = r < NXCD ? NXCD : (r > GRAM_MAXBLK ? GRAM_MAXBLK : r);
    } else {
      resident = 256;
    }
  }
  if (want > resident) want = resident;
  if (want >= NXCD) want = want / NXCD * NXCD;
  return (int)(want < 1 ? 1 : want);
}

template <typename VT, int KB, typename TX, bool MR>
static int gram_launch(const CsrView &A, const TX *Q1, int64_t ld, const double *b, int cnt, double *partials,
                       const Ctl *ctl, hipStream_t st) {
  const int nb = gram_grid<VT, KB, TX, MR>(A.n);
  hipLaunchKernelGGL((k_spmm_gram<VT, KB, TX, MR>), dim3(nb), dim3(GRAM_TPB), 0, st, A.rowptr, A.col,
                     (const VT *)A.val, Q1, b, A.n, ld, cnt, partials, ctl);
  return nb;
}

template <typename VT, typename TX>
static int gram_launch_vt(const CsrView &A, const TX *Q1, int64_t ld, const double *b, int cnt, int minres,
                          double *partials, const Ctl *ctl, hipStream_t st) {
  if (cnt <= 16)
    return minres ? gram_launch<VT, 16, TX, true>(A, Q1, ld, b, cnt, partials, ctl, st)
                  : gram_launch<VT, 16, TX, false>(A, Q1, ld, b, cnt, partials, ctl, st);
  return minres ? gram_launch<VT, 32, TX, true>(A, Q1, ld, b, cnt, partials, ctl, st)
                : gram_launch<VT, 32, TX, false>(A, Q1, ld, b, cnt, partials, ctl, st);
}

template <typename TX>
hipError_t launch_spmm_gram(const CsrView &A, const TX *Q1, int64_t ld, const double *b, int cnt, int minres,
                            double *partials, int *nblk_out, Ctl *ctl, hipStream_t st) {
  *nblk_out = A.fp32 ? gram_launch_vt<float, TX>(A, Q1, ld, b, cnt, minres, partials, ctl, st)
                     : gram_launch_vt<double, TX>(A, Q1, ld, b, cnt, minres, partials, ctl, st);
  return hipGetLastError();
}

int gram_width(int cnt, int minres) { return cnt * (2 * cnt + 1) + (minres ? cnt * (cnt + 1) : 0); }

// ============================================================================ POD (Alg. 2)
// The POD basis is formed from the Gram matrix of the history: G = X^T X (this kernel,
// partial rows reduced by k_colsum), G = V diag(lam) V^T by cyclic Jacobi rotations on one
// workgroup (k_pod_eig), T1 = V_k diag(lam_k)^(-1/2) for the k leading eigenvalues, so
// Q1 = X T1 holds the k leading left singular vectors of X.
//
// Gram: a wave owns tiles of 16 rows; v_mfma_f64_16x16x4f64 accumulates the blocks on and
// above the diagonal over the tile's four row quads, the operands read straight from X
// (A[i][kq] from lane i + 16 kq, B[kq][j] from lane j + 16 kq); the waves' blocks are added
// in wave order and the block writes its partial row P[a + c cnt], a, c < cnt.
template <int KB, typename TX>
__global__ __launch_bounds__(GRAM_TPB) void k_gram_x(const TX *X, int64_t n, int64_t ld, int cnt,
                                                     double *partials) {
  constexpr int NA = KB / 16, NG = NA * (NA + 1) / 2;
  __shared__ double comb[NG * 256];
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  const int i16 = lane % 16, kq = lane / 16;
  const int na = (cnt + 15) / 16;
  d4 acc[NG];
#pragma unroll
  for (int e = 0; e < NG; ++e) acc[e] = (d4){0.0, 0.0, 0.0, 0.0};
  const int64_t T = (n + GRAM_ROWS - 1) / GRAM_ROWS;
  const int groups = gridDim.x >= NXCD ? NXCD : 1;
  const int64_t per = (T + groups - 1) / groups;
  const int64_t tlo = (int64_t)(blockIdx.x % groups) * per;
  const int64_t thi = tlo + per < T ? tlo + per : T;
  const int64_t tstep = (int64_t)(gridDim.x / groups) * GRAM_NW;
  for (int64_t t = tlo + (int64_t)(blockIdx.x / groups) * GRAM_NW + wid; t < thi; t += tstep) {
    double xv[GRAM_ROWS / 4][NA];
#pragma unroll
    for (int s4 = 0; s4 < GRAM_ROWS / 4; ++s4) {
      const int64_t row = t * GRAM_ROWS + 4 * s4 + kq;
      const int64_t rq = row < n ? row : n - 1;
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const int c = a * 16 + i16;
        const double v = (double)X[(size_t)(c < cnt ? c : cnt - 1) * ld + rq];
        xv[s4][a] = (c < cnt && row < n) ? v : 0.0;
      }
    }
#pragma unroll
    for (int s4 = 0; s4 < GRAM_ROWS / 4; ++s4)
#pragma unroll
      for (int a = 0; a < NA; ++a)
        if (a < na)
#pragma unroll
          for (int bq = a; bq < NA; ++bq)
            if (bq < na)
              acc[gram_gidx(a, bq, NA)] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(xv[s4][a], xv[s4][bq], acc[gram_gidx(a, bq, NA)], 0, 0, 0);
  }
  for (int wv = 0; wv < GRAM_NW; ++wv) {
    if (wid == wv)
#pragma unroll
      for (int e = 0; e < NG; ++e)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double *dst = comb + (size_t)e * 256 + (lane / 16 + 4 * v) * 16 + lane % 16;
          *dst = wv == 0 ? acc[e][v] : *dst + acc[e][v];
        }
    __syncthreads();
  }
  double *out = partials + (size_t)blockIdx.x * cnt * cnt;
  for (int e = threadIdx.x; e < cnt * cnt; e += blockDim.x) {
    const int a = e % cnt, c = e / cnt;
    const int r = a <= c ? a : c, q = a <= c ? c : a;
    out[e] = comb[(size_t)gram_gidx(r / 16, q / 16, NA) * 256 + (r % 16) * 16 + q % 16];
  }
}

template <int KB, typename TX>
static int gram_x_launch(const TX *X, int64_t n, int64_t ld, int cnt, double *partials, hipStream_t st) {
  const int64_t T = (n + GRAM_ROWS - 1) / GRAM_ROWS;
  int64_t nb = (T + GRAM_NW - 1) / GRAM_NW;
  if (nb > 512) nb = 512;
  if (nb >= NXCD) nb = nb / NXCD * NXCD;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL((k_gram_x<KB, TX>), dim3(nb), dim3(GRAM_TPB), 0, st, X, n, ld, cnt, partials);
  return (int)nb;
}

template <typename TX>
hipError_t launch_gram_x(const TX *X, int64_t n, int64_t ld, int cnt, double *partials, int *nblk_out,
                         hipStream_t st) {
  *nblk_out = cnt <= 16 ? gram_x_launch<16, TX>(X, n, ld, cnt, partials, st)
                        : gram_x_launch<32, TX>(X, n, ld, cnt, partials, st);
  return hipGetLastError();
}

// One workgroup: eigen-decomposition of the Gram matrix in ctl->gram (cnt x cnt) by cyclic
// Jacobi rotations, the round-robin ordering giving cnt / 2 disjoint pairs per round (all
// pairs' rotations from the same matrix, then the rows, then the columns and V); sweeps
// until the off-diagonal norm is at most 1e-15 of the Frobenius norm, at most 30.  The
// eigenvalues in descending order (lowest index first among equal ones); k = the leading
// count with lam_j > tau lam_1, at most m; T1[:, c] = V[:, c] / sqrt(lam_c).
__global__ __launch_bounds__(TPB) void k_pod_eig(int cnt, int m, double tau, Ctl *ctl) {
  constexpr int N = MAXM;  // padded order (even)
  __shared__ double A[N][N + 1], V[N][N + 1];
  __shared__ double cs[N / 2], sn[N / 2];
  __shared__ int pp[N / 2], qq[N / 2];
  __shared__ double lam[N];
  __shared__ int order[N];
  __shared__ int s_bad, s_done;
  __shared__ double s_red[TPB / WAVE];
  const int tid = threadIdx.x, lane = tid % WAVE, wid = tid / WAVE;
  const int np = cnt + (cnt & 1);  // even order for the tournament (a zero row and column added)
  for (int e = tid; e < N * N; e += blockDim.x) {
    const int a = e % N, b = e / N;
    double g = 0.0;
    if (a < cnt && b < cnt) g = 0.5 * (ctl->gram[a + b * cnt] + ctl->gram[b + a * cnt]);
    A[a][b] = g;
    V[a][b] = a == b ? 1.0 : 0.0;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int e = tid; e < cnt * cnt; e += blockDim.x)
    if (!isfinite(A[e % cnt][e / cnt])) s_bad = 1;
  __syncthreads();
  if (s_bad || cnt == 0) {
    for (int e = tid; e < MAXM * MAXM; e += blockDim.x) ctl->T1[e] = 0.0;
    if (tid == 0) {
      ctl->k = 0;
      ctl->nonfinite = s_bad;
    }
    return;
  }
  // Frobenius norm (fixed order: each wave sums its rows, waves in order)
  double fro2 = 0.0;
  {
    double part = 0.0;
    for (int e = tid; e < np * np; e += blockDim.x) part += A[e % np][e / np] * A[e % np][e / np];
    part = wave_sum(part);
    if (lane == 0) s_red[wid] = part;
    __syncthreads();
    for (int w = 0; w < (int)blockDim.x / WAVE; ++w) fro2 += s_red[w];
    __syncthreads();
  }
  for (int sweep = 0; sweep < 30 && np > 1; ++sweep) {
    for (int r = 0; r < np - 1; ++r) {
      if (tid < np / 2) {
        const int i = tid;
        int p = i == 0 ? r % (np - 1) : (r + i) % (np - 1);
        int q = i == 0 ? np - 1 : (r - i + np - 1) % (np - 1);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        const double apq = A[p][q];
        double c = 1.0, sv = 0.0;
        if (apq != 0.0) {
          const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          sv = t * c;
        }
        pp[i] = p;
        qq[i] = q;
        cs[i] = c;
        sn[i] = sv;
      }
      __syncthreads();
      // rows p, q of every pair: row_p <- c row_p - s row_q, row_q <- s row_p + c row_q
      for (int e = tid; e < (np / 2) * np; e += blockDim.x) {
        const int i = e / np, j = e % np;
        const int p = pp[i], q = qq[i];
        const double c = cs[i], sv = sn[i], ap = A[p][j], aq = A[q][j];
        A[p][j] = c * ap - sv * aq;
        A[q][j] = sv * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of every pair, and of V
      for (int e = tid; e < (np / 2) * np; e += blockDim.x) {
        const int i = e / np, j = e % np;
        const int p = pp[i], q = qq[i];
        const double c = cs[i], sv = sn[i];
        const double ap = A[j][p], aq = A[j][q];
        A[j][p] = c * ap - sv * aq;
        A[j][q] = sv * ap + c * aq;
        const double vp = V[j][p], vq = V[j][q];
        V[j][p] = c * vp - sv * vq;
        V[j][q] = sv * vp + c * vq;
      }
      __syncthreads();
    }
    // off-diagonal norm after the sweep
    double part = 0.0;
    for (int e = tid; e < np * np; e += blockDim.x) {
      const int a = e % np, b = e / np;
      if (a != b) part += A[a][b] * A[a][b];
    }
    part = wave_sum(part);
    if (lane == 0) s_red[wid] = part;
    __syncthreads();
    if (tid == 0) {
      double off = 0.0;
      for (int w = 0; w < (int)blockDim.x / WAVE; ++w) off += s_red[w];
      s_done = off <= 1e-30 * fro2;
    }
    __syncthreads();
    if (s_done) break;
  }
  // eigenvalues of the cnt real columns, descending (selection by the wave argmax,
  // lowest index among equal values), on wave 0
  if (wid == 0) {
    double v = lane < cnt ? A[lane][lane] : -INFINITY;
    for (int j = 0; j < cnt; ++j) {
      const int imax = wave_argmax(v, lane);
      if (lane == 0) {
        order[j] = imax;
        lam[j] = A[imax][imax];
      }
      if (lane == imax) v = -INFINITY;
    }
  }
  __syncthreads();
  int k = 0;
  if (lam[0] > 0.0)
    while (k < cnt && k < m && lam[k] > tau * lam[0]) ++k;
  for (int e = tid; e < MAXM * MAXM; e += blockDim.x) {
    const int row = e % MAXM, c = e / MAXM;
    double t = 0.0;
    if (c < k && row < cnt) t = V[row][order[c]] / sqrt(lam[c]);
    ctl->T1[e] = t;
  }
  if (tid == 0) {
    ctl->k = k;
    ctl->nonfinite = 0;
  }
}

hipError_t launch_pod_eig(int cnt, int m, double tau, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_pod_eig, dim3(1), dim3(TPB), 0, st, cnt, m, tau, ctl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- column sums
// gram[e] = sum_b partials[b][e]; block = 16 entries x 16 block-groups (block bx: entries
// 16 bx ..).
__device__ __forceinline__ void colsum_body(int bx, const double *partials, int nblk, int W, Ctl *ctl) {
  __shared__ double sc[TPB];
  const int e = bx * 16 + threadIdx.x % 16, grp = threadIdx.x / 16;
  double s = 0.0;
  // (unrolled so that a thread's row loads go out together: 18.8 -> 6.7 us over 768 rows)
  if (e < W)
#pragma unroll 16
    for (int b = grp; b < nblk; b += 16) s += partials[(size_t)b * W + e];
  sc[threadIdx.x] = s;
  __syncthreads();
  for (int off = 8; off > 0; off >>= 1) {
    if (grp < off) sc[threadIdx.x] += sc[threadIdx.x + off * 16];
    __syncthreads();
  }
  if (threadIdx.x < 16 && e < W) ctl->gram[e] = sc[threadIdx.x];
}

__global__ __launch_bounds__(TPB) void k_colsum(const double *partials, int nblk, int W, Ctl *ctl) {
  colsum_body(blockIdx.x, partials, nblk, W, ctl);
}

// many sequences' column sums in one launch: grid row y runs job y (blocks past a job's
// entries write nothing)
__global__ __launch_bounds__(TPB) void k_colsum_batch(const SolveJob *__restrict__ jobs) {
  const SolveJob &j = jobs[blockIdx.y];
  colsum_body(blockIdx.x, j.partials, j.nblk, j.W, j.ctl);
}

hipError_t launch_colsum(const double *partials, int nblk, int W, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3((W + 15) / 16), dim3(TPB), 0, st, partials, nblk, W, ctl);
  return hipGetLastError();
}

hipError_t launch_colsum_batch(const SolveJob *jobs_dev, const SolveJob *jobs_host, int njobs, hipStream_t st) {
  int gx = 1;
  for (int i = 0; i < njobs; ++i) gx = std::max(gx, (jobs_host[i].W + 15) / 16);
  if (njobs > 0) hipLaunchKernelGGL(k_colsum_batch, dim3(gx, njobs), dim3(TPB), 0, st, jobs_dev);
  return hipGetLastError();
}

// ============================================================================ small reduced solve
// One workgroup.  gram holds P = Q1^T [Q1 | W | b] with ld cnt: G = P[:, 0:k],
// Ht = P[:, cnt:cnt+k], gt = P[:, 2 cnt]; for the minimum residual it is followed by
// K = W^T [W | b] (ld cnt), and Ht, gt are taken from K instead: K[:, 0:k], K[:, cnt]
// (the normal equations of min ||A Q y - b||).  Pivoted Cholesky of G with threshold
// tau_c max(diag G) gives R2 (k2 x k2) and perm2; H = R2^-T Ht_pp R2^-1,
// g = R2^-T gt_p; H y = g by Cholesky (SPD path, and always for the minimum residual)
// or LU with partial pivoting; c[perm2[i]] = (R2^-1 y)_i, cX = T1 c.
__device__ __forceinline__ void small_solve_body(int cnt, int minres, int spd, double tau_c, Ctl *ctl) {
  extern __shared__ double sh[];
  const int k = ctl->k;
  const int tid = threadIdx.x, lane = tid % WAVE, wid = tid / WAVE;
  __shared__ int perm[MAXM];
  __shared__ double gv[MAXM], yv[MAXM], cv[MAXM];
  __shared__ int s_k2, s_fail;
  __shared__ double s_dmax;
  double *Gm = sh;                  // k x k, ld k  (-> R2 in its leading k2 x k2, upper part)
  double *Ri = sh + (size_t)k * k;  // k2 x k2, ld k
  double *Hm = sh + (size_t)2 * k * k;  // k x k, ld k
  double *P = sh + (size_t)3 * cnt * cnt;  // LDS copy of the reduced Gram block (ld cnt)
  // column 0 of the reduced matrix and the column of its right-hand side inside P
  const int hoff = minres ? cnt * (2 * cnt + 1) : cnt * cnt;
  const int goff = minres ? cnt * (2 * cnt + 1) + cnt * cnt : 2 * cnt * cnt;
  {
    // the reduced Gram block, 16 entries per thread and round requested together
    const int tot = cnt * (2 * cnt + 1) + (minres ? cnt * (cnt + 1) : 0);
    for (int e0 = 0; e0 < tot; e0 += 16 * (int)blockDim.x) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = e0 + u * (int)blockDim.x + tid;
        v[u] = ctl->gram[e < tot ? e : tot - 1];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = e0 + u * (int)blockDim.x + tid;
        if (e < tot) P[e] = v[u];
      }
    }
  }
  __syncthreads();
  if (k == 0) {
    for (int c = tid; c < MAXM; c += blockDim.x) {
      ctl->c[c] = 0.0;
      ctl->cX[c] = 0.0;
    }
    if (tid == 0) {
      const int fb = ctl->nonfinite;
      ctl->k2 = 0;
      ctl->fallback = fb;
      if (int *hi = ctl->hinfo) {
        ((volatile int *)hi)[0] = 0;
        ((volatile int *)hi)[1] = 0;
        ((volatile int *)hi)[2] = fb;
      }
    }
    return;
  }
  for (int e = tid; e < k * k; e += blockDim.x) {
    const int a = e % k, b = e / k;
    Gm[a + b * k] = P[a + b * cnt];
  }
  for (int a = tid; a < k; a += blockDim.x) perm[a] = a;
  if (tid == 0) {
    s_fail = 0;
    double dm = 0.0;
    for (int a = 0; a < k; ++a) dm = fmax(dm, P[a + a * cnt]);
    s_dmax = dm;
    s_k2 = k;
  }
  __syncthreads();
  // pivoted Cholesky, outer-product form, in place on the full symmetric matrix; the
  // pivot (largest remaining diagonal, lowest index among equal ones) found by every
  // wave on its own
  for (int j = 0; j < k; ++j) {
    const int p = wave_argmax((j + lane < k) ? Gm[(j + lane) * (k + 1)] : -INFINITY, j + lane);
    const bool stop = !(Gm[p * (k + 1)] > tau_c * s_dmax);
    __syncthreads();  // every wave has read the diagonal before the swaps below
    if (stop) {
      if (tid == 0) s_k2 = j;
      break;
    }
    if (tid == 0 && p != j) {
      int t = perm[j];
      perm[j] = perm[p];
      perm[p] = t;
    }
    if (p != j) {
      for (int a = tid; a < k; a += blockDim.x) {  // swap rows j, p
        double t = Gm[j + a * k];
        Gm[j + a * k] = Gm[p + a * k];
        Gm[p + a * k] = t;
      }
      __syncthreads();
      for (int a = tid; a < k; a += blockDim.x) {  // swap columns j, p
        double t = Gm[a + j * k];
        Gm[a + j * k] = Gm[a + p * k];
        Gm[a + p * k] = t;
      }
      __syncthreads();
    }
    const double d = sqrt(Gm[j + j * k]);
    __syncthreads();
    for (int a = j + 1 + tid; a < k; a += blockDim.x) Gm[j + a * k] /= d;
    if (tid == 0) Gm[j + j * k] = d;
    __syncthreads();
    for (int e = tid; e < (k - j - 1) * (k - j - 1); e += blockDim.x) {
      const int a = j + 1 + e % (k - j - 1), b = j + 1 + e / (k - j - 1);
      Gm[a + b * k] -= Gm[j + a * k] * Gm[j + b * k];
    }
    __syncthreads();
  }
  __syncthreads();
  const int k2 = s_k2;
  // Ri = R2^-1 (upper triangular, ld k) on wave 0, lane c = column c, row by row from the
  // bottom (each entry the same ascending sum as a per-column back substitution)
  if (wid == 0) {
    const int c = lane;
    if (c < k2) {
      for (int i = 0; i < k2; ++i) Ri[i + c * k] = 0.0;
      Ri[c + c * k] = 1.0 / Gm[c + c * k];
    }
    for (int i = k2 - 2; i >= 0; --i) {
      if (c > i && c < k2) {
        double acc = 0.0;
#pragma unroll 4
        for (int l = i + 1; l <= c; ++l) acc += Gm[i + l * k] * Ri[l + c * k];
        Ri[i + c * k] = -acc / Gm[i + i * k];
      }
    }
  }
  __syncthreads();
  // Hm = Ht_pp Ri  (Ht_pp[a][b] = Ht[perm a][perm b]); reuse Gm for the result of Ri^T (.)
  for (int e = tid; e < k2 * k2; e += blockDim.x) {
    const int a = e % k2, b = e / k2;
    double acc = 0.0;
    for (int l = 0; l <= b; ++l) acc += P[hoff + perm[a] + perm[l] * cnt] * Ri[l + b * k];
    Hm[a + b * k] = acc;
  }
  for (int a = tid; a < k2; a += blockDim.x) {
    double acc = 0.0;
    for (int l = 0; l <= a; ++l) acc += Ri[l + a * k] * P[goff + perm[l]];
    gv[a] = acc;
  }
  __syncthreads();
  for (int e = tid; e < k2 * k2; e += blockDim.x) {
    const int a = e % k2, b = e / k2;
    double acc = 0.0;
    for (int l = 0; l <= a; ++l) acc += Ri[l + a * k] * Hm[l + b * k];
    Gm[a + b * k] = acc;  // H (k2 x k2, ld k)
  }
  __syncthreads();
  if (spd) {
    for (int e = tid; e < k2 * k2; e += blockDim.x) {
      const int a = e % k2, b = e / k2;
      if (a < b) {
        const double m = 0.5 * (Gm[a + b * k] + Gm[b + a * k]);
        Gm[a + b * k] = m;
        Gm[b + a * k] = m;
      }
    }
    __syncthreads();
    // Cholesky H = L L^T in the lower triangle
    for (int j = 0; j < k2; ++j) {
      if (tid == 0) {
        const double d = Gm[j + j * k];
        if (!(d > 0.0) || !isfinite(d)) s_fail = 1;
        Gm[j + j * k] = sqrt(d);
      }
      __syncthreads();
      if (s_fail) break;
      const double d = Gm[j + j * k];
      for (int a = j + 1 + tid; a < k2; a += blockDim.x) Gm[a + j * k] /= d;
      __syncthreads();
      for (int e = tid; e < (k2 - j - 1) * (k2 - j - 1); e += blockDim.x) {
        const int a = j + 1 + e % (k2 - j - 1), b = j + 1 + e / (k2 - j - 1);
        if (a >= b) Gm[a + b * k] -= Gm[a + j * k] * Gm[b + j * k];
      }
      __syncthreads();
    }
    __syncthreads();
    // L L^T y = g on wave 0 by columns, lane a = entry a: forward (terms in ascending
    // order), then backward from the last entry
    if (wid == 0 && !s_fail) {
      const int a = lane;
      double acc = a < k2 ? gv[a] : 0.0;
      for (int l = 0; l < k2; ++l) {
        if (a == l) acc = acc / Gm[a + a * k];
        const double yl = lane_bcast(acc, l);
        if (a > l && a < k2) acc -= Gm[a + l * k] * yl;
      }
      for (int l = k2 - 1; l >= 0; --l) {
        if (a == l) acc = acc / Gm[a + a * k];
        const double yl = lane_bcast(acc, l);
        if (a < l) acc -= Gm[l + a * k] * yl;
      }
      if (a < k2) yv[a] = acc;
    }
  } else {
    // LU with partial pivoting, row interchanges applied to the whole rows
    for (int j = 0; j < k2; ++j) {
      // pivot: largest |entry| of column j at or below the diagonal, lowest index among
      // equal ones (every wave on its own)
      const int p = wave_argmax((j + lane < k2) ? fabs(Gm[j + lane + j * k]) : -1.0, j + lane);
      const double gp = Gm[p + j * k];
      const bool fail = !(gp != 0.0) || !isfinite(gp);
      __syncthreads();  // every wave has read column j before the swap below
      if (fail) {
        if (tid == 0) s_fail = 1;
        break;
      }
      if (tid == 0 && p != j) {
        double t = gv[j];
        gv[j] = gv[p];
        gv[p] = t;
      }
      if (p != j)
        for (int b = tid; b < k2; b += blockDim.x) {
          double t = Gm[j + b * k];
          Gm[j + b * k] = Gm[p + b * k];
          Gm[p + b * k] = t;
        }
      __syncthreads();
      const double d = Gm[j + j * k];
      for (int a = j + 1 + tid; a < k2; a += blockDim.x) Gm[a + j * k] /= d;
      __syncthreads();
      for (int e = tid; e < (k2 - j - 1) * (k2 - j - 1); e += blockDim.x) {
        const int a = j + 1 + e % (k2 - j - 1), b = j + 1 + e / (k2 - j - 1);
        Gm[a + b * k] -= Gm[a + j * k] * Gm[j + b * k];
      }
      __syncthreads();
    }
    __syncthreads();
    // L U y = g on wave 0 by columns, lane a = entry a: forward (unit lower, terms in
    // ascending order), then backward from the last entry
    if (wid == 0 && !s_fail) {
      const int a = lane;
      double acc = a < k2 ? gv[a] : 0.0;
      for (int l = 0; l < k2; ++l) {
        const double yl = lane_bcast(acc, l);
        if (a > l && a < k2) acc -= Gm[a + l * k] * yl;
      }
      for (int l = k2 - 1; l >= 0; --l) {
        if (a == l) acc = acc / Gm[a + a * k];
        const double yl = lane_bcast(acc, l);
        if (a < l) acc -= Gm[a + l * k] * yl;
      }
      if (a < k2) yv[a] = acc;
    }
  }
  __syncthreads();
  for (int a = tid; a < MAXM; a += blockDim.x) cv[a] = 0.0;
  __syncthreads();
  if (!s_fail)
    for (int a = tid; a < k2; a += blockDim.x) {
      double acc = 0.0;
      for (int l = a; l < k2; ++l) acc += Ri[a + l * k] * yv[l];
      cv[perm[a]] = acc;
    }
  __syncthreads();
  if (tid == 0) {
    int bad = s_fail;
    for (int a = 0; a < k; ++a)
      if (!isfinite(cv[a])) bad = 1;
    s_fail = bad;
  }
  __syncthreads();
  for (int a = tid; a < MAXM; a += blockDim.x) ctl->c[a] = s_fail ? 0.0 : cv[a];
  for (int l = tid; l < MAXM; l += blockDim.x) {
    double acc = 0.0;
    if (!s_fail && l < cnt)
      // T1's row l in rounds of 16 entries requested together (one load at a time would
      // wait for each in turn); the terms are added in column order
      for (int c0 = 0; c0 < k; c0 += 16) {
        double tv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) tv[u] = ctl->T1[l + (c0 + u < k ? c0 + u : k - 1) * MAXM];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (c0 + u < k) acc += tv[u] * cv[c0 + u];
      }
    ctl->cX[l] = acc;
  }
  if (tid == 0) {
    ctl->k2 = k2;
    ctl->fallback = s_fail;
    // the ranks and the decision of this guess, for the host (read after the solve)
    if (int *hi = ctl->hinfo) {
      ((volatile int *)hi)[0] = k;
      ((volatile int *)hi)[1] = k2;
      ((volatile int *)hi)[2] = s_fail;
    }
  }
}

__global__ __launch_bounds__(TPB) void k_small_solve(int cnt, int minres, int spd, double tau_c, Ctl *ctl) {
  small_solve_body(cnt, minres, spd, tau_c, ctl);
}

// many sequences' reduced solves in one launch: block b runs job b
__global__ __launch_bounds__(TPB) void k_small_solve_batch(const SolveJob *__restrict__ jobs) {
  const SolveJob &j = jobs[blockIdx.x];
  small_solve_body(j.cnt, j.minres, j.minres ? 1 : j.spd, j.tau_c, j.ctl);
}

static size_t small_solve_lds(int cnt, int minres) {
  const size_t lds = ((size_t)3 * cnt * cnt + (size_t)gram_width(cnt, minres)) * sizeof(double);
  return lds == 0 ? sizeof(double) : lds;
}

hipError_t launch_small_solve(int cnt, int minres, int spd, double tau_c, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(TPB), small_solve_lds(cnt, minres), st, cnt, minres,
                     minres ? 1 : spd, tau_c, ctl);
  return hipGetLastError();
}

hipError_t launch_small_solve_batch(const SolveJob *jobs_dev, const SolveJob *jobs_host, int njobs, hipStream_t st) {
  size_t lds = sizeof(double);
  for (int i = 0; i < njobs; ++i) lds = std::max(lds, small_solve_lds(jobs_host[i].cnt, jobs_host[i].minres));
  if (njobs > 0) hipLaunchKernelGGL(k_small_solve_batch, dim3(njobs), dim3(TPB), lds, st, jobs_dev);
  return hipGetLastError();
}

// ============================================================================ x0
template <int MC, typename TX>
__device__ __forceinline__ void x0_body(const TX *Q1, const TX *X, double *x0, int64_t n, int64_t ld,
                                        const Ctl *ctl) {
  __shared__ double cc[MC];
  const int k = ctl->k;
  const int fb = ctl->fallback;
  const int newest = ctl->newest;
  const int newest_ok = ctl->newest_ok;
  for (int c = threadIdx.x; c < MC; c += blockDim.x) cc[c] = (c < k) ? ctl->c[c] : 0.0;
  __syncthreads();
  GRID_ROWS(i, n) {
    double s = 0.0;
    if (fb) {
      s = (newest >= 0 && newest_ok) ? (double)X[(size_t)newest * ld + i] : 0.0;
    } else {
      for (int c = 0; c < k; ++c) s += (double)Q1[(size_t)c * ld + i] * cc[c];
    }
    x0[i] = s;
  }
}

template <int MC, typename TX>
__global__ __launch_bounds__(TPB) void k_x0(const TX *Q1, const TX *X, double *x0, int64_t n, int64_t ld,
                                            const Ctl *ctl) {
  x0_body<MC, TX>(Q1, X, x0, n, ld, ctl);
}

// many sequences' x0 in one launch: grid row y runs job y over its rows
template <typename TX>
__global__ __launch_bounds__(TPB) void k_x0_batch(const X0Job *__restrict__ jobs) {
  const X0Job &j = jobs[blockIdx.y];
  x0_body<MAXM, TX>((const TX *)j.Q1, (const TX *)j.X, j.x0, j.n, j.ld, j.ctl);
}

template <typename TX>
hipError_t launch_x0(const TX *Q1, const TX *X, double *x0, int64_t n, int64_t ld, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL((k_x0<MAXM, TX>), dim3(stream_blocks(n)), dim3(TPB), 0, st, Q1, X, x0, n, ld, ctl);
  return hipGetLastError();
}

template <typename TX>
hipError_t launch_x0_batch(const X0Job *jobs_dev, const X0Job *jobs_host, int njobs, hipStream_t st) {
  int64_t nmax = 1;
  for (int i = 0; i < njobs; ++i) nmax = std::max(nmax, jobs_host[i].n);
  if (njobs > 0) hipLaunchKernelGGL((k_x0_batch<TX>), dim3(stream_blocks(nmax), njobs), dim3(TPB), 0, st, jobs_dev);
  return hipGetLastError();
}

// y = (double) x  (the "previous solution" guess from an FP32 history column)
template <typename TX>
__global__ __launch_bounds__(TPB) void k_to_double(const TX *x, double *y, int64_t n) {
  GRID_ROWS(i, n) y[i] = (double)x[i];
}

template <typename TX>
hipError_t launch_to_double(const TX *x, double *y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_double<TX>, dim3(stream_blocks(n)), dim3(TPB), 0, st, x, y, n);
  return hipGetLastError();
}

// ============================================================================ iterative refinement
// Outer residual of the mixed mode: r = b - A32 x in FP64 (the FP32 matrix values are
// exact in FP64), the inner right-hand side r32 = fl32(r), and partial sums of
// ||r||^2 and ||b||^2.
template <typename VT, int C>
__global__ __launch_bounds__(TPB) void k_ir_resid(const int *rowptr, const int *col, const VT *val,
                                                  const double *b, const double *x, float *r32, int64_t n,
                                                  double *partials) {
  __shared__ double red[NWAVE * 2];
  __shared__ int lcol[NWAVE * WT_CAP];
  __shared__ VT lval[NWAVE * WT_CAP];
  const int wid = threadIdx.x / WAVE;
  double acc[2] = {0.0, 0.0};
  const WaveTiles wt = wave_tiles(n);
  wave_tiles_spmv<C>(
      rowptr, col, val, Gather1<double>{x}, n, wt.t, wt.end, wt.step, lcol + wid * WT_CAP, lval + wid * WT_CAP,
      [&](int64_t i) { return b[i]; },
      [&](int64_t i, double bi, double ax) {
        const double ri = bi - ax;
        r32[i] = (float)ri;
        acc[0] += ri * ri;
        acc[1] += bi * bi;
      });
  block_sum_store<2>(acc, 2, red, partials + (size_t)blockIdx.x * 2);
}

template <typename VT, int C>
static int ir_resid_c(const CsrView &A, const double *b, const double *x, float *r32, double *partials,
                      hipStream_t st) {
  static int cache = 0;
  const int nb = wave_grid((const void *)k_ir_resid<VT, C>, A.n, cache, IR_MAXBLK);
  const int *colp = A.nnz > 0 ? A.col : A.rowptr;
  const VT *valp = A.nnz > 0 ? (const VT *)A.val : (const VT *)x;
  hipLaunchKernelGGL((k_ir_resid<VT, C>), dim3(nb), dim3(TPB), 0, st, A.rowptr, colp, valp, b, x, r32, A.n,
                     partials);
  return nb;
}

template <typename VT>
static int ir_resid_vt(const CsrView &A, const double *b, const double *x, float *r32, double *partials,
                       hipStream_t st) {
  const int C = wave_tile_chunk(A.n, A.nnz);
  if (C <= 5) return ir_resid_c<VT, 5>(A, b, x, r32, partials, st);
  if (C <= 7) return ir_resid_c<VT, 7>(A, b, x, r32, partials, st);
  return ir_resid_c<VT, 9>(A, b, x, r32, partials, st);
}

// One block: the outer stopping test ||r|| <= tol ||b|| (first sweep also sets ||b||
// and relres0).  sweep = refinement sweeps done; state RUN means "refine again".
__global__ __launch_bounds__(TPB) void k_ir_close(const double *partials, int nblk, int sweep, int max_refine,
                                                  Ctl *ctl) {
  __shared__ double outv[2];
  __shared__ double scratch[TPB];
  final_sum(partials, nblk, 2, 2, outv, scratch);
  if (threadIdx.x != 0) return;
  if (sweep == 0) ctl->bnorm = sqrt(outv[1]);
  const double bn = ctl->bnorm, nr = sqrt(outv[0]);
  const double rel = bn > 0.0 ? nr / bn : 0.0;
  ctl->relres = rel;
  if (sweep == 0) ctl->relres0 = rel;
  if (bn == 0.0)
    ctl->state = ST_ZERO_RHS;
  else if (nr <= ctl->tol * bn)
    ctl->state = ST_CONV;
  else if (!isfinite(nr))
    ctl->state = ST_BREAK;
  else
    ctl->state = sweep >= max_refine ? ST_MAXIT : ST_RUN;
}

__global__ __launch_bounds__(TPB) void k_ir_update(double *x, const float *d, int64_t n) {
  GRID_ROWS(i, n) x[i] += (double)d[i];
}

hipError_t launch_ir_resid(const CsrView &A, const double *b, const double *x, float *r32, double *partials,
                           int sweep, int max_refine, Ctl *ctl, hipStream_t st) {
  const int nb = A.fp32 ? ir_resid_vt<float>(A, b, x, r32, partials, st)
                        : ir_resid_vt<double>(A, b, x, r32, partials, st);
  hipLaunchKernelGGL(k_ir_close, dim3(1), dim3(TPB), 0, st, partials, nb, sweep, max_refine, ctl);
  return hipGetLastError();
}

hipError_t launch_ir_update(double *x, const float *d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_ir_update, dim3(stream_blocks(n)), dim3(TPB), 0, st, x, d, n);
  return hipGetLastError();
}

// ============================================================================ control block reset
// Fill kernels rather than a memset, so that the call also stays valid in a captured
// stream: the grid clears every word, then one thread sets the solver settings.
__global__ __launch_bounds__(TPB) void k_ctl_clear(unsigned long long *w, int64_t nw) {
  GRID_ROWS(e, nw) w[e] = 0ull;
}

__global__ void k_ctl_set(Ctl *ctl, double tol, int maxit, int restart, int trust_est) {
  ctl->tol = tol;
  ctl->maxit = maxit;
  ctl->restart = restart;
  ctl->trust_est = trust_est;
  ctl->state = ST_CONV;
  ctl->newest = -1;
}

hipError_t launch_ctl_reset(Ctl *ctl, double tol, int maxit, int restart, int trust_est, hipStream_t st) {
  static_assert(sizeof(Ctl) % sizeof(unsigned long long) == 0, "control block of whole words");
  const int64_t nw = (int64_t)(sizeof(Ctl) / sizeof(unsigned long long));
  hipLaunchKernelGGL(k_ctl_clear, dim3(stream_blocks(nw)), dim3(TPB), 0, st, (unsigned long long *)ctl, nw);
  hipLaunchKernelGGL(k_ctl_set, dim3(1), dim3(1), 0, st, ctl, tol, maxit, restart, trust_est);
  return hipGetLastError();
}

// one word of device state set by a kernel (instead of a small host-to-device copy)
__global__ void k_set_int(int *p, int v) {
  if (threadIdx.x == 0) *p = v;
}

hipError_t launch_set_int(int *p, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(TPB) void k_zero(double *x, int64_t n) {
  GRID_ROWS(i, n) x[i] = 0.0;
}

hipError_t launch_zero(double *x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3(stream_blocks(n)), dim3(TPB), 0, st, x, n);
  return hipGetLastError();
}

#define SACC_INSTANTIATE_PROJ(TX)                                                                              \
  template hipError_t launch_push_bf16<TX>(const double *, TX *, const unsigned short *, double *, int64_t,       \
                                           int64_t, int, int, double *, const Ctl *, int, hipStream_t);           \
  template hipError_t launch_push<TX>(const double *, TX *, double *, int64_t, int64_t, int, int, int, uint64_t, \
                                      const long long *, const unsigned long long *, double *, const Ctl *, int, \
                                      hipStream_t);                                                            \
  template hipError_t launch_basis<TX>(const TX *, TX *, int64_t, int64_t, int, Ctl *, hipStream_t);           \
  template hipError_t launch_spmm_gram<TX>(const CsrView &, const TX *, int64_t, const double *, int, int,    \
                                           double *, int *, Ctl *, hipStream_t);                               \
  template hipError_t launch_x0<TX>(const TX *, const TX *, double *, int64_t, int64_t, Ctl *, hipStream_t);   \
  template hipError_t launch_x0_batch<TX>(const X0Job *, const X0Job *, int, hipStream_t);                     \
  template hipError_t launch_gram_x<TX>(const TX *, int64_t, int64_t, int, double *, int *, hipStream_t);     \
  template hipError_t launch_to_double<TX>(const TX *, double *, int64_t, hipStream_t);

SACC_INSTANTIATE_PROJ(double)
SACC_INSTANTIATE_PROJ(float)

size_t partials_doubles(int64_t n, int M, int s) {
  (void)n;
  size_t a = krylov_partials_doubles();                                 // Krylov dots
  size_t b = (size_t)MAXBLK * SKETCH_RG;                                // sketch
  size_t c = (size_t)GRAM_MAXBLK * M * (3 * M + 2);                     // Gram (minimum residual)
  (void)s;
  size_t m = a > b ? a : b;
  return m > c ? m : c;
}

}  // namespace sacc
