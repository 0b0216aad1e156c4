// Device helpers shared by the kernels: launch geometry, deterministic reductions,
// the Philox4x64-10 counter-based generator and the sketch entries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sacc {

constexpr int TPB = 256;          // threads per block of the streaming kernels
constexpr int WAVE = 64;          // CDNA wavefront width
constexpr int NWAVE = TPB / WAVE;
constexpr int MAXBLK = 512;       // cap on blocks of a streaming kernel (grid-stride beyond)
constexpr int MAXM = 64;          // longest history
constexpr int MAXS = 256;         // most sketch rows
constexpr int MAXR = 64;          // longest GMRES cycle
constexpr int SKETCH_RG = 16;     // sketch rows per block row-group

// Solver states kept in the device control block.
enum : int {
  ST_RUN = 0,      // iterating
  ST_CHECK = 1,    // recursive residual met the tolerance: confirm with the true residual
  ST_CONV = 2,     // converged (true residual)
  ST_MAXIT = 3,    // iteration cap reached
  ST_BREAK = 4,    // breakdown (CG p^T A p <= 0, non-finite numbers)
  ST_ZERO_RHS = 5  // b = 0: the solution is x = 0
};

// Per-sequence control block in device memory.  Scalars of the Krylov recurrences,
// the small dense factors of the projection and the reduction counters live here so
// that no host round trip is needed inside a step.
struct Ctl {
  // Krylov state (read by the host poll: state .. pad0 are contiguous)
  double bnorm, relres0, relres, tol;
  int state, iters, restarts, maxit;
  int active, jend, restart, pad0;
  double rho[4], beta[4];       // CG: r^T r and beta of iteration k in slot k & 3
  double h1[MAXR + 1];          // GMRES: first Gram-Schmidt pass of the current step
  double cs[MAXR], sn[MAXR];    // Givens rotations
  double gam[MAXR + 1];         // rotated right-hand side (final entries)
  double gnext[MAXR + 2];       // carried entry g_{j} before rotation j
  double y[MAXR], vs[MAXR + 1]; // cycle solution; scale of each unnormalised V column
  double Hraw[(MAXR + 1) * MAXR];  // column-major raw Hessenberg columns
  double R[(MAXR + 1) * MAXR];     // column-major rotated columns (upper triangular)
  // projection
  int k, k2, fallback, cnt;
  int newest, nonfinite, newest_ok, pad1;
  double T1[MAXM * MAXM];  // M x M column-major; row = ring slot, column = basis index
  double c[MAXM];          // x0 = Q1 c
  double cX[MAXM];         // x0 = X cX (ring-slot coordinates)
  double gram[MAXM * MAXM * 3 + 2 * MAXM];  // reduced G | Ht | gt  (| K | ht for MINRES)
};

// ---------------------------------------------------------------- launch geometry
inline int stream_blocks(int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  return (int)(b > MAXBLK ? MAXBLK : b);
}

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Block-reduce K per-thread values (fixed butterfly + fixed wave order) and store the
// block's sums at out[0..kc).  `red` is LDS of at least NWAVE * K doubles.
template <int K>
__device__ inline void block_sum_store(const double (&v)[K], int kc, double *red, double *out) {
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
#pragma unroll
  for (int e = 0; e < K; ++e) {
    if (e < kc) {
      double s = wave_sum(v[e]);
      if (lane == 0) red[wid * K + e] = s;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kc; e += blockDim.x) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) s += red[w * K + e];
    out[e] = s;
  }
}

// Cross-block results never use device-scope fences (on a multi-XCD part each one
// writes back the L2): a kernel's per-block partial rows are reduced by the next
// kernel, whose launch orders them.
//
// Sums over nblk rows of partials[nblk][W] for entries e < kc, in
// a fixed order (strided per-thread sums, then a fixed tree), into LDS out[0..kc).
// `scratch` is LDS of blockDim.x doubles; blockDim.x must be a power of two.
__device__ inline void final_sum(const double *partials, int nblk, int W, int kc, double *out,
                                 double *scratch) {
  for (int e0 = 0; e0 < kc; e0 += 32) {
    const int ec = kc - e0 < 32 ? kc - e0 : 32;
    int ep = 1;
    while (ep < ec) ep <<= 1;
    const int ngrp = blockDim.x / ep;
    const int e = threadIdx.x % ep, grp = threadIdx.x / ep;
    // four independent accumulators keep several loads in flight
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (e < ec) {
      int b = grp;
      for (; b + 3 * ngrp < nblk; b += 4 * ngrp) {
        s0 += partials[(size_t)b * W + e0 + e];
        s1 += partials[(size_t)(b + ngrp) * W + e0 + e];
        s2 += partials[(size_t)(b + 2 * ngrp) * W + e0 + e];
        s3 += partials[(size_t)(b + 3 * ngrp) * W + e0 + e];
      }
      for (; b < nblk; b += ngrp) s0 += partials[(size_t)b * W + e0 + e];
    }
    scratch[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int off = ngrp / 2; off > 0; off >>= 1) {
      if (grp < off) scratch[threadIdx.x] += scratch[threadIdx.x + off * ep];
      __syncthreads();
    }
    if (threadIdx.x < ec) out[e0 + threadIdx.x] = scratch[threadIdx.x];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- CSR stream SpMV
constexpr int SPMV_CAP = 4096;  // nonzeros of one row tile staged in LDS (32 KB)

// (A x)_i for row i = r0 + threadIdx.x of the row tile [r0, r0 + blockDim.x) (0 beyond
// n).  Every thread of the block must call it for the same r0.  The tile's val/col
// are read with consecutive threads on consecutive nonzeros (coalesced) and the
// products staged in LDS; each thread then sums its row in column order.  Tiles with
// more than SPMV_CAP nonzeros read their rows directly.
template <typename VT, typename TX>
__device__ inline double tile_spmv(const int *__restrict__ rowptr, const int *__restrict__ col,
                                   const VT *__restrict__ val, const TX *__restrict__ x, int64_t n,
                                   int64_t r0, double *prod) {
  const int t = threadIdx.x;
  const int64_t i = r0 + t;
  const int64_t rl = (r0 + (int64_t)blockDim.x < n) ? r0 + (int64_t)blockDim.x : n;
  const int p0 = rowptr[r0], p1 = rowptr[rl];
  int a = 0, b = 0;
  if (i < n) {
    a = rowptr[i];
    b = rowptr[i + 1];
  }
  double s = 0.0;
  if (p1 - p0 <= SPMV_CAP) {
    for (int p = p0 + t; p < p1; p += blockDim.x) prod[p - p0] = (double)val[p] * (double)x[col[p]];
    __syncthreads();
    for (int p = a; p < b; ++p) s += prod[p - p0];
    __syncthreads();
  } else {
    for (int p = a; p < b; ++p) s += (double)val[p] * (double)x[col[p]];
  }
  return s;
}

// ---------------------------------------------------------------- Philox4x64-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11.
struct U64x4 {
  uint64_t v[4];
};

__device__ inline U64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                   uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U64x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// ((w >> 12) + 1/2) 2^-52: exact binary64 in (0, 1).
__device__ inline double unit_open(uint64_t w) {
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

enum : uint64_t { STREAM_GAUSS_SKETCH = 1, STREAM_SRHT_SIGNS = 2, STREAM_SRHT_ROWS = 3 };

// Four Box-Muller normals of block (c0, c1, stream): (cos0, sin0, cos1, sin1).
__device__ inline void normals4(uint64_t c0, uint64_t c1, uint64_t stream, uint64_t seed, double g[4]) {
  U64x4 w = philox4x64(c0, c1, stream, 0, seed, 0);
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    double rad = sqrt(-2.0 * log(unit_open(w.v[2 * p])));
    double sv, cv;
    sincospi(2.0 * unit_open(w.v[2 * p + 1]), &sv, &cv);
    g[2 * p] = rad * cv;
    g[2 * p + 1] = rad * sv;
  }
}

// SRHT sign d_j in {+1, -1}.
__device__ inline double srht_sign(uint64_t j, uint64_t seed) {
  U64x4 w = philox4x64(j >> 8, 0, STREAM_SRHT_SIGNS, 0, seed, 0);
  uint64_t word = w.v[(j & 255) >> 6];
  return ((word >> (j & 63)) & 1ull) ? -1.0 : 1.0;
}

}  // namespace sacc
