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
constexpr int MAXR = 32;          // longest GMRES cycle
constexpr int SKETCH_RG = 16;     // sketch rows per block row-group
constexpr int WORK_LOG = 4096;    // timed launches logged per solve
constexpr int LHIST_MAX = 16;     // ring of learned-predictor targets

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
  int active, jend, restart, col16_ok;  // col16_ok: the packed column offsets of the current
                                         // matrix fit in 16 bits (mixed CG)
  int kcur;                     // CG: number of the iteration in flight
  int fresh_at;                 // CG: iteration whose direction restarts from p = r
  int ibase;                    // GMRES: iterations done before the current cycle
  int trust_est;                // inner solves: accept the recursive residual estimate
  int conv_pending;             // GMRES: the last cycle ended on the estimate (trust_est)
  int pad2;
  double rho[4];                // CG: r^T r after iteration k in slot k & 3
  double cg_alpha;              // CG: alpha of iteration cg_xk, whose x += alpha p is pending
  int cg_xk, cg_xdone;          // CG: iteration of the pending x update; last one applied by
                                // the fix-up kernel (the next p / q kernel applies it otherwise)
  unsigned long long *mirror;   // host-visible progress word (pinned host memory), or null
  int *hinfo;                   // host-visible guess record (pinned host memory), or null:
                                // [0] k, [1] k2, [2] fallback (reduced solve), [4] learned used
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
  // kernel timing: launch l of a timed solve sets work_log[l] = 1 when it did its work
  int work_log[WORK_LOG];
  // learned predictor: targets of past steps (lag order), last decision and residuals
  double lhist[LHIST_MAX * MAXM];
  double learned_r2[2];
  int learned_used, pad3;
};

// Progress word the host reads while it enqueues a solve (pinned host memory, one
// 64-bit store, so the serial and the flags arrive together): the serial number the
// host gave the last step kernel that ran, and what that kernel saw.  A kernel cannot
// complete before its store to host memory is acknowledged, so steps without news
// report only every MIR_EVERY serials; any flag is reported at once.
// MIR_EST_CONV comes with MIR_CYCLE_END when the cycle ended on its residual estimate
// (the restart's true residual will most likely end the solve).
enum : unsigned { MIR_STOPPED = 1u, MIR_CYCLE_END = 2u, MIR_CHECK = 4u, MIR_EST_CONV = 8u };
constexpr int MIR_EVERY = 8;

// A serial with MIR_REPORT set asks for a report even without news (the host waits for it).
constexpr int MIR_REPORT = 1 << 30;

__device__ inline void mirror_report(unsigned long long *m, int serial, unsigned flags) {
  const bool force = (serial & MIR_REPORT) != 0;
  serial &= ~MIR_REPORT;
  if (m && serial > 0 && (force || flags != 0u || serial % MIR_EVERY == 0))
    *(volatile unsigned long long *)m = ((unsigned long long)(unsigned)serial << 32) | flags;
}

// ---------------------------------------------------------------- launch geometry
inline int stream_blocks(int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  return (int)(b > MAXBLK ? MAXBLK : b);
}

// Blocks of `kernel` with `threads` threads the device holds at once (0 when the runtime
// cannot say); `cache` is the caller's per-kernel slot, filled on the first call.
inline int resident_blocks(const void *kernel, int threads, int &cache) {
  if (cache == 0) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1)
      return 0;
    cache = per * ncu;
  }
  return cache;
}

// grid-stride loop over rows
#define GRID_ROWS(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// ---------------------------------------------------------------- control-block reads
// Reads of control-block fields through the vector memory path: the index is a register
// the compiler cannot prove uniform, so the read is a global load counted with the other
// vector loads.  A scalar load shares its wait counter with the kernel-argument and LDS
// traffic, so the first wait for an argument or an LDS result after it would also wait
// for a control-block read still on its way from memory (one more trip before the
// kernel's main loads go out).
__device__ inline int vzero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}
template <typename T>
__device__ inline T vread(const T *p, int z) {
  return p[z];
}

// ---------------------------------------------------------------- reductions
// Cross-lane exchanges without the LDS unit: v_permlane32_swap / v_permlane16_swap
// (gfx950) for partners 32 and 16 lanes apart, DPP row controls inside a row of 16
// (row_mirror, row_half_mirror, two quad permutations).  Each pairs every lane with
// a partner in the other half of its current group, which is all a fixed-order
// recursive reduction needs.
__device__ inline unsigned dlo(double v) { return (unsigned)__double2loint(v); }
__device__ inline unsigned dhi(double v) { return (unsigned)__double2hiint(v); }
__device__ inline double dmake(unsigned lo, unsigned hi) { return __hiloint2double((int)hi, (int)lo); }

// lane i's value of v, in every lane (i uniform)
__device__ inline double lane_bcast(double v, int i) {
  const int lo = __builtin_amdgcn_readlane((int)dlo(v), i), hi = __builtin_amdgcn_readlane((int)dhi(v), i);
  return dmake((unsigned)lo, (unsigned)hi);
}

// x' + y' after exchanging the upper half of x's lane group with the lower half of
// y's: lanes in a lower half get the pair sum of x, lanes in an upper half the pair
// sum of y.  W = 32 (halves of the wave) or 16 (rows).
template <int W>
__device__ inline double swap_sum(double x, double y) {
  static_assert(W == 32 || W == 16, "permlane swaps exchange 32- or 16-lane groups");
  if constexpr (W == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(dlo(x), dlo(y), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(dhi(x), dhi(y), false, false);
    return dmake(lo[0], hi[0]) + dmake(lo[1], hi[1]);
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(dlo(x), dlo(y), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(dhi(x), dhi(y), false, false);
    return dmake(lo[0], hi[0]) + dmake(lo[1], hi[1]);
  }
}

// the partner's value under a DPP row control
template <int CTRL>
__device__ inline double dpp_partner(double v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)dlo(v), CTRL, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)dhi(v), CTRL, 0xF, 0xF, true);
  return dmake(lo, hi);
}

// Largest value over the wave's lanes and its index, the lowest index among equal values
// (values not NaN); every lane returns the index.  Exchanges: permlane32 / permlane16
// swaps, then DPP row rotations by 8, 4, 2, 1 (a total order, so every lane ends with
// the same pair).
__device__ inline void argmax_take(double &v, int &i, double ov, int oi) {
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}
template <int W>
__device__ inline void argmax_swap_step(double &v, int &i) {
  const bool up = (threadIdx.x & W) != 0;
  unsigned lo0, lo1, hi0, hi1, i0, i1;
  if constexpr (W == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(dlo(v), dlo(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(dhi(v), dhi(v), false, false);
    const auto ix = __builtin_amdgcn_permlane32_swap((unsigned)i, (unsigned)i, false, false);
    lo0 = lo[0]; lo1 = lo[1]; hi0 = hi[0]; hi1 = hi[1]; i0 = ix[0]; i1 = ix[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(dlo(v), dlo(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(dhi(v), dhi(v), false, false);
    const auto ix = __builtin_amdgcn_permlane16_swap((unsigned)i, (unsigned)i, false, false);
    lo0 = lo[0]; lo1 = lo[1]; hi0 = hi[0]; hi1 = hi[1]; i0 = ix[0]; i1 = ix[1];
  }
  // lower lanes find the partner's value in the second result, upper lanes in the first
  const double ov = up ? dmake(lo0, hi0) : dmake(lo1, hi1);
  const int oi = (int)(up ? i0 : i1);
  argmax_take(v, i, ov, oi);
}
template <int D>
__device__ inline void argmax_ror_step(double &v, int &i) {
  const double ov = dpp_partner<0x120 + D>(v);
  const int oi = __builtin_amdgcn_update_dpp(0, i, 0x120 + D, 0xF, 0xF, true);
  argmax_take(v, i, ov, oi);
}
__device__ inline int wave_argmax(double v, int i) {
  argmax_swap_step<32>(v, i);
  argmax_swap_step<16>(v, i);
  argmax_ror_step<8>(v, i);
  argmax_ror_step<4>(v, i);
  argmax_ror_step<2>(v, i);
  argmax_ror_step<1>(v, i);
  return __builtin_amdgcn_readfirstlane(i);
}

// Level L = 0..5 of the wave reduction splits lane groups of 64 >> L at lane bit
// 32 >> L: partners by permlane32 / permlane16 swaps, then row_mirror (lane i <-> 15 - i),
// row_half_mirror (i <-> 7 - i), quad permutations [3,2,1,0] and [1,0,3,2].
constexpr int DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141, DPP_QUAD_3210 = 0x1B, DPP_QUAD_1032 = 0xB1;

template <int L>
__device__ inline double level_partner(double v) {
  if constexpr (L == 2) return dpp_partner<DPP_ROW_MIRROR>(v);
  else if constexpr (L == 3) return dpp_partner<DPP_ROW_HALF_MIRROR>(v);
  else if constexpr (L == 4) return dpp_partner<DPP_QUAD_3210>(v);
  else return dpp_partner<DPP_QUAD_1032>(v);
}

// keep one of (lo, hi) by this lane's half and add the partner's other one
template <int L>
__device__ inline double level_halve(double lo, double hi, int lane) {
  if constexpr (L == 0) return swap_sum<32>(lo, hi);
  else if constexpr (L == 1) return swap_sum<16>(lo, hi);
  else {
    const bool up = (lane & (32 >> L)) != 0;
    const double send = up ? lo : hi, keep = up ? hi : lo;
    return keep + level_partner<L>(send);
  }
}

// v + the partner's v
template <int L>
__device__ inline double level_full(double v) {
  if constexpr (L == 0) return swap_sum<32>(v, v);
  else if constexpr (L == 1) return swap_sum<16>(v, v);
  else return v + level_partner<L>(v);
}

template <int K, int L>
__device__ inline void wave_level(double (&v)[K], int lane) {
  if constexpr (L < 6) {
    constexpr int LOGK = K >= 64 ? 6 : K >= 32 ? 5 : K >= 16 ? 4 : K >= 8 ? 3 : K >= 4 ? 2 : K >= 2 ? 1 : 0;
    if constexpr (L < LOGK) {
      constexpr int H = K >> (L + 1);
#pragma unroll
      for (int i = 0; i < H; ++i) v[i] = level_halve<L>(v[i], v[i + H], lane);
    } else {
      v[0] = level_full<L>(v[0]);
    }
    wave_level<K, L + 1>(v, lane);
  }
}

// Sums over the 64 lanes of a wave of K per-lane values (K a power of two <= 64) by
// recursive halving: at each level a lane keeps half of its entries and adds its
// partner's copy of that half, so K - 1 + log2(64 / K) exchanges replace 6 K.  On
// return lane l holds in v[0] the total of entry l / (64 / K).  Fixed order.
template <int K>
__device__ inline void wave_sum_multi(double (&v)[K]) {
  static_assert(K >= 1 && K <= WAVE && (K & (K - 1)) == 0, "K must be a power of two <= 64");
  wave_level<K, 0>(v, (int)(threadIdx.x % WAVE));
}

// total over the wave, in every lane
__device__ inline double wave_sum(double v) {
  double a[1] = {v};
  wave_sum_multi<1>(a);
  return a[0];
}

// Block-reduce K per-thread values (K a power of two; fixed butterfly and fixed wave
// order) and store the block's sums at out[0..kc).  `red` is LDS of at least
// (blockDim.x / 64) * K doubles.  The values in v are consumed.
template <int K>
__device__ inline void block_sum_store(double (&v)[K], int kc, double *red, double *out) {
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  constexpr int STEP = WAVE / K;
  wave_sum_multi<K>(v);
  if (lane % STEP == 0) red[wid * K + lane / STEP] = v[0];
  __syncthreads();
  for (int e = threadIdx.x; e < kc; e += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w * K + e];
    out[e] = s;
  }
}

// Cross-block results never use device-scope fences (on a multi-XCD part each one
// writes back the L2): a kernel's per-block partial rows are reduced by the next
// kernel, whose launch orders them.
//
// Sums over nblk rows of partials[nblk][W] for entries e < kc, in a fixed order
// (per-thread sums over a strided set of rows, all loads of a thread issued
// together, then the fixed tree of final_tree), into LDS out[0..kc), 64 entries at a
// time.  `scratch` is LDS of blockDim.x doubles; blockDim.x must be a multiple of 64.
template <int U = 32>
__device__ inline double final_part(const double *partials, int nblk, int W, int kc);
__device__ inline void final_tree(double s, int kc, double *out, double *scratch);
__device__ inline void final_sum(const double *partials, int nblk, int W, int kc, double *out,
                                 double *scratch) {
  for (int e0 = 0; e0 < kc; e0 += WAVE) {
    const int ec = kc - e0 < WAVE ? kc - e0 : WAVE;
    final_tree(final_part(partials + e0, nblk, W, ec), ec, out + e0, scratch);
  }
}

// final_sum for kc <= 64 entries in two halves, so that a kernel can issue the loads
// of its partial rows before it knows whether it runs (together with its control-block
// reads: one trip to memory instead of two).  final_part: this thread's sum over its
// rows (the same rows and order as final_sum); final_tree: the fixed tree into LDS
// out[0..kc), identical results to final_sum.
template <int U>
__device__ inline double final_part(const double *partials, int nblk, int W, int kc) {
  int ep = 1;
  while (ep < kc) ep <<= 1;
  const int ngrp = blockDim.x / ep;
  const int e = threadIdx.x % ep, grp = threadIdx.x / ep;
  double s = 0.0;
  if (e < kc) {
    for (int b0 = grp; b0 < nblk; b0 += U * ngrp) {
      double t[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int b = b0 + u * ngrp;
        const double x = partials[(size_t)(b < nblk ? b : nblk - 1) * W + e];
        t[u] = b < nblk ? x : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) s += t[u];
    }
  }
  return s;
}

// final_part in two halves, so that the loads of the partial rows go out with a
// kernel's other first-trip loads and the sum runs after a barrier: final_part_load
// issues U rows per thread (every thread, no branch around the loads: entries and rows
// past the valid ranges re-read valid ones), final_part_sum adds them (masked) and any
// further rows, in final_part's order and with its result.  U is chosen by the caller
// from the entry count it expects (nblk <= U * blockDim.x / ep rows in one round).
template <int U>
__device__ inline void final_part_load(const double *partials, int nblk, int W, int kc, double (&t)[U]) {
  int ep = 1;
  while (ep < kc) ep <<= 1;
  const int ngrp = blockDim.x / ep;
  const int e = threadIdx.x % ep, grp = threadIdx.x / ep;
  const int ec = e < kc ? e : kc - 1;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int b = grp + u * ngrp;
    t[u] = partials[(size_t)(b < nblk ? b : nblk - 1) * W + ec];
  }
}

template <int U>
__device__ inline double final_part_sum(const double *partials, int nblk, int W, int kc, const double (&t)[U]) {
  int ep = 1;
  while (ep < kc) ep <<= 1;
  const int ngrp = blockDim.x / ep;
  const int e = threadIdx.x % ep, grp = threadIdx.x / ep;
  double s = 0.0;
  if (e < kc) {
#pragma unroll
    for (int u = 0; u < U; ++u) s += (grp + u * ngrp < nblk) ? t[u] : 0.0;
    for (int b = grp + U * ngrp; b < nblk; b += ngrp) s += partials[(size_t)b * W + e];
  }
  return s;
}

// One folding step of final_tree: v plus the value of the lane D apart in the same
// entry (lane % ep), for D = 32, 16 (permlane swaps) and 8, 4, 2, 1 (DPP row_ror:D,
// rotation inside rows of 16).  Applied from D = 32 down to ep, every lane ends with
// the sum over the lanes of its wave that hold its entry, the same value in each.
template <int D>
__device__ inline double tree_fold(double v) {
  if constexpr (D == 32) return swap_sum<32>(v, v);
  else if constexpr (D == 16) return swap_sum<16>(v, v);
  else return v + dpp_partner<0x120 + D>(v);
}

// Fixed tree over the threads' sums s of entry threadIdx.x % ep (ep = kc rounded up to
// a power of two, kc <= 64): folded inside each wave, then the waves' sums added in
// wave order, into LDS out[0..kc).  Called by every thread of the block.
__device__ inline void final_tree(double s, int kc, double *out, double *scratch) {
  int ep = 1;
  while (ep < kc) ep <<= 1;
  if (ep <= 32) s = tree_fold<32>(s);
  if (ep <= 16) s = tree_fold<16>(s);
  if (ep <= 8) s = tree_fold<8>(s);
  if (ep <= 4) s = tree_fold<4>(s);
  if (ep <= 2) s = tree_fold<2>(s);
  if (ep <= 1) s = tree_fold<1>(s);
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  if (lane < ep) scratch[wid * ep + lane] = s;
  __syncthreads();
  if (threadIdx.x < kc) {
    double a = 0.0;
    for (int w = 0; w < nw; ++w) a += scratch[w * ep + threadIdx.x];
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- CSR stream SpMV
constexpr int SPMV_CAP = 4096;  // nonzeros of one row tile staged in LDS (32 KB)

// CSR row tile [r0, r0 + NT) for NT = threads of the block, row i = r0 + threadIdx.x.
// Stage: the tile's col/val are read with consecutive threads on consecutive nonzeros
// (coalesced), a chunk of C per thread issued before the first is used (indices past
// the tile re-read its last entry and are dropped), then the gathers, and the
// products are written to LDS.  Sum (after a barrier): each thread adds its row in
// column order.  Tiles with more than SPMV_CAP nonzeros read their rows directly in
// the sum.  `gx(c)` returns the source vector's entry c in double.  Every thread of
// the block must take part, for the same r0.
struct TileRows {
  int a, b, p0, direct;
};

template <int NT, typename VT, typename G>
__device__ inline TileRows tile_spmv_stage(const int *__restrict__ rowptr, const int *__restrict__ col,
                                           const VT *__restrict__ val, const G &gx, int64_t n, int64_t r0,
                                           double *prod) {
  constexpr int C = 6;
  const int t = threadIdx.x;
  const int64_t i = r0 + t;
  const int64_t rl = (r0 + (int64_t)NT < n) ? r0 + (int64_t)NT : n;
  const int p0 = rowptr[r0], p1 = rowptr[rl];
  TileRows tr{0, 0, p0, 0};
  if (i < n) {
    tr.a = rowptr[i];
    tr.b = rowptr[i + 1];
  }
  if (p1 - p0 > SPMV_CAP) {
    tr.direct = 1;
    return tr;
  }
  for (int base = p0; base < p1; base += C * NT) {
    int cc[C];
    double vv[C], xx[C];
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int p = base + t + u * NT;
      const int pc = p < p1 ? p : p1 - 1;
      cc[u] = col[pc];
      vv[u] = (double)val[pc];
    }
#pragma unroll
    for (int u = 0; u < C; ++u) xx[u] = gx(cc[u]);
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int p = base + t + u * NT;
      if (p < p1) prod[p - p0] = vv[u] * xx[u];
    }
  }
  return tr;
}

template <typename VT, typename G>
__device__ inline double tile_spmv_sum(const TileRows &tr, const int *__restrict__ col, const VT *__restrict__ val,
                                       const G &gx, const double *prod) {
  double s = 0.0;
  if (!tr.direct) {
    for (int p = tr.a; p < tr.b; ++p) s += prod[p - tr.p0];
  } else {
    for (int p = tr.a; p < tr.b; ++p) s += (double)val[p] * gx(col[p]);
  }
  return s;
}

// (A x)_i of the tile in one call (stage, barrier, sum, barrier)
template <int NT, typename VT, typename G>
__device__ inline double tile_spmv_g(const int *__restrict__ rowptr, const int *__restrict__ col,
                                     const VT *__restrict__ val, const G &gx, int64_t n, int64_t r0,
                                     double *prod) {
  const TileRows tr = tile_spmv_stage<NT>(rowptr, col, val, gx, n, r0, prod);
  __syncthreads();
  const double s = tile_spmv_sum(tr, col, val, gx, prod);
  __syncthreads();
  return s;
}

// Row tile of R NT rows [r0, r0 + R NT): thread t owns rows r0 + u NT + t, u < R.
// The same stage / sum scheme as above for all R rows at once (one row-pointer trip,
// one column / value trip, one gather trip for the whole tile); CAP = nonzeros staged
// in LDS (prod holds CAP doubles).
template <int R>
struct TileRowsR {
  int a[R], b[R];
  int p0, direct;
};

template <int NT, int R, int CAP, typename VT, typename G>
__device__ inline TileRowsR<R> tile_spmv_stage_r(const int *__restrict__ rowptr, const int *__restrict__ col,
                                                 const VT *__restrict__ val, const G &gx, int64_t n, int64_t r0,
                                                 double *prod) {
  constexpr int C = 6;
  const int t = threadIdx.x;
  const int64_t rl = (r0 + (int64_t)R * NT < n) ? r0 + (int64_t)R * NT : n;
  const int p0 = rowptr[r0], p1 = rowptr[rl];
  TileRowsR<R> tr;
  tr.p0 = p0;
  tr.direct = 0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int64_t i = r0 + (int64_t)u * NT + t;
    const int64_t ic = i < n ? i : n - 1;
    const int a = rowptr[ic], b = rowptr[ic + 1];
    tr.a[u] = i < n ? a : 0;
    tr.b[u] = i < n ? b : 0;
  }
  if (p1 - p0 > CAP) {
    tr.direct = 1;
    return tr;
  }
  // rounds of C nonzeros per thread, software-pipelined: a round's gathers and the next
  // round's column / value loads are in flight together, so a round costs one trip to
  // memory instead of two (loads past the range re-read an in-bounds entry)
  int cc[C];
  double vv[C];
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const int p = p0 + t + u * NT;
    const int pc = p < p1 ? p : (p1 > 0 ? p1 - 1 : 0);
    cc[u] = col[pc];
    vv[u] = (double)val[pc];
  }
  for (int base = p0; base < p1; base += C * NT) {
    double xx[C];
#pragma unroll
    for (int u = 0; u < C; ++u) xx[u] = gx(cc[u]);
    int cn[C];
    double vn[C];
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int p = base + C * NT + t + u * NT;
      const int pc = p < p1 ? p : p1 - 1;
      cn[u] = col[pc];
      vn[u] = (double)val[pc];
    }
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int p = base + t + u * NT;
      if (p < p1) prod[p - p0] = vv[u] * xx[u];
    }
#pragma unroll
    for (int u = 0; u < C; ++u) {
      cc[u] = cn[u];
      vv[u] = vn[u];
    }
  }
  return tr;
}

template <int R, typename VT, typename G>
__device__ inline void tile_spmv_sum_r(const TileRowsR<R> &tr, const int *__restrict__ col,
                                       const VT *__restrict__ val, const G &gx, const double *prod,
                                       double (&s)[R]) {
#pragma unroll
  for (int u = 0; u < R; ++u) {
    double acc = 0.0;
    if (!tr.direct) {
      for (int p = tr.a[u]; p < tr.b[u]; ++p) acc += prod[p - tr.p0];
    } else {
      for (int p = tr.a[u]; p < tr.b[u]; ++p) acc += (double)val[p] * gx(col[p]);
    }
    s[u] = acc;
  }
}

template <typename TX>
struct Gather1 {
  const TX *__restrict__ x;
  __device__ double operator()(int c) const { return (double)x[c]; }
};

template <int NT, typename VT, typename TX>
__device__ inline double tile_spmv(const int *__restrict__ rowptr, const int *__restrict__ col,
                                   const VT *__restrict__ val, const TX *__restrict__ x, int64_t n,
                                   int64_t r0, double *prod) {
  return tile_spmv_g<NT>(rowptr, col, val, Gather1<TX>{x}, n, r0, prod);
}

// ---------------------------------------------------------------- wave-tile CSR SpMV
// A wave owns a tile of 64 consecutive rows (lane l: row r0 + l) and works on it alone:
// no block barrier, so the waves of a block (and the several blocks a compute unit
// holds) overlap each other's memory trips.  Stage: the tile's nonzeros [p0, p1) are
// read with consecutive lanes on consecutive nonzeros (coalesced), C per lane per round,
// and the column indices and values go to the wave's own LDS slices.  Gather: each lane
// then walks its own row, C entries at a time, all gathers of a step issued together,
// so that lane l's k-th gather sits next to lane l+1's whenever neighbouring rows have
// neighbouring columns (a stencil): a gather instruction then touches two or three
// cache lines instead of one per row it crosses.  Each lane adds its row's products in
// column order, each product rounded before it is added (no fused multiply-add, the
// rounding of a plain CSR product loop).  Tiles with more than WT_CAP nonzeros read
// their rows directly.  `gx(c)` returns the source vector's entry c (double, or the
// vector's own type).
constexpr int WT_CAP = 512;  // nonzeros of one wave tile staged in LDS
constexpr int NXCD = 8;      // accelerator complex dies (each with its own L2) of the MI355X

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave's loop over its tiles t, t + step, ... < end.  Per tile: the next tile's row
// pointers go out first; this tile's first round of columns / values (requested while
// the previous tile was summed) goes to LDS, later rounds of a long tile load inline;
// then the next tile's first round is requested, then this tile's gathers and `pre`
// (a load of the row's own entries), so the next tile's index stream overlaps this
// tile's gathers.  `epi(i, pre value, (A x)_i)` runs for every row i < n.  Loads are
// unconditional (a load under a branch makes the compiler count the memory queue as if
// it had not gone out, so its later waits drain the queue): slots past a tile re-read
// its last entry, a tile with no nonzero up to it re-reads entry 0, so col and val must
// hold at least one entry even for a matrix without nonzeros (callers pass stand-ins),
// and the loads of the last tile's successor re-read the last tile.  lcol / lval: the
// wave's LDS slices of WT_CAP entries.  IT: the column index type, int (columns) or
// short (each entry's column minus its row, for matrices whose offsets fit in 16 bits:
// half the index bytes; the products and their order are the same).
// The row pointers of a wave's first tile, for a caller that requests them before its
// own prologue (wave_tiles_spmv's `first` argument); in bounds for any t.
struct TileRows0 {
  int a, b;
};
__device__ inline TileRows0 wave_tile_first_rows(const int *__restrict__ rowptr, int64_t n, int64_t t) {
  const int64_t i = t * WAVE + threadIdx.x % WAVE;
  const int64_t ic = i < n ? i : n - 1;
  return TileRows0{rowptr[ic], rowptr[ic + 1]};
}

template <int C, typename IT, typename VT, typename G, typename PRE, typename EPI>
__device__ inline void wave_tiles_spmv(const int *__restrict__ rowptr, const IT *__restrict__ col,
                                       const VT *__restrict__ val, const G &gx, int64_t n, int64_t t, int64_t end,
                                       int64_t step, int *lcol, VT *lval, const PRE &pre, const EPI &epi,
                                       const TileRows0 *first = nullptr) {
  using XT = decltype(gx(0));
  constexpr bool REL = sizeof(IT) == 2;
  const int lane = threadIdx.x % WAVE;
  if (t >= end) return;
  int a, b, p0, p1, cc[C];
  VT vv[C];
  auto load_rows = [&](int64_t tt, int &ra, int &rb) {
    const int64_t i = tt * WAVE + lane;
    const int64_t ic = i < n ? i : n - 1;
    ra = rowptr[ic];
    rb = rowptr[ic + 1];
  };
  auto tile_range = [&](int64_t tt, int ra, int rb, int &q0, int &q1) {
    const int64_t r0 = tt * WAVE;
    const int last = (int)((n - r0 < WAVE ? n - r0 : WAVE) - 1);
    q0 = __builtin_amdgcn_readfirstlane(ra);
    q1 = __builtin_amdgcn_readlane(rb, last);
  };
  auto load_round = [&](int base, int q1, int (&c)[C], VT (&v)[C]) {
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int pp = base + u * WAVE + lane;
      const int pc = pp < q1 ? pp : (q1 > 0 ? q1 - 1 : 0);
      c[u] = col[(unsigned)pc];
      v[u] = val[(unsigned)pc];
    }
  };
  auto stage = [&](int base, int q0, int q1, const int (&c)[C], const VT (&v)[C]) {
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int pp = base + u * WAVE + lane;
      if (pp < q1) {
        lcol[pp - q0] = c[u];
        lval[pp - q0] = v[u];
      }
    }
  };
  if (first) {
    a = first->a;
    b = first->b;
  } else {
    load_rows(t, a, b);
  }
  tile_range(t, a, b, p0, p1);
  load_round(p0, p1, cc, vv);
  for (;;) {
    const int64_t i = t * WAVE + lane;
    const int64_t ic = i < n ? i : n - 1;
    const int64_t tn = t + step;
    const bool more = tn < end;
    int an, bn;
    load_rows(more ? tn : t, an, bn);
    // the row pointers go out ahead of this tile's remaining loads
    __builtin_amdgcn_sched_barrier(0);
    const bool staged = p1 - p0 <= WT_CAP;
    if (staged) {
      stage(p0, p0, p1, cc, vv);
      for (int base = p0 + C * WAVE; base < p1; base += C * WAVE) {
        int c2[C];
        VT v2[C];
        load_round(base, p1, c2, v2);
        stage(base, p0, p1, c2, v2);
      }
      wave_lds_sync();
    }
    int p0n, p1n;
    tile_range(more ? tn : t, an, bn, p0n, p1n);
    load_round(p0n, p1n, cc, vv);
    const int len = i < n ? b - a : 0;
    const int off = a - p0;
    const double own = pre(ic);
    double s = 0.0;
    if (staged) {
      for (int k0 = 0; __any(k0 < len); k0 += C) {
        int c[C];
        VT v[C];
        XT x[C];
#pragma unroll
        for (int u = 0; u < C; ++u) {
          const int k = k0 + u;
          const int idx = k < len ? off + k : 0;
          c[u] = k < len ? (REL ? (int)ic + lcol[idx] : lcol[idx]) : (int)ic;
          v[u] = lval[idx];
        }
#pragma unroll
        for (int u = 0; u < C; ++u) x[u] = gx(c[u]);
#pragma unroll
        for (int u = 0; u < C; ++u)
          if (k0 + u < len) s += __dmul_rn((double)v[u], (double)x[u]);
      }
      wave_lds_sync();  // the slices are rewritten by the wave's next tile
    } else {
      for (int pp = a; pp < a + len; ++pp)
        s += __dmul_rn((double)val[pp], (double)gx(REL ? (int)ic + (int)col[pp] : (int)col[pp]));
    }
    if (i < n) epi(i, own, s);
    if (!more) break;
    t = tn;
    a = an;
    b = bn;
    p0 = p0n;
    p1 = p1n;
  }
}

// The wave tiles of a launch in an XCD-aware order.  Blocks are dispatched to the dies
// round robin by block index, so blocks with equal blockIdx.x % 8 share an L2; each
// such group takes one contiguous eighth of the tiles (a stencil's neighbour rows are
// then mostly in the same L2) and its waves take those tiles round robin.  The grid is
// a multiple of 8 blocks, or fewer than 8 (one group).
struct WaveTiles {
  int64_t t, end, step;
};
__device__ inline WaveTiles wave_tiles(int64_t n) {
  const int nw = blockDim.x / WAVE, wid = threadIdx.x / WAVE;
  const int64_t T = (n + WAVE - 1) / WAVE;
  const int groups = gridDim.x >= NXCD ? NXCD : 1;
  const int g = blockIdx.x % groups;
  const int64_t per = (T + groups - 1) / groups;
  const int64_t lo = g * per;
  const int64_t hi = lo + per < T ? lo + per : T;
  const int64_t idx = (int64_t)(blockIdx.x / groups) * nw + wid;
  return WaveTiles{lo + idx, hi, (int64_t)(gridDim.x / groups) * nw};
}

// grid of a wave-tile launch: enough blocks of `threads` for one tile per wave, at most
// maxblk, rounded to a multiple of NXCD once it reaches NXCD
inline int wave_tile_blocks(int64_t n, int threads, int maxblk) {
  const int64_t T = (n + WAVE - 1) / WAVE;
  const int64_t nw = threads / WAVE;
  int64_t b = (T + nw - 1) / nw;
  if (b > maxblk) b = maxblk;
  if (b < 1) b = 1;
  if (b >= NXCD) b = (b + NXCD - 1) / NXCD * NXCD;
  if (b > maxblk) b = maxblk / NXCD * NXCD;
  return (int)b;
}

// gathers per lane and round of a wave tile (5, 7 or 9): the matrix's average row
// length rounded up, so that one round covers an average tile
inline int wave_tile_chunk(int64_t n, int64_t nnz) {
  const int64_t c = n > 0 ? (nnz + n - 1) / n : 1;
  return c <= 5 ? 5 : (c <= 7 ? 7 : 9);
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

enum : uint64_t { STREAM_GAUSS_SKETCH = 1, STREAM_SRHT_SIGNS = 2, STREAM_SRHT_ROWS = 3, STREAM_RANGE_Z = 4 };

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

// The bit words srht_sign draws from, word w = bits of entries 64 w .. 64 w + 63 (bit set:
// sign -1); a sequence stores them once, so a push reads one word per 64 entries instead
// of evaluating the generator.
__device__ inline unsigned long long srht_sign_word(uint64_t w, uint64_t seed) {
  return philox4x64(w >> 2, 0, STREAM_SRHT_SIGNS, 0, seed, 0).v[w & 3];
}
__device__ inline bool srht_negative(const unsigned long long *words, uint64_t j) {
  return ((words[j >> 6] >> (j & 63)) & 1ull) != 0;
}

}  // namespace sacc
