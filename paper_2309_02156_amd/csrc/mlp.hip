// Learned coefficient predictor: MLP forward, backward and Adam kernels, and the
// device side of the learned initial guess (not in arXiv 2309.02156; it predicts the
// coefficients of the next solution in the history basis of Alg. 1 and is kept only
// when its residual is below the projection's).
//
// Numerics: weights are float32 masters used in bfloat16; every matrix product takes
// bf16-rounded operands (round to nearest, ties to even) and accumulates in float32;
// biases, activations (SiLU), the loss and Adam are float32.
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace sacc {

__device__ inline float bf16r(float x) {
  if (isnan(x)) return x;
  const unsigned u = __float_as_uint(x);
  const unsigned r = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(r);
}

__device__ inline float silu_f(float z) { return z / (1.0f + expf(-z)); }

__device__ inline float silu_grad_f(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

enum { EPI_FWD = 0, EPI_STORE = 1, EPI_DA = 2 };

constexpr int GT = 32;  // C tile of the small GEMM: GT x GT, 256 threads (one 16 x 16 quarter per wave)
constexpr int GTP = GT + 4;  // LDS row stride of the staged tiles (16-bit words)

typedef short mlp_s4 __attribute__((ext_vector_type(4)));
typedef float mlp_f4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_word(float x) { return (unsigned short)(__float_as_uint(bf16r(x)) >> 16); }

// C[m][n] = sum_k bf16(L(m, k)) bf16(R(k, n)), float32 accumulate, with
// L(m, k) = L[m lsm + k lsk] and R(k, n) = R[k rsk + n rsn]; epilogues:
//   EPI_FWD:   Z = C + bias[n]; Aout = act ? silu(Z) : Z  (row-major M x N)
//   EPI_STORE: Out = C
//   EPI_DA:    Out = C * silu'(Zprev)
// The block stages GT x GT tiles of L and of R (transposed) in LDS as BF16 words (the
// strides and the bounds are handled there) and each wave accumulates one 16 x 16
// quarter of the C tile with v_mfma_f32_16x16x16bf16_1k, two per staged tile.  Operand
// layout: A[i][4 kq + e] from lane i + 16 kq, B[4 kq + e][j] from lane j + 16 kq
// (e = 0..3), D[4 kq + v][j] in lane j + 16 kq, element v.  The products of two BF16
// values are exact in float32; only the order of the float32 sums differs from a plain
// loop over k.
template <int EPI>
__global__ __launch_bounds__(256) void k_mlp_gemm(int M, int N, int K, const float *L, int lsm, int lsk,
                                                  const float *R, int rsk, int rsn, const float *bias, float *Z,
                                                  float *Aout, int act, const float *Zprev, float *Out) {
  __shared__ __align__(8) unsigned short Ls[GT][GTP], Rt[GT][GTP];  // Rt[n][k]: R transposed
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  const int i16 = lane % 16, kq = lane / 16;
  const int wm = wid / 2, wn = wid % 2;  // the wave's quarter of the C tile
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  mlp_f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += GT) {
    for (int e = threadIdx.x; e < GT * GT; e += 256) {
      const int r = e / GT, c = e % GT;
      const int m = m0 + r, kk = k0 + c;
      Ls[r][c] = (m < M && kk < K) ? bf16_word(L[(size_t)m * lsm + (size_t)kk * lsk]) : (unsigned short)0;
      const int kr = k0 + r, n = n0 + c;
      Rt[c][r] = (kr < K && n < N) ? bf16_word(R[(size_t)kr * rsk + (size_t)n * rsn]) : (unsigned short)0;
    }
    __syncthreads();
#pragma unroll
    for (int kh = 0; kh < GT; kh += 16) {
      const mlp_s4 a = *(const mlp_s4 *)&Ls[wm * 16 + i16][kh + 4 * kq];
      const mlp_s4 b = *(const mlp_s4 *)&Rt[wn * 16 + i16][kh + 4 * kq];
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = m0 + wm * 16 + 4 * kq + v, n = n0 + wn * 16 + i16;
    if (m >= M || n >= N) continue;
    const size_t o = (size_t)m * N + n;
    if (EPI == EPI_FWD) {
      const float z = acc[v] + bias[n];
      Z[o] = z;
      Aout[o] = act ? silu_f(z) : z;
    } else if (EPI == EPI_STORE) {
      Out[o] = acc[v];
    } else {
      Out[o] = acc[v] * silu_grad_f(Zprev[o]);
    }
  }
}

template <int EPI>
static void gemm(int M, int N, int K, const float *L, int lsm, int lsk, const float *R, int rsk, int rsn,
                 const float *bias, float *Z, float *Aout, int act, const float *Zprev, float *Out, hipStream_t st) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  hipLaunchKernelGGL(k_mlp_gemm<EPI>, grid, dim3(256), 0, st, M, N, K, L, lsm, lsk, R, rsk, rsn, bias, Z, Aout, act,
                     Zprev, Out);
}

// standardise rows: Y[m][j] = (X[m][j] - mu[j]) / sd[j]
__global__ void k_mlp_scale(const float *X, int B, int D, const float *mu, const float *sd, float *Y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < B * D) Y[e] = (X[e] - mu[e % D]) / sd[e % D];
}

// dZ = 2 (y - t) / (B n_out), loss = mean (y - t)^2 (one block)
__global__ __launch_bounds__(256) void k_mlp_loss(const float *Y, const float *T, int count, float *dZ,
                                                  float *loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int e = threadIdx.x; e < count; e += 256) {
    const float d = Y[e] - T[e];
    dZ[e] = 2.f * d / (float)count;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / (float)count;
}

// db[n] = sum_m dZ[m][n]
__global__ void k_mlp_bias_grad(const float *dZ, int B, int N, float *db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < B; ++m) s += dZ[(size_t)m * N + n];
  db[n] = s;
}

__global__ void k_mlp_adam(float *P, const float *G, float *Mo, float *Vo, size_t count, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const float g = G[e];
  const float m = b1 * Mo[e] + (1.f - b1) * g;
  const float v = b2 * Vo[e] + (1.f - b2) * g * g;
  Mo[e] = m;
  Vo[e] = v;
  P[e] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

size_t mlp_param_count(const MlpDims &d) {
  size_t c = 0;
  for (int l = 0; l <= d.n_layers; ++l) {
    const int in = l == 0 ? d.n_in : d.n_hidden, out = l == d.n_layers ? d.n_out : d.n_hidden;
    c += (size_t)out * in + out;
  }
  return c;
}

// offsets of W_l and b_l in the parameter vector
static void layer_off(const MlpDims &d, int l, size_t *w, size_t *b, int *in, int *out) {
  size_t c = 0;
  for (int i = 0; i < l; ++i) {
    const int ii = i == 0 ? d.n_in : d.n_hidden, oo = i == d.n_layers ? d.n_out : d.n_hidden;
    c += (size_t)oo * ii + oo;
  }
  *in = l == 0 ? d.n_in : d.n_hidden;
  *out = l == d.n_layers ? d.n_out : d.n_hidden;
  *w = c;
  *b = c + (size_t)(*out) * (*in);
}

hipError_t launch_mlp_forward(const MlpDims &d, const MlpBuffers &m, int B, hipStream_t st) {
  for (int l = 0; l <= d.n_layers; ++l) {
    size_t wo, bo;
    int in, out;
    layer_off(d, l, &wo, &bo, &in, &out);
    const float *A = l == 0 ? m.xs : m.act[l - 1];
    gemm<EPI_FWD>(B, out, in, A, in, 1, m.P + wo, 1, in, m.P + bo, m.z[l], m.act[l], l < d.n_layers ? 1 : 0,
                  nullptr, nullptr, st);
  }
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const MlpDims &d, const MlpBuffers &m, int B, float *loss, hipStream_t st) {
  const int L = d.n_layers;
  const int cnt = B * d.n_out;
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, m.act[L], m.ts, cnt, m.dz[L & 1], loss);
  for (int l = L; l >= 0; --l) {
    size_t wo, bo;
    int in, out;
    layer_off(d, l, &wo, &bo, &in, &out);
    const float *dZ = m.dz[l & 1];
    const float *A = l == 0 ? m.xs : m.act[l - 1];
    // dW_l (out x in) = dZ^T A
    gemm<EPI_STORE>(out, in, B, dZ, 1, out, A, in, 1, nullptr, nullptr, nullptr, 0, nullptr, m.G + wo, st);
    hipLaunchKernelGGL(k_mlp_bias_grad, dim3((out + 127) / 128), dim3(128), 0, st, dZ, B, out, m.G + bo);
    if (l > 0)  // dZ_{l-1} (B x in) = (dZ W_l) * silu'(Z_{l-1})
      gemm<EPI_DA>(B, in, out, dZ, out, 1, m.P + wo, in, 1, nullptr, nullptr, nullptr, 0, m.z[l - 1],
                   m.dz[(l - 1) & 1], st);
  }
  return hipGetLastError();
}

hipError_t launch_mlp_adam(const MlpDims &d, const MlpBuffers &m, float lr, float b1, float b2, float eps, int t,
                           hipStream_t st) {
  const size_t cnt = mlp_param_count(d);
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, m.P, m.G, m.am, m.av, cnt, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_scale(const float *X, int B, int D, const float *mu, const float *sd, float *Y, hipStream_t st) {
  const int cnt = B * D;
  if (cnt > 0) hipLaunchKernelGGL(k_mlp_scale, dim3((cnt + 255) / 256), dim3(256), 0, st, X, B, D, mu, sd, Y);
  return hipGetLastError();
}

// ============================================================================ learned guess
// Target of one step, at the push of its solution x: the coefficients c (lag order) of
// the sketched least-squares fit of x by the history that step used, argmin over the
// basis kept by the sketched QR of ||S X c - S x||, i.e. c = T1 T1^T (S X)^T (S x) (the
// sketched basis S X T1 is orthonormal).  S x comes from the push partials (reduced
// here, read-only); SX and T1 still hold the step's history.  Written to the history
// ring of targets at position `pos` (ring of LHIST_MAX entries).  One block.
__global__ __launch_bounds__(TPB) void k_learn_target(const double *SX, int s, const double *partials, int nbx,
                                                      int cnt_old, int newest_old, int M, int pos, Ctl *ctl) {
  __shared__ double v[MAXS], u[MAXM], z[MAXM], c[MAXM];
  __shared__ double scratch[TPB];
  const int tid = threadIdx.x;
  const int ng = (s + SKETCH_RG - 1) / SKETCH_RG;
  for (int g = 0; g < ng; ++g) {
    const int r0 = g * SKETCH_RG;
    const int rc = (s - r0) < SKETCH_RG ? (s - r0) : SKETCH_RG;
    final_sum(partials + (size_t)g * nbx * SKETCH_RG, nbx, SKETCH_RG, rc, v + r0, scratch);
  }
  const double inv = 1.0 / sqrt((double)s);
  const int k = (cnt_old > 0 && !ctl->nonfinite) ? ctl->k : 0;
  // u[slot] = SX[:, slot]^T S x over the old history's slots (the ring fills slots
  // 0, 1, ... in order, so the live slots are 0 .. cnt_old - 1)
  for (int sl = tid; sl < M; sl += blockDim.x) {
    double a = 0.0;
    if (sl < cnt_old)
      for (int r = 0; r < s; ++r) a += SX[(size_t)sl * s + r] * v[r] * inv;
    u[sl] = a;
  }
  __syncthreads();
  for (int b = tid; b < MAXM; b += blockDim.x) {
    double a = 0.0;
    if (b < k)
      for (int sl = 0; sl < M; ++sl) a += ctl->T1[sl + b * MAXM] * u[sl];
    z[b] = a;
  }
  __syncthreads();
  for (int sl = tid; sl < M; sl += blockDim.x) {
    double a = 0.0;
    for (int b = 0; b < k; ++b) a += ctl->T1[sl + b * MAXM] * z[b];
    c[sl] = a;
  }
  __syncthreads();
  // lag order: lag l (0 = oldest) is slot (newest_old - cnt_old + 1 + l) mod M
  double *out = ctl->lhist + (size_t)(pos % LHIST_MAX) * MAXM;
  for (int l = tid; l < MAXM; l += blockDim.x) {
    double a = 0.0;
    if (l < cnt_old) a = c[((newest_old - cnt_old + 1 + l) % M + M) % M];
    out[l] = a;
  }
}

hipError_t launch_learn_target(const double *SX, int s, const double *partials, int nbx, int cnt_old, int newest_old,
                               int M, int pos, Ctl *ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_learn_target, dim3(1), dim3(TPB), 0, st, SX, s, partials, nbx, cnt_old, newest_old, M, pos,
                     ctl);
  return hipGetLastError();
}

// MLP input of step `pos`: the targets of steps pos - H .. pos - 1 (oldest first), each
// M coefficients in lag order, then sin t, cos t; standardised.
__global__ void k_learn_features(const Ctl *ctl, int H, int M, int pos, double t, const float *mu, const float *sd,
                                 float *xs) {
  const int D = H * M + 2;
  for (int e = threadIdx.x; e < D; e += blockDim.x) {
    double val;
    if (e < H * M) {
      const int h = e / M, l = e % M;
      const int p = pos - H + h;
      val = ctl->lhist[(size_t)(((p % LHIST_MAX) + LHIST_MAX) % LHIST_MAX) * MAXM + l];
    } else {
      val = e == H * M ? sin(t) : cos(t);
    }
    xs[e] = ((float)val - mu[e]) / sd[e];
  }
}

hipError_t launch_learn_features(const Ctl *ctl, int H, int M, int pos, double t, const float *mu, const float *sd,
                                 float *xs, hipStream_t st) {
  hipLaunchKernelGGL(k_learn_features, dim3(1), dim3(256), 0, st, ctl, H, M, pos, t, mu, sd, xs);
  return hipGetLastError();
}

// x_pred = X c with c = y * sd + mu (lag order -> ring slots), rows of X in TX
template <typename TX>
__global__ __launch_bounds__(TPB) void k_learn_xpred(const TX *X, int64_t n, int64_t ld, int cnt, int newest, int M,
                                                     const float *y, const float *mu, const float *sd, double *xp) {
  __shared__ double cs[MAXM];
  for (int l = threadIdx.x; l < MAXM; l += blockDim.x) {
    double c = 0.0;
    if (l < cnt) c = (double)y[l] * (double)sd[l] + (double)mu[l];
    cs[l] = c;
  }
  __syncthreads();
  GRID_ROWS(i, n) {
    double a = 0.0;
    for (int l = 0; l < cnt; ++l) {
      const int sl = ((newest - cnt + 1 + l) % M + M) % M;
      a += cs[l] * (double)X[(size_t)sl * ld + i];
    }
    xp[i] = a;
  }
}

template <typename TX>
hipError_t launch_learn_xpred(const TX *X, int64_t n, int64_t ld, int cnt, int newest, int M, const float *y,
                              const float *mu, const float *sd, double *xp, hipStream_t st) {
  hipLaunchKernelGGL(k_learn_xpred<TX>, dim3(stream_blocks(n)), dim3(TPB), 0, st, X, n, ld, cnt, newest, M, y, mu, sd,
                     xp);
  return hipGetLastError();
}

// partial ||b - A x0||^2 and ||b - A xp||^2 (row tiles)
template <typename VT>
__global__ __launch_bounds__(TPB) void k_learn_resid(const int *rowptr, const int *col, const VT *val,
                                                     const double *b, const double *x0, const double *xp, int64_t n,
                                                     double *partials) {
  __shared__ double red[NWAVE * 2];
  __shared__ double prod[SPMV_CAP];
  double acc[2] = {0.0, 0.0};
  for (int64_t r0 = (int64_t)blockIdx.x * TPB; r0 < n; r0 += (int64_t)gridDim.x * TPB) {
    const double a0 = tile_spmv<TPB>(rowptr, col, val, x0, n, r0, prod);
    const double ap = tile_spmv<TPB>(rowptr, col, val, xp, n, r0, prod);
    const int64_t i = r0 + threadIdx.x;
    if (i < n) {
      const double r0v = b[i] - a0, rpv = b[i] - ap;
      acc[0] += r0v * r0v;
      acc[1] += rpv * rpv;
    }
  }
  block_sum_store<2>(acc, 2, red, partials + (size_t)blockIdx.x * 2);
}

// every block: keep x_pred when its residual is strictly smaller (finite); block 0
// records the decision
__global__ __launch_bounds__(TPB) void k_learn_choose(const double *partials, int nblk, double *x0, const double *xp,
                                                      int64_t n, Ctl *ctl) {
  __shared__ double outv[2];
  __shared__ double scratch[TPB];
  final_sum(partials, nblk, 2, 2, outv, scratch);
  const bool take = isfinite(outv[1]) && outv[1] < outv[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->learned_used = take ? 1 : 0;
    if (int *hi = ctl->hinfo) ((volatile int *)hi)[4] = take ? 1 : 0;
    ctl->learned_r2[0] = outv[0];
    ctl->learned_r2[1] = outv[1];
  }
  if (!take) return;
  GRID_ROWS(i, n) x0[i] = xp[i];
}

hipError_t launch_learn_pick(const CsrView &A, const double *b, double *x0, const double *xp, double *partials,
                             Ctl *ctl, hipStream_t st) {
  const int nb = stream_blocks(A.n);
  if (A.fp32)
    hipLaunchKernelGGL(k_learn_resid<float>, dim3(nb), dim3(TPB), 0, st, A.rowptr, A.col, (const float *)A.val, b, x0,
                       xp, A.n, partials);
  else
    hipLaunchKernelGGL(k_learn_resid<double>, dim3(nb), dim3(TPB), 0, st, A.rowptr, A.col, (const double *)A.val, b,
                       x0, xp, A.n, partials);
  hipLaunchKernelGGL(k_learn_choose, dim3(nb), dim3(TPB), 0, st, partials, nb, x0, xp, A.n, ctl);
  return hipGetLastError();
}

template hipError_t launch_learn_xpred<double>(const double *, int64_t, int64_t, int, int, int, const float *,
                                               const float *, const float *, double *, hipStream_t);
template hipError_t launch_learn_xpred<float>(const float *, int64_t, int64_t, int, int, int, const float *,
                                              const float *, const float *, double *, hipStream_t);

}  // namespace sacc
