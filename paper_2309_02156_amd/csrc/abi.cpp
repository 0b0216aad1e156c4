// C-ABI of the sequence solver: sequence state, workspace carving and the per-step
// orchestration of the device kernels (Alg. 1 of arXiv 2309.02156, Section 2).
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sacc.h"
#include "kernels.h"

using namespace sacc;

// Per-kernel timing of the dominant Krylov kernels (sa_profile_enable): HIP events
// around each launch, kept only for launches that logged real work.
struct KernelProfile {
  bool on = false;
  std::vector<hipEvent_t> ev;  // two per timed launch
  std::vector<int> cls;        // record index per timed launch
  std::vector<double> bytes;   // algorithmic bytes per timed launch
  int n = 0;                   // timed launches of the current solve
  std::vector<sa_kernel_prof> rec;
};

// Learned coefficient predictor: an MLP with its parameters, Adam state, scaling of
// inputs and outputs and per-layer work buffers for up to max_batch rows (device).
struct sa_mlp {
  MlpDims d{};
  MlpBuffers b{};
  float *mu_in = nullptr, *sd_in = nullptr, *mu_out = nullptr, *sd_out = nullptr;
  float *xraw = nullptr;  // one raw output row for the learned guess
  float lr = 1e-3f, beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  int t = 0;  // Adam steps taken
  std::vector<void *> allocs;
};

struct sa_seq {
  sa_config cfg;
  bool mixed = false;  // SA_MIXED or SA_MIXED_KRYLOV: float32 operator and inner Krylov vectors, FP64 refinement
  bool x32 = false;    // SA_MIXED: history and basis stored in float32 too
  char *ws = nullptr;
  size_t ws_bytes = 0;
  void *X = nullptr, *Q1 = nullptr;  // double or float storage
  double *SX = nullptr, *partials = nullptr;
  void *kry = nullptr;               // Krylov vectors (double, or float for inner solves)
  float *r32 = nullptr, *d32 = nullptr;  // mixed: inner right-hand side and correction
  size_t q1_bytes = 0;     // bytes of the workspace region of Q1 (the packed column
                           // offsets of a mixed CG solve use it during the solve)
  long long *srht_rows = nullptr;
  unsigned long long *srht_signs = nullptr;  // SRHT sign words (one bit per row of x)
  unsigned short *sketch_bf16 = nullptr;     // SA_MIXED Gaussian sketch: BF16 normals (MFMA push)
  bool tune = true;  // the CG kernels' tile autotuner may run (not in the allocation-free solve)
  Ctl *ctl = nullptr;     // device control block (projection + outer solve)
  Ctl *ctl_in = nullptr;  // device control block of the inner solves (mixed)
  int *hbuf = nullptr;    // pinned host mirror of solver state (128 ints; from int 64 on the
                          // snapshot of the last poll: norms, then the state words)
  const Ctl *snap_ctl = nullptr;  // control block of that snapshot
  const Ctl *poll_ctl = nullptr;  // control block of the snapshot copy in flight (ev_poll)
  unsigned long long *mir[2] = {nullptr, nullptr};  // progress words of ctl and ctl_in (pinned)
  long long pushes = 0;
  long long basis_for = -1;  // Q1 holds X T1 of the history after this many pushes
  int64_t ld = 0;  // leading dimension of X, Q1 and the Krylov vectors
  double tau_s = 1e-12, tau_c = 1e-12;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_poll = nullptr;  // completion of the last snapshot copy
  hipStream_t poll_stream = nullptr;  // stream of the snapshot copy in flight
  bool sync_poll = false;  // no event: the host waits for the whole stream after a snapshot copy
  KernelProfile prof;
  sa_mlp *mlp = nullptr;  // learned guess (sa_learned_attach)
  int lhist = 0;          // targets per MLP input
  long long ltargets = 0; // targets written (one per push while attached)
  double t_now = 0.0;     // time of the next system (sa_set_time)
  // range finder (1 <= m < M): the Gaussian row each history column carries, in lag
  // order (oldest first), the stream's epoch, pushes since its draw and its next row
  std::vector<int> zrows;
  int z_epoch = 0, z_since = 0, z_drawn = 0;
  bool alive = true;
};

namespace {

constexpr size_t ALIGN = 256;
constexpr double kPodTau = 1e-14;  // POD: eigenvalues of X^T X kept above this times the largest
inline size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Host Philox4x64-10 (Salmon et al., SC'11): used for the SRHT row sample only.
void philox4x64_host(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    unsigned __int128 p0 = (unsigned __int128)M0 * c[0];
    unsigned __int128 p1 = (unsigned __int128)M1 * c[2];
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// s distinct rows of 0..n-1: partial Fisher-Yates, step i swaps i with
// i + ((word0 >> 32) * (n - i) >> 32), word0 from block (i, 0, STREAM_SRHT_ROWS, 0).
void srht_rows_host(int64_t n, int s, uint64_t seed, std::vector<long long> &out) {
  std::vector<long long> perm((size_t)n);
  for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = i;
  out.resize(s);
  for (int i = 0; i < s; ++i) {
    uint64_t c[4] = {(uint64_t)i, 0, (uint64_t)STREAM_SRHT_ROWS, 0};
    philox4x64_host(c, seed, 0);
    uint64_t hi = c[0] >> 32;
    int64_t j = i + (int64_t)((hi * (uint64_t)(n - i)) >> 32);
    long long t = perm[(size_t)i];
    perm[(size_t)i] = perm[(size_t)j];
    perm[(size_t)j] = t;
    out[i] = perm[(size_t)i];
  }
}

struct Layout {
  size_t X, SX, Q1, kry, partials, rows, signs, r32, d32, gbf16, total;
};

// the mixed mode applies its Gaussian sketch in BF16 on the matrix cores, from normals
// generated once into the workspace
inline bool bf16_sketch(const sa_config *c) {
  return c->precision == SA_MIXED && c->sketch == SA_SKETCH_GAUSSIAN;
}

int validate(const sa_config *c) {
  if (!c) return SA_EINVAL;
  if (c->n < 1 || c->n > ((int64_t)1 << 31) - 1) return SA_EINVAL;
  if (c->M < 1 || c->M > 32) return SA_EINVAL;
  if (c->s < c->M || c->s > MAXS || (int64_t)c->s * c->M > 8192) return SA_EINVAL;
  if (c->sketch != SA_SKETCH_GAUSSIAN && c->sketch != SA_SKETCH_SRHT) return SA_EINVAL;
  if (c->sketch == SA_SKETCH_SRHT && (c->n & (c->n - 1)) != 0) return SA_EINVAL;
  if (c->sketch == SA_SKETCH_SRHT && c->s > c->n) return SA_EINVAL;
  if (c->projection != SA_GALERKIN && c->projection != SA_MINRES) return SA_EINVAL;
  if (c->solver != SA_CG && c->solver != SA_GMRES) return SA_EINVAL;
  if (c->solver == SA_GMRES && (c->restart < 1 || c->restart > MAXR)) return SA_EINVAL;
  if (!(c->tol > 0.0) || c->maxit < 0) return SA_EINVAL;
  if (c->precision != SA_FP64 && c->precision != SA_MIXED && c->precision != SA_MIXED_KRYLOV) return SA_EINVAL;
  if (c->precision != SA_FP64 && (!(c->inner_tol > 0.0) || !(c->inner_tol < 1.0) || c->max_refine < 1))
    return SA_EINVAL;
  if (c->guess < SA_GUESS_PROJECTION || c->guess > SA_GUESS_PREVIOUS) return SA_EINVAL;
  if (c->m < 0 || c->m > c->M) return SA_EINVAL;
  if (c->m > 0 && c->m < c->M && (int64_t)c->s * (c->M + 2 * c->m) + (int64_t)c->m * c->m > 12288) return SA_EINVAL;
  if (c->basis != SA_BASIS_SKETCHED_QR && c->basis != SA_BASIS_POD) return SA_EINVAL;
  if (c->precond != SA_PRECOND_NONE && c->precond != SA_PRECOND_JACOBI) return SA_EINVAL;
  return SA_OK;
}

// columns of ld rows in the Krylov block: GMRES V (restart + 1 columns) and a scratch
// column, CG r, two p and q; then D^-1 with the Jacobi preconditioner
size_t krylov_columns(const sa_config *c) {
  const size_t kv = c->solver == SA_GMRES ? (size_t)(c->restart + 2) : 4;
  return kv + (c->precond == SA_PRECOND_JACOBI ? 1 : 0);
}

Layout layout(const sa_config *c) {
  Layout L;
  const size_t M = (size_t)c->M;
  const bool mixed = c->precision != SA_FP64;
  const size_t wx = c->precision == SA_MIXED ? sizeof(float) : sizeof(double);  // history / basis word
  const size_t wk = mixed ? sizeof(float) : sizeof(double);                      // Krylov word
  const size_t ld = (size_t)padded_ld(c->n);
  size_t off = 0;
  L.X = off;
  off += up(ld * M * wx);
  L.SX = off;
  off += up((size_t)c->s * M * sizeof(double));
  L.Q1 = off;
  off += up(ld * M * wx);
  L.kry = off;
  off += up(ld * krylov_columns(c) * wk);
  L.partials = off;
  off += up(partials_doubles(c->n, c->M, c->s) * sizeof(double));
  L.rows = off;
  off += up((size_t)c->s * sizeof(long long));
  L.signs = off;
  off += up((size_t)(c->n + 63) / 64 * sizeof(unsigned long long));
  L.r32 = L.d32 = 0;
  if (mixed) {
    L.r32 = off;
    off += up(ld * sizeof(float));
    L.d32 = off;
    off += up(ld * sizeof(float));
  }
  L.gbf16 = 0;
  if (bf16_sketch(c)) {
    L.gbf16 = off;
    off += up((size_t)sketch_bf16_rows(c->s) * (size_t)sketch_bf16_ld(c->n) * sizeof(unsigned short));
  }
  L.total = off;
  return L;
}

inline int hipok(hipError_t e) { return e == hipSuccess ? SA_OK : SA_EHIP; }
#define HIP_TRY(expr)                      \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return SA_EHIP;  \
  } while (0)
#define SA_TRY(expr)             \
  do {                           \
    int rc_ = (expr);            \
    if (rc_ != SA_OK) return rc_; \
  } while (0)

int check_csr(const sa_seq *q, const sa_csr *A) {
  if (!A || !A->rowptr_dev || !A->col_dev || !A->val_dev) return SA_EINVAL;
  if (A->n != q->cfg.n || A->nnz < 0) return SA_EINVAL;
  if (q->mixed && !A->val_is_fp32) return SA_EINVAL;  // the mixed mode solves A32
  return SA_OK;
}

CsrView view(const sa_csr *A) {
  CsrView v;
  v.n = A->n;
  v.nnz = A->nnz;
  v.rowptr = A->rowptr_dev;
  v.col = A->col_dev;
  v.val = A->val_dev;
  v.fp32 = A->val_is_fp32 ? 1 : 0;
  return v;
}

inline int count(const sa_seq *q) { return (int)(q->pushes < q->cfg.M ? q->pushes : q->cfg.M); }

// solver state of a control block, read after all enqueued work: one copy of the norms
// (bnorm, relres0, relres, tol) and the state words that follow them (state, iters,
// restarts, maxit, active, jend, restart, pad0); the state words land in hbuf[0..7]
static_assert(offsetof(Ctl, state) == offsetof(Ctl, bnorm) + 4 * sizeof(double), "norms then state words");
inline double *snapshot(sa_seq *q) { return (double *)(q->hbuf + 64); }
// poll = poll_enqueue (the copy, then an event) + poll_wait (the host waits for that event
// only, so work enqueued after the copy keeps the device busy meanwhile)
int poll_enqueue(sa_seq *q, Ctl *ctl, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(snapshot(q), &ctl->bnorm, 4 * sizeof(double) + 8 * sizeof(int), hipMemcpyDeviceToHost,
                         st));
  if (!q->sync_poll) HIP_TRY(hipEventRecord(q->ev_poll, st));
  q->poll_ctl = ctl;
  q->poll_stream = st;
  return SA_OK;
}
int poll_wait(sa_seq *q) {
  if (q->sync_poll)
    HIP_TRY(hipStreamSynchronize(q->poll_stream));
  else
    HIP_TRY(hipEventSynchronize(q->ev_poll));
  memcpy(q->hbuf, snapshot(q) + 4, 8 * sizeof(int));
  q->snap_ctl = q->poll_ctl;
  return SA_OK;
}
int poll(sa_seq *q, Ctl *ctl, hipStream_t st) {
  SA_TRY(poll_enqueue(q, ctl, st));
  return poll_wait(q);
}

// control block in device memory, with its progress word in pinned host memory
int init_ctl(Ctl **out, unsigned long long **mir_out, double tol, int maxit, int restart, int trust_est,
             hipStream_t st) {
  Ctl *d = nullptr;
  unsigned long long *mh = nullptr, *md = nullptr;
  if (hipHostMalloc((void **)&mh, 64, hipHostMallocDefault) != hipSuccess) return SA_EHIP;
  *mh = 0;
  if (hipHostGetDevicePointer((void **)&md, mh, 0) != hipSuccess || hipMalloc((void **)&d, sizeof(Ctl)) != hipSuccess) {
    (void)hipHostFree(mh);
    return SA_EHIP;
  }
  Ctl *h = new (std::nothrow) Ctl();
  if (!h) {
    (void)hipFree(d);
    (void)hipHostFree(mh);
    return SA_ENOMEM;
  }
  memset((void *)h, 0, sizeof(Ctl));
  h->mirror = md;
  h->hinfo = (int *)(md + 2);  // same pinned block, bytes 16..47
  h->tol = tol;
  h->maxit = maxit;
  h->restart = restart;
  h->trust_est = trust_est;
  h->newest = -1;
  h->state = ST_CONV;
  hipError_t e = hipMemcpyAsync(d, h, sizeof(Ctl), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  delete h;
  if (e != hipSuccess) {
    (void)hipFree(d);
    (void)hipHostFree(mh);
    return SA_EHIP;
  }
  *out = d;
  *mir_out = mh;
  return SA_OK;
}

// ---------------------------------------------------------------------------- Krylov host loops
// CG on control block `ctl` for A x = b from the iterate in x; final state in q->hbuf[0],
// iterations in q->hbuf[1], restarts in q->hbuf[2].
// ---- kernel timing
constexpr int PROF_LAUNCHES = 1024;

int prof_class(sa_seq *q, const std::string &name) {
  auto &rec = q->prof.rec;
  for (size_t i = 0; i < rec.size(); ++i)
    if (name == rec[i].name) return (int)i;
  sa_kernel_prof r;
  memset(&r, 0, sizeof(r));
  strncpy(r.name, name.c_str(), sizeof(r.name) - 1);
  rec.push_back(r);
  return (int)rec.size() - 1;
}

// a timing slot for the next launch, or null when timing is off or the slots are used up
const KTiming *prof_slot(sa_seq *q, const std::string &name, double bytes, KTiming *tm) {
  KernelProfile &P = q->prof;
  if (!P.on || P.n >= PROF_LAUNCHES || P.n >= WORK_LOG) return nullptr;
  const int i = P.n++;
  P.cls[i] = prof_class(q, name);
  P.bytes[i] = bytes;
  tm->e0 = P.ev[2 * i];
  tm->e1 = P.ev[2 * i + 1];
  tm->lidx = i;
  return tm;
}

int prof_begin(sa_seq *q, Ctl *ctl, hipStream_t st) {
  if (!q->prof.on) return SA_OK;
  q->prof.n = 0;
  HIP_TRY(hipMemsetAsync(ctl->work_log, 0, sizeof(ctl->work_log), st));
  return SA_OK;
}

// after the solve has completed on the stream
int prof_end(sa_seq *q, Ctl *ctl, hipStream_t st) {
  KernelProfile &P = q->prof;
  if (!P.on || P.n == 0) return SA_OK;
  std::vector<int> log(P.n);
  HIP_TRY(hipMemcpyAsync(log.data(), ctl->work_log, P.n * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < P.n; ++i) {
    if (!log[i]) continue;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, P.ev[2 * i], P.ev[2 * i + 1]));
    sa_kernel_prof &r = P.rec[P.cls[i]];
    r.launches += 1;
    r.ms += ms;
    r.bytes += P.bytes[i];
  }
  P.n = 0;
  return SA_OK;
}

inline const char *tname(size_t w) { return w == 4 ? "float" : "double"; }

// Progress of a solve as the device reports it.  The host enqueues a solve step by
// step and tags each step kernel with a serial number; the kernel writes the serial and
// what it saw (solve stopped, GMRES cycle ended, CG check pending) into the control
// block's progress word in pinned host memory.  The host keeps up to `poll` (at least
// MIR_EVERY) steps in front of the device and stops enqueueing as soon as the device reports the end of
// the solve (or of a GMRES cycle), without copies or events inside the loop.  It only
// waits on the device's own progress: once the stream is idle every kernel has run,
// and if the word still lags the state is read from the control block instead.  The
// final state of a solve is always read from the control block.
struct Progress {
  volatile unsigned long long *w;
  int serial = 0;  // last serial handed out
  void reset() {
    *w = 0ull;
    serial = 0;
  }
  int next() { return ++serial; }
};

inline Progress progress_of(sa_seq *q, Ctl *ctl) { return Progress{ctl == q->ctl ? q->mir[0] : q->mir[1]}; }

// Waits until the device has run the step with serial `target`, or reports a flag in
// `mask` (MIR_CYCLE_END counts only from serial `cycle_first` on), or the stream is idle.
int progress_wait(sa_seq *q, Ctl *ctl, const Progress &pg, int target, int cycle_first, unsigned mask,
                  hipStream_t st, int *seen, unsigned *flags) {
  // the stream is asked whether it is idle only after 50 us without news, then every
  // 50 us (the query takes the runtime's locks, which other threads launching on
  // other streams need)
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto next_check = t0 + std::chrono::microseconds(50);
  for (unsigned spin = 1;; ++spin) {
    const unsigned long long v = *pg.w;
    *seen = (int)(v >> 32);
    *flags = (unsigned)v;
    if (*seen >= target) return SA_OK;
    const unsigned f = *flags & mask & (*seen >= cycle_first ? ~0u : ~(unsigned)MIR_CYCLE_END);
    if (f) return SA_OK;
    if ((spin & 31) == 0 && clk::now() >= next_check) {
      next_check = clk::now() + std::chrono::microseconds(50);
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        SA_TRY(poll(q, ctl, st));
        const int state = q->hbuf[0];
        *seen = pg.serial;
        *flags = state == ST_RUN ? 0u : (state == ST_CHECK ? (unsigned)MIR_CHECK : (unsigned)MIR_STOPPED);
        return SA_OK;
      }
      if (e != hipErrorNotReady) return SA_EHIP;
      std::this_thread::yield();
    }
    __builtin_ia32_pause();
  }
}

// CG to the tolerance (or maxit); final state words in q->hbuf[0..7].
template <typename TV>
int run_cg(sa_seq *q, const CsrView &v, Ctl *ctl, const TV *b, TV *x, int maxit, hipStream_t st, const TV *dinv) {
  const sa_config &c = q->cfg;
  int *hs = q->hbuf;
  TV *r = (TV *)q->kry, *p2 = r + q->ld, *qq = r + 3 * q->ld;
  SA_TRY(prof_begin(q, ctl, st));
  const size_t w = sizeof(TV), wv = v.fp32 ? 4 : 8;
  const double wi = v.col16 ? 2.0 : 4.0;  // bytes per column index
  const double csr = 4.0 * (v.n + 1) + (wi + wv) * v.nnz;
  // wave-tile shape of the CG kernels: tuned on first use of this operator shape
  const int chunk = q->tune ? cg_tile_tune<TV>(v, b, x, r, q->partials, ctl, st) : cg_tile_chunk(v.n, v.nnz);
  const std::string pname = std::string("k_cg_p<") + tname(wv) + ", " + tname(w) + ", " + std::to_string(chunk) +
                            (v.col16 ? ", i16>" : ">");
  Progress pg = progress_of(q, ctl);
  pg.reset();
  const int ahead = c.poll > MIR_EVERY ? c.poll : MIR_EVERY;  // progress arrives every MIR_EVERY steps
  HIP_TRY(launch_cg_start_k<TV>(v, b, x, r, 0, q->partials, ctl, st, pg.next(), dinv, chunk));
  // every launched iteration is productive, or a no-op while a check or the end of the
  // solve is on its way to the host (at most `poll` of them each time)
  const long long cap = 2LL * maxit + 64LL * c.poll + 1024;
  for (long long launched = 0;; ++launched) {
    if (launched > cap) return SA_EHIP;
    int seen;
    unsigned fl;
    SA_TRY(progress_wait(q, ctl, pg, pg.serial - ahead, INT_MAX, MIR_STOPPED | MIR_CHECK, st, &seen, &fl));
    if (fl & MIR_STOPPED) break;
    if (fl & MIR_CHECK) {
      // the recursive residual met the tolerance: confirm with the true residual and
      // wait for the decision
      HIP_TRY(launch_cg_xfix<TV>(v, x, p2, ctl, st));
      HIP_TRY(launch_cg_start_k<TV>(v, b, x, r, 1, q->partials, ctl, st, pg.next(), dinv, chunk));
      SA_TRY(progress_wait(q, ctl, pg, pg.serial, INT_MAX, MIR_STOPPED, st, &seen, &fl));
      if (fl & MIR_STOPPED) break;
      continue;
    }
    KTiming tm;
    // gathers r and p, writes p and q
    // r and p gathered, p and q written, x read and written (the previous iteration's
    // x += alpha p)
    const KTiming *tp = prof_slot(q, pname, csr + (dinv ? 7.0 : 6.0) * w * v.n, &tm);
    HIP_TRY(launch_cg_iter<TV>(v, x, r, p2, qq, q->partials, ctl, st, tp, pg.next(), dinv, chunk));
  }
  // the last x += alpha p (no-op when the check before the stop applied it)
  HIP_TRY(launch_cg_xfix<TV>(v, x, p2, ctl, st));
  SA_TRY(poll(q, ctl, st));
  if (hs[0] == ST_MAXIT || hs[0] == ST_BREAK) {
    HIP_TRY(launch_cg_start_k<TV>(v, b, x, r, 2, q->partials, ctl, st, 0, dinv, chunk));
    SA_TRY(poll(q, ctl, st));
  }
  return prof_end(q, ctl, st);
}

// GMRES(m) to the tolerance (or maxit); final state words in q->hbuf[0..7].
template <typename TV>
int run_gmres(sa_seq *q, const CsrView &v, Ctl *ctl, const TV *b, TV *x, int maxit, hipStream_t st, const TV *dinv,
              bool defer = false) {
  const sa_config &c = q->cfg;
  TV *V = (TV *)q->kry;
  TV *T = V + (size_t)(c.restart + 1) * q->ld;
  SA_TRY(prof_begin(q, ctl, st));
  const size_t w = sizeof(TV), wv = v.fp32 ? 4 : 8;
  const double csr = 4.0 * (v.n + 1) + (4.0 + wv) * v.nnz;
  Progress pg = progress_of(q, ctl);
  pg.reset();
  const int ahead = c.poll > MIR_EVERY ? c.poll : MIR_EVERY;  // progress arrives every MIR_EVERY steps
  HIP_TRY(launch_gm_start<TV>(v, b, x, V, 0, q->partials, ctl, st));
  bool stop = false;
  bool est_end = false;  // the last cycle ended on its residual estimate
  const bool from_g = gm_norm_in_g(c.restart);  // G(m - 1) records ||w'_m||^2 (no F(m))
  // every cycle either adds an iteration or ends the solve in its first step
  for (long long cycle = 0; !stop; ++cycle) {
    if (cycle > (long long)maxit + 4) return SA_EHIP;
    const int first = pg.serial + 1;
    bool cut = false;  // the cycle ended before its last step: its last close ran in G
    for (int j = 0; j < c.restart; ++j) {
      int seen;
      unsigned fl;
      // after a cycle that ended on its estimate, the restart's decision (reported by
      // its first step) is awaited before more steps go out: most likely it ends the solve
      const int target = (est_end && j == 1) ? pg.serial : pg.serial - ahead;
      SA_TRY(progress_wait(q, ctl, pg, target, first, MIR_STOPPED | MIR_CYCLE_END, st, &seen, &fl));
      if (fl & MIR_STOPPED) {
        stop = true;
        break;
      }
      if ((fl & MIR_CYCLE_END) && seen >= first) {  // the rest of this cycle would be no-ops
        cut = true;
        est_end = (fl & MIR_EST_CONV) != 0;
        break;
      }
      if (j == 1) est_end = false;
      KTiming tm;
      const KTiming *tp = nullptr;
      if (q->prof.on) {
        // SpMV of the source column, columns 0..j-1, the finalised column and y
        const int rb = j <= 8 ? 8 : (j <= 16 ? 16 : 32);
        const double bytes = csr + ((j == 0 ? 2.0 : (double)(j + 3)) + (dinv ? 1.0 : 0.0)) * w * v.n;
        const std::string name = std::string("k_gm_f<") + tname(wv) + ", " + tname(w) + ", " + std::to_string(rb) +
                                 ", " + std::to_string(gm_f_rows_per_thread(v.n, rb)) + ">";
        tp = prof_slot(q, name, bytes, &tm);
      }
      // (the restart's first step reports in any case when the host will wait for it)
      const int serial = pg.next() | ((est_end && j == 0) ? MIR_REPORT : 0);
      HIP_TRY(launch_gm_step<TV>(v, V, T, q->ld, j, cycle > 0 ? 1 : 0, q->partials, ctl, st, tp, serial,
                                 from_g && j + 1 == c.restart, dinv));
    }
    if (stop) break;
    // a full cycle: the update closes step m - 1 itself, from G(m - 1)'s partial rows
    // (||w''_m|| from ||w'_m|| and the second-pass coefficients) or after a finalise F(m)
    if (!cut && !from_g) HIP_TRY(launch_gm_finish<TV>(v, V, T, q->ld, c.restart, q->partials, ctl, st, false));
    HIP_TRY(launch_gm_update<TV>(x, V, v.n, q->ld, c.restart, ctl, st, q->partials, !cut, from_g, dinv));
    HIP_TRY(launch_gm_start<TV>(v, b, x, V, 1, q->partials, ctl, st));
  }
  // defer: only enqueue the final read of the state (poll_wait reads it); the GMRES
  // state needs no action after it
  if (defer && !q->prof.on) return poll_enqueue(q, ctl, st);
  SA_TRY(poll(q, ctl, st));
  return prof_end(q, ctl, st);
}

// Jacobi preconditioner of the operator of a solve: D^-1 in the last Krylov column
// (null without a preconditioner)
template <typename TV>
int jacobi_setup(sa_seq *q, const CsrView &v, hipStream_t st, const TV **dinv) {
  *dinv = nullptr;
  if (q->cfg.precond != SA_PRECOND_JACOBI) return SA_OK;
  TV *d = (TV *)q->kry + (krylov_columns(&q->cfg) - 1) * (size_t)q->ld;
  HIP_TRY(launch_jacobi_dinv<TV>(v, d, st));
  *dinv = d;
  return SA_OK;
}

template <typename TV>
int run_krylov(sa_seq *q, const CsrView &v, Ctl *ctl, const TV *b, TV *x, int maxit, hipStream_t st) {
  const TV *dinv;
  SA_TRY(jacobi_setup<TV>(q, v, st, &dinv));
  return q->cfg.solver == SA_CG ? run_cg<TV>(q, v, ctl, b, x, maxit, st, dinv)
                                : run_gmres<TV>(q, v, ctl, b, x, maxit, st, dinv);
}

// read (bnorm, relres0, relres) of a control block
int read_norms(sa_seq *q, Ctl *ctl, double d[4], hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(d, &ctl->bnorm, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SA_OK;
}

int status_of(int state) {
  if (state == ST_MAXIT) return SA_NOTCONV;
  if (state == ST_BREAK) return SA_EBREAKDOWN;
  return SA_OK;
}

// The basis Q1 = X T1 of the current history: T1 from the sketched QR of the last push,
// or for POD (Alg. 2) from the eigen-decomposition of X^T X formed here.
template <typename TX>
int basis_enqueue(sa_seq *q, int cnt, hipStream_t st) {
  const sa_config &c = q->cfg;
  if (c.basis == SA_BASIS_POD) {
    int nb = 0;
    HIP_TRY(launch_gram_x<TX>((const TX *)q->X, c.n, q->ld, cnt, q->partials, &nb, st));
    HIP_TRY(launch_colsum(q->partials, nb, cnt * cnt, q->ctl, st));
    HIP_TRY(launch_pod_eig(cnt, c.m > 0 ? c.m : c.M, kPodTau, q->ctl, st));
  }
  HIP_TRY(launch_basis<TX>((const TX *)q->X, (TX *)q->Q1, c.n, q->ld, cnt, q->ctl, st));
  q->basis_for = q->pushes;
  return SA_OK;
}

// Alg. 1 (basis and reduced problem) on the device: Q1 = X T1, SpMM + Gram, reduced solve,
// x0 = Q1 c.  guess_projection_begin enqueues the basis (when the history changed since
// it was formed) and the SpMM + Gram pass and describes the column sums of its partial
// rows and the reduced solve in *job (the caller launches them alone or batched with
// other sequences'); guess_projection_finish enqueues x0.
template <typename TX>
int guess_projection_begin(sa_seq *q, const CsrView &v, const double *b, int cnt, hipStream_t st, SolveJob *job) {
  const sa_config &c = q->cfg;
  int nblk = 0;
  if (q->basis_for != q->pushes) SA_TRY(basis_enqueue<TX>(q, cnt, st));
  const int mr = c.projection == SA_MINRES ? 1 : 0;
  HIP_TRY(launch_spmm_gram<TX>(v, (const TX *)q->Q1, q->ld, b, cnt, mr, q->partials, &nblk, q->ctl, st));
  job->partials = q->partials;
  job->nblk = nblk;
  job->W = gram_width(cnt, mr);
  job->cnt = cnt;
  job->minres = mr;
  job->spd = c.solver == SA_CG ? 1 : 0;
  job->tau_c = q->tau_c;
  job->ctl = q->ctl;
  return SA_OK;
}

template <typename TX>
int guess_projection_finish(sa_seq *q, double *x0, hipStream_t st) {
  HIP_TRY(launch_x0<TX>((const TX *)q->Q1, (const TX *)q->X, x0, q->cfg.n, q->ld, q->ctl, st));
  return SA_OK;
}

// Learned guess on top of the projection: MLP input from the last lhist targets and
// the time, prediction x_pred = X c, kept instead of the projection's x0 when its
// residual is smaller.  The Krylov vectors' memory serves as scratch for x_pred.
int guess_learned(sa_seq *q, const CsrView &v, const double *b, double *x0, int cnt, hipStream_t st) {
  const sa_config &c = q->cfg;
  sa_mlp *m = q->mlp;
  const int newest = (int)((q->pushes - 1) % c.M);
  double *xp = (double *)q->kry;
  HIP_TRY(launch_learn_features(q->ctl, q->lhist, c.M, (int)q->ltargets, q->t_now, m->mu_in, m->sd_in, m->b.xs, st));
  HIP_TRY(launch_mlp_forward(m->d, m->b, 1, st));
  const float *y = m->b.act[m->d.n_layers];
  if (q->x32)
    HIP_TRY(launch_learn_xpred<float>((const float *)q->X, c.n, q->ld, cnt, newest, c.M, y, m->mu_out, m->sd_out, xp,
                                      st));
  else
    HIP_TRY(launch_learn_xpred<double>((const double *)q->X, c.n, q->ld, cnt, newest, c.M, y, m->mu_out, m->sd_out,
                                       xp, st));
  HIP_TRY(launch_learn_pick(v, b, x0, xp, q->partials, q->ctl, st));
  return SA_OK;
}

}  // namespace

extern "C" {

int sa_workspace_bytes(const sa_config *cfg, size_t *bytes) {
  int rc = validate(cfg);
  if (rc != SA_OK) return rc;
  if (!bytes) return SA_EINVAL;
  *bytes = layout(cfg).total;
  return SA_OK;
}

int sa_init_sequence(const sa_config *cfg, void *dev_ws, size_t ws_bytes, void *stream, sa_seq **out) {
  int rc = validate(cfg);
  if (rc != SA_OK) return rc;
  if (!out || !dev_ws || ((uintptr_t)dev_ws % ALIGN) != 0) return SA_EINVAL;
  Layout L = layout(cfg);
  if (ws_bytes < L.total) return SA_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  sa_seq *q = new (std::nothrow) sa_seq();
  if (!q) return SA_ENOMEM;
  q->cfg = *cfg;
  q->mixed = cfg->precision != SA_FP64;
  q->x32 = cfg->precision == SA_MIXED;
  if (q->cfg.poll <= 0) q->cfg.poll = 8;
  q->tau_s = cfg->rank_tol_sketch > 0.0 ? cfg->rank_tol_sketch : 1e-12;
  q->tau_c = cfg->rank_tol_chol > 0.0 ? cfg->rank_tol_chol : 1e-12;
  q->ws = (char *)dev_ws;
  q->ws_bytes = ws_bytes;
  q->ld = padded_ld(cfg->n);
  q->X = q->ws + L.X;
  q->SX = (double *)(q->ws + L.SX);
  q->Q1 = q->ws + L.Q1;
  q->q1_bytes = L.kry - L.Q1;
  q->kry = q->ws + L.kry;
  q->partials = (double *)(q->ws + L.partials);
  q->srht_rows = (long long *)(q->ws + L.rows);
  q->srht_signs = (unsigned long long *)(q->ws + L.signs);
  if (q->mixed) {
    q->r32 = (float *)(q->ws + L.r32);
    q->d32 = (float *)(q->ws + L.d32);
  }
  if (bf16_sketch(cfg)) q->sketch_bf16 = (unsigned short *)(q->ws + L.gbf16);
  bool ok = hipHostMalloc((void **)&q->hbuf, 128 * sizeof(int), hipHostMallocDefault) == hipSuccess;
  for (int e = 0; ok && e < 4; ++e) ok = hipEventCreate(&q->ev[e]) == hipSuccess;
  if (ok) ok = hipEventCreateWithFlags(&q->ev_poll, hipEventDisableTiming) == hipSuccess;
  if (ok) ok = init_ctl(&q->ctl, &q->mir[0], cfg->tol, cfg->maxit, cfg->restart, 0, st) == SA_OK;
  if (ok && q->mixed)
    ok = init_ctl(&q->ctl_in, &q->mir[1], cfg->inner_tol, cfg->maxit, cfg->restart, 1, st) == SA_OK;
  if (!ok) {
    sa_destroy_sequence(q);
    return SA_EHIP;
  }
  std::vector<long long> rows;
  if (cfg->sketch == SA_SKETCH_SRHT) srht_rows_host(cfg->n, cfg->s, cfg->seed, rows);
  hipError_t e = hipSuccess;
  if (!rows.empty())
    e = hipMemcpyAsync(q->srht_rows, rows.data(), rows.size() * sizeof(long long), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && cfg->sketch == SA_SKETCH_SRHT) e = launch_srht_signs(q->srht_signs, cfg->n, cfg->seed, st);
  if (e == hipSuccess && q->sketch_bf16) e = launch_gen_sketch_bf16(q->sketch_bf16, cfg->n, cfg->s, cfg->seed, st);
  const size_t w = q->x32 ? sizeof(float) : sizeof(double);
  if (e == hipSuccess) e = hipMemsetAsync(q->X, 0, (size_t)q->ld * cfg->M * w, st);
  if (e == hipSuccess) e = hipMemsetAsync(q->SX, 0, (size_t)cfg->s * cfg->M * sizeof(double), st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    sa_destroy_sequence(q);
    return SA_EHIP;
  }
  *out = q;
  return SA_OK;
}

}  // extern "C"

namespace {

// The range finder's rows after a push (q->pushes already counts it), in ring-slot
// order for the QR kernel (Alg. 3): while the window fills and every `refresh` pushes
// after, a new epoch gives the window's columns rows 0..cnt-1 in lag order; otherwise
// the oldest column leaves with its row and the new column takes the epoch's next row.
ZRows zrows_push(sa_seq *q) {
  const sa_config &c = q->cfg;
  ZRows z;
  memset(&z, 0, sizeof(z));
  if (!(c.m > 0 && c.m < c.M) || c.basis != SA_BASIS_SKETCHED_QR) return z;
  const int cnt = count(q);
  const int refresh = c.refresh > 0 ? c.refresh : 50;
  auto scratch = [&](int k) {
    q->z_epoch += 1;
    q->zrows.resize(k);
    for (int l = 0; l < k; ++l) q->zrows[l] = l;
    q->z_drawn = k;
    q->z_since = 0;
  };
  if ((int)q->zrows.size() < c.M) {
    scratch((int)q->zrows.size() + 1);
  } else {
    q->zrows.erase(q->zrows.begin());
    q->z_since += 1;
    if (q->z_since >= refresh) {
      scratch(c.M);
    } else {
      q->zrows.push_back(q->z_drawn);
      q->z_drawn += 1;
    }
  }
  for (int l = 0; l < cnt; ++l) z.row[(q->pushes - cnt + l) % c.M] = q->zrows[l];
  z.m = c.m;
  z.epoch = (unsigned)q->z_epoch;
  return z;
}

// push x into the history; zero_rhs: push zero if the last solve ended with b = 0
// A push up to its sketched QR, which it describes in *job (launched alone by
// push_enqueue, or batched with other sequences' by the segmented batch step)
int push_begin(sa_seq *q, const void *x_dev, int zero_rhs, hipStream_t st, QrcpJob *job) {
  const sa_config &c = q->cfg;
  const int slot = (int)(q->pushes % c.M);
  if (q->sketch_bf16)
    HIP_TRY(launch_push_bf16<float>((const double *)x_dev, (float *)q->X, q->sketch_bf16, q->SX, c.n, q->ld, slot,
                                    c.s, q->partials, q->ctl, zero_rhs, st));
  else if (q->x32)
    HIP_TRY(launch_push<float>((const double *)x_dev, (float *)q->X, q->SX, c.n, q->ld, slot, c.s, c.sketch, c.seed,
                               q->srht_rows, q->srht_signs, q->partials, q->ctl, zero_rhs, st));
  else
    HIP_TRY(launch_push<double>((const double *)x_dev, (double *)q->X, q->SX, c.n, q->ld, slot, c.s, c.sketch,
                                c.seed, q->srht_rows, q->srht_signs, q->partials, q->ctl, zero_rhs, st));
  if (q->mlp) {
    // target of the step whose solution this is: its sketched least-squares
    // coordinates in that step's history (before this push changes SX and T1)
    const int cnt_old = count(q);
    const int newest_old = cnt_old > 0 ? (int)((q->pushes - 1) % c.M) : -1;
    HIP_TRY(launch_learn_target(q->SX, c.s, q->partials, push_blocks_x(c.n, c.s), cnt_old, newest_old, c.M,
                                (int)(q->ltargets % LHIST_MAX), q->ctl, st));
    q->ltargets += 1;
  }
  q->pushes += 1;
  job->SX = q->SX;
  job->s = c.s;
  job->cnt = count(q);
  job->newest = slot;
  job->tau = q->tau_s;
  job->partials = q->partials;
  job->nbx = push_blocks_x(c.n, c.s);
  job->ctl = q->ctl;
  job->zr = zrows_push(q);
  job->seed = c.seed;
  return SA_OK;
}

int push_enqueue(sa_seq *q, const void *x_dev, int zero_rhs, hipStream_t st) {
  QrcpJob j;
  SA_TRY(push_begin(q, x_dev, zero_rhs, st, &j));
  HIP_TRY(launch_qrcp(j.SX, j.s, j.cnt, j.newest, j.tau, j.partials, q->cfg.n, j.ctl, j.zr, j.seed, st));
  return SA_OK;
}

}  // namespace

extern "C" {

int sa_push_solution(sa_seq *q, const void *x_dev, void *stream) {
  if (!q || !q->alive) return SA_ESTATE;
  if (!x_dev) return SA_EINVAL;
  return push_enqueue(q, x_dev, 0, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Enqueues the initial guess of the next step into x0; with `want_info` also its timing
// events (the reduced solve and the learned choice write their ranks and decision into
// the pinned guess record, read by guess_info after the stream has passed them).
// *cnt = history columns used.  guess_begin enqueues it up to the SpMM + Gram pass of a
// projection guess (then *deferred = true and *job describes the column sums and the
// reduced solve, which the caller launches alone or batched), guess_finish the rest
// (x0 unless the caller has launched it, the learned choice, the closing event).
int guess_begin(sa_seq *q, const sa_csr *A, const void *b_dev, void *x0_dev, bool want_info, hipStream_t st,
                int *cnt_out, SolveJob *job, bool *deferred) {
  *deferred = false;
  int rc = check_csr(q, A);
  if (rc != SA_OK) return rc;
  if (!b_dev || !x0_dev) return SA_EINVAL;
  const sa_config &c = q->cfg;
  const int cnt = count(q);
  *cnt_out = cnt;
  const size_t nb = (size_t)c.n * sizeof(double);
  if (want_info) HIP_TRY(hipEventRecord(q->ev[0], st));
  const int newest = cnt > 0 ? (int)((q->pushes - 1) % c.M) : -1;
  if (cnt == 0 || c.guess == SA_GUESS_ZERO) {
    HIP_TRY(hipMemsetAsync(x0_dev, 0, nb, st));
  } else if (c.guess == SA_GUESS_PREVIOUS) {
    if (q->x32)
      HIP_TRY(launch_to_double<float>((const float *)q->X + (size_t)newest * q->ld, (double *)x0_dev, c.n, st));
    else
      HIP_TRY(hipMemcpyAsync(x0_dev, (const double *)q->X + (size_t)newest * q->ld, nb, hipMemcpyDeviceToDevice,
                             st));
  } else {
    CsrView v = view(A);
    if (q->x32)
      SA_TRY(guess_projection_begin<float>(q, v, (const double *)b_dev, cnt, st, job));
    else
      SA_TRY(guess_projection_begin<double>(q, v, (const double *)b_dev, cnt, st, job));
    *deferred = true;
  }
  return SA_OK;
}

int guess_finish(sa_seq *q, const sa_csr *A, const void *b_dev, void *x0_dev, bool want_info, hipStream_t st,
                 int cnt, bool x0_done) {
  const sa_config &c = q->cfg;
  if (cnt > 0 && c.guess == SA_GUESS_PROJECTION) {
    if (!x0_done) {
      if (q->x32)
        SA_TRY(guess_projection_finish<float>(q, (double *)x0_dev, st));
      else
        SA_TRY(guess_projection_finish<double>(q, (double *)x0_dev, st));
    }
    if (q->mlp && q->ltargets >= q->lhist)
      SA_TRY(guess_learned(q, view(A), (const double *)b_dev, (double *)x0_dev, cnt, st));
  }
  if (want_info) HIP_TRY(hipEventRecord(q->ev[1], st));
  return SA_OK;
}

int guess_enqueue(sa_seq *q, const sa_csr *A, const void *b_dev, void *x0_dev, bool want_info, hipStream_t st,
                  int *cnt_out) {
  SolveJob job;
  bool deferred = false;
  SA_TRY(guess_begin(q, A, b_dev, x0_dev, want_info, st, cnt_out, &job, &deferred));
  if (deferred) {
    HIP_TRY(launch_colsum(job.partials, job.nblk, job.W, job.ctl, st));
    HIP_TRY(launch_small_solve(job.cnt, job.minres, job.spd, job.tau_c, job.ctl, st));
  }
  return guess_finish(q, A, b_dev, x0_dev, want_info, st, *cnt_out, false);
}

// After a step's push: the next projection guess's basis Q1 = X T1 depends on the history
// only, so it is enqueued at once (it runs while the host returns and prepares the next
// system); guess_projection_begin then skips it.
int basis_ahead(sa_seq *q, hipStream_t st) {
  const int cnt = count(q);
  if (cnt == 0 || q->cfg.guess != SA_GUESS_PROJECTION) return SA_OK;
  return q->x32 ? basis_enqueue<float>(q, cnt, st) : basis_enqueue<double>(q, cnt, st);
}

// the guess fields of info, after the stream has synchronized past guess_enqueue
// (timed: ms_guess from the guess's events; otherwise the caller fills it)
int guess_info(sa_seq *q, int cnt, sa_info *info, bool timed = true) {
  const sa_config &c = q->cfg;
  float ms = 0.f;
  if (timed) HIP_TRY(hipEventElapsedTime(&ms, q->ev[0], q->ev[1]));
  const bool proj = cnt > 0 && c.guess == SA_GUESS_PROJECTION;
  const volatile int *rec = (const volatile int *)(q->mir[0] + 2);  // the pinned guess record
  info->k_sketch = proj ? rec[0] : 0;
  info->k_eff = proj ? rec[1] : 0;
  info->used_fallback = proj ? rec[2] : 0;
  info->history = cnt;
  info->used_learned = (q->mlp && proj && q->ltargets >= q->lhist) ? rec[4] : 0;
  info->ms_guess = ms;
  return SA_OK;
}

}  // namespace

extern "C" {

int sa_initial_guess(sa_seq *q, const sa_csr *A, const void *b_dev, void *x0_dev, sa_info *info, void *stream) {
  if (!q || !q->alive) return SA_ESTATE;
  hipStream_t st = (hipStream_t)stream;
  int cnt = 0;
  SA_TRY(guess_enqueue(q, A, b_dev, x0_dev, info != nullptr, st, &cnt));
  if (info) {
    HIP_TRY(hipStreamSynchronize(st));
    SA_TRY(guess_info(q, cnt, info));
  }
  return SA_OK;
}

// Mixed mode: FP64 iterative refinement around FP32-stored inner solves of A32 d = r.
// iterations of one inner solve: inner_maxit, or by default 10 GMRES cycles / 1000 CG
// iterations (float32 storage may keep the inner residual from ever reaching inner_tol)
static int inner_cap(const sa_config &c) {
  if (c.inner_maxit > 0) return c.inner_maxit;
  return c.solver == SA_GMRES ? 10 * c.restart : 1000;
}

// Mixed CG: the inner solves' kernels read the matrix's column indices as 16-bit offsets
// from the row (half the index bytes of the bandwidth-bound SpMV) when every offset fits;
// packed once per solve into the workspace region of the basis Q1 (free from the guess's
// last use of Q1 to the next basis, which the next guess then recomputes), the fit
// reported with the first residual's poll.  Matrices with more than q1_bytes / 2
// nonzeros keep the 32-bit indices; SACC_NO_COL16 turns the packing off.
static int col16_prepare(sa_seq *q, const CsrView &v, hipStream_t st) {
  const bool want = q->cfg.solver == SA_CG && v.nnz > 0 && (size_t)v.nnz * sizeof(short) <= q->q1_bytes &&
                    !getenv("SACC_NO_COL16");
  HIP_TRY(launch_set_int(&q->ctl->col16_ok, want ? 1 : 0, st));
  if (want) {
    HIP_TRY(launch_col_rel16(v, (short *)q->Q1, &q->ctl->col16_ok, st));
    q->basis_for = -1;  // Q1's space holds the offsets now
  }
  return SA_OK;
}

static int solve_mixed(sa_seq *q, const CsrView &v, const double *b, double *x, int *iters, int *restarts,
                       int *sweeps, hipStream_t st) {
  const sa_config &c = q->cfg;
  int *hs = q->hbuf;
  *iters = *restarts = *sweeps = 0;
  SA_TRY(col16_prepare(q, v, st));
  CsrView vi = v;  // the inner solves' view
  for (int sweep = 0;; ++sweep) {
    HIP_TRY(launch_ir_resid(v, b, x, q->r32, q->partials, sweep, c.max_refine, q->ctl, st));
    SA_TRY(poll(q, q->ctl, st));
    if (sweep == 0 && hs[7] == 1) vi.col16 = (const short *)q->Q1;
    const int outer = hs[0];
    if (outer < ST_RUN || outer > ST_ZERO_RHS) return SA_EHIP;
    if (outer != ST_RUN || *iters >= c.maxit) {
      if (outer == ST_RUN) {  // iteration budget spent: report as not converged
        HIP_TRY(launch_set_int(&q->ctl->state, ST_MAXIT, st));
        HIP_TRY(hipStreamSynchronize(st));
        hs[0] = ST_MAXIT;
      }
      break;
    }
    // inner solve from d = 0 with the remaining iteration budget, at most inner_maxit
    hs[40] = c.maxit - *iters < inner_cap(c) ? c.maxit - *iters : inner_cap(c);
    HIP_TRY(launch_set_int(&q->ctl_in->maxit, hs[40], st));
    HIP_TRY(hipMemsetAsync(q->d32, 0, (size_t)c.n * sizeof(float), st));
    SA_TRY(run_krylov<float>(q, vi, q->ctl_in, q->r32, q->d32, hs[40], st));
    const int inner_state = hs[0];
    *iters += hs[1];
    *restarts += hs[2];
    if (inner_state == ST_BREAK) {
      hs[0] = ST_BREAK;
      return SA_OK;
    }
    HIP_TRY(launch_ir_update(x, q->d32, c.n, st));
    *sweeps = sweep + 1;
  }
  return SA_OK;
}

int sa_solve(sa_seq *q, const sa_csr *A, const void *b_dev, void *x_dev, sa_info *info, void *stream) {
  if (!q || !q->alive) return SA_ESTATE;
  int rc = check_csr(q, A);
  if (rc != SA_OK) return rc;
  if (!b_dev || !x_dev) return SA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const sa_config &c = q->cfg;
  const int64_t n = c.n;
  CsrView v = view(A);
  const double *b = (const double *)b_dev;
  double *x = (double *)x_dev;
  if (info) HIP_TRY(hipEventRecord(q->ev[2], st));
  int *hs = q->hbuf;
  q->snap_ctl = nullptr;
  int iters = 0, restarts = 0, sweeps = 0;
  if (q->mixed) {
    SA_TRY(solve_mixed(q, v, b, x, &iters, &restarts, &sweeps, st));
  } else {
    SA_TRY(run_krylov<double>(q, v, q->ctl, b, x, c.maxit, st));
    iters = hs[1];
    restarts = hs[2];
  }
  const int state = hs[0];
  if (state < ST_RUN || state > ST_ZERO_RHS) return SA_EHIP;
  if (state == ST_ZERO_RHS) HIP_TRY(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
  const int ret = status_of(state);
  if (info) {
    HIP_TRY(hipEventRecord(q->ev[3], st));
    double d[4];  // bnorm, relres0, relres, tol
    if (q->snap_ctl == q->ctl) {
      // the solve ended with a poll of this control block: its norms are final
      memcpy(d, snapshot(q), sizeof(d));
      HIP_TRY(hipEventSynchronize(q->ev[3]));
    } else {
      SA_TRY(read_norms(q, q->ctl, d, st));
    }
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, q->ev[2], q->ev[3]));
    info->iters = iters;
    info->restarts = restarts;
    info->refinements = sweeps;
    info->relres0 = d[1];
    info->relres = state == ST_ZERO_RHS ? 0.0 : d[2];
    info->status = ret;
    info->ms_solve = ms;
  }
  return ret;
}

int sa_step(sa_seq *q, const sa_csr *A, const void *b_dev, void *x_dev, sa_info *info, void *stream) {
  if (!q || !q->alive) return SA_ESTATE;
  hipStream_t st = (hipStream_t)stream;
  const sa_config &c = q->cfg;
  int cnt = 0;
  SA_TRY(guess_enqueue(q, A, b_dev, x_dev, info != nullptr, st, &cnt));
  if (q->mixed || c.solver != SA_GMRES || q->prof.on) {
    // with info the solve returns with the stream synchronized, past the guess
    const int rs = sa_solve(q, A, b_dev, x_dev, info, st);
    if (rs != SA_OK && rs != SA_NOTCONV && rs != SA_EBREAKDOWN) return rs;
    if (info) SA_TRY(guess_info(q, cnt, info));
    SA_TRY(push_enqueue(q, x_dev, 0, st));
    SA_TRY(basis_ahead(q, st));
    return rs;
  }
  // GMRES: the solve, the read of its final state and the push are all enqueued before
  // the host waits, for the read only, so the push runs while the host takes the result
  // and enqueues the next step.  (A solve that ended with b = 0 pushes zero: its x is
  // zeroed below, after the push in stream order.)
  if (info) HIP_TRY(hipEventRecord(q->ev[2], st));
  q->snap_ctl = nullptr;
  const double *dinv;
  SA_TRY(jacobi_setup<double>(q, view(A), st, &dinv));
  SA_TRY(run_gmres<double>(q, view(A), q->ctl, (const double *)b_dev, (double *)x_dev, c.maxit, st, dinv, true));
  if (info) HIP_TRY(hipEventRecord(q->ev[3], st));
  SA_TRY(push_enqueue(q, x_dev, 1, st));
  SA_TRY(basis_ahead(q, st));
  SA_TRY(poll_wait(q));
  const int state = q->hbuf[0];
  if (state < ST_RUN || state > ST_ZERO_RHS) return SA_EHIP;
  if (state == ST_ZERO_RHS) HIP_TRY(hipMemsetAsync(x_dev, 0, (size_t)c.n * sizeof(double), st));
  const int ret = status_of(state);
  if (info) {
    HIP_TRY(hipEventSynchronize(q->ev[3]));
    double d[4];  // bnorm, relres0, relres, tol
    memcpy(d, snapshot(q), sizeof(d));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, q->ev[2], q->ev[3]));
    info->iters = q->hbuf[1];
    info->restarts = q->hbuf[2];
    info->refinements = 0;
    info->relres0 = d[1];
    info->relres = state == ST_ZERO_RHS ? 0.0 : d[2];
    info->status = ret;
    info->ms_solve = ms;
    SA_TRY(guess_info(q, cnt, info));
  }
  return ret;
}

int sa_destroy_sequence(sa_seq *q) {
  if (!q) return SA_EINVAL;
  q->alive = false;
  if (q->ctl) (void)hipFree(q->ctl);
  if (q->ctl_in) (void)hipFree(q->ctl_in);
  if (q->hbuf) (void)hipHostFree(q->hbuf);
  for (auto m : q->mir)
    if (m) (void)hipHostFree(m);
  for (int e = 0; e < 4; ++e)
    if (q->ev[e]) (void)hipEventDestroy(q->ev[e]);
  if (q->ev_poll) (void)hipEventDestroy(q->ev_poll);
  for (auto &e : q->prof.ev)
    if (e) (void)hipEventDestroy(e);
  delete q;
  return SA_OK;
}

// ---------------------------------------------------------------- learned predictor
static void mlp_free(sa_mlp *m) {
  for (void *p : m->allocs) (void)hipFree(p);
  m->allocs.clear();
}

static float *mlp_alloc(sa_mlp *m, size_t count, bool *ok) {
  void *p = nullptr;
  if (!*ok || hipMalloc(&p, count * sizeof(float)) != hipSuccess) {
    *ok = false;
    return nullptr;
  }
  m->allocs.push_back(p);
  return (float *)p;
}

int sa_mlp_create(const sa_mlp_config *cfg, const float *init_params, sa_mlp **out) {
  if (!cfg || !init_params || !out) return SA_EINVAL;
  if (cfg->n_in < 1 || cfg->n_hidden < 1 || cfg->n_out < 1 || cfg->n_layers < 0 ||
      cfg->n_layers + 1 > MLP_MAXL || cfg->max_batch < 1 || !(cfg->lr >= 0.f))
    return SA_EINVAL;
  sa_mlp *m = new (std::nothrow) sa_mlp();
  if (!m) return SA_ENOMEM;
  m->d = MlpDims{cfg->n_in, cfg->n_hidden, cfg->n_layers, cfg->n_out, cfg->max_batch};
  m->lr = cfg->lr;
  m->beta1 = cfg->beta1;
  m->beta2 = cfg->beta2;
  m->eps = cfg->eps;
  const size_t np = mlp_param_count(m->d);
  const int B = cfg->max_batch;
  const int wmax = cfg->n_hidden > cfg->n_out ? (cfg->n_hidden > cfg->n_in ? cfg->n_hidden : cfg->n_in)
                                              : (cfg->n_out > cfg->n_in ? cfg->n_out : cfg->n_in);
  bool ok = true;
  m->b.P = mlp_alloc(m, np, &ok);
  m->b.G = mlp_alloc(m, np, &ok);
  m->b.am = mlp_alloc(m, np, &ok);
  m->b.av = mlp_alloc(m, np, &ok);
  m->b.xs = mlp_alloc(m, (size_t)B * cfg->n_in, &ok);
  m->b.ts = mlp_alloc(m, (size_t)B * cfg->n_out, &ok);
  for (int l = 0; l <= cfg->n_layers; ++l) {
    const int w = l == cfg->n_layers ? cfg->n_out : cfg->n_hidden;
    m->b.z[l] = mlp_alloc(m, (size_t)B * w, &ok);
    m->b.act[l] = mlp_alloc(m, (size_t)B * w, &ok);
  }
  m->b.dz[0] = mlp_alloc(m, (size_t)B * wmax, &ok);
  m->b.dz[1] = mlp_alloc(m, (size_t)B * wmax, &ok);
  m->mu_in = mlp_alloc(m, cfg->n_in, &ok);
  m->sd_in = mlp_alloc(m, cfg->n_in, &ok);
  m->mu_out = mlp_alloc(m, cfg->n_out, &ok);
  m->sd_out = mlp_alloc(m, cfg->n_out, &ok);
  m->xraw = mlp_alloc(m, cfg->n_in, &ok);
  if (ok) {
    std::vector<float> zero(np, 0.f), one_in(cfg->n_in, 1.f), one_out(cfg->n_out, 1.f);
    ok = hipMemcpy(m->b.P, init_params, np * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->b.am, zero.data(), np * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->b.av, zero.data(), np * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->b.G, zero.data(), np * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->mu_in, zero.data(), cfg->n_in * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->sd_in, one_in.data(), cfg->n_in * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->mu_out, zero.data(), cfg->n_out * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->sd_out, one_out.data(), cfg->n_out * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) {
    mlp_free(m);
    delete m;
    return SA_EHIP;
  }
  *out = m;
  return SA_OK;
}

int sa_mlp_destroy(sa_mlp *m) {
  if (!m) return SA_EINVAL;
  mlp_free(m);
  delete m;
  return SA_OK;
}

int sa_mlp_set_scaling(sa_mlp *m, const float *mu_in, const float *sd_in, const float *mu_out, const float *sd_out) {
  if (!m || !mu_in || !sd_in || !mu_out || !sd_out) return SA_EINVAL;
  for (int j = 0; j < m->d.n_in; ++j)
    if (!(sd_in[j] > 0.f)) return SA_EINVAL;
  for (int j = 0; j < m->d.n_out; ++j)
    if (!(sd_out[j] > 0.f)) return SA_EINVAL;
  const size_t a = m->d.n_in * sizeof(float), b = m->d.n_out * sizeof(float);
  HIP_TRY(hipMemcpy(m->mu_in, mu_in, a, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->sd_in, sd_in, a, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->mu_out, mu_out, b, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->sd_out, sd_out, b, hipMemcpyHostToDevice));
  return SA_OK;
}

int sa_mlp_forward(sa_mlp *m, const float *x_dev, int batch, float *y_dev, void *stream) {
  if (!m || !x_dev || !y_dev || batch < 1 || batch > m->d.max_batch) return SA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_mlp_scale(x_dev, batch, m->d.n_in, m->mu_in, m->sd_in, m->b.xs, st));
  HIP_TRY(launch_mlp_forward(m->d, m->b, batch, st));
  HIP_TRY(hipMemcpyAsync(y_dev, m->b.act[m->d.n_layers], (size_t)batch * m->d.n_out * sizeof(float),
                         hipMemcpyDeviceToDevice, st));
  return SA_OK;
}

int sa_mlp_train_step(sa_mlp *m, const float *x_dev, const float *t_dev, int batch, float *loss_dev, void *stream) {
  if (!m || !x_dev || !t_dev || batch < 1 || batch > m->d.max_batch) return SA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_mlp_scale(x_dev, batch, m->d.n_in, m->mu_in, m->sd_in, m->b.xs, st));
  HIP_TRY(launch_mlp_scale(t_dev, batch, m->d.n_out, m->mu_out, m->sd_out, m->b.ts, st));
  HIP_TRY(launch_mlp_forward(m->d, m->b, batch, st));
  HIP_TRY(launch_mlp_backward(m->d, m->b, batch, loss_dev, st));
  m->t += 1;
  HIP_TRY(launch_mlp_adam(m->d, m->b, m->lr, m->beta1, m->beta2, m->eps, m->t, st));
  return SA_OK;
}

int sa_mlp_get(sa_mlp *m, int what, float *host, size_t count, void *stream) {
  if (!m || !host) return SA_EINVAL;
  const size_t np = mlp_param_count(m->d);
  const float *src = what == 0 ? m->b.P : what == 1 ? m->b.G : what == 2 ? m->b.am : what == 3 ? m->b.av : nullptr;
  if (!src || count < np) return SA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(host, src, np * sizeof(float), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SA_OK;
}

int sa_learned_attach(sa_seq *q, sa_mlp *m, int n_hist) {
  if (!q || !q->alive) return SA_ESTATE;
  if (!m) {
    q->mlp = nullptr;
    return SA_OK;
  }
  if (n_hist < 1 || n_hist > LHIST_MAX || m->d.n_in != n_hist * q->cfg.M + 2 || m->d.n_out != q->cfg.M ||
      q->cfg.guess != SA_GUESS_PROJECTION)
    return SA_EINVAL;
  if (q->pushes != 0) return SA_ESTATE;
  q->mlp = m;
  q->lhist = n_hist;
  q->ltargets = 0;
  return SA_OK;
}

int sa_set_time(sa_seq *q, double t) {
  if (!q || !q->alive) return SA_ESTATE;
  q->t_now = t;
  return SA_OK;
}

int sa_profile_enable(sa_seq *q, int enable) {
  if (!q || !q->alive) return SA_ESTATE;
  KernelProfile &P = q->prof;
  if (enable && P.ev.empty()) {
    P.ev.assign(2 * PROF_LAUNCHES, nullptr);
    for (auto &e : P.ev)
      if (hipEventCreate(&e) != hipSuccess) return SA_EHIP;
    P.cls.assign(PROF_LAUNCHES, 0);
    P.bytes.assign(PROF_LAUNCHES, 0.0);
  }
  P.on = enable != 0;
  P.n = 0;
  P.rec.clear();
  return SA_OK;
}

int sa_profile_read(sa_seq *q, sa_kernel_prof *out, int max, int *count) {
  if (!q || !q->alive) return SA_ESTATE;
  if (!count || max < 0 || (max > 0 && !out)) return SA_EINVAL;
  const int n = (int)q->prof.rec.size();
  *count = n;
  for (int i = 0; i < n && i < max; ++i) out[i] = q->prof.rec[i];
  return SA_OK;
}

const char *sa_status_string(int code) {
  switch (code) {
    case SA_OK: return "ok";
    case SA_NOTCONV: return "not converged within maxit";
    case SA_EINVAL: return "invalid argument";
    case SA_ENOMEM: return "workspace too small";
    case SA_EHIP: return "HIP runtime error";
    case SA_ESTATE: return "call out of order";
    case SA_EBREAKDOWN: return "breakdown";
    case SA_ETOOBIG: return "problem larger than the fixed scratch of an allocation-free call";
    default: return "unknown status";
  }
}

int sa_spmv(const sa_csr *A, const void *x_dev, void *y_dev, void *stream) {
  if (!A || !A->rowptr_dev || !A->col_dev || !A->val_dev || !x_dev || !y_dev || A->n < 0) return SA_EINVAL;
  if (A->n == 0) return SA_OK;
  return hipok(launch_spmv(view(A), (const double *)x_dev, (double *)y_dev, (hipStream_t)stream));
}

int sa_copy_state(sa_seq *q, int what, void *host_dst, size_t bytes, void *stream) {
  if (!q || !q->alive) return SA_ESTATE;
  if (!host_dst) return SA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const sa_config &c = q->cfg;
  const size_t w = q->x32 ? sizeof(float) : sizeof(double);
  if (what == 4) {  // the learned target written by the last push (M float64, lag order)
    if (!q->mlp || q->ltargets == 0) return SA_ESTATE;
    if (bytes < (size_t)c.M * sizeof(double)) return SA_EINVAL;
    HIP_TRY(hipMemcpyAsync(host_dst, q->ctl->lhist + (size_t)((q->ltargets - 1) % LHIST_MAX) * MAXM,
                           (size_t)c.M * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SA_OK;
  }
  if (what == 0 || what == 1 || what == 2) {
    size_t need = what == 0 ? (size_t)c.s * c.M * sizeof(double)
                 : what == 1 ? (size_t)c.n * c.M * w
                             : (size_t)c.M * sizeof(double);
    if (bytes < need) return SA_EINVAL;
    if (what == 1)
      HIP_TRY(hipMemcpy2DAsync(host_dst, (size_t)c.n * w, q->X, (size_t)q->ld * w, (size_t)c.n * w, (size_t)c.M,
                               hipMemcpyDeviceToHost, st));
    else
      HIP_TRY(hipMemcpyAsync(host_dst, what == 0 ? (const void *)q->SX : (const void *)q->ctl->cX, need,
                             hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SA_OK;
  }
  if (what == 3) {
    if (bytes < (size_t)c.M * sizeof(int32_t)) return SA_EINVAL;
    int32_t *o = (int32_t *)host_dst;
    const int cnt = count(q);
    for (int i = 0; i < c.M; ++i) o[i] = -1;
    for (int i = 0; i < cnt; ++i) o[i] = (int32_t)((q->pushes - cnt + i) % c.M);
    return SA_OK;
  }
  return SA_EINVAL;
}

}  // extern "C"

// ============================================================================ checkpoint / resume
// The state a sequence carries from one step to the next: the history X (n x M in ring
// slots), its sketch S X, the push count (which fixes the ring order), the sketched QR
// of the history (T1, rank, newest slot and its finiteness) and the learned predictor's
// target ring.  Everything else (Krylov vectors, partial sums, the basis Q1) is rebuilt
// by the next step, and the sketch's random entries follow from the configuration.
namespace {

constexpr uint64_t kStateMagic = 0x3130746174734153ull;  // "SAstat01"

struct StateHeader {
  uint64_t magic;
  sa_config cfg;
  int64_t pushes, ltargets;
  double t_now;
  uint64_t x_bytes, sx_bytes, ctl_bytes;
  int32_t z_epoch, z_since, z_drawn, z_count;
  int32_t zrows[MAXM];
};

// the control-block fields of the projection state, one contiguous range
constexpr size_t kCtlLo = offsetof(Ctl, k);
constexpr size_t kCtlHi = offsetof(Ctl, c);
static_assert(offsetof(Ctl, T1) > kCtlLo && offsetof(Ctl, T1) < kCtlHi, "T1 inside the saved range");

size_t state_bytes(const sa_seq *q) {
  const size_t w = q->x32 ? sizeof(float) : sizeof(double);
  return sizeof(StateHeader) + (size_t)q->cfg.n * q->cfg.M * w + (size_t)q->cfg.s * q->cfg.M * sizeof(double) +
         (kCtlHi - kCtlLo) + sizeof(((Ctl *)0)->lhist);
}

bool same_method(const sa_config &a, const sa_config &b) {
  return a.n == b.n && a.M == b.M && a.s == b.s && a.sketch == b.sketch && a.precision == b.precision &&
         a.seed == b.seed && a.m == b.m && a.refresh == b.refresh && a.basis == b.basis;
}

}  // namespace

extern "C" {

int sa_state_bytes(const sa_seq *q, size_t *bytes) {
  if (!q || !q->alive) return SA_ESTATE;
  if (!bytes) return SA_EINVAL;
  *bytes = state_bytes(q);
  return SA_OK;
}

int sa_export_state(sa_seq *q, void *host_dst, size_t bytes, void *stream) {
  if (!q || !q->alive) return SA_ESTATE;
  if (!host_dst || bytes < state_bytes(q)) return SA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const sa_config &c = q->cfg;
  const size_t w = q->x32 ? sizeof(float) : sizeof(double);
  StateHeader h;
  memset(&h, 0, sizeof(h));
  h.magic = kStateMagic;
  h.cfg = c;
  h.pushes = q->pushes;
  h.ltargets = q->ltargets;
  h.t_now = q->t_now;
  h.x_bytes = (uint64_t)c.n * c.M * w;
  h.sx_bytes = (uint64_t)c.s * c.M * sizeof(double);
  h.ctl_bytes = (uint64_t)(kCtlHi - kCtlLo) + sizeof(((Ctl *)0)->lhist);
  h.z_epoch = q->z_epoch;
  h.z_since = q->z_since;
  h.z_drawn = q->z_drawn;
  h.z_count = (int32_t)q->zrows.size();
  for (int l = 0; l < h.z_count && l < MAXM; ++l) h.zrows[l] = q->zrows[l];
  char *o = (char *)host_dst;
  memcpy(o, &h, sizeof(h));
  o += sizeof(h);
  HIP_TRY(hipMemcpy2DAsync(o, (size_t)c.n * w, q->X, (size_t)q->ld * w, (size_t)c.n * w, (size_t)c.M,
                           hipMemcpyDeviceToHost, st));
  o += h.x_bytes;
  HIP_TRY(hipMemcpyAsync(o, q->SX, h.sx_bytes, hipMemcpyDeviceToHost, st));
  o += h.sx_bytes;
  HIP_TRY(hipMemcpyAsync(o, (const char *)q->ctl + kCtlLo, kCtlHi - kCtlLo, hipMemcpyDeviceToHost, st));
  o += kCtlHi - kCtlLo;
  HIP_TRY(hipMemcpyAsync(o, q->ctl->lhist, sizeof(((Ctl *)0)->lhist), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SA_OK;
}

int sa_import_state(sa_seq *q, const void *host_src, size_t bytes, void *stream) {
  if (!q || !q->alive) return SA_ESTATE;
  if (!host_src || bytes < sizeof(StateHeader)) return SA_EINVAL;
  StateHeader h;
  memcpy(&h, host_src, sizeof(h));
  if (h.magic != kStateMagic || !same_method(h.cfg, q->cfg) || bytes < state_bytes(q) || h.pushes < 0 ||
      h.z_count < 0 || h.z_count > MAXM)
    return SA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const sa_config &c = q->cfg;
  const size_t w = q->x32 ? sizeof(float) : sizeof(double);
  const char *in = (const char *)host_src + sizeof(h);
  HIP_TRY(hipMemcpy2DAsync(q->X, (size_t)q->ld * w, in, (size_t)c.n * w, (size_t)c.n * w, (size_t)c.M,
                           hipMemcpyHostToDevice, st));
  in += h.x_bytes;
  HIP_TRY(hipMemcpyAsync(q->SX, in, h.sx_bytes, hipMemcpyHostToDevice, st));
  in += h.sx_bytes;
  HIP_TRY(hipMemcpyAsync((char *)q->ctl + kCtlLo, in, kCtlHi - kCtlLo, hipMemcpyHostToDevice, st));
  in += kCtlHi - kCtlLo;
  HIP_TRY(hipMemcpyAsync(q->ctl->lhist, in, sizeof(((Ctl *)0)->lhist), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  q->pushes = h.pushes;
  q->z_epoch = h.z_epoch;
  q->z_since = h.z_since;
  q->z_drawn = h.z_drawn;
  q->zrows.assign(h.zrows, h.zrows + h.z_count);
  q->ltargets = q->mlp ? h.ltargets : 0;
  q->t_now = h.t_now;
  q->basis_for = -1;
  return SA_OK;
}

}  // extern "C"

// ============================================================================ allocation-free solve
// sa_solve_static: the Krylov solve of sa_solve for callers that cannot allocate.  Its
// control block, partial sums and Krylov vectors live in one file-scope device array
// (each device holds its own copy for the life of the process); the host state is a
// stack object.  Without a progress word in pinned memory the host keeps `poll` steps
// in flight, waits for the stream to drain and reads the state with a copy.
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (null: not resolved)

// the device address of the current device's scratch array, resolved once per device
int scratch_base(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SA_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SA_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SA_OK;
}

struct StaticLayout {
  size_t ctl, partials, kry, total;
};

StaticLayout static_layout(const sa_config *c) {
  StaticLayout L;
  size_t off = 0;
  L.ctl = off;
  off += up(sizeof(Ctl));
  L.partials = off;
  off += up(krylov_partials_doubles() * sizeof(double));
  L.kry = off;
  off += up((size_t)padded_ld(c->n) * krylov_columns(c) * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

int sa_static_scratch_bytes(const sa_config *cfg, size_t *need, size_t *capacity) {
  int rc = validate(cfg);
  if (rc != SA_OK) return rc;
  if (!need || !capacity) return SA_EINVAL;
  *need = static_layout(cfg).total;
  *capacity = kScratchBytes;
  return SA_OK;
}

int sa_solve_static(const sa_config *cfg, const sa_csr *A, const void *b_dev, void *x_dev, sa_info *info,
                    void *stream) {
  int rc = validate(cfg);
  if (rc != SA_OK) return rc;
  if (cfg->precision != SA_FP64 || !b_dev || !x_dev) return SA_EINVAL;
  const StaticLayout L = static_layout(cfg);
  if (L.total > kScratchBytes) return SA_ETOOBIG;
  sa_seq q;  // host state on the stack
  q.cfg = *cfg;
  if (q.cfg.poll <= 0) q.cfg.poll = 8;
  rc = check_csr(&q, A);
  if (rc != SA_OK) return rc;
  void *base = nullptr;
  SA_TRY(scratch_base(&base));
  hipStream_t st = (hipStream_t)stream;
  alignas(64) int hb[128] = {0};
  unsigned long long progress = 0ull;  // never written by the device (no mirror)
  q.hbuf = hb;
  q.mir[0] = &progress;
  q.sync_poll = true;
  q.tune = false;  // the autotuner creates events
  q.ld = padded_ld(cfg->n);
  q.ctl = (Ctl *)((char *)base + L.ctl);
  q.partials = (double *)((char *)base + L.partials);
  q.kry = (char *)base + L.kry;
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(launch_ctl_reset(q.ctl, cfg->tol, cfg->maxit, cfg->restart, 0, st));
  SA_TRY(run_krylov<double>(&q, view(A), q.ctl, (const double *)b_dev, (double *)x_dev, cfg->maxit, st));
  const int state = hb[0];
  if (state < ST_RUN || state > ST_ZERO_RHS) return SA_EHIP;
  if (state == ST_ZERO_RHS) HIP_TRY(launch_zero((double *)x_dev, cfg->n, st));
  const int ret = status_of(state);
  if (info) {
    double d[4];  // bnorm, relres0, relres, tol: the last poll's snapshot of this control block
    memcpy(d, snapshot(&q), sizeof(d));
    HIP_TRY(hipStreamSynchronize(st));
    memset(info, 0, sizeof(*info));
    info->iters = hb[1];
    info->restarts = hb[2];
    info->relres0 = d[1];
    info->relres = state == ST_ZERO_RHS ? 0.0 : d[2];
    info->status = ret;
    info->ms_solve = (float)(1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  }
  q.hbuf = nullptr;  // not owned
  q.mir[0] = nullptr;
  q.ctl = nullptr;
  return ret;
}

}  // extern "C"

// ============================================================================ batches
// Batched execution of many independent sequences (the paper's Section 5 setting:
// 64 independent poloidal-plane sequences advanced together): one step of every
// sequence, spread over several HIP streams so the small per-sequence kernels of
// different sequences run concurrently, with a longest-processing-time assignment of
// sequences to streams and a plan (streams, poll batch) chosen by timing candidates
// on the first steps after the histories are full.

namespace batchplan {

// streams: host threads / streams in use; poll: Krylov steps enqueued ahead (stream
// plans); seg: the solves run in the segmented engine (the streams then carry the
// guesses and pushes up to their batched QRCP, column-sum, reduced-solve and x0
// launches); over: the engine's data grid in multiples of the resident blocks; rows:
// its work-item rows (512 or 1024)
struct Plan {
  int streams, poll, seg, over, rows;
};

// candidates the autotuner times, one step each (after the history is full); the
// segmented ones only where every sequence can use the engine
const Plan kCandidates[] = {{1, 8, 0, 0, 0},     {2, 8, 0, 0, 0},     {4, 8, 0, 0, 0},    {4, 4, 0, 0, 0},
                            {4, 16, 0, 0, 0},    {4, 30, 0, 0, 0},    {2, 16, 0, 0, 0},   {8, 8, 0, 0, 0},
                            {8, 16, 0, 0, 0},    {4, 8, 1, 8, 1024},  {8, 8, 1, 4, 1024}, {8, 8, 1, 8, 1024},
                            {8, 8, 1, 16, 1024}, {8, 8, 1, 4, 512},   {8, 8, 1, 8, 512}};
constexpr int kNumCandidates = sizeof(kCandidates) / sizeof(kCandidates[0]);

}  // namespace batchplan

using batchplan::Plan;
using batchplan::kCandidates;
using batchplan::kNumCandidates;

// The batch's host threads: one per stream beyond the caller's, created with the batch
// and kept; a step hands each of them its list through a generation counter.
struct BatchPool {
  std::vector<std::thread> th;
  std::mutex mu;
  std::condition_variable go, done;
  long long gen = 0;
  int active = 0, pending = 0;
  bool stop = false;
  std::function<void(int)> job;
};

struct sa_batch {
  std::vector<sa_seq *> seqs;
  std::vector<hipStream_t> streams;
  BatchPool pool;
  std::vector<double> cost;  // estimated cost of a sequence's step (nnz x (iterations + 10))
  Plan plan{4, 8, 0, 0, 0};
  int tune_next = 0;        // next candidate to time; kNumCandidates when tuned
  int tune_warm = 0;        // steps before timing starts (history filling)
  double tune_best = 1e300;
  Plan tune_best_plan{4, 8, 0, 0, 0};
  long long steps = 0;
  int mode = SA_BATCH_AUTO;
  bool seg_ok = false;        // every sequence is mixed-precision without a preconditioner
  SegEngine *seg = nullptr;   // the segmented engine (created with the batch when seg_ok)
  // the segmented step's batched QRCP and reduced-solve launches: per-stream events,
  // the batch stream's event, pinned staging and device copies of the jobs
  std::vector<hipEvent_t> sev;
  hipEvent_t bev = nullptr;
  SolveJob *hsolve = nullptr, *dsolve = nullptr;
  X0Job *hx0 = nullptr, *dx0 = nullptr;
  QrcpJob *hqrcp = nullptr, *dqrcp = nullptr;
  double seg_bytes = 0.0, seg_ms = 0.0;  // the last step's segmented solve (0 after a stream step)
};

namespace {

// job(s) for s in [0, nthreads) on the batch's threads (job(0) on the caller's)
void pool_run(sa_batch *b, int nthreads, const std::function<void(int)> &job) {
  BatchPool &P = b->pool;
  {
    std::lock_guard<std::mutex> lk(P.mu);
    P.job = job;
    P.active = nthreads;
    P.pending = nthreads - 1;
    P.gen += 1;
  }
  P.go.notify_all();
  job(0);
  std::unique_lock<std::mutex> lk(P.mu);
  P.done.wait(lk, [&] { return P.pending == 0; });
  P.job = nullptr;
}

void guess_into(sa_info &dst, const sa_info &g) {
  dst.k_eff = g.k_eff;
  dst.k_sketch = g.k_sketch;
  dst.used_fallback = g.used_fallback;
  dst.history = g.history;
  dst.ms_guess = g.ms_guess;
}

// One step with the solves in the segmented engine: the guesses on the plan's streams
// (each stream waits for its own), the solves of all sequences together on stream 0,
// then the pushes on the plan's streams.
int batch_step_seg(sa_batch *b, const Plan &plan, const std::vector<std::vector<int>> &lists, const sa_csr *const *A,
                   const void *const *rhs, void *const *x, std::vector<sa_info> &inf, bool graph) {
  const int nseq = (int)b->seqs.size();
  std::vector<int> rc(plan.streams, SA_OK);
  hipStream_t bs = b->streams[0];  // the batched launches' stream
  // the guesses up to their SpMM + Gram passes, every sequence of a stream's list
  // enqueued on it; then on the batch stream every sequence's column sums, reduced solve
  // and x0 in one launch each, the learned choices, one wait, and the guess records
  // (ms_guess: the whole guess phase's wall time, as ms_solve is the engine's)
  const auto tg0 = std::chrono::steady_clock::now();
  std::vector<int> cnts(nseq, 0);
  std::vector<SolveJob> sj(nseq);
  std::vector<char> deferred(nseq, 0);
  pool_run(b, plan.streams, [&](int s) {
    hipStream_t st = b->streams[s];
    int r = SA_OK;
    for (size_t k = 0; k < lists[s].size() && r == SA_OK; ++k) {
      const int i = lists[s][k];
      memset(&inf[i], 0, sizeof(sa_info));
      bool d = false;
      r = b->seqs[i]->alive ? guess_begin(b->seqs[i], A[i], rhs[i], x[i], false, st, &cnts[i], &sj[i], &d)
                            : SA_ESTATE;
      deferred[i] = d ? 1 : 0;
    }
    if (r == SA_OK) r = hipEventRecord(b->sev[s], st) == hipSuccess ? SA_OK : SA_EHIP;
    if (r != SA_OK) rc[s] = r;
  });
  for (int r : rc)
    if (r != SA_OK) return r;
  for (int s = 1; s < plan.streams; ++s) HIP_TRY(hipStreamWaitEvent(bs, b->sev[s], 0));
  {
    int nj = 0, n32 = 0, n64 = 0;
    for (int i = 0; i < nseq; ++i)
      if (deferred[i]) b->hsolve[nj++] = sj[i];
    // x0 jobs: float32 histories first, then float64 ones
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < nseq; ++i) {
        const sa_seq *q = b->seqs[i];
        if (!deferred[i] || q->x32 != (pass == 0)) continue;
        b->hx0[n32 + n64] = X0Job{q->Q1, q->X, (double *)x[i], q->cfg.n, q->ld, q->ctl};
        (pass == 0 ? n32 : n64) += 1;
      }
    if (nj > 0) {
      HIP_TRY(hipMemcpyAsync(b->dsolve, b->hsolve, nj * sizeof(SolveJob), hipMemcpyHostToDevice, bs));
      HIP_TRY(hipMemcpyAsync(b->dx0, b->hx0, nj * sizeof(X0Job), hipMemcpyHostToDevice, bs));
      HIP_TRY(launch_colsum_batch(b->dsolve, b->hsolve, nj, bs));
      HIP_TRY(launch_small_solve_batch(b->dsolve, b->hsolve, nj, bs));
      if (n32 > 0) HIP_TRY(launch_x0_batch<float>(b->dx0, b->hx0, n32, bs));
      if (n64 > 0) HIP_TRY(launch_x0_batch<double>(b->dx0 + n32, b->hx0 + n32, n64, bs));
    }
    for (int i = 0; i < nseq; ++i) SA_TRY(guess_finish(b->seqs[i], A[i], rhs[i], x[i], false, bs, cnts[i], true));
    HIP_TRY(hipStreamSynchronize(bs));
    const float gms = (float)(1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - tg0).count());
    for (int i = 0; i < nseq; ++i) {
      sa_info g;
      memset(&g, 0, sizeof(g));
      SA_TRY(guess_info(b->seqs[i], cnts[i], &g, false));
      g.ms_guess = gms;
      guess_into(inf[i], g);
    }
  }
  if (!b->seg) return SA_ESTATE;
  int64_t tn = 0, tnnz = 0;
  for (int i = 0; i < nseq; ++i) {
    tn += A[i]->n;
    tnnz += A[i]->nnz;
  }
  std::vector<SegDesc> desc(nseq);
  for (int i = 0; i < nseq; ++i) {
    const sa_seq *q = b->seqs[i];
    const sa_config &c = q->cfg;
    SegDesc &d = desc[i];
    memset(&d, 0, sizeof(d));
    d.rowptr = A[i]->rowptr_dev;
    d.col = A[i]->col_dev;
    d.val = (const float *)A[i]->val_dev;
    d.b = (const double *)rhs[i];
    d.x = (double *)x[i];
    d.kry = (float *)q->kry;
    d.r32 = q->r32;
    d.d32 = q->d32;
    d.n = c.n;
    d.ld = q->ld;
    d.nnz = A[i]->nnz;
    d.solver = c.solver;
    d.m = c.solver == SA_GMRES ? c.restart : 0;
    d.max_refine = c.max_refine;
    d.maxit = c.maxit;
    d.icap = inner_cap(c);
    d.tol = c.tol;
    d.itol = c.inner_tol;
  }
  hipStream_t st = b->streams[0];
  std::vector<SegResult> res(nseq);
  const auto t0 = std::chrono::steady_clock::now();
  if (seg_engine_solve(b->seg, desc.data(), graph, plan.over, wave_tile_chunk(tn, tnnz), plan.rows, st, res.data()) !=
      hipSuccess)
    return SA_EHIP;
  for (int i = 0; i < nseq; ++i)
    if (res[i].state == ST_ZERO_RHS) HIP_TRY(hipMemsetAsync(x[i], 0, (size_t)desc[i].n * sizeof(double), st));
  HIP_TRY(hipStreamSynchronize(st));
  const float ms = (float)(1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  b->seg_bytes = 0.0;
  for (int i = 0; i < nseq; ++i) b->seg_bytes += res[i].bytes;
  b->seg_ms = ms;
  for (int i = 0; i < nseq; ++i) {
    const SegResult &r = res[i];
    if (r.state < ST_RUN || r.state > ST_ZERO_RHS) return SA_EHIP;
    inf[i].iters = r.iters;
    inf[i].restarts = r.restarts;
    inf[i].refinements = r.sweeps;
    inf[i].relres0 = r.relres0;
    inf[i].relres = r.state == ST_ZERO_RHS ? 0.0 : r.relres;
    inf[i].status = status_of(r.state);
    inf[i].ms_solve = ms;
  }
  // the pushes up to their sketched QRs on the streams, then every QRCP in one launch
  // (the small instantiation's jobs first) and one wait
  std::vector<QrcpJob> qj(nseq);
  pool_run(b, plan.streams, [&](int s) {
    hipStream_t sp = b->streams[s];
    int r = SA_OK;
    for (size_t k = 0; k < lists[s].size() && r == SA_OK; ++k) {
      const int i = lists[s][k];
      r = b->seqs[i]->alive ? push_begin(b->seqs[i], x[i], 0, sp, &qj[i]) : SA_ESTATE;
    }
    if (r == SA_OK) r = hipEventRecord(b->sev[s], sp) == hipSuccess ? SA_OK : SA_EHIP;
    if (r != SA_OK) rc[s] = r;
  });
  for (int r : rc)
    if (r != SA_OK) return r;
  int nj = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int i = 0; i < nseq; ++i)
      if (qrcp_job_small(qj[i]) == (pass == 0)) b->hqrcp[nj++] = qj[i];
  for (int s = 1; s < plan.streams; ++s) HIP_TRY(hipStreamWaitEvent(bs, b->sev[s], 0));
  HIP_TRY(hipMemcpyAsync(b->dqrcp, b->hqrcp, nj * sizeof(QrcpJob), hipMemcpyHostToDevice, bs));
  HIP_TRY(launch_qrcp_batch(b->dqrcp, b->hqrcp, nj, bs));
  HIP_TRY(hipStreamSynchronize(bs));
  return SA_OK;
}

}  // namespace

namespace {

// the segmented step's engine and batched-launch resources (each released if present)
void batch_seg_free(sa_batch *b) {
  if (b->seg) seg_engine_destroy(b->seg);
  b->seg = nullptr;
  for (auto &e : b->sev)
    if (e) (void)hipEventDestroy(e);
  b->sev.clear();
  if (b->bev) (void)hipEventDestroy(b->bev);
  if (b->hsolve) (void)hipHostFree(b->hsolve);
  if (b->dsolve) (void)hipFree(b->dsolve);
  if (b->hx0) (void)hipHostFree(b->hx0);
  if (b->dx0) (void)hipFree(b->dx0);
  b->hx0 = b->dx0 = nullptr;
  if (b->hqrcp) (void)hipHostFree(b->hqrcp);
  if (b->dqrcp) (void)hipFree(b->dqrcp);
  b->bev = nullptr;
  b->hsolve = b->dsolve = nullptr;
  b->hqrcp = b->dqrcp = nullptr;
}

}  // namespace

extern "C" {

int sa_batch_create(sa_seq *const *seqs, int nseq, int max_streams, int tune_warmup, sa_batch **out) {
  if (!seqs || nseq < 1 || !out || max_streams < 1 || max_streams > 16 || tune_warmup < 0) return SA_EINVAL;
  for (int i = 0; i < nseq; ++i)
    if (!seqs[i]) return SA_EINVAL;
  sa_batch *b = new (std::nothrow) sa_batch();
  if (!b) return SA_ENOMEM;
  b->seqs.assign(seqs, seqs + nseq);
  b->cost.assign(nseq, 1.0);
  b->streams.resize(max_streams, nullptr);
  for (auto &s : b->streams)
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto &t : b->streams)
        if (t) (void)hipStreamDestroy(t);
      delete b;
      return SA_EHIP;
    }
  b->plan = Plan{max_streams, 8, 0, 0, 0};
  b->seg_ok = true;
  for (int i = 0; i < nseq; ++i)
    b->seg_ok = b->seg_ok && seqs[i]->mixed && seqs[i]->cfg.precond == SA_PRECOND_NONE;
  if (b->seg_ok) {
    std::vector<int64_t> ns(nseq);
    for (int i = 0; i < nseq; ++i) ns[i] = seqs[i]->cfg.n;
    bool ok = seg_engine_create(ns.data(), nseq, &b->seg) == 0;
    b->sev.assign(max_streams, nullptr);
    for (auto &e : b->sev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->bev, hipEventDisableTiming) == hipSuccess &&
         hipHostMalloc((void **)&b->hsolve, nseq * sizeof(SolveJob), hipHostMallocDefault) == hipSuccess &&
         hipMalloc((void **)&b->dsolve, nseq * sizeof(SolveJob)) == hipSuccess &&
         hipHostMalloc((void **)&b->hx0, nseq * sizeof(X0Job), hipHostMallocDefault) == hipSuccess &&
         hipMalloc((void **)&b->dx0, nseq * sizeof(X0Job)) == hipSuccess &&
         hipHostMalloc((void **)&b->hqrcp, nseq * sizeof(QrcpJob), hipHostMallocDefault) == hipSuccess &&
         hipMalloc((void **)&b->dqrcp, nseq * sizeof(QrcpJob)) == hipSuccess;
    if (!ok) {
      batch_seg_free(b);
      for (auto &t : b->streams) (void)hipStreamDestroy(t);
      delete b;
      return SA_ENOMEM;
    }
  }
  b->tune_warm = tune_warmup;
  b->tune_next = 0;
  BatchPool &P = b->pool;
  for (int s = 1; s < max_streams; ++s)
    P.th.emplace_back([&P, s] {
      long long seen = 0;
      for (;;) {
        std::unique_lock<std::mutex> lk(P.mu);
        P.go.wait(lk, [&] { return P.stop || P.gen != seen; });
        if (P.stop) return;
        seen = P.gen;
        const bool mine = s < P.active;
        lk.unlock();
        if (mine) {
          P.job(s);
          std::lock_guard<std::mutex> g(P.mu);
          if (--P.pending == 0) P.done.notify_one();
        }
      }
    });
  *out = b;
  return SA_OK;
}

int sa_batch_destroy(sa_batch *b) {
  if (!b) return SA_EINVAL;
  {
    std::lock_guard<std::mutex> lk(b->pool.mu);
    b->pool.stop = true;
  }
  b->pool.go.notify_all();
  for (auto &t : b->pool.th) t.join();
  batch_seg_free(b);
  for (auto &s : b->streams)
    if (s) (void)hipStreamDestroy(s);
  delete b;
  return SA_OK;
}

int sa_batch_plan(const sa_batch *b, int *streams, int *poll, int *tuned, int *segmented) {
  if (!b || !streams || !poll || !tuned || !segmented) return SA_EINVAL;
  *streams = b->plan.streams;
  *poll = b->plan.poll;
  *tuned = (b->mode != SA_BATCH_AUTO || b->tune_next >= kNumCandidates) ? 1 : 0;
  *segmented = b->plan.seg ? (b->plan.rows == 512 ? 512 : 1024) : 0;
  return SA_OK;
}

int sa_batch_solve_stats(const sa_batch *b, double *bytes, double *ms) {
  if (!b || !bytes || !ms) return SA_EINVAL;
  *bytes = b->seg_bytes;
  *ms = b->seg_ms;
  return SA_OK;
}

int sa_batch_set_mode(sa_batch *b, int mode) {
  if (!b || mode < SA_BATCH_AUTO || mode > SA_BATCH_SEGMENTED_EAGER) return SA_EINVAL;
  if ((mode == SA_BATCH_SEGMENTED || mode == SA_BATCH_SEGMENTED_EAGER) && !b->seg_ok) return SA_EINVAL;
  b->mode = mode;
  if (mode != SA_BATCH_AUTO) {
    const bool sg = mode != SA_BATCH_STREAMS;
    b->plan = Plan{(int)b->streams.size(), 8, sg ? 1 : 0, sg ? 8 : 0, sg ? 1024 : 0};
  }
  return SA_OK;
}

int sa_batch_step(sa_batch *b, const sa_csr *const *A, const void *const *rhs, void *const *x, sa_info *info) {
  if (!b || !A || !rhs || !x) return SA_EINVAL;
  const int nseq = (int)b->seqs.size();
  for (int i = 0; i < nseq; ++i)
    if (!A[i] || !rhs[i] || !x[i]) return SA_EINVAL;
  // plan of this step: a candidate while tuning, else the chosen one (segmented
  // candidates are skipped for a batch the engine cannot take)
  if (b->mode == SA_BATCH_AUTO && !b->seg_ok)
    while (b->tune_next < kNumCandidates && kCandidates[b->tune_next].seg) ++b->tune_next;
  const bool timing = b->mode == SA_BATCH_AUTO && b->steps >= b->tune_warm && b->tune_next < kNumCandidates;
  Plan plan = b->plan;
  if (timing) plan = kCandidates[b->tune_next];
  if (plan.streams > (int)b->streams.size()) plan.streams = (int)b->streams.size();
  // the engine needs at least one nonzero per matrix (its SpMV tiles read entry 0)
  bool seg = plan.seg != 0 && b->seg_ok;
  for (int i = 0; i < nseq && seg; ++i) seg = A[i]->nnz > 0 && A[i]->val_is_fp32 && A[i]->n == b->seqs[i]->cfg.n;
  // longest processing time first: sequences by decreasing cost to the least loaded stream
  std::vector<int> order(nseq);
  for (int i = 0; i < nseq; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int c) { return b->cost[a] > b->cost[c]; });
  std::vector<std::vector<int>> lists(plan.streams);
  std::vector<double> load(plan.streams, 0.0);
  for (int i : order) {
    int best = 0;
    for (int s = 1; s < plan.streams; ++s)
      if (load[s] < load[best]) best = s;
    lists[best].push_back(i);
    load[best] += b->cost[i];
  }
  std::vector<sa_info> inf(nseq);
  std::vector<int> rc(plan.streams, SA_OK);
  auto worker = [&](int s) {
    hipStream_t st = b->streams[s];
    for (int i : lists[s]) {
      sa_seq *q = b->seqs[i];
      q->cfg.poll = plan.poll;
      memset(&inf[i], 0, sizeof(sa_info));
      sa_info g;
      memset(&g, 0, sizeof(g));
      int r = sa_initial_guess(q, A[i], rhs[i], x[i], &g, st);
      if (r == SA_OK) {
        r = sa_solve(q, A[i], rhs[i], x[i], &inf[i], st);
        if (r == SA_NOTCONV || r == SA_EBREAKDOWN) r = SA_OK;  // reported in info
      }
      if (r == SA_OK) r = sa_push_solution(q, x[i], st);
      if (r == SA_OK) r = hipStreamSynchronize(st) == hipSuccess ? SA_OK : SA_EHIP;
      guess_into(inf[i], g);
      if (r != SA_OK) {
        rc[s] = r;
        return;
      }
    }
  };
  const auto t0 = std::chrono::steady_clock::now();
  b->seg_bytes = b->seg_ms = 0.0;
  if (seg) {
    const int r = batch_step_seg(b, plan, lists, A, rhs, x, inf, b->mode != SA_BATCH_SEGMENTED_EAGER);
    if (r != SA_OK) return r;
  } else {
    pool_run(b, plan.streams, worker);
  }
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int s = 0; s < plan.streams; ++s)
    if (rc[s] != SA_OK) return rc[s];
  long long its = 0;
  for (int i = 0; i < nseq; ++i) {
    its += inf[i].iters;
    b->cost[i] = (double)A[i]->nnz * (double)(inf[i].iters + 10);
  }
  if (timing) {
    // seconds per Krylov iteration of the whole batch (steps differ in iterations)
    const double per = sec / (double)(its > 0 ? its : 1);
    if (per < b->tune_best) {
      b->tune_best = per;
      b->tune_best_plan = plan;
    }
    if (++b->tune_next >= kNumCandidates) b->plan = b->tune_best_plan;
  }
  b->steps += 1;
  if (info)
    for (int i = 0; i < nseq; ++i) info[i] = inf[i];
  return SA_OK;
}

}  // extern "C"
