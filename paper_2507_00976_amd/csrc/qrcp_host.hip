// Host driver of the C ABI (include/qrcp.h): argument checks, workspace
// layout, the per-block loop of the blocked randomized QRCP and the unpivoted
// Householder QR baseline.  All device work goes to the caller's stream; the
// loop reads one small status record back per block (block rank after the
// Cholesky step, error status), so the host knows the block rank k before it
// enqueues the k-dependent launches of the block.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "steps.hpp"

namespace qrcp {

size_t hh_leaf_records_bytes(i64 mi);
int launch_hh_leaf(double* A, i64 lda, i64 mi, int ib, double* tau, uint64_t* rec,
                   size_t rec_bytes, int* status, hipStream_t st, double* tout = nullptr,
                   i64 ldt = 0);

static thread_local std::string g_last_error;

Gate& current_gate() {
  static thread_local Gate g{nullptr, 0, kGateRun};
  return g;
}

int launch_resident(const void* fn, dim3 grid, dim3 block, void** params, size_t smem,
                    hipStream_t st) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, unsigned, size_t, int>, int> cache;
  int dev = 0;
  QRCP_HIP(hipGetDevice(&dev));
  int fit = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(fn, block.x, smem, dev);
    auto it = cache.find(key);
    if (it != cache.end()) {
      fit = it->second;
    } else {
      int cus = 0, per = 0;
      QRCP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      QRCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, (int)block.x, smem));
      fit = cus * per;
      cache[key] = fit;
    }
  }
  if ((int)(grid.x * grid.y * grid.z) > fit) return QRCP_ERR_UNSUPPORTED;
  QRCP_HIP(hipLaunchKernel(fn, grid, block, params, smem, st));
  return QRCP_OK;
}

void note_hip_error(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
}

// ---------------------------------------------------------------------------
// Optional stage timing with HIP events (qrcp_profile_*).  Mode 1 records only
// the trailing-update product (the dominant kernel); mode 2 every stage.
// Events are recorded on the caller's stream, so they time the device work of
// each stage; the accumulated records are read back by qrcp_profile_read().
// ---------------------------------------------------------------------------
enum Stage {
  kStSketch, kStLu, kStPerm, kStSketchQr, kStCholGram, kStCholQ, kStRecon, kStLarft,
  kStTrailW, kStTrailUpdate, kStSketchUpdate, kStFinal, kStGeqrfPanel, kNumStages
};
static const char* kStageNames[kNumStages] = {
    "sketch", "lu_pivots", "permute", "sketch_qr", "precondition_gram_potrf", "cholqr_q",
    "reconstruct_r11", "larft", "trailing_w", "trailing_update", "sketch_update", "finalize",
    "geqrf_panel"};

struct Profiler {
  int mode = 0;
  struct Rec {
    hipEvent_t a, b;
    int stage;
    double flops;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};
static Profiler g_prof;

struct ProfScope {
  int stage;
  double flops;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(int s, double f, hipStream_t stream) : stage(s), flops(f), st(stream) {
    if (g_prof.mode == 2 || (g_prof.mode == 1 && s == kStTrailUpdate)) {
      a = g_prof.get();
      if (a) hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = g_prof.get();
    if (!b) return;
    hipEventRecord(b, st);
    g_prof.recs.push_back({a, b, stage, flops});
  }
};

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kSplitBytes = 112u << 20;  // split-K partials (any shape fits, see gemm_pick_splits)

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct FactorWs {
  double* big;  // max(m d, m n): S^T at the start, final-permutation scratch at the end
  double *sk0, *sk1, *xw;
  uint64_t* rec;
  size_t rec_bytes;
  i64 *J[2], *phys[2], *inv, *plan, *ipiv, *jsk;
  double *tmp, *Y;  // m x b each
  double *G, *Rc, *Rinv, *Tm, *P, *X, *Uinv, *R11inv, *R2, *RcN;
  double* dsig;
  double *W, *W2;
  double* Z;       // b x n: Q2^T C2 of the Cholesky-QR panel (formed beside the reconstruction)
  double* split2;  // split-K partials of that product (2 b n doubles)
  double *colss, *ref;
  int *status, *kdev, *info;
  double* split;
  void* skqr;
  size_t skqr_bytes;
  uint64_t* hrec;
  size_t hrec_bytes;
  void* gq;
  size_t gq_bytes;
  double* psave;   // the panel as placed, for a block that stops before its width
  LoopCtl* ctl;    // control record of the device-driven loop
  CallResult* result;  // rank and status of the call
};

size_t carve_factor(char* base, i64 m, i64 n, i64 b, int d, FactorWs* w, bool hqr = false) {
  Carver c{base};
  const i64 bb = std::max<i64>(b, 1);
  w->big = c.take<double>((size_t)std::max(m * (i64)d, m * n));
  w->sk0 = c.take<double>((size_t)d * n);
  w->sk1 = c.take<double>((size_t)d * n);
  w->xw = c.take<double>((size_t)d * n);
  w->rec_bytes = lu_records_bytes_upto(d, n);
  w->rec = c.take<uint64_t>(w->rec_bytes / 8 + 1);
  for (int i = 0; i < 2; ++i) {
    w->J[i] = c.take<i64>(n + 1);
    w->phys[i] = c.take<i64>(n + 1);
  }
  w->inv = c.take<i64>(n + 1);
  w->plan = c.take<i64>(8 + 3 * bb);
  w->ipiv = c.take<i64>(d + 1);
  w->jsk = c.take<i64>(n + 1);
  w->tmp = c.take<double>((size_t)m * bb);
  w->Y = c.take<double>((size_t)m * bb);
  double** sq[] = {&w->G, &w->Rc, &w->Rinv, &w->Tm, &w->P, &w->X, &w->Uinv, &w->R11inv, &w->R2, &w->RcN};
  for (double** p : sq) *p = c.take<double>((size_t)bb * bb);
  w->dsig = c.take<double>(bb);
  w->W = c.take<double>((size_t)bb * n);
  w->W2 = c.take<double>((size_t)bb * n);
  w->Z = c.take<double>((size_t)bb * n);
  w->split2 = c.take<double>((size_t)2 * bb * n);
  w->colss = c.take<double>(n + 1);
  w->ref = c.take<double>(1);
  w->status = c.take<int>(4);
  w->kdev = c.take<int>(4);
  w->info = c.take<int>(4);
  w->split = c.take<double>(kSplitBytes / 8);
  w->skqr_bytes = sketch_qr_ws_bytes(d, n);
  w->skqr = c.take<char>(w->skqr_bytes);
  // column-pivoted sketch QR scratch (qrcp_wide = 1): reflector scalars and arg-max partials
  w->gq_bytes = sketch_geqp3_ws_bytes(d);
  w->gq = c.take<char>(w->gq_bytes);
  w->psave = c.take<double>((size_t)m * bb);
  w->ctl = c.take<LoopCtl>(1);
  w->result = c.take<CallResult>(1);
  // exchange records of the Householder panel's leaf kernel (qr_tall = 1)
  w->hrec_bytes = hqr ? hh_leaf_records_bytes(m) : 0;
  w->hrec = hqr ? c.take<uint64_t>(w->hrec_bytes / 8 + 1) : nullptr;
  return c.off + kAlign;
}

int sketch_rows(i64 b, double gamma) {
  return (int)std::ceil(gamma * (double)b - 1e-12);
}

qrcp_opts defaults() {
  qrcp_opts o;
  o.struct_size = sizeof(qrcp_opts);
  o.cholqr_passes = 1;
  o.sketch_precision = 0;
  o.trailing_precision = 0;
  o.pivot_base = 0;
  o.pivot_steps = 0;
  o.qr_tall = 0;
  o.qrcp_wide = 0;
  o.max_rank = 0;
  return o;
}

qrcp_opts read_opts(const qrcp_opts* p) {
  qrcp_opts o = defaults();
  if (!p) return o;
  const int sz = p->struct_size;
  if (sz >= (int)(offsetof(qrcp_opts, cholqr_passes) + 4)) o.cholqr_passes = p->cholqr_passes;
  if (sz >= (int)(offsetof(qrcp_opts, sketch_precision) + 4)) o.sketch_precision = p->sketch_precision;
  if (sz >= (int)(offsetof(qrcp_opts, trailing_precision) + 4)) o.trailing_precision = p->trailing_precision;
  if (sz >= (int)(offsetof(qrcp_opts, pivot_base) + 4)) o.pivot_base = p->pivot_base;
  if (sz >= (int)(offsetof(qrcp_opts, pivot_steps) + 4)) o.pivot_steps = p->pivot_steps;
  if (sz >= (int)(offsetof(qrcp_opts, qr_tall) + 4)) o.qr_tall = p->qr_tall;
  if (sz >= (int)(offsetof(qrcp_opts, qrcp_wide) + 4)) o.qrcp_wide = p->qrcp_wide;
  if (sz >= (int)(offsetof(qrcp_opts, max_rank) + 8)) o.max_rank = p->max_rank;
  return o;
}

int read_back(void* host, const void* dev, size_t bytes, hipStream_t st) {
  QRCP_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, st));
  QRCP_HIP(hipStreamSynchronize(st));
  return QRCP_OK;
}

int zero_int(int* p, hipStream_t st) { return launch_fill_u64((uint64_t*)p, 1, 0ull, st); }

GemmArgs ga(int M, int N, int K, const double* A, i64 lda, const double* B, i64 ldb, double* C,
            i64 ldc, double alpha = 1.0, double beta = 0.0) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta;
  return g;
}

// First half of (H_0..H_{k-1})^T C for a clean unit lower trapezoidal Y
// (mi x k, ldy): T from the UT transform of Y^T Y, W = Y^T C, W2 = T^T W.
// T of the compact WY form of (H_0..H_{k-1}) from the UT transform of Y^T Y.
int apply_qt_t(const double* Y, i64 mi, int k, i64 ldy, const double* tau, double* G, double* T,
               i64 ldk, double* split, size_t split_bytes, hipStream_t st) {
  if (k <= 0 || mi <= 0) return QRCP_OK;
  ProfScope ps(kStLarft, 2.0 * mi * k * k, st);
  QRCP_TRY(gemm(true, false, Prec::F64, ga(k, k, (int)mi, Y, ldy, Y, ldy, G, ldk), split, split_bytes, st));
  QRCP_TRY(launch_ut_tinv(G, ldk, tau, k, st));
  QRCP_TRY(launch_trinv_upper(G, ldk, k, T, ldk, st));
  QRCP_TRY(launch_ut_zero_diag(T, ldk, tau, k, st));
  return QRCP_OK;
}

// W = Y^T C, W2 = -T^T W (so that the update is C += Y W2, accumulated onto C).
int apply_qt_wt(const double* Y, i64 mi, int k, i64 ldy, const double* T, i64 ldk, const double* C,
                i64 nc, i64 ldc, Prec prec, double* W, double* W2, double* split,
                size_t split_bytes, hipStream_t st) {
  if (k <= 0 || nc <= 0 || mi <= 0) return QRCP_OK;
  ProfScope ps(kStTrailW, 2.0 * mi * k * nc + 2.0 * k * k * nc, st);
  GemmArgs w = ga(k, (int)nc, (int)mi, Y, ldy, C, ldc, W, k);
  w.kind = GemmKind::TrailingW;
  QRCP_TRY(gemm(true, false, prec, w, split, split_bytes, st));
  QRCP_TRY(gemm(true, false, prec, ga(k, (int)nc, k, T, ldk, W, k, W2, k, -1.0, 0.0), split,
                split_bytes, st));
  return QRCP_OK;
}

int apply_qt_w(const double* Y, i64 mi, int k, i64 ldy, const double* tau, const double* C,
               i64 nc, i64 ldc, Prec prec, double* G, double* T, i64 ldk, double* W, double* W2,
               double* split, size_t split_bytes, hipStream_t st) {
  if (k <= 0 || nc <= 0 || mi <= 0) return QRCP_OK;
  QRCP_TRY(apply_qt_t(Y, mi, k, ldy, tau, G, T, ldk, split, split_bytes, st));
  return apply_qt_wt(Y, mi, k, ldy, T, ldk, C, nc, ldc, prec, W, W2, split, split_bytes, st);
}

// Second half, rows r0 .. r1 of C: C(r0:r1, :) += Y(r0:r1, :) W2 (W2 = -T^T Y^T C).
int apply_qt_rows(const double* Y, i64 r0, i64 r1, int k, i64 ldy, double* C, i64 nc, i64 ldc,
                  Prec prec, const double* W2, hipStream_t st) {
  if (k <= 0 || nc <= 0 || r1 <= r0) return QRCP_OK;
  ProfScope ps(kStTrailUpdate, 2.0 * (r1 - r0) * k * nc, st);
  GemmArgs u = ga((int)(r1 - r0), (int)nc, k, Y + r0, ldy, W2, k, C + r0, ldc, 1.0, 1.0);
  u.kind = GemmKind::TrailingUpdate;
  QRCP_TRY(gemm(false, false, prec, u, nullptr, 0, st));
  return QRCP_OK;
}

int apply_qt_clean(const double* Y, i64 mi, int k, i64 ldy, const double* tau, double* C, i64 nc,
                   i64 ldc, Prec prec, double* G, double* T, i64 ldk, double* W, double* W2,
                   double* split, size_t split_bytes, hipStream_t st) {
  QRCP_TRY(apply_qt_w(Y, mi, k, ldy, tau, C, nc, ldc, prec, G, T, ldk, W, W2, split, split_bytes, st));
  return apply_qt_rows(Y, 0, mi, k, ldy, C, nc, ldc, prec, W2, st);
}

// apply_qt_clean for a Householder leaf whose kernel left the T of its
// compact WY form in T (no Gram product, no separate triangular inverse).
int apply_qt_leaf(const double* Y, i64 mi, int k, i64 ldy, double* C, i64 nc, i64 ldc,
                  const double* T, i64 ldk, double* W, double* W2, double* split,
                  size_t split_bytes, hipStream_t st) {
  if (k <= 0 || mi <= 0 || nc <= 0) return QRCP_OK;
  QRCP_TRY(apply_qt_wt(Y, mi, k, ldy, T, ldk, C, nc, ldc, Prec::F64, W, W2, split, split_bytes, st));
  return apply_qt_rows(Y, 0, mi, k, ldy, C, nc, ldc, Prec::F64, W2, st);
}

// A second stream of the calling thread on the current device, with a fork
// and a join event, for the rank-k update that overlaps the next block's
// pivot selection.  Created on first use, kept until the thread ends.
struct AuxStream {
  int dev = -1;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  void release() {
    if (s) hipStreamDestroy(s);
    for (hipEvent_t e : {fork, join})
      if (e) hipEventDestroy(e);
    s = nullptr;
    fork = join = nullptr;
    dev = -1;
  }
  ~AuxStream() { release(); }
};

int aux_stream(AuxStream** out) {
  static thread_local AuxStream a;
  int dev = 0;
  QRCP_HIP(hipGetDevice(&dev));
  if (a.dev != dev) {
    a.release();
    QRCP_HIP(hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking));
    QRCP_HIP(hipEventCreateWithFlags(&a.fork, hipEventDisableTiming));
    QRCP_HIP(hipEventCreateWithFlags(&a.join, hipEventDisableTiming));
    a.dev = dev;
  }
  *out = &a;
  return QRCP_OK;
}

// A pinned host word of the calling thread that the blocking form polls: the
// loop's decision kernel writes the block count there once the loop stops, so
// the host stops enqueueing blocks whose launches would only return at once.
struct StopFlag {
  int dev = -1;
  int* host = nullptr;
  int* devp = nullptr;
  void release() {
    if (host) (void)hipHostFree(host);
    host = devp = nullptr;
    dev = -1;
  }
  ~StopFlag() { release(); }
};

int stop_flag(StopFlag** out) {
  static thread_local StopFlag f;
  int dev = 0;
  QRCP_HIP(hipGetDevice(&dev));
  if (f.dev != dev) {
    f.release();
    void* h = nullptr;
    QRCP_HIP(hipHostMalloc(&h, 64, hipHostMallocMapped));
    f.host = (int*)h;
    void* dp = nullptr;
    QRCP_HIP(hipHostGetDevicePointer(&dp, h, 0));
    f.devp = (int*)dp;
    f.dev = dev;
  }
  *out = &f;
  return QRCP_OK;
}

// Makes the caller's stream wait for the overlapped update on every exit path.
struct JoinGuard {
  hipStream_t st;
  AuxStream* aux;
  bool pending = false;
  int join() {
    if (!pending) return QRCP_OK;
    pending = false;
    QRCP_HIP(hipStreamWaitEvent(st, aux->join, 0));
    return QRCP_OK;
  }
  ~JoinGuard() { join(); }
};

}  // namespace
}  // namespace qrcp

using namespace qrcp;

extern "C" {

const char* qrcp_status_string(int status) {
  switch (status) {
    case QRCP_OK: return "success";
    case QRCP_ERR_WORKSPACE: return "workspace missing or too small";
    case QRCP_ERR_HIP: return "HIP runtime error";
    case QRCP_ERR_NONFINITE: return "non-finite value in the input or the sketch";
    case QRCP_ERR_UNSUPPORTED: return "unsupported shape or option";
    case QRCP_ERR_TIMEOUT: return "cross-workgroup wait timed out";
    default: return status < 0 ? "illegal argument" : "unknown status";
  }
}

const char* qrcp_last_error(void) { return g_last_error.c_str(); }

size_t qrcp_workspace_size(int64_t m, int64_t n, int64_t block_size, double sketch_factor,
                           const qrcp_opts* opts) {
  if (m < 0 || n < 0 || block_size < 1 || !(sketch_factor >= 1.0)) return 0;
  FactorWs w;
  const int d = sketch_rows(block_size, sketch_factor);
  const qrcp_opts o = read_opts(opts);
  const i64 b = std::min<i64>(block_size, std::max<i64>(n, 1));
  return carve_factor(nullptr, m, n, b, d, &w, o.qr_tall == 1);
}

}  // extern "C"

namespace qrcp {
namespace {

// Library resources a call may use (factor_impl's uses):
//   kResAux  - run the deferred rank-k update on the library's second stream
//              (created on first use); without it every launch goes to the
//              caller's stream in the same order, with the same arithmetic
//              (the results are bitwise the same);
//   kResStop - a pinned host word of the calling thread (allocated on first
//              use) through which the device tells the blocking form to stop
//              enqueueing blocks once the loop has stopped.
enum : unsigned { kResAux = 1u, kResStop = 2u };

// The factorization behind qrcp_factor, qrcp_factor_async, qrcp_factor_noalloc
// and the request server.
int factor_impl(double* A, int64_t m, int64_t n, int64_t lda, int64_t block_size,
                double sketch_factor, uint64_t seed, double tol, int64_t* jpiv, double* tau,
                const qrcp_opts* opts_in, void* workspace, size_t workspace_bytes, void* stream,
                unsigned uses, int64_t* rank_host, int64_t* rank_dev, int32_t* status_dev) {
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (lda < std::max<int64_t>(1, m)) return -4;
  if (block_size < 1) return -5;
  if (!(sketch_factor >= 1.0)) return -6;
  if (!(tol >= 0.0)) return -8;
  const qrcp_opts o = read_opts(opts_in);
  if (o.cholqr_passes != 1 && o.cholqr_passes != 2) return -12;
  if (o.sketch_precision < 0 || o.sketch_precision > 1) return -12;
  if (o.trailing_precision < 0 || o.trailing_precision > 1) return -12;
  if (o.pivot_base != 0 && o.pivot_base != 1) return -12;
  if (o.pivot_steps != 0 && o.pivot_steps != 1) return -12;
  if (o.qr_tall != 0 && o.qr_tall != 1) return -12;
  if (o.qrcp_wide != 0 && o.qrcp_wide != 1) return -12;
  if (o.max_rank < 0) return -12;
  if (rank_host) *rank_host = 0;
  if (n == 0) {
    if (rank_dev || status_dev) QRCP_TRY(launch_set_result(rank_dev, status_dev, (hipStream_t)stream));
    return QRCP_OK;
  }
  if (!A && m > 0) return -1;
  if (!jpiv) return -9;
  if (!tau && m > 0) return -10;
  const i64 b = std::min<i64>(block_size, n);
  const int d = sketch_rows(block_size, sketch_factor);
  // the pivot selection of the first block (n_i = n) must fit its resident grid
  if (d > 1024 || lu_resident_groups(n) == 0) return QRCP_ERR_UNSUPPORTED;
  // the Householder panel's leaf kernel keeps one row per thread resident
  if (o.qr_tall == 1 && m > 65536) return QRCP_ERR_UNSUPPORTED;
  FactorWs w;
  const size_t need = carve_factor(nullptr, m, n, b, d, &w, o.qr_tall == 1);
  if (!workspace || workspace_bytes < need) return QRCP_ERR_WORKSPACE;
  carve_factor((char*)workspace, m, n, b, d, &w, o.qr_tall == 1);
  // columns the loop factors at most: min(m, n), or fewer in truncated mode
  const i64 mn = std::min(m, n);
  const i64 lim = o.max_rank > 0 ? std::min(mn, (i64)o.max_rank) : mn;
  hipStream_t st = (hipStream_t)stream;
  const Prec tprec = o.trailing_precision ? Prec::F32 : Prec::F64;
  // every launch below passes a gate on the loop's control record
  GateScope open_gate(Gate{nullptr, 0, kGateRun});
  QRCP_TRY(launch_loop_init(w.ctl, st));
  QRCP_TRY(zero_int(w.status, st));
  QRCP_TRY(launch_iota(w.J[0], n, st));
  QRCP_TRY(launch_iota(w.phys[0], n, st));
  QRCP_TRY(launch_iota(w.inv, n, st));

  // ---- sketch M^sk = S A (S generated once, stored transposed) ----
  if (lim > 0) {
    ProfScope ps(kStSketch, 2.0 * d * m * n, st);
    // the BF16 product holding all d rows per tile (S generated in BF16), else
    // the general one
    int rc = QRCP_ERR_UNSUPPORTED;
    if (o.sketch_precision)
      rc = launch_sketch_bf16(A, m, n, lda, d, seed, w.sk0, d, w.big,
                              (size_t)std::max(m * (i64)d, m * n) * sizeof(double), w.split, kSplitBytes, st);
    if (rc == QRCP_ERR_UNSUPPORTED) {
      QRCP_TRY(launch_sketch_operator(w.big, m, d, m, seed, st));
      GemmArgs g = ga(d, (int)n, (int)m, w.big, m, A, lda, w.sk0, d);
      g.kind = GemmKind::Sketch;
      QRCP_TRY(gemm(true, false, o.sketch_precision ? Prec::BF16 : Prec::F64, g, w.split, kSplitBytes, st));
    } else {
      QRCP_TRY(rc);
    }
    QRCP_TRY(launch_sketch_ref(w.sk0, d, d, n, w.colss, w.ref, st));
  }

  AuxStream* aux = nullptr;
  bool lookahead = (uses & kResAux) != 0;
  if (getenv("QRCP_NO_LOOKAHEAD")) lookahead = false;
  if (lookahead) QRCP_TRY(aux_stream(&aux));
  JoinGuard jg{st, aux};
  // the blocking form with the library's own resources stops enqueueing once
  // the device reports that the loop has stopped (the async and no-alloc
  // forms enqueue every block)
  volatile int* stop_host = nullptr;
  int* stop_dev = nullptr;
  if (rank_host && (uses & kResStop)) {
    StopFlag* sf = nullptr;
    QRCP_TRY(stop_flag(&sf));
    *sf->host = INT_MAX;
    stop_host = sf->host;
    stop_dev = sf->devp;
  }
  // the previous block's rank-k update of rows s+k .. m, started on the
  // second stream once the next block's pivots are known (its kernels carry
  // the gate of the block they belong to)
  struct Pending {
    bool on = false;
    int blk = 0;
    i64 r0 = 0, r1 = 0, nc = 0;
    int k = 0;
    double* C = nullptr;
  } pend;
  auto start_pending = [&]() -> int {
    if (!pend.on) return QRCP_OK;
    pend.on = false;
    GateScope gs(Gate{w.ctl, pend.blk, kGateRun});
    if (!lookahead)
      return apply_qt_rows(w.Y, pend.r0, pend.r1, pend.k, m, pend.C, pend.nc, lda, tprec, w.W2, st);
    QRCP_HIP(hipEventRecord(aux->fork, st));
    QRCP_HIP(hipStreamWaitEvent(aux->s, aux->fork, 0));
    QRCP_TRY(apply_qt_rows(w.Y, pend.r0, pend.r1, pend.k, m, pend.C, pend.nc, lda, tprec, w.W2, aux->s));
    QRCP_HIP(hipEventRecord(aux->join, aux->s));
    jg.pending = true;
    return QRCP_OK;
  };
  const int* keff = &w.ctl->k;  // the block's effective width, on the device
  int cur = 0;
  // pivot_steps = 1 runs only the block's k_max elimination steps of the
  // GETRF of the sketch (the selected columns are the same; the order of the
  // columns no block selects is not that of Alg. 2)
  const bool lu_all_steps = o.pivot_steps == 0;
  // Every block is enqueued without reading anything back: each block's
  // launches are sized for its full width k_max; a one-thread kernel after the
  // panel's Cholesky factorization (tri_rank for the Householder panel)
  // records the effective width k and whether the loop stops here.  Later
  // blocks' kernels then return at once (gate kGateRun); in the block that
  // stops, columns k .. k_max of the panel become identity reflectors (their
  // factors padded with the identity, tau = 0), and those panel columns,
  // saved before the panel QR, get the k reflectors applied like the rest of
  // the trailing matrix (gate kGateExit); the sketch update runs only in
  // blocks the loop continues past (gate kGateGoOn).
  int blk = 0;
  for (i64 s = 0; s < lim; ++blk) {
    if (stop_host && *stop_host <= blk) break;  // the rest would return at once
    const i64 ni = n - s, mi = m - s;
    const int kmax = (int)std::min<i64>(std::min<i64>(b, lim - s), std::min(ni, mi));
    const i64 c = s + kmax;
    const bool last = c >= lim;
    const Gate run{w.ctl, blk, kGateRun}, ex{w.ctl, blk, kGateExit}, goon{w.ctl, blk, kGateGoOn};
    GateScope gs(run);
    // elimination steps of the sketch's GETRF: all min(d, n_i), bounded by
    // m_i (the sketch of an m_i-row matrix has rank <= m_i: beyond it the
    // Schur complement is zero in exact arithmetic, only a wide matrix's last
    // blocks have m_i < min(d, n_i)); or the block's kmax with pivot_steps = 1
    int lu_steps = 0;
    if (!lu_all_steps) lu_steps = kmax;
    else if (mi < std::min<i64>(d, ni)) lu_steps = (int)mi;
    double* Ablk = A + s + s * lda;  // panel top-left (rows s.., physical column s)
    const i64 nc = n - c;
    double* Ct = A + s + c * lda;  // trailing columns c .. n-1, rows s..m-1
    // W of the trailing update split as Y1^T C1 + U^{-T} (Q2^T C2) (Cholesky-QR
    // panel, FP64 update, rows below the panel and columns right of it)
    const bool zsplit = o.qr_tall == 0 && tprec == Prec::F64 && mi > kmax && nc > 0;
    // 1. pivots of the sketch (Alg. 2 GETRF on the transpose, or GEQP3)
    if (o.qrcp_wide == 1) {
      // column-pivoted QR of the sketch (GEQP3): pivots and R^sk in one pass,
      // pivoting over the same rank bound as the LU (min(d, n_i, m_i) steps)
      {
        ProfScope ps(kStLu, 4.0 * d * d * ni, st);
        QRCP_TRY(launch_sketch_geqp3(w.sk0 + s * d, d, ni, d, (int)std::min<i64>(std::min<i64>(d, ni), mi),
                                     w.sk1 + s * d, w.sk0 + s * d, d, w.jsk, w.gq, w.gq_bytes,
                                     w.status, st));
      }
      {
        ProfScope ps(kStPerm, 0.0, st);
        QRCP_TRY(launch_perm_plan(w.jsk, s, n, kmax, w.J[cur], w.J[1 - cur], w.phys[cur],
                                  w.phys[1 - cur], w.inv, w.plan, st));
      }
      QRCP_TRY(start_pending());
      cur = 1 - cur;
    } else {
      {
        ProfScope ps(kStLu, 2.0 * ni * d * (lu_steps ? lu_steps : std::min<i64>(d, ni)), st);
        QRCP_TRY(launch_lu_pivots(w.sk0 + s * d, d, ni, d, w.xw, w.rec, w.rec_bytes, w.ipiv, w.jsk,
                                  w.status, st, lu_steps));
      }
      // 2. logical maps and the placement plan; 3. permuted sketch
      {
        ProfScope ps(kStPerm, 0.0, st);
        QRCP_TRY(launch_perm_plan(w.jsk, s, n, kmax, w.J[cur], w.J[1 - cur], w.phys[cur],
                                  w.phys[1 - cur], w.inv, w.plan, st));
        QRCP_TRY(launch_sketch_permute(w.sk0 + s * d, w.sk1 + s * d, d, d, ni, w.jsk, st));
      }
      // The previous block's update runs beside the sketch QR and tri_rank
      // (which touch only the sketch buffers), not beside the pivot selection,
      // whose per-step exchange is slowed by the update's memory traffic.
      QRCP_TRY(start_pending());
      cur = 1 - cur;
      // 4. R factor of the permuted sketch (back into sk0, logical positions)
      {
        ProfScope ps(kStSketchQr, 2.0 * d * d * ni, st);
        QRCP_TRY(run_sketch_qr(w.sk1 + s * d, d, ni, d, w.sk0 + s * d, d, w.skqr, w.skqr_bytes,
                               w.status, st));
      }
    }
    const double* Rsk = w.sk0 + s * d;
    // 5. tri_rank
    QRCP_TRY(launch_trirank(Rsk, d, kmax, tol, w.ref, w.kdev, st));
    // 6. place the panel columns (all m rows): needs the previous block's update
    QRCP_TRY(jg.join());
    {
      ProfScope ps(kStPerm, 0.0, st);
      QRCP_TRY(launch_place_columns(A, lda, m, s, kmax, w.plan, w.tmp, m, st));
    }
    if (o.qr_tall == 1) {
      // Householder QR of the panel (GEQRF; Sec. 2.3), 32-column leaves each
      // applied to the rest of the panel; tri_rank's k is the block's width
      QRCP_TRY(launch_loop_decide(w.ctl, w.status, w.kdev, blk, kmax, s, c, lim, false, stop_dev, st));
      {
        GateScope gx(ex);
        QRCP_TRY(launch_copy2d(Ablk, lda, w.psave, m, mi, kmax, st));
      }
      ProfScope ps(kStGeqrfPanel, 2.0 * mi * kmax * kmax - 2.0 * kmax * kmax * kmax / 3.0, st);
      for (int s2 = 0; s2 < kmax; s2 += 32) {
        const int ib = std::min(32, kmax - s2);
        double* Al = Ablk + s2 + (i64)s2 * lda;
        QRCP_TRY(launch_hh_leaf(Al, lda, mi - s2, ib, tau + s + s2, w.hrec, w.hrec_bytes, w.status, st,
                                w.Rc, b));
        if (s2 + ib < kmax) {
          QRCP_TRY(launch_copy2d(Al, lda, w.tmp, m, mi - s2, ib, st));
          QRCP_TRY(launch_unit_lower(Al, lda, ib, w.tmp, m, st));
          QRCP_TRY(apply_qt_leaf(w.tmp, mi - s2, ib, m, Al + (i64)ib * lda, kmax - s2 - ib, lda, w.Rc,
                                 b, w.W, w.W2, w.split, kSplitBytes, st));
        }
      }
      {
        GateScope gx(ex);
        QRCP_TRY(launch_zero_tail(tau + s, kmax, keff, st));
      }
      // clean Y (unit lower trapezoidal) for the trailing update; R11 stays
      // in place on and above the panel's diagonal
      QRCP_TRY(launch_copy2d(Ablk, lda, w.Y, m, mi, kmax, st));
      QRCP_TRY(launch_unit_lower(Ablk, lda, kmax, w.Y, m, st));
    } else {
      {
        ProfScope ps(kStCholGram, 4.0 * mi * kmax * kmax, st);
        // 7. precondition with the leading k x k block of Rsk (k on the device)
        QRCP_TRY(launch_trinv_upper(Rsk, d, kmax, w.Rinv, b, st));
        QRCP_TRY(launch_mask_k(w.Rinv, b, kmax, w.kdev, st));
        QRCP_TRY(gemm(false, false, Prec::F64, ga((int)mi, kmax, kmax, Ablk, lda, w.Rinv, b, w.Y, m),
                      nullptr, 0, st));
        // 8. Gram and Cholesky; a breakdown (or the rank cut) ends the factor at info
        QRCP_TRY(gemm(true, false, Prec::F64, ga(kmax, kmax, (int)mi, w.Y, m, w.Y, m, w.G, b), w.split,
                      kSplitBytes, st));
        QRCP_TRY(launch_potrf_mw(w.G, b, kmax, w.info, w.split, kSplitBytes, st));
        QRCP_TRY(launch_loop_decide(w.ctl, w.status, w.info, blk, kmax, s, c, lim, false, stop_dev, st));
        GateScope gx(ex);
        QRCP_TRY(launch_copy2d(Ablk, lda, w.psave, m, mi, kmax, st));
        QRCP_TRY(launch_pad_identity(w.G, b, kmax, keff, st));
      }
      // Q = M^pre Rc^{-1}
      {
        ProfScope psq(kStCholQ, 2.0 * mi * kmax * kmax, st);
        QRCP_TRY(launch_trinv_upper(w.G, b, kmax, w.Rinv, b, st));
        {
          GateScope gx(ex);
          QRCP_TRY(launch_mask_k(w.Rinv, b, kmax, keff, st));
        }
        if (o.cholqr_passes == 2) {
          QRCP_TRY(gemm(false, false, Prec::F64, ga((int)mi, kmax, kmax, w.Y, m, w.Rinv, b, w.tmp, m),
                        nullptr, 0, st));
          QRCP_TRY(gemm(true, false, Prec::F64, ga(kmax, kmax, (int)mi, w.tmp, m, w.tmp, m, w.R2, b),
                        w.split, kSplitBytes, st));
          QRCP_TRY(launch_potrf_mw(w.R2, b, kmax, w.info, w.split, kSplitBytes, st));
          QRCP_TRY(launch_loop_decide(w.ctl, w.status, w.info, blk, kmax, s, c, lim, true, stop_dev, st));
          {
            // a second-pass breakdown shrinks the width: redo the first pass's
            // inverse and Q with it (the block then stops the loop)
            GateScope gx(ex);
            QRCP_TRY(launch_pad_identity(w.G, b, kmax, keff, st));
            QRCP_TRY(launch_trinv_upper(w.G, b, kmax, w.Rinv, b, st));
            QRCP_TRY(launch_mask_k(w.Rinv, b, kmax, keff, st));
            QRCP_TRY(gemm(false, false, Prec::F64, ga((int)mi, kmax, kmax, w.Y, m, w.Rinv, b, w.tmp, m),
                          nullptr, 0, st));
            QRCP_TRY(launch_pad_identity(w.R2, b, kmax, keff, st));
          }
          QRCP_TRY(launch_trinv_upper(w.R2, b, kmax, w.Uinv, b, st));
          {
            GateScope gx(ex);
            QRCP_TRY(launch_mask_k(w.Uinv, b, kmax, keff, st));
          }
          QRCP_TRY(gemm(false, false, Prec::F64, ga((int)mi, kmax, kmax, w.tmp, m, w.Uinv, b, Ablk, lda),
                        nullptr, 0, st));
          // Rc <- R2 Rc
          QRCP_TRY(gemm(false, false, Prec::F64, ga(kmax, kmax, kmax, w.R2, b, w.G, b, w.RcN, b), nullptr,
                        0, st));
          QRCP_TRY(launch_copy2d(w.RcN, b, w.G, b, kmax, kmax, st));
        } else {
          QRCP_TRY(gemm(false, false, Prec::F64, ga((int)mi, kmax, kmax, w.Y, m, w.Rinv, b, Ablk, lda),
                        nullptr, 0, st));
        }
      }
      // W = Y^T C of the trailing update, with Y = [Y1; Q2 U^{-1}] from the
      // reconstruction below, is Y1^T C1 + U^{-T} (Q2^T C2): the large product
      // Z = Q2^T C2 needs only the Cholesky-QR panel, so it runs on the second
      // stream beside the reconstruction and T (on the caller's stream in
      // order when there is no second stream: the same arithmetic)
      if (zsplit) {
        hipStream_t zs = st;
        if (lookahead) {
          QRCP_HIP(hipEventRecord(aux->fork, st));
          QRCP_HIP(hipStreamWaitEvent(aux->s, aux->fork, 0));
          zs = aux->s;
        }
        {
          ProfScope psz(kStTrailW, 2.0 * (mi - kmax) * kmax * nc, zs);
          GemmArgs z = ga(kmax, (int)nc, (int)(mi - kmax), Ablk + kmax, lda, Ct + kmax, lda, w.Z, kmax);
          z.kind = GemmKind::TrailingW;
          QRCP_TRY(gemm(true, false, Prec::F64, z, w.split2, (size_t)2 * b * n * sizeof(double), zs));
        }
        if (lookahead) {
          QRCP_HIP(hipEventRecord(aux->join, zs));
          jg.pending = true;
        }
      }
      // 9. Householder reconstruction: sign-modified LU of the head, Y2 = Q2 U^{-1}
      {
        ProfScope psr(kStRecon, 2.0 * (mi - kmax) * kmax * kmax + 2.0 * kmax * kmax * kmax, st);
        QRCP_TRY(launch_headlu_mw(Ablk, lda, kmax, w.dsig, w.split, kSplitBytes, w.status, st));
        QRCP_TRY(launch_tau_from_u(Ablk, lda, kmax, w.dsig, tau + s, st));
        {
          GateScope gx(ex);
          QRCP_TRY(launch_zero_tail(tau + s, kmax, keff, st));
        }
        QRCP_TRY(launch_trinv_upper(Ablk, lda, kmax, w.Uinv, b, st));
        if (mi > kmax) {
          QRCP_TRY(gemm(false, false, Prec::F64,
                        ga((int)(mi - kmax), kmax, kmax, Ablk + kmax, lda, w.Uinv, b, w.Y + kmax, m),
                        nullptr, 0, st));
          // Y2 into the output below the head (after Z, which still reads Q2 there)
          if (!zsplit) QRCP_TRY(launch_copy2d(w.Y + kmax, m, Ablk + kmax, lda, mi - kmax, kmax, st));
        }
        QRCP_TRY(launch_unit_lower(Ablk, lda, kmax, w.Y, m, st));
        //    R11 = diag(D) Rc Rsk(0:k, 0:k)
        QRCP_TRY(gemm(false, false, Prec::F64, ga(kmax, kmax, kmax, w.G, b, Rsk, d, w.P, b), nullptr, 0, st));
        QRCP_TRY(launch_write_r11(w.P, b, kmax, w.dsig, Ablk, lda, st));
      }
    }
    // 10-11. trailing update of the physical columns c .. n-1 (rows s..m-1)
    if (zsplit) {
      QRCP_TRY(apply_qt_t(w.Y, mi, kmax, m, tau + s, w.Tm, w.R11inv, b, w.split, kSplitBytes, st));
      QRCP_TRY(jg.join());
      QRCP_TRY(launch_copy2d(w.Y + kmax, m, Ablk + kmax, lda, mi - kmax, kmax, st));
      ProfScope psw(kStTrailW, 4.0 * kmax * kmax * nc, st);
      // W = U^{-T} Z + Y1^T C1, W2 = -T^T W
      QRCP_TRY(gemm(true, false, Prec::F64, ga(kmax, (int)nc, kmax, w.Uinv, b, w.Z, kmax, w.W, kmax),
                    nullptr, 0, st));
      QRCP_TRY(gemm(true, false, Prec::F64,
                    ga(kmax, (int)nc, kmax, w.Y, m, Ct, lda, w.W, kmax, 1.0, 1.0), nullptr, 0, st));
      QRCP_TRY(gemm(true, false, Prec::F64,
                    ga(kmax, (int)nc, kmax, w.R11inv, b, w.W, kmax, w.W2, kmax, -1.0, 0.0), nullptr, 0,
                    st));
    } else {
      QRCP_TRY(apply_qt_w(w.Y, mi, kmax, m, tau + s, Ct, nc, lda, tprec, w.Tm, w.R11inv, b, w.W,
                          w.W2, w.split, kSplitBytes, st));
    }
    {
      // a block that stops before its width: the k reflectors applied to the
      // saved panel columns k .. k_max, which become R(0:k, k:k_max) and the
      // residual rows
      GateScope gx(ex);
      QRCP_TRY(apply_qt_wt(w.Y, mi, kmax, m, w.R11inv, b, w.psave, kmax, m, tprec, w.X, w.R2, w.split,
                           kSplitBytes, st));
      QRCP_TRY(apply_qt_rows(w.Y, 0, mi, kmax, m, w.psave, kmax, m, tprec, w.R2, st));
      QRCP_TRY(launch_copy_cols_from(w.psave, m, Ablk, lda, mi, kmax, keff, st));
    }
    if (last) {
      QRCP_TRY(apply_qt_rows(w.Y, 0, mi, kmax, m, Ct, nc, lda, tprec, w.W2, st));
      break;
    }
    // rows s .. s+k (R12) now: the sketch update needs them
    QRCP_TRY(apply_qt_rows(w.Y, 0, kmax, kmax, m, Ct, nc, lda, tprec, w.W2, st));
    // 12. sketch update: M^sk(0:b, c:) = Rsk12 - Rsk11 R11^{-1} R12 (R12 read through the map)
    {
      GateScope gg(goon);
      ProfScope psu(kStSketchUpdate, 2.0 * b * b * (n - c), st);
      if (o.cholqr_passes == 1 && o.qr_tall == 0) {
        // R11 = diag(D) Rc Rsk11, so Rsk11 R11^{-1} = Rc^{-1} diag(D): the
        // inverse of the Cholesky factor is at hand (Q = M^pre Rc^{-1})
        QRCP_TRY(launch_scale_upper_cols(w.Rinv, b, w.dsig, (int)b, w.X, b, st));
      } else {
        QRCP_TRY(launch_trinv_upper(Ablk, lda, (int)b, w.R11inv, b, st));
        QRCP_TRY(gemm(false, false, Prec::F64, ga((int)b, (int)b, (int)b, Rsk, d, w.R11inv, b, w.X, b),
                      nullptr, 0, st));
      }
      GemmArgs g = ga((int)b, (int)(n - c), (int)b, w.X, b, A + s, lda, w.sk0 + c * d, d, -1.0, 1.0);
      g.bcol = w.phys[cur] + c;
      QRCP_TRY(gemm(false, false, Prec::F64, g, nullptr, 0, st));
    }
    // rows s+k .. m: deferred to the next block, on the second stream
    // (QRCP_NO_LOOKAHEAD=1 keeps them on the caller's stream, for diagnosis)
    pend.on = true;
    pend.blk = blk;
    pend.r0 = kmax;
    pend.r1 = mi;
    pend.k = kmax;
    pend.C = Ct;
    pend.nc = nc;
    s = c;
  }
  QRCP_TRY(start_pending());
  QRCP_TRY(jg.join());
  // the live maps
  QRCP_TRY(launch_loop_pick(w.ctl, w.J[0], w.J[1], w.phys[0], w.phys[1], n, st));
  // tau(l:) = 0, the unplaced columns in logical order, rank and status
  i64* rdev = rank_dev ? rank_dev : (i64*)&w.result->rank;
  int* sdev = status_dev ? status_dev : &w.result->status;
  QRCP_TRY(launch_loop_final(w.ctl, A, lda, m, n, w.phys[0], tau, mn, w.big, w.status, rdev, sdev,
                             st));
  QRCP_TRY(launch_jpiv_out(w.J[0], n, o.pivot_base, jpiv, st));
  if (!rank_host) return QRCP_OK;
  // the blocking form: one read-back of rank and status for the whole call
  CallResult res{};
  if (rank_dev || status_dev) {
    QRCP_TRY(launch_copy_result(rdev, sdev, w.result, st));
  }
  QRCP_TRY(read_back(&res, w.result, sizeof(CallResult), st));
  *rank_host = res.rank;
  return res.status;
}
}  // namespace

int factor_served(double* A, int64_t m, int64_t n, int64_t lda, int64_t block_size,
                  double sketch_factor, uint64_t seed, double tol, int64_t* jpiv, double* tau,
                  int64_t* rank, const qrcp_opts* opts, void* workspace, size_t workspace_bytes,
                  void* stream) {
  if (!rank) return -11;
  return factor_impl(A, m, n, lda, block_size, sketch_factor, seed, tol, jpiv, tau, opts, workspace,
                     workspace_bytes, stream, kResStop, rank, nullptr, nullptr);
}
}  // namespace qrcp

extern "C" {

int qrcp_factor(double* A, int64_t m, int64_t n, int64_t lda, int64_t block_size,
                double sketch_factor, uint64_t seed, double tol, int64_t* jpiv, double* tau,
                int64_t* rank, const qrcp_opts* opts, void* workspace, size_t workspace_bytes,
                void* stream) {
  if (!rank) return -11;
  return factor_impl(A, m, n, lda, block_size, sketch_factor, seed, tol, jpiv, tau, opts, workspace,
                     workspace_bytes, stream, kResAux | kResStop, rank, nullptr, nullptr);
}

int qrcp_factor_async(double* A, int64_t m, int64_t n, int64_t lda, int64_t block_size,
                      double sketch_factor, uint64_t seed, double tol, int64_t* jpiv, double* tau,
                      int64_t* rank_dev, int32_t* status_dev, const qrcp_opts* opts,
                      void* workspace, size_t workspace_bytes, void* stream) {
  if (!rank_dev) return -11;
  if (!status_dev) return -12;
  return factor_impl(A, m, n, lda, block_size, sketch_factor, seed, tol, jpiv, tau, opts, workspace,
                     workspace_bytes, stream, kResAux, nullptr, rank_dev, status_dev);
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Allocation-free factorization: the workspace is a fixed device array of this
// library, so the call needs no caller buffer and allocates nothing.
// ----------------------------------------------------------------------------
namespace qrcp {
namespace {

constexpr size_t kNoAllocBytes = size_t(192) << 20;

// One copy per GPU (each device that loads the library holds its own until the
// process ends).  Host code never passes this name to a kernel: it is only the
// symbol looked up by hipGetSymbolAddress for the device-side address.
__device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_address(void** out) {
  int dev = 0;
  QRCP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return QRCP_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    QRCP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return QRCP_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QRCP_OK;
}

}  // namespace
}  // namespace qrcp

extern "C" {

size_t qrcp_noalloc_max_bytes(void) { return kNoAllocBytes; }

int qrcp_factor_noalloc(double* A, int64_t m, int64_t n, int64_t lda, int64_t block_size,
                        double sketch_factor, uint64_t seed, double tol, int64_t* jpiv,
                        double* tau, int64_t* rank, const qrcp_opts* opts, void* stream) {
  // qrcp_factor's own checks, all on the host before any launch: without a
  // workspace the call ends at the workspace check if everything else holds
  if (!rank) return -11;
  const int pre = factor_impl(A, m, n, lda, block_size, sketch_factor, seed, tol, jpiv, tau, opts,
                              nullptr, 0, stream, 0u, rank, nullptr, nullptr);
  if (pre != QRCP_ERR_WORKSPACE) return pre;
  const size_t need = qrcp_workspace_size(m, n, block_size, sketch_factor, opts);
  if (need > kNoAllocBytes) {
    g_last_error = "qrcp_factor_noalloc: these sizes need " + std::to_string(need) +
                   " bytes of workspace, above the fixed " + std::to_string(kNoAllocBytes) +
                   "-byte device array";
    return QRCP_ERR_WORKSPACE;
  }
  void* ws = nullptr;
  QRCP_TRY(scratch_address(&ws));
  // no second stream: the library creates nothing on this path
  return factor_impl(A, m, n, lda, block_size, sketch_factor, seed, tol, jpiv, tau, opts, ws,
                     kNoAllocBytes, stream, 0u, rank, nullptr, nullptr);
}

// ----------------------------------------------------------------------------
// Unpivoted blocked Householder QR (GEQRF storage).
// ----------------------------------------------------------------------------
}  // extern "C"

namespace qrcp {
namespace {

constexpr size_t kSplitBytesSmall = 32u << 20;  // split-K partials of the panel-side products

struct GeqrfWs {
  double* Yc[2];  // clean reflectors of the current and the previous panel
  double* T[2];   // their compact WY factors
  double *G, *Wn, *W2n;      // panel-side: Gram, next panel's W and W2
  double *W, *W2;            // second stream: the rest of the trailing matrix
  double *Yl, *Gl, *Tl, *Wl, *W2l;  // inside a panel: 32-column leaves
  uint64_t* rec;
  size_t rec_bytes;
  int* status;
  double *split, *split2;
};

size_t carve_geqrf(char* base, i64 m, i64 n, i64 nb, GeqrfWs* w) {
  Carver c{base};
  for (int i = 0; i < 2; ++i) {
    w->Yc[i] = c.take<double>((size_t)m * nb);
    w->T[i] = c.take<double>((size_t)nb * nb);
  }
  w->G = c.take<double>((size_t)nb * nb);
  w->Wn = c.take<double>((size_t)nb * nb);
  w->W2n = c.take<double>((size_t)nb * nb);
  w->W = c.take<double>((size_t)nb * n);
  w->W2 = c.take<double>((size_t)nb * n);
  w->Yl = c.take<double>((size_t)m * 32);
  w->Gl = c.take<double>(32 * 32);
  w->Tl = c.take<double>(32 * 32);
  w->Wl = c.take<double>((size_t)32 * nb);
  w->W2l = c.take<double>((size_t)32 * nb);
  w->rec_bytes = hh_leaf_records_bytes(m);
  w->rec = c.take<uint64_t>(w->rec_bytes / 8 + 1);
  w->status = c.take<int>(4);
  w->split = c.take<double>(kSplitBytes / 8);
  w->split2 = c.take<double>(kSplitBytesSmall / 8);
  return c.off + kAlign;
}

}  // namespace
}  // namespace qrcp

extern "C" {

size_t qrcp_geqrf_workspace_size(int64_t m, int64_t n, int64_t nb) {
  if (m < 0 || n < 0 || nb < 1) return 0;
  GeqrfWs w;
  return carve_geqrf(nullptr, m, n, std::min<i64>(nb, std::max<i64>(n, 1)), &w);
}

// Blocked Householder QR with lookahead: after panel i is factored, the next
// panel's columns are updated on the caller's stream and the rest of the
// trailing matrix on the library's second stream, so the update of the far
// columns runs beside the factorization of panel i+1 (joined before panel
// i+1 updates panel i+2, whose columns that update writes).
int qrcp_geqrf(double* A, int64_t m, int64_t n, int64_t lda, double* tau, int64_t nb,
               void* workspace, size_t workspace_bytes, void* stream) {
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (lda < std::max<int64_t>(1, m)) return -4;
  if (nb < 1) return -6;
  if (m < n) return QRCP_ERR_UNSUPPORTED;
  if (n == 0) return QRCP_OK;
  if (!A) return -1;
  if (!tau) return -5;
  if (m > 65536) return QRCP_ERR_UNSUPPORTED;
  nb = std::min<i64>(nb, n);
  GeqrfWs w;
  const size_t need = carve_geqrf(nullptr, m, n, nb, &w);
  if (!workspace || workspace_bytes < need) return QRCP_ERR_WORKSPACE;
  carve_geqrf((char*)workspace, m, n, nb, &w);
  hipStream_t st = (hipStream_t)stream;
  QRCP_TRY(zero_int(w.status, st));
  AuxStream* aux = nullptr;
  const bool lookahead = getenv("QRCP_NO_LOOKAHEAD") == nullptr;
  if (lookahead) QRCP_TRY(aux_stream(&aux));
  JoinGuard jg{st, aux};
  constexpr int IB = 32;
  int blk = 0;
  for (i64 s = 0; s < n; s += nb, ++blk) {
    const i64 kb = std::min<i64>(nb, n - s), mi = m - s;
    double* Ap = A + s + s * lda;
    {
      ProfScope ps(kStGeqrfPanel, 2.0 * mi * kb * kb, st);
      for (i64 s2 = 0; s2 < kb; s2 += IB) {
        const int ib = (int)std::min<i64>(IB, kb - s2);
        double* Al = Ap + s2 + s2 * lda;
        QRCP_TRY(launch_hh_leaf(Al, lda, mi - s2, ib, tau + s + s2, w.rec, w.rec_bytes, w.status, st,
                                w.Tl, 32));
        if (s2 + ib < kb) {
          // clean copy of the leaf's reflectors, then update the rest of the panel
          QRCP_TRY(launch_copy2d(Al, lda, w.Yl, m, mi - s2, ib, st));
          QRCP_TRY(launch_unit_lower(Al, lda, ib, w.Yl, m, st));
          QRCP_TRY(apply_qt_leaf(w.Yl, mi - s2, ib, m, Al + ib * lda, kb - s2 - ib, lda, w.Tl, 32, w.Wl,
                                 w.W2l, w.split2, kSplitBytesSmall, st));
        }
      }
    }
    if (s + kb >= n) break;
    double* Y = w.Yc[blk & 1];
    double* T = w.T[blk & 1];
    QRCP_TRY(launch_copy2d(Ap, lda, Y, m, mi, kb, st));
    QRCP_TRY(launch_unit_lower(Ap, lda, (int)kb, Y, m, st));
    QRCP_TRY(apply_qt_t(Y, mi, (int)kb, m, tau + s, w.G, T, nb, w.split2, kSplitBytesSmall, st));
    // the next panel's columns: the previous block's far update wrote them
    QRCP_TRY(jg.join());
    const i64 nn = lookahead ? std::min<i64>(nb, n - s - kb) : n - s - kb;
    double* Cn = Ap + kb * lda;
    QRCP_TRY(apply_qt_wt(Y, mi, (int)kb, m, T, nb, Cn, nn, lda, Prec::F64, w.Wn, w.W2n, w.split2,
                         kSplitBytesSmall, st));
    QRCP_TRY(apply_qt_rows(Y, 0, mi, (int)kb, m, Cn, nn, lda, Prec::F64, w.W2n, st));
    const i64 nf = n - s - kb - nn;
    if (nf > 0) {
      double* Cf = Ap + (kb + nn) * lda;
      QRCP_HIP(hipEventRecord(aux->fork, st));
      QRCP_HIP(hipStreamWaitEvent(aux->s, aux->fork, 0));
      QRCP_TRY(apply_qt_wt(Y, mi, (int)kb, m, T, nb, Cf, nf, lda, Prec::F64, w.W, w.W2, w.split,
                           kSplitBytes, aux->s));
      QRCP_TRY(apply_qt_rows(Y, 0, mi, (int)kb, m, Cf, nf, lda, Prec::F64, w.W2, aux->s));
      QRCP_HIP(hipEventRecord(aux->join, aux->s));
      jg.pending = true;
    }
  }
  QRCP_TRY(jg.join());
  int hs = 0;
  QRCP_TRY(read_back(&hs, w.status, sizeof(int), st));
  return hs;
}

// ----------------------------------------------------------------------------
// Step entry points
// ----------------------------------------------------------------------------
int qrcp_sketch_operator(double* St, int64_t m, int64_t d, int64_t ldst, uint64_t seed,
                         void* stream) {
  if (!St && m * d > 0) return -1;
  if (m < 0) return -2;
  if (d < 0) return -3;
  if (ldst < std::max<int64_t>(1, m)) return -4;
  QRCP_TRY(launch_sketch_operator(St, m, (int)d, ldst, seed, (hipStream_t)stream));
  QRCP_HIP(hipStreamSynchronize((hipStream_t)stream));
  return QRCP_OK;
}

int qrcp_philox(const uint32_t* ctr, int64_t count, uint32_t key0, uint32_t key1, uint32_t* out,
                void* stream) {
  if (count < 0) return -2;
  QRCP_TRY(launch_philox(ctr, count, key0, key1, out, (hipStream_t)stream));
  QRCP_HIP(hipStreamSynchronize((hipStream_t)stream));
  return QRCP_OK;
}

int qrcp_sketch(const double* A, int64_t m, int64_t n, int64_t lda, int64_t d, uint64_t seed,
                int32_t precision, double* Msk, int64_t ldmsk, void* workspace,
                size_t workspace_bytes, void* stream) {
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (lda < std::max<int64_t>(1, m)) return -4;
  if (d < 1) return -5;
  if (precision != 0 && precision != 1) return -7;
  if (ldmsk < d) return -9;
  constexpr size_t kSketchSplitBytes = 40u << 20;  // the sketch product's split-K partials
  const size_t need = (size_t)m * d * 8 + kSketchSplitBytes + 2 * kAlign;
  if (!workspace || workspace_bytes < need) return QRCP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Carver c{(char*)workspace};
  double* St = c.take<double>((size_t)m * d);
  double* split = c.take<double>(kSketchSplitBytes / 8);
  int rc = QRCP_ERR_UNSUPPORTED;
  if (precision)
    rc = launch_sketch_bf16(A, m, n, lda, (int)d, seed, Msk, ldmsk, St, (size_t)m * d * 8, split,
                            kSketchSplitBytes, st);
  if (rc == QRCP_ERR_UNSUPPORTED) {
    QRCP_TRY(launch_sketch_operator(St, m, (int)d, m, seed, st));
    QRCP_TRY(gemm(true, false, precision ? Prec::BF16 : Prec::F64,
                  ga((int)d, (int)n, (int)m, St, m, A, lda, Msk, ldmsk), split, kSketchSplitBytes, st));
  } else {
    QRCP_TRY(rc);
  }
  QRCP_HIP(hipStreamSynchronize(st));
  return QRCP_OK;
}

size_t qrcp_lu_workspace_size(int64_t d, int64_t ni) {
  if (d < 1 || ni < 0) return 0;
  return (size_t)d * ni * 8 + lu_records_bytes((int)d, ni) + 4 * kAlign + 64;
}

int qrcp_lu_pivots(const double* Msk, int64_t d, int64_t ni, int64_t ldmsk, int64_t* ipiv,
                   int64_t* jsk, void* workspace, size_t workspace_bytes, void* stream) {
  if (d < 1) return -2;
  if (ni < 0) return -3;
  if (ldmsk < d) return -4;
  if (ni == 0) return QRCP_OK;
  if (ni > 65536) return QRCP_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < qrcp_lu_workspace_size(d, ni)) return QRCP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Carver c{(char*)workspace};
  double* xw = c.take<double>((size_t)d * ni);
  const size_t rb = lu_records_bytes((int)d, ni);
  uint64_t* rec = c.take<uint64_t>(rb / 8);
  int* status = c.take<int>(4);
  QRCP_TRY(zero_int(status, st));
  QRCP_TRY(launch_lu_pivots(Msk, (int)d, ni, ldmsk, xw, rec, rb, ipiv, jsk, status, st));
  int hs = 0;
  QRCP_TRY(read_back(&hs, status, sizeof(int), st));
  return hs;
}

size_t qrcp_sketch_qr_workspace_size(int64_t d, int64_t ni) {
  if (d < 1 || ni < 0) return 0;
  return sketch_qr_ws_bytes((int)d, ni) + 2 * kAlign + 64;
}

int qrcp_sketch_qr(const double* B, int64_t d, int64_t ni, int64_t ldb, double* R, int64_t ldr,
                   void* workspace, size_t workspace_bytes, void* stream) {
  if (d < 1) return -2;
  if (ni < 0) return -3;
  if (ldb < d) return -4;
  if (ldr < d) return -6;
  if (ni == 0) return QRCP_OK;
  if (!workspace || workspace_bytes < qrcp_sketch_qr_workspace_size(d, ni)) return QRCP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Carver c{(char*)workspace};
  int* status = c.take<int>(4);
  void* ws = c.take<char>(sketch_qr_ws_bytes((int)d, ni));
  QRCP_TRY(zero_int(status, st));
  QRCP_TRY(run_sketch_qr(B, (int)d, ni, ldb, R, ldr, ws, sketch_qr_ws_bytes((int)d, ni), status, st));
  int hs = 0;
  QRCP_TRY(read_back(&hs, status, sizeof(int), st));
  return hs;
}

size_t qrcp_panel_workspace_size(int64_t mi, int64_t k) {
  if (mi < 0 || k < 0) return 0;
  const size_t kk = (size_t)std::max<int64_t>(k, 1);
  return (size_t)mi * kk * 8 * 2 + 6 * kk * kk * 8 + kk * 8 + kSplitBytes + 16 * kAlign;
}

int qrcp_cholqr(double* P, int64_t mi, int64_t k, int64_t ldp, const double* Rs, int64_t ldrs,
                double* Rc, int64_t ldrc, int32_t passes, int64_t* keff, void* workspace,
                size_t workspace_bytes, void* stream) {
  if (mi < 0) return -2;
  if (k < 0 || k > mi) return -3;
  if (ldp < std::max<int64_t>(1, mi)) return -4;
  if (ldrs < std::max<int64_t>(1, k)) return -6;
  if (ldrc < std::max<int64_t>(1, k)) return -8;
  if (passes != 1 && passes != 2) return -9;
  if (!keff) return -10;
  *keff = 0;
  if (k == 0) return QRCP_OK;
  if (k > 1024) return QRCP_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < qrcp_panel_workspace_size(mi, k)) return QRCP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Carver c{(char*)workspace};
  double* Mp = c.take<double>((size_t)mi * k);
  double* Q1 = c.take<double>((size_t)mi * k);
  double* Rinv = c.take<double>((size_t)k * k);
  double* G = c.take<double>((size_t)k * k);
  double* G2 = c.take<double>((size_t)k * k);
  double* Rn = c.take<double>((size_t)k * k);
  int* info = c.take<int>(4);
  double* split = c.take<double>(kSplitBytes / 8);
  const int kk = (int)k;
  QRCP_TRY(launch_trinv_upper(Rs, ldrs, kk, Rinv, k, st));
  QRCP_TRY(gemm(false, false, Prec::F64, ga((int)mi, kk, kk, P, ldp, Rinv, k, Mp, mi), nullptr, 0, st));
  QRCP_TRY(gemm(true, false, Prec::F64, ga(kk, kk, (int)mi, Mp, mi, Mp, mi, G, k), split, kSplitBytes, st));
  QRCP_TRY(launch_potrf_mw(G, k, kk, info, split, kSplitBytes, st));
  int t = 0;
  QRCP_TRY(read_back(&t, info, sizeof(int), st));
  if (t < 0) return QRCP_ERR_TIMEOUT;
  if (t < kk) {
    *keff = t;
    QRCP_TRY(launch_copy2d(G, k, Rc, ldrc, t, t, st));
    QRCP_HIP(hipStreamSynchronize(st));
    return QRCP_OK;
  }
  QRCP_TRY(launch_trinv_upper(G, k, kk, Rinv, k, st));
  if (passes == 2) {
    QRCP_TRY(gemm(false, false, Prec::F64, ga((int)mi, kk, kk, Mp, mi, Rinv, k, Q1, mi), nullptr, 0, st));
    QRCP_TRY(gemm(true, false, Prec::F64, ga(kk, kk, (int)mi, Q1, mi, Q1, mi, G2, k), split, kSplitBytes, st));
    QRCP_TRY(launch_potrf_mw(G2, k, kk, info, split, kSplitBytes, st));
    QRCP_TRY(read_back(&t, info, sizeof(int), st));
    if (t < 0) return QRCP_ERR_TIMEOUT;
    if (t < kk) {
      *keff = t;
      QRCP_TRY(launch_copy2d(G, k, Rc, ldrc, t, t, st));
      QRCP_HIP(hipStreamSynchronize(st));
      return QRCP_OK;
    }
    QRCP_TRY(launch_trinv_upper(G2, k, kk, Rinv, k, st));
    QRCP_TRY(gemm(false, false, Prec::F64, ga((int)mi, kk, kk, Q1, mi, Rinv, k, P, ldp), nullptr, 0, st));
    QRCP_TRY(gemm(false, false, Prec::F64, ga(kk, kk, kk, G2, k, G, k, Rn, k), nullptr, 0, st));
    QRCP_TRY(launch_copy2d(Rn, k, Rc, ldrc, k, k, st));
  } else {
    QRCP_TRY(gemm(false, false, Prec::F64, ga((int)mi, kk, kk, Mp, mi, Rinv, k, P, ldp), nullptr, 0, st));
    QRCP_TRY(launch_copy2d(G, k, Rc, ldrc, k, k, st));
  }
  *keff = k;
  QRCP_HIP(hipStreamSynchronize(st));
  return QRCP_OK;
}

int qrcp_reconstruct(double* Q, int64_t mi, int64_t k, int64_t ldq, double* tau, double* dsig,
                     void* workspace, size_t workspace_bytes, void* stream) {
  if (mi < 0) return -2;
  if (k < 0 || k > mi) return -3;
  if (ldq < std::max<int64_t>(1, mi)) return -4;
  if (k == 0) return QRCP_OK;
  if (k > 1024) return QRCP_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < qrcp_panel_workspace_size(mi, k)) return QRCP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Carver c{(char*)workspace};
  double* Yt = c.take<double>((size_t)mi * k);
  double* Uinv = c.take<double>((size_t)k * k);
  int* stat = c.take<int>(4);
  double* scratch = c.take<double>(kSplitBytes / 8);
  const int kk = (int)k;
  QRCP_TRY(zero_int(stat, st));
  QRCP_TRY(launch_headlu_mw(Q, ldq, kk, dsig, scratch, kSplitBytes, stat, st));
  QRCP_TRY(launch_tau_from_u(Q, ldq, kk, dsig, tau, st));
  QRCP_TRY(launch_trinv_upper(Q, ldq, kk, Uinv, k, st));
  if (mi > k) {
    QRCP_TRY(gemm(false, false, Prec::F64, ga((int)(mi - k), kk, kk, Q + k, ldq, Uinv, k, Yt, mi), nullptr, 0, st));
    QRCP_TRY(launch_copy2d(Yt, mi, Q + k, ldq, mi - k, k, st));
  }
  int fin = QRCP_OK;
  QRCP_TRY(read_back(&fin, stat, sizeof(int), st));
  return fin;
}

size_t qrcp_apply_qt_workspace_size(int64_t mi, int64_t k, int64_t nc) {
  if (mi < 0 || k < 0 || nc < 0) return 0;
  const size_t kk = (size_t)std::max<int64_t>(k, 1);
  return (size_t)mi * kk * 8 + 2 * kk * kk * 8 + 2 * kk * (size_t)std::max<int64_t>(nc, 1) * 8 +
         kSplitBytes + 10 * kAlign;
}

int qrcp_apply_qt(const double* Y, int64_t mi, int64_t k, int64_t ldy, const double* tau,
                  double* C, int64_t nc, int64_t ldc, int32_t precision, void* workspace,
                  size_t workspace_bytes, void* stream) {
  if (mi < 0) return -2;
  if (k < 0 || k > mi) return -3;
  if (ldy < std::max<int64_t>(1, mi)) return -4;
  if (nc < 0) return -7;
  if (ldc < std::max<int64_t>(1, mi)) return -8;
  if (precision != 0 && precision != 1) return -9;
  if (k == 0 || nc == 0) return QRCP_OK;
  if (k > 1024) return QRCP_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < qrcp_apply_qt_workspace_size(mi, k, nc)) return QRCP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Carver c{(char*)workspace};
  double* Yc = c.take<double>((size_t)mi * k);
  double* G = c.take<double>((size_t)k * k);
  double* T = c.take<double>((size_t)k * k);
  double* W = c.take<double>((size_t)k * nc);
  double* W2 = c.take<double>((size_t)k * nc);
  double* split = c.take<double>(kSplitBytes / 8);
  QRCP_TRY(launch_copy2d(Y, ldy, Yc, mi, mi, k, st));
  QRCP_TRY(launch_unit_lower(Y, ldy, (int)k, Yc, mi, st));
  QRCP_TRY(apply_qt_clean(Yc, mi, (int)k, mi, tau, C, nc, ldc, precision ? Prec::F32 : Prec::F64, G,
                          T, k, W, W2, split, kSplitBytes, st));
  QRCP_HIP(hipStreamSynchronize(st));
  return QRCP_OK;
}

int qrcp_sketch_update(double* Rsk, int64_t d, int64_t b, int64_t nt, int64_t ldrsk,
                       const double* R11, int64_t ldr11, const double* R12, int64_t ldr12,
                       void* workspace, size_t workspace_bytes, void* stream) {
  if (d < 1) return -2;
  if (b < 1 || b > d) return -3;
  if (nt < 0) return -4;
  if (ldrsk < d) return -5;
  if (ldr11 < b) return -7;
  if (ldr12 < b) return -9;
  if (nt == 0) return QRCP_OK;
  if (b > 1024) return QRCP_ERR_UNSUPPORTED;
  const size_t need = 2 * (size_t)b * b * 8 + 4 * kAlign;
  if (!workspace || workspace_bytes < need) return QRCP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Carver c{(char*)workspace};
  double* Rinv = c.take<double>((size_t)b * b);
  double* X = c.take<double>((size_t)b * b);
  const int bb = (int)b;
  QRCP_TRY(launch_trinv_upper(R11, ldr11, bb, Rinv, b, st));
  QRCP_TRY(gemm(false, false, Prec::F64, ga(bb, bb, bb, Rsk, ldrsk, Rinv, b, X, b), nullptr, 0, st));
  QRCP_TRY(gemm(false, false, Prec::F64,
                ga(bb, (int)nt, bb, X, b, R12, ldr12, Rsk + b * ldrsk, ldrsk, -1.0, 1.0), nullptr, 0, st));
  QRCP_HIP(hipStreamSynchronize(st));
  return QRCP_OK;
}

int qrcp_sketch_update_chol(double* Rsk, int64_t d, int64_t b, int64_t nt, int64_t ldrsk,
                            const double* Rc, int64_t ldrc, const double* dsig, const double* R12,
                            int64_t ldr12, void* workspace, size_t workspace_bytes, void* stream) {
  if (d < 1) return -2;
  if (b < 1 || b > d) return -3;
  if (nt < 0) return -4;
  if (ldrsk < d) return -5;
  if (ldrc < b) return -7;
  if (ldr12 < b) return -10;
  if (nt == 0) return QRCP_OK;
  if (b > 1024) return QRCP_ERR_UNSUPPORTED;
  const size_t need = 2 * (size_t)b * b * 8 + 4 * kAlign;
  if (!workspace || workspace_bytes < need) return QRCP_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Carver c{(char*)workspace};
  double* Rinv = c.take<double>((size_t)b * b);
  double* X = c.take<double>((size_t)b * b);
  const int bb = (int)b;
  // the kernels of qrcp_factor's one-pass sample update: X = Rc^{-1} diag(D)
  QRCP_TRY(launch_trinv_upper(Rc, ldrc, bb, Rinv, b, st));
  QRCP_TRY(launch_scale_upper_cols(Rinv, b, dsig, bb, X, b, st));
  QRCP_TRY(gemm(false, false, Prec::F64,
                ga(bb, (int)nt, bb, X, b, R12, ldr12, Rsk + b * ldrsk, ldrsk, -1.0, 1.0), nullptr, 0, st));
  QRCP_HIP(hipStreamSynchronize(st));
  return QRCP_OK;
}

// ----------------------------------------------------------------------------
// Stage timing
// ----------------------------------------------------------------------------
int qrcp_profile_enable(int32_t mode) {
  if (mode < 0 || mode > 2) return -1;
  g_prof.mode = mode;
  g_prof.recs.clear();
  g_prof.used = 0;
  return QRCP_OK;
}

int32_t qrcp_profile_num_stages(void) { return kNumStages; }

const char* qrcp_profile_stage_name(int32_t stage) {
  return (stage >= 0 && stage < kNumStages) ? kStageNames[stage] : "";
}

int qrcp_profile_read(int32_t stage, double* ms, int64_t* count, double* flops) {
  if (stage < 0 || stage >= kNumStages) return -1;
  double t = 0.0, f = 0.0;
  int64_t c = 0;
  for (auto& r : g_prof.recs) {
    if (r.stage != stage) continue;
    QRCP_HIP(hipEventSynchronize(r.b));
    float e = 0.f;
    QRCP_HIP(hipEventElapsedTime(&e, r.a, r.b));
    t += e;
    f += r.flops;
    ++c;
  }
  if (ms) *ms = t;
  if (count) *count = c;
  if (flops) *flops = f;
  return QRCP_OK;
}

}  // extern "C"
