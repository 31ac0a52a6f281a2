// Small per-block kernels of the QRCP loop: the reference scale of the rank
// test, tri_rank, masking by the device-side block rank, and the clean copy
// of the reflector block.
#include <algorithm>
#include <climits>

#include "common.hpp"
#include "kernels.hpp"
#include "steps.hpp"

namespace qrcp {

// colss[j] = sum_i X(i,j)^2 (one wave per column)
__global__ void colss_kernel(Gate gt, const double* X, long ld, int rows, long cols, double* colss) {
  QRCP_GATE(gt);
  const long j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= cols) return;
  double s = 0.0;
  for (int i = lane; i < rows; i += 64) {
    const double v = X[i + j * ld];
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) colss[j] = s;
}

// ref = sqrt(max_j colss[j]) by one workgroup, fixed order
__global__ __launch_bounds__(1024) void ref_kernel(Gate gt, const double* colss, long cols, double* ref) {
  QRCP_GATE(gt);
  __shared__ double red[16];
  double m = 0.0;
  for (long j = threadIdx.x; j < cols; j += blockDim.x) m = fmax(m, colss[j]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, red[i]);
    *ref = sqrt(r);
  }
}

int launch_sketch_ref(const double* X, i64 ld, int rows, i64 cols, double* colss, double* ref,
                      hipStream_t st) {
  if (cols <= 0) {
    hipLaunchKernelGGL(ref_kernel, dim3(1), dim3(1024), 0, st, current_gate(), colss, 0, ref);
    QRCP_LAUNCHED("ref");
    return QRCP_OK;
  }
  hipLaunchKernelGGL(colss_kernel, dim3((cols + 3) / 4), dim3(256), 0, st, current_gate(), X, ld, rows, cols,
                     colss);
  hipLaunchKernelGGL(ref_kernel, dim3(1), dim3(1024), 0, st, current_gate(), colss, cols, ref);
  QRCP_LAUNCHED("sketch_ref");
  return QRCP_OK;
}

// k = first t < kmax with !(|R(t,t)| > tol * ref) (NaN fails), else kmax
__global__ __launch_bounds__(256) void trirank_kernel(Gate gt, const double* R, long ldr, int kmax,
                                                      double tol, const double* ref, int* kdev) {
  QRCP_GATE(gt);
  __shared__ int kmin;
  if (threadIdx.x == 0) kmin = kmax;
  __syncthreads();
  const double thr = tol * (*ref);
  for (int t = threadIdx.x; t < kmax; t += blockDim.x) {
    const double v = fabs(R[t + (long)t * ldr]);
    if (!(v > thr)) atomicMin(&kmin, t);
  }
  __syncthreads();
  if (threadIdx.x == 0) *kdev = kmin;
}

int launch_trirank(const double* R, i64 ldr, int kmax, double tol, const double* ref, int* kdev,
                   hipStream_t st) {
  hipLaunchKernelGGL(trirank_kernel, dim3(1), dim3(256), 0, st, current_gate(), R, ldr, kmax, tol, ref, kdev);
  QRCP_LAUNCHED("trirank");
  return QRCP_OK;
}

// X(i,j) = 0 when i >= k or j >= k (k read from the device)
__global__ void mask_k_kernel(Gate gt, double* X, long ld, int n, const int* kdev) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)n * n) return;
  const int i = idx % n, j = idx / n;
  const int k = *kdev;
  if (i >= k || j >= k) X[i + (long)j * ld] = 0.0;
}

int launch_mask_k(double* X, i64 ld, int n, const int* kdev, hipStream_t st) {
  if (n <= 0) return QRCP_OK;
  hipLaunchKernelGGL(mask_k_kernel, dim3(((long)n * n + 255) / 256), dim3(256), 0, st, current_gate(), X, ld, n,
                     kdev);
  QRCP_LAUNCHED("mask_k");
  return QRCP_OK;
}

// Clean reflector block: Y(0:k, 0:k) = unit lower part of the head H (strictly
// lower entries of H, ones on the diagonal, zeros above).
__global__ void unit_lower_kernel(Gate gt, const double* H, long ldh, int k, double* Y, long ldy) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)k * k) return;
  const int i = idx % k, j = idx / k;
  Y[i + (long)j * ldy] = (i > j) ? H[i + (long)j * ldh] : (i == j ? 1.0 : 0.0);
}

int launch_unit_lower(const double* H, i64 ldh, int k, double* Y, i64 ldy, hipStream_t st) {
  if (k <= 0) return QRCP_OK;
  hipLaunchKernelGGL(unit_lower_kernel, dim3(((long)k * k + 255) / 256), dim3(256), 0, st, current_gate(), H, ldh,
                     k, Y, ldy);
  QRCP_LAUNCHED("unit_lower");
  return QRCP_OK;
}

// ---------------------------------------------------------------------------
// Control of the device-driven block loop (LoopCtl in common.hpp).
// ---------------------------------------------------------------------------
__global__ void loop_init_kernel(LoopCtl* ctl) {
  ctl->nblk = INT_MAX;
  ctl->exit_blk = -1;
  ctl->k = 0;
  ctl->status = QRCP_OK;
  ctl->ell = 0;
  ctl->perms = 0;
  ctl->kmax = 0;
}

// After block blk's panel factorization: the block's effective width k (the
// Cholesky QR's count of factored columns, or tri_rank's for the Householder
// panel), errors, and whether the loop stops at this block.
// host_nblk (may be null): a word in pinned host memory that the blocking
// form polls to stop enqueueing blocks once the loop has stopped
__global__ void loop_decide_kernel(Gate gt, LoopCtl* ctl, const int* status, const int* kdev, int blk,
                                   int kmax, long s, long c, long lim, int second, int* host_nblk) {
  QRCP_GATE(gt);
  const int st = *status;
  const int k = *kdev;
  if (st != QRCP_OK || k < 0) {
    ctl->status = st != QRCP_OK ? st : QRCP_ERR_TIMEOUT;
    ctl->nblk = blk;
    ctl->exit_blk = -1;
    ctl->ell = s;
  } else {
    // the second Cholesky pass can only shrink the width found by the first
    const int kk = second ? min(k, ctl->k) : k;
    ctl->k = kk;
    ctl->kmax = kmax;
    if (kk < kmax || c >= lim) {
      ctl->exit_blk = blk;
      ctl->nblk = blk + 1;
      ctl->ell = s + kk;
    } else {
      ctl->ell = c;
    }
  }
  if (host_nblk && ctl->nblk != INT_MAX)
    __hip_atomic_store(host_nblk, ctl->nblk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// X(i, j) = delta_ij wherever i or j >= k (the trailing part of a factor
// beyond the block's width becomes the identity)
__global__ void pad_identity_kernel(Gate gt, double* X, long ld, int n, const int* kdev) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)n * n) return;
  const int i = idx % n, j = idx / n;
  const int k = *kdev;
  if (i >= k || j >= k) X[i + (long)j * ld] = (i == j) ? 1.0 : 0.0;
}

// v[j] = 0 for k <= j < n
__global__ void zero_tail_kernel(Gate gt, double* v, int n, const int* kdev) {
  QRCP_GATE(gt);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n && j >= *kdev) v[j] = 0.0;
}

// dst(:, j) = src(:, j) for the columns k <= j < cols
__global__ void copy_cols_from_kernel(Gate gt, const double* src, long lds, double* dst, long ldd,
                                      long rows, int cols, const int* kdev) {
  QRCP_GATE(gt);
  const int j = blockIdx.y;
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= cols || j < *kdev || r >= rows) return;
  dst[r + j * ldd] = src[r + j * lds];
}

// the live column maps (index perms % 2) moved into slot 0
__global__ void pick_maps_kernel(const LoopCtl* ctl, long* J0, const long* J1, long* P0,
                                 const long* P1, long n) {
  if (!(ctl->perms & 1)) return;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    J0[i] = J1[i];
    P0[i] = P1[i];
  }
}

// tau(ell : mn) = 0 after a successful run
__global__ void tau_tail_kernel(const LoopCtl* ctl, double* tau, long mn) {
  if (ctl->status != QRCP_OK) return;
  for (long i = ctl->ell + blockIdx.x * (long)blockDim.x + threadIdx.x; i < mn;
       i += (long)gridDim.x * blockDim.x)
    tau[i] = 0.0;
}

// the physical columns ell .. n-1 put in logical order: gather into tmp, then
// scatter back (two launches, grid-stride over the columns the loop did not
// place)
__global__ void final_gather_dyn_kernel(const LoopCtl* ctl, const double* A, long lda, long m, long n,
                                        const long* phys, double* tmp) {
  if (ctl->status != QRCP_OK) return;
  const long l = ctl->ell;
  for (long t = l + blockIdx.y; t < n; t += gridDim.y)
    for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < m; r += (long)gridDim.x * blockDim.x)
      tmp[r + (t - l) * m] = A[r + phys[t] * lda];
}

__global__ void final_scatter_dyn_kernel(const LoopCtl* ctl, double* A, long lda, long m, long n,
                                         const double* tmp) {
  if (ctl->status != QRCP_OK) return;
  const long l = ctl->ell;
  for (long t = l + blockIdx.y; t < n; t += gridDim.y)
    for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < m; r += (long)gridDim.x * blockDim.x)
      A[r + t * lda] = tmp[r + (t - l) * m];
}

// rank and status of the call into the caller's device words (a wait that
// timed out after the block loop's last check reports itself here)
__global__ void loop_finish_kernel(const LoopCtl* ctl, const int* status, i64* rank_dev,
                                   int* status_dev) {
  if (rank_dev) *rank_dev = ctl->ell;
  if (status_dev) *status_dev = ctl->status != QRCP_OK ? ctl->status : *status;
}

int launch_loop_init(LoopCtl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(loop_init_kernel, dim3(1), dim3(1), 0, st, ctl);
  QRCP_LAUNCHED("loop_init");
  return QRCP_OK;
}

int launch_loop_decide(LoopCtl* ctl, const int* status, const int* kdev, int blk, int kmax, i64 s,
                       i64 c, i64 lim, bool second, int* host_nblk, hipStream_t st) {
  hipLaunchKernelGGL(loop_decide_kernel, dim3(1), dim3(1), 0, st, current_gate(), ctl, status, kdev,
                     blk, kmax, (long)s, (long)c, (long)lim, second ? 1 : 0, host_nblk);
  QRCP_LAUNCHED("loop_decide");
  return QRCP_OK;
}

int launch_pad_identity(double* X, i64 ld, int n, const int* kdev, hipStream_t st) {
  if (n <= 0) return QRCP_OK;
  hipLaunchKernelGGL(pad_identity_kernel, dim3(((long)n * n + 255) / 256), dim3(256), 0, st,
                     current_gate(), X, ld, n, kdev);
  QRCP_LAUNCHED("pad_identity");
  return QRCP_OK;
}

int launch_zero_tail(double* v, int n, const int* kdev, hipStream_t st) {
  if (n <= 0) return QRCP_OK;
  hipLaunchKernelGGL(zero_tail_kernel, dim3((n + 255) / 256), dim3(256), 0, st, current_gate(), v, n,
                     kdev);
  QRCP_LAUNCHED("zero_tail");
  return QRCP_OK;
}

int launch_copy_cols_from(const double* src, i64 lds, double* dst, i64 ldd, i64 rows, int cols,
                          const int* kdev, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return QRCP_OK;
  hipLaunchKernelGGL(copy_cols_from_kernel, dim3((rows + 255) / 256, cols), dim3(256), 0, st,
                     current_gate(), src, lds, dst, ldd, rows, cols, kdev);
  QRCP_LAUNCHED("copy_cols_from");
  return QRCP_OK;
}

int launch_loop_pick(const LoopCtl* ctl, i64* J0, const i64* J1, i64* P0, const i64* P1, i64 n,
                     hipStream_t st) {
  hipLaunchKernelGGL(pick_maps_kernel, dim3(64), dim3(256), 0, st, ctl, (long*)J0, (const long*)J1,
                     (long*)P0, (const long*)P1, (long)n);
  QRCP_LAUNCHED("loop_pick");
  return QRCP_OK;
}

int launch_loop_final(const LoopCtl* ctl, double* A, i64 lda, i64 m, i64 n, const i64* P0,
                      double* tau, i64 mn, double* tmp, const int* status, i64* rank_dev,
                      int* status_dev, hipStream_t st) {
  if (mn > 0)
    hipLaunchKernelGGL(tau_tail_kernel, dim3(16), dim3(256), 0, st, ctl, tau, (long)mn);
  if (m > 0) {
    const dim3 grid((unsigned)std::min<i64>((m + 255) / 256, 16), (unsigned)std::min<i64>(n, 4096));
    hipLaunchKernelGGL(final_gather_dyn_kernel, grid, dim3(256), 0, st, ctl, (const double*)A,
                       (long)lda, (long)m, (long)n, (const long*)P0, tmp);
    hipLaunchKernelGGL(final_scatter_dyn_kernel, grid, dim3(256), 0, st, ctl, A, (long)lda, (long)m,
                       (long)n, (const double*)tmp);
  }
  hipLaunchKernelGGL(loop_finish_kernel, dim3(1), dim3(1), 0, st, ctl, status, rank_dev, status_dev);
  QRCP_LAUNCHED("loop_final");
  return QRCP_OK;
}

__global__ void set_result_kernel(i64* rank_dev, int* status_dev) {
  if (rank_dev) *rank_dev = 0;
  if (status_dev) *status_dev = QRCP_OK;
}

__global__ void copy_result_kernel(const i64* rank_dev, const int* status_dev, CallResult* out) {
  out->rank = rank_dev ? *rank_dev : 0;
  out->status = status_dev ? *status_dev : QRCP_OK;
}

int launch_set_result(i64* rank_dev, int* status_dev, hipStream_t st) {
  hipLaunchKernelGGL(set_result_kernel, dim3(1), dim3(1), 0, st, rank_dev, status_dev);
  QRCP_LAUNCHED("set_result");
  return QRCP_OK;
}

int launch_copy_result(const i64* rank_dev, const int* status_dev, CallResult* out, hipStream_t st) {
  hipLaunchKernelGGL(copy_result_kernel, dim3(1), dim3(1), 0, st, rank_dev, status_dev, out);
  QRCP_LAUNCHED("copy_result");
  return QRCP_OK;
}

}  // namespace qrcp
