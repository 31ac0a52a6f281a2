// Small per-block kernels of the QRCP loop: the reference scale of the rank
// test, tri_rank, masking by the device-side block rank, and the clean copy
// of the reflector block.
#include "common.hpp"
#include "kernels.hpp"
#include "steps.hpp"

namespace qrcp {

// colss[j] = sum_i X(i,j)^2 (one wave per column)
__global__ void colss_kernel(const double* X, long ld, int rows, long cols, double* colss) {
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
__global__ __launch_bounds__(1024) void ref_kernel(const double* colss, long cols, double* ref) {
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
    hipLaunchKernelGGL(ref_kernel, dim3(1), dim3(1024), 0, st, colss, 0, ref);
    QRCP_LAUNCHED("ref");
    return QRCP_OK;
  }
  hipLaunchKernelGGL(colss_kernel, dim3((cols + 3) / 4), dim3(256), 0, st, X, ld, rows, cols,
                     colss);
  hipLaunchKernelGGL(ref_kernel, dim3(1), dim3(1024), 0, st, colss, cols, ref);
  QRCP_LAUNCHED("sketch_ref");
  return QRCP_OK;
}

// k = first t < kmax with !(|R(t,t)| > tol * ref) (NaN fails), else kmax
__global__ __launch_bounds__(256) void trirank_kernel(const double* R, long ldr, int kmax,
                                                      double tol, const double* ref, int* kdev) {
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
  hipLaunchKernelGGL(trirank_kernel, dim3(1), dim3(256), 0, st, R, ldr, kmax, tol, ref, kdev);
  QRCP_LAUNCHED("trirank");
  return QRCP_OK;
}

// X(i,j) = 0 when i >= k or j >= k (k read from the device)
__global__ void mask_k_kernel(double* X, long ld, int n, const int* kdev) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)n * n) return;
  const int i = idx % n, j = idx / n;
  const int k = *kdev;
  if (i >= k || j >= k) X[i + (long)j * ld] = 0.0;
}

int launch_mask_k(double* X, i64 ld, int n, const int* kdev, hipStream_t st) {
  if (n <= 0) return QRCP_OK;
  hipLaunchKernelGGL(mask_k_kernel, dim3(((long)n * n + 255) / 256), dim3(256), 0, st, X, ld, n,
                     kdev);
  QRCP_LAUNCHED("mask_k");
  return QRCP_OK;
}

// Clean reflector block: Y(0:k, 0:k) = unit lower part of the head H (strictly
// lower entries of H, ones on the diagonal, zeros above).
__global__ void unit_lower_kernel(const double* H, long ldh, int k, double* Y, long ldy) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)k * k) return;
  const int i = idx % k, j = idx / k;
  Y[i + (long)j * ldy] = (i > j) ? H[i + (long)j * ldh] : (i == j ? 1.0 : 0.0);
}

int launch_unit_lower(const double* H, i64 ldh, int k, double* Y, i64 ldy, hipStream_t st) {
  if (k <= 0) return QRCP_OK;
  hipLaunchKernelGGL(unit_lower_kernel, dim3(((long)k * k + 255) / 256), dim3(256), 0, st, H, ldh,
                     k, Y, ldy);
  QRCP_LAUNCHED("unit_lower");
  return QRCP_OK;
}

}  // namespace qrcp
