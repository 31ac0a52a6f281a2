// Column bookkeeping of the QRCP loop.
//
// The paper permutes all trailing columns of M by J^sk at every block (Alg. 1
// permutation steps; Alg. 5 on the GPU, with a full copy of M).  Here columns
// move lazily: a map phys[pos] gives the physical column holding logical
// position pos.  Per block only the k_max panel columns are placed at their
// final physical positions s..c-1 (all m rows, so the R entries of earlier
// blocks travel with them); the columns they displace move into the vacated
// slots.  Columns never placed (the residual block after an early stop) are
// put in logical order by one final pass.  The sketch itself (d rows) is
// permuted eagerly, since it is small and the LU needs logical positions for
// its tie-break.
#include "common.hpp"
#include "kernels.hpp"

namespace qrcp {

// plan layout: plan[0] = nD; plan[8 + t] = source column of panel slot t;
// plan[8 + kmax + q] = displaced slot D[q]; plan[8 + 2 kmax + q] = free slot F[q].
__global__ __launch_bounds__(1024) void perm_plan_kernel(Gate gt, const long* jsk, long s, long n, int kmax,
                                                        const long* J0, long* J1,
                                                        const long* phys0, long* phys1, long* inv,
                                                        long* plan) {
  QRCP_GATE(gt);
  extern __shared__ long sm[];
  long* src = sm;              // kmax: physical column of panel slot t
  long* dsl = src + kmax;      // kmax: displaced slots, in increasing order
  long* fsl = dsl + kmax;      // kmax: free slots, in panel-slot order
  int* mark = (int*)(fsl + kmax);
  __shared__ int wcnt[2][16];
  __shared__ int base[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long ni = n - s;
  const long c = s + kmax;
  for (long p = tid; p < s; p += blockDim.x) {
    J1[p] = J0[p];
    phys1[p] = phys0[p];
  }
  for (long t = tid; t < ni; t += blockDim.x) {
    const long from = s + jsk[t];
    J1[s + t] = J0[from];
    phys1[s + t] = phys0[from];
  }
  __syncthreads();
  for (long p = s + tid; p < n; p += blockDim.x) inv[phys1[p]] = p;
  for (int t = tid; t < kmax; t += blockDim.x) mark[t] = 0;
  if (tid == 0) base[0] = base[1] = 0;
  __syncthreads();
  for (int t = tid; t < kmax; t += blockDim.x) {
    src[t] = phys1[s + t];
    plan[8 + t] = src[t];
    if (src[t] < c) mark[src[t] - s] = 1;
  }
  __syncthreads();
  // stable compactions (ballot ranks within a wave, wave counts through LDS):
  // D = unmarked panel slots in increasing order, F = sources beyond the panel
  // in panel-slot order
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int x0 = 0; x0 < kmax; x0 += blockDim.x) {
    const int x = x0 + tid;
    const bool fd = x < kmax && !mark[x];
    const bool ff = x < kmax && src[x] >= c;
    const unsigned long long bd = __ballot(fd), bf = __ballot(ff);
    if (lane == 0) {
      wcnt[0][wave] = __popcll(bd);
      wcnt[1][wave] = __popcll(bf);
    }
    __syncthreads();
    int od = base[0], of = base[1];
    for (int w = 0; w < wave; ++w) {
      od += wcnt[0][w];
      of += wcnt[1][w];
    }
    if (fd) dsl[od + __popcll(bd & below)] = s + x;
    if (ff) fsl[of + __popcll(bf & below)] = src[x];
    __syncthreads();
    if (tid == 0) {
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        base[0] += wcnt[0][w];
        base[1] += wcnt[1][w];
      }
    }
    __syncthreads();
  }
  const int nd = base[0];  // equals the number of free slots
  if (tid == 0) plan[0] = nd;
  // displaced logical columns take the free slots; the displaced slots lie in
  // [s, c) and the free ones at c or beyond, so the pairs are independent
  for (int q = tid; q < nd; q += blockDim.x) {
    const long dslot = dsl[q], fslot = fsl[q];
    plan[8 + kmax + q] = dslot;
    plan[8 + 2 * kmax + q] = fslot;
    const long lg = inv[dslot];
    phys1[lg] = fslot;
    inv[fslot] = lg;
  }
  __syncthreads();
  for (int t = tid; t < kmax; t += blockDim.x) {
    phys1[s + t] = s + t;
    inv[s + t] = s + t;
  }
  // one more map update: the live maps alternate between the two buffers
  if (tid == 0 && gt.ctl) const_cast<LoopCtl*>(gt.ctl)->perms += 1;
}

int launch_perm_plan(const i64* jsk, i64 s, i64 n, int kmax, const i64* J0, i64* J1,
                     const i64* phys0, i64* phys1, i64* inv, i64* plan, hipStream_t st) {
  const size_t smem = (size_t)kmax * 8 * 3 + (size_t)kmax * 4 + 16;
  if (smem > 64 * 1024) return QRCP_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(perm_plan_kernel, dim3(1), dim3(1024), smem, st, current_gate(), (const long*)jsk, s, n, kmax,
                     (const long*)J0, (long*)J1, (const long*)phys0, (long*)phys1, (long*)inv,
                     (long*)plan);
  QRCP_LAUNCHED("perm_plan");
  return QRCP_OK;
}

// dst(:, t) = src(:, jsk[t]) for t < ni (d rows, same leading dimension)
__global__ void sketch_permute_kernel(Gate gt, const double* src, double* dst, int d, long ld, long ni,
                                      const long* jsk) {
  QRCP_GATE(gt);
  const long t = blockIdx.x;
  if (t >= ni) return;
  const double* a = src + jsk[t] * ld;
  double* b = dst + t * ld;
  for (int r = threadIdx.x; r < d; r += blockDim.x) b[r] = a[r];
}

int launch_sketch_permute(const double* src, double* dst, int d, i64 ld, i64 ni, const i64* jsk,
                          hipStream_t st) {
  if (ni <= 0) return QRCP_OK;
  hipLaunchKernelGGL(sketch_permute_kernel, dim3(ni), dim3(128), 0, st, current_gate(), src, dst, d, ld, ni,
                     (const long*)jsk);
  QRCP_LAUNCHED("sketch_permute");
  return QRCP_OK;
}

// column copies driven by the plan; grid.y = column slot, grid.x = row blocks
__global__ void place_gather_kernel(Gate gt, const double* A, long lda, long m, int kmax, const long* plan,
                                    double* tmp, long ldt) {
  QRCP_GATE(gt);
  const int t = blockIdx.y;
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r >= m) return;
  tmp[r + t * ldt] = A[r + plan[8 + t] * lda];
}

__global__ void place_displace_kernel(Gate gt, double* A, long lda, long m, int kmax, const long* plan) {
  QRCP_GATE(gt);
  const int q = blockIdx.y;
  if (q >= plan[0]) return;
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r >= m) return;
  const long dslot = plan[8 + kmax + q], fslot = plan[8 + 2 * kmax + q];
  A[r + fslot * lda] = A[r + dslot * lda];
}

__global__ void place_scatter_kernel(Gate gt, double* A, long lda, long m, long s, const double* tmp,
                                     long ldt) {
  QRCP_GATE(gt);
  const int t = blockIdx.y;
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r >= m) return;
  A[r + (s + t) * lda] = tmp[r + t * ldt];
}

int launch_place_columns(double* A, i64 lda, i64 m, i64 s, int kmax, const i64* plan, double* tmp,
                         i64 ldt, hipStream_t st) {
  if (kmax <= 0 || m <= 0) return QRCP_OK;
  dim3 grid((m + 255) / 256, kmax);
  hipLaunchKernelGGL(place_gather_kernel, grid, dim3(256), 0, st, current_gate(), A, lda, m, kmax,
                     (const long*)plan, tmp, ldt);
  hipLaunchKernelGGL(place_displace_kernel, grid, dim3(256), 0, st, current_gate(), A, lda, m, kmax,
                     (const long*)plan);
  hipLaunchKernelGGL(place_scatter_kernel, grid, dim3(256), 0, st, current_gate(), A, lda, m, s, tmp, ldt);
  QRCP_LAUNCHED("place_columns");
  return QRCP_OK;
}

__global__ void final_gather_kernel(Gate gt, const double* A, long lda, long m, long l, const long* phys,
                                    double* tmp) {
  QRCP_GATE(gt);
  const long t = blockIdx.y;
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r >= m) return;
  tmp[r + t * m] = A[r + phys[l + t] * lda];
}

__global__ void final_scatter_kernel(Gate gt, double* A, long lda, long m, long l, const double* tmp) {
  QRCP_GATE(gt);
  const long t = blockIdx.y;
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r >= m) return;
  A[r + (l + t) * lda] = tmp[r + t * m];
}

int launch_final_permute(double* A, i64 lda, i64 m, i64 l, i64 n, const i64* phys, double* tmp,
                         hipStream_t st) {
  const i64 cnt = n - l;
  if (cnt <= 0 || m <= 0) return QRCP_OK;
  for (i64 c0 = 0; c0 < cnt; c0 += 65535) {
    const i64 cc = std::min<i64>(65535, cnt - c0);
    dim3 grid((m + 255) / 256, cc);
    hipLaunchKernelGGL(final_gather_kernel, grid, dim3(256), 0, st, current_gate(), A, lda, m, l + c0,
                       (const long*)phys, tmp + c0 * m);
  }
  for (i64 c0 = 0; c0 < cnt; c0 += 65535) {
    const i64 cc = std::min<i64>(65535, cnt - c0);
    dim3 grid((m + 255) / 256, cc);
    hipLaunchKernelGGL(final_scatter_kernel, grid, dim3(256), 0, st, current_gate(), A, lda, m, l + c0,
                       tmp + c0 * m);
  }
  QRCP_LAUNCHED("final_permute");
  return QRCP_OK;
}

__global__ void jpiv_out_kernel(Gate gt, const long* J, long n, long base, long* out) {
  QRCP_GATE(gt);
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) out[i] = J[i] + base;
}

int launch_jpiv_out(const i64* J, i64 n, i64 base, i64* out, hipStream_t st) {
  if (n <= 0) return QRCP_OK;
  hipLaunchKernelGGL(jpiv_out_kernel, dim3((n + 255) / 256), dim3(256), 0, st, current_gate(), (const long*)J, n,
                     base, (long*)out);
  QRCP_LAUNCHED("jpiv_out");
  return QRCP_OK;
}

__global__ void iota_kernel(Gate gt, long* x, long n) {
  QRCP_GATE(gt);
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) x[i] = i;
}

int launch_iota(i64* x, i64 n, hipStream_t st) {
  if (n <= 0) return QRCP_OK;
  hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, st, current_gate(), (long*)x, n);
  QRCP_LAUNCHED("iota");
  return QRCP_OK;
}

}  // namespace qrcp
