// Column-pivoted Householder QR of the sketch (GEQP3 semantics): the
// alternative wide QRCP of the method (Sec. 2.1; Alg. 2 is the LU-based one).
// Businger-Golub pivoting: at step j the column of largest norm over rows
// j..d-1 among columns j..n_i-1 moves to position j (ties to the smallest
// position); the norms are recomputed exactly after every step (no
// downdating); the reflectors follow LAPACK's DLARFG convention
// (beta = -sign(alpha) ||[alpha; x]||, sign(0) = +1, tau = 0 when x = 0).
//
// The d x n_i sketch (d <= 1024) is worked on in place in a column-major copy.
// Per step two launches:
//  * update: reflector j-1 applied to every later column and the column's norm
//    over rows j.. formed from the updated values in the same pass (a wave per
//    column: one read and one write of the column), with a per-workgroup
//    arg-max of the norms;
//  * pivot: one workgroup reduces the arg-max, swaps the pivot column (and its
//    index) into position j and builds reflector j in place (v below the
//    diagonal, beta on it, tau aside).
// Only the first `psteps` steps pivot (the rest keep the column order); the
// upper trapezoid of the result is R^sk.
#include <cfloat>

#include "common.hpp"
#include "kernels.hpp"

namespace qrcp {
namespace {

constexpr int NT = 256;
constexpr int kWavesPerGroup = NT / 64;
constexpr int kMaxParts = 1024;

// a beats b: larger norm, or the same norm at a smaller position
__device__ __forceinline__ bool beats(double va, long ia, double vb, long ib) {
  return ib < 0 || (ia >= 0 && (va > vb || (va == vb && ia < ib)));
}

__global__ __launch_bounds__(NT) void geqp3_update_kernel(Gate gt, double* X, long ld, int d, long ni,
                                                          int refl, const double* tau, long c0,
                                                          double* part_v, long* part_i,
                                                          int* status) {
  QRCP_GATE(gt);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long nw = (long)gridDim.x * kWavesPerGroup;
  const int r0 = refl + 1;  // the norms are over rows r0 .. d-1
  const double t = refl >= 0 ? tau[refl] : 0.0;
  const double* v = X + (long)(refl >= 0 ? refl : 0) * ld;
  double bv = 0.0;
  long bi = -1;
  bool bad = false;
  for (long c = c0 + (long)blockIdx.x * kWavesPerGroup + wave; c < ni; c += nw) {
    double* col = X + c * ld;
    double ss = 0.0;
    if (refl >= 0 && t != 0.0) {
      // w = v^T x over rows refl .. d-1 (v(refl) = 1), then x -= tau w v
      double w = 0.0;
      for (int r = refl + lane; r < d; r += 64) w += (r == refl ? 1.0 : v[r]) * col[r];
      w = wave_sum(w);
      const double tw = t * w;
      for (int r = refl + lane; r < d; r += 64) {
        const double x = col[r] - tw * (r == refl ? 1.0 : v[r]);
        col[r] = x;
        if (r >= r0) ss += x * x;
      }
    } else {
      for (int r = (r0 > 0 ? r0 : 0) + lane; r < d; r += 64) {
        const double x = col[r];
        ss += x * x;
      }
    }
    ss = wave_sum(ss);
    const double nrm = sqrt(ss);
    if (!(nrm <= DBL_MAX)) bad = true;
    if (beats(nrm, c, bv, bi)) {
      bv = nrm;
      bi = c;
    }
  }
  if (bad && lane == 0) store_agent_i32(status, QRCP_ERR_NONFINITE);
  __shared__ double sv[kWavesPerGroup];
  __shared__ long si[kWavesPerGroup];
  if (lane == 0) {
    sv[wave] = bv;
    si[wave] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v0 = sv[0];
    long i0 = si[0];
    for (int w2 = 1; w2 < kWavesPerGroup; ++w2)
      if (beats(sv[w2], si[w2], v0, i0)) {
        v0 = sv[w2];
        i0 = si[w2];
      }
    part_v[blockIdx.x] = v0;
    part_i[blockIdx.x] = i0;
  }
}

__global__ __launch_bounds__(NT) void geqp3_pivot_kernel(Gate gt, double* X, long ld, int d, int j, int pivot,
                                                         const double* part_v, const long* part_i,
                                                         int nparts, i64* jsk, double* tau) {
  QRCP_GATE(gt);
  __shared__ double sv[NT];
  __shared__ long si[NT];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  long p = j;
  if (pivot) {
    double bv = 0.0;
    long bi = -1;
    for (int q = tid; q < nparts; q += NT)
      if (beats(part_v[q], part_i[q], bv, bi)) {
        bv = part_v[q];
        bi = part_i[q];
      }
    sv[tid] = bv;
    si[tid] = bi;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (tid < o && beats(sv[tid + o], si[tid + o], sv[tid], si[tid])) {
        sv[tid] = sv[tid + o];
        si[tid] = si[tid + o];
      }
      __syncthreads();
    }
    p = si[0] >= 0 ? si[0] : j;
  }
  double* cj = X + (long)j * ld;
  if (p != j) {
    double* cp = X + p * ld;
    for (int r = tid; r < d; r += NT) {
      const double a = cj[r];
      cj[r] = cp[r];
      cp[r] = a;
    }
    if (tid == 0) {
      const i64 a = jsk[j];
      jsk[j] = jsk[p];
      jsk[p] = a;
    }
  }
  __syncthreads();
  // reflector j from column j, rows j .. d-1
  double xs = 0.0;
  for (int r = j + 1 + tid; r < d; r += NT) xs += cj[r] * cj[r];
  const double xx = block_sum<NT>(xs, red);
  const double alpha = cj[j];
  if (xx == 0.0) {
    if (tid == 0) tau[j] = 0.0;
    return;
  }
  const double beta = -copysign(sqrt(alpha * alpha + xx), alpha != 0.0 ? alpha : 1.0);
  const double den = alpha - beta;
  for (int r = j + 1 + tid; r < d; r += NT) cj[r] = cj[r] / den;
  if (tid == 0) {
    tau[j] = (beta - alpha) / beta;
    cj[j] = beta;
  }
}

int parts_for(long cols) {
  const long g = (cols + kWavesPerGroup - 1) / kWavesPerGroup;
  return (int)std::max<long>(1, std::min<long>(g, kMaxParts));
}

}  // namespace

size_t sketch_geqp3_ws_bytes(int d) {
  return (size_t)(d + 2 * kMaxParts) * sizeof(double) + 256;
}

int launch_sketch_geqp3(const double* Msk, int d, i64 ni, i64 ld, int psteps, double* X,
                        double* R, i64 ldr, i64* jsk, void* ws, size_t ws_bytes, int* status,
                        hipStream_t st) {
  if (ni <= 0) return QRCP_OK;
  if (d < 1 || d > 1024) return QRCP_ERR_UNSUPPORTED;
  if (ws_bytes < sketch_geqp3_ws_bytes(d)) return QRCP_ERR_WORKSPACE;
  double* tau = (double*)ws;
  double* part_v = tau + d;
  long* part_i = (long*)(part_v + kMaxParts);
  QRCP_TRY(launch_copy2d(Msk, ld, X, d, d, ni, st));
  QRCP_TRY(launch_iota(jsk, ni, st));
  const int steps = (int)std::min<i64>(d, ni);
  // norms of all columns over all rows, for the first pivot
  int parts = parts_for(ni);
  hipLaunchKernelGGL(geqp3_update_kernel, dim3(parts), dim3(NT), 0, st, current_gate(), X, (long)d, d, (long)ni, -1,
                     (const double*)tau, 0L, part_v, part_i, status);
  QRCP_LAUNCHED("geqp3_update");
  for (int j = 0; j < steps; ++j) {
    hipLaunchKernelGGL(geqp3_pivot_kernel, dim3(1), dim3(NT), 0, st, current_gate(), X, (long)d, d, j,
                       j < psteps ? 1 : 0, (const double*)part_v, (const long*)part_i, parts, jsk,
                       tau);
    QRCP_LAUNCHED("geqp3_pivot");
    if (j + 1 < ni) {
      parts = parts_for(ni - j - 1);
      hipLaunchKernelGGL(geqp3_update_kernel, dim3(parts), dim3(NT), 0, st, current_gate(), X, (long)d, d,
                         (long)ni, j, (const double*)tau, (long)(j + 1), part_v, part_i, status);
      QRCP_LAUNCHED("geqp3_update");
    }
  }
  // R^sk: the upper trapezoid, exact zeros below the diagonal
  return launch_triu_copy(X, d, R, ldr, d, ni, st);
}

}  // namespace qrcp
