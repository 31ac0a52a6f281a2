// Factorizations and inverses of a 32 x 32 block by one 64-lane wave.
//
// A block in registers uses 32 registers per lane, in one of two layouts:
//   column layout: lane c holds column c, x[r] = M(r, c);
//   row layout:    lane r holds row r,    x[c] = M(r, c).
// Lanes 32..63 carry zeros and their results are ignored.  Every loop index is
// a compile-time constant after unrolling; the rows or columns that every lane
// needs at a factorization step are broadcast through a small LDS buffer of
// the calling wave (written and read by the same wave, so no barrier is
// involved) or read from their lane as scalars, the inverses request the next row of the triangle while applying
// the current one, and the updates are written without per-element branches:
// entries outside the triangle that a caller uses may hold garbage, which
// never flows into the triangle.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace qrcp {

constexpr int W32 = 32;

// Value of v in lane l (l wave-uniform).
__device__ __forceinline__ double rdlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Newton-Raphson refinements of the hardware approximations (each step
// roughly doubles the number of correct bits; two steps from the hardware
// estimate reach double precision up to a unit or two in the last place).
// Arguments outside [2^-1000, 2^1000] take the exact library operations, so
// neither the estimate nor its square can leave the normal range.
__device__ __forceinline__ bool nr_range(double a) {
  const double m = fabs(a);
  return m >= 0x1p-1000 && m <= 0x1p1000;
}
// 1 / sqrt(d) for d > 0
__device__ __forceinline__ double nr_rsqrt(double d) {
  if (!nr_range(d)) return 1.0 / sqrt(d);
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);  // 1 - d y^2
    y = fma(0.5 * y, e, y);
  }
  return y;
}
// 1 / a for a != 0
__device__ __forceinline__ double nr_rcp(double a) {
  if (!nr_range(a)) return 1.0 / a;
  double y = __builtin_amdgcn_rcp(a);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-a, y, 1.0);  // 1 - a y
    y = fma(y, e, y);
  }
  return y;
}

// Cholesky of the upper triangle, column layout, in place: on return
// x[r] = R(r, c) for r <= c (the entries below the diagonal are garbage).
// With y = 1/sqrt(pivot) (refined hardware estimate), row t is x(t, c) y off
// the diagonal and pivot * y on it: a handful of dependent operations per step
// instead of a square root followed by a division.
// Returns the first column t whose pivot is not positive (breakdown), else
// nb; from the breakdown on, columns are left as they were at that point.
// sb: 64 doubles of LDS owned by the calling wave.
__device__ __forceinline__ int wave_potrf32_col(double (&x)[W32], int nb, double* sb) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < W32; ++t) {
    if (t < nb) {
      const double d = rdlane(x[t], t);
      if (!(d > 0.0)) return t;
      const double y = nr_rsqrt(d);
      const double r = d * y;
      const double q = x[t] * y;
      x[t] = (lane == t) ? r : ((lane > t) ? q : x[t]);
      sb[lane] = x[t];  // row t of R: R(t, c) in lane c
      wave_lds_sync();
      // G(rr, c) -= R(t, rr) R(t, c) for t < rr <= c
#pragma unroll
      for (int rr = t + 1; rr < W32; ++rr) x[rr] = fma(-sb[rr], x[t], x[rr]);
      wave_lds_sync();
    }
  }
  return nb;
}

// Cholesky as wave_potrf32_col, for wave 0 of a workgroup whose wave 1 builds
// the inverse meanwhile (wave_inv_upper32_follow): each finished row t of R
// (R(t, c), c >= t, at sRows[t * ldr + c]; ldr >= 33) is published with
// *flag = t + 1 (LDS, release) before it is applied; a breakdown publishes -1.
// *flag must be 0 when both waves start.
__device__ __forceinline__ int wave_potrf32_col_pub(double (&x)[W32], int nb, double* sRows,
                                                    int ldr, int* flag) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < W32; ++t) {
    if (t < nb) {
      const double d = rdlane(x[t], t);
      if (!(d > 0.0)) {
        if (lane == 0) __hip_atomic_store(flag, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        return t;
      }
      const double y = nr_rsqrt(d);
      const double r = d * y;
      const double q = x[t] * y;
      x[t] = (lane == t) ? r : ((lane > t) ? q : x[t]);
      if (lane < W32) sRows[t * ldr + lane] = x[t];
      wave_lds_sync();
      if (lane == 0) __hip_atomic_store(flag, t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      // G(rr, c) -= R(t, rr) R(t, c) for t < rr <= c
#pragma unroll
      for (int rr = t + 1; rr < W32; ++rr) x[rr] = fma(-sRows[t * ldr + rr], x[t], x[rr]);
    }
  }
  return nb;
}

// R^{-1} for the R that wave_potrf32_col_pub is producing, built as the forward
// substitution of R^T: as soon as row t of R is published, row t of R^{-T}
// follows (lane j: R^{-1}(j, t) = -(sum_{s<t} R(s, t) R^{-1}(j, s)) / R(t, t),
// 1 / R(t, t) on the diagonal, 0 for j > t).  Lane j ends with row j of R^{-1},
// stored to sInv[j * ldi + t] (zero outside nb x nb).  Returns false, storing
// nothing, when the factorization breaks down.
__device__ __forceinline__ bool wave_inv_upper32_follow(const double* sRows, int ldr, double* sInv,
                                                        int ldi, int nb, int* flag) {
  const int lane = threadIdx.x & 63;
  double z[W32];
#pragma unroll
  for (int t = 0; t < W32; ++t) z[t] = 0.0;
#pragma unroll
  for (int t = 0; t < W32; ++t) {
    if (t < nb) {
      long spins = 0;
      int f = __hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
      while (f >= 0 && f <= t) {
        if (++spins > kSpinLimit) {
          f = -1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        f = __hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      if (f < 0) return false;
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < t; ++s) s4[s & 3] = fma(sRows[s * ldr + t], z[s], s4[s & 3]);
      const double dinv = 1.0 / sRows[t * ldr + t];
      const double v = -((s4[0] + s4[1]) + (s4[2] + s4[3])) * dinv;
      z[t] = (lane == t) ? dinv : ((lane < t) ? v : 0.0);
    }
  }
  if (lane < W32) {
#pragma unroll
    for (int t = 0; t < W32; ++t) sInv[lane * ldi + t] = z[t];
  }
  return true;
}

// y = R^{-1} (column layout) for the upper triangle of R held in LDS,
// row-major with stride ld (only entries on and above the diagonal are
// read): back substitution R X = I, one column of X per lane, four partial
// sums per dot product.  The reciprocals of the diagonal are formed first, all
// lanes at once, so each row costs a multiplication instead of a division.
__device__ __forceinline__ void wave_inv_upper32(const double* sR, int ld, double (&y)[W32],
                                                 int nb) {
  const int lane = threadIdx.x & 63;
  wave_lds_sync();
  const double dinv = (lane < nb) ? 1.0 / sR[lane * ld + lane] : 0.0;  // lane i: 1 / R(i, i)
  // row i - 1 of R is requested while row i is applied
  double cur[W32], nxt[W32];
  nxt[W32 - 1] = sR[(W32 - 2) * ld + W32 - 1];
#pragma unroll
  for (int i = 0; i < W32; ++i) y[i] = 0.0;
#pragma unroll
  for (int i = W32 - 1; i >= 0; --i) {
#pragma unroll
    for (int l = i + 1; l < W32; ++l) cur[l] = nxt[l];
    if (i >= 1) {
#pragma unroll
      for (int l = i; l < W32; ++l) nxt[l] = sR[(i - 1) * ld + l];
    }
    if (i < nb) {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int l = i + 1; l < W32; ++l) s4[l & 3] = fma(cur[l], y[l], s4[l & 3]);
      const double di = rdlane(dinv, i);
      const double v = -((s4[0] + s4[1]) + (s4[2] + s4[3])) * di;
      const double keep = (lane > i && lane < nb) ? v : 0.0;
      y[i] = (lane == i) ? di : keep;
    }
  }
}

// y = L^{-1} (column layout) for the unit lower triangle of L held in LDS,
// row-major with stride ld (only entries strictly below the diagonal are
// read): forward substitution.
__device__ __forceinline__ void wave_inv_unit_lower32(const double* sL, int ld, double (&y)[W32],
                                                      int nb) {
  const int lane = threadIdx.x & 63;
  wave_lds_sync();
  // row i + 1 of L is requested while row i is applied
  double cur[W32], nxt[W32];
  nxt[0] = sL[1 * ld + 0];
#pragma unroll
  for (int i = 0; i < W32; ++i) {
#pragma unroll
    for (int l = 0; l < i; ++l) cur[l] = nxt[l];
    if (i + 1 < W32) {
#pragma unroll
      for (int l = 0; l <= i; ++l) nxt[l] = sL[(i + 1) * ld + l];
    }
    if (i < nb) {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int l = 0; l < i; ++l) s4[l & 3] = fma(cur[l], y[l], s4[l & 3]);
      const double v = -((s4[0] + s4[1]) + (s4[2] + s4[3]));
      const double keep = (lane < i) ? v : 0.0;
      y[i] = (lane == i) ? 1.0 : keep;
    } else {
      y[i] = 0.0;
    }
  }
}

// LU without pivoting with the sign modification of the Householder
// reconstruction (row layout, in place): at step t, D_t = -sgn(M(t,t))
// (sgn(0) = +1), the pivot becomes M(t,t) - D_t, the column below it is
// scaled by the pivot's (refined) reciprocal and the trailing block updated.  Lane 0 stores D_t to
// dj[t].  sb is not used.
__device__ __forceinline__ void wave_lu32_signmod_row(double (&x)[W32], int nb, double* dj,
                                                      double* sb) {
  (void)sb;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < W32; ++t) {
    if (t < nb) {
      const double a = rdlane(x[t], t);
      const double d = (a >= 0.0) ? -1.0 : 1.0;
      const double piv = a - d;
      if (lane == 0) dj[t] = d;
      const double q = x[t] * nr_rcp(piv);
      x[t] = (lane == t) ? piv : ((lane > t) ? q : x[t]);
      // row t of U is lane t's registers, read as scalars (one lane would
      // otherwise write it to LDS element by element)
      const double l = (lane > t) ? x[t] : 0.0;  // rows at and above t keep their values
#pragma unroll
      for (int c = t + 1; c < W32; ++c) x[c] = fma(-l, rdlane(x[c], t), x[c]);
    }
  }
}

}  // namespace qrcp
