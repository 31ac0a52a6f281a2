// Factorizations and inverses of a 32 x 32 block by one 64-lane wave.
//
// A block in registers uses 32 registers per lane, in one of two layouts:
//   column layout: lane c holds column c, x[r] = M(r, c);
//   row layout:    lane r holds row r,    x[c] = M(r, c).
// Lanes 32..63 carry zeros and their results are ignored.  Every loop index is
// a compile-time constant after unrolling; the rows or columns that every lane
// needs are broadcast through a small LDS buffer of the calling wave (written
// and read by the same wave, so no barrier is involved), and the updates are
// written without per-element branches: entries outside the triangle that a
// caller uses may hold garbage, which never flows into the triangle.
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

// Cholesky of the upper triangle, column layout, in place: on return
// x[r] = R(r, c) for r <= c (the entries below the diagonal are garbage).
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
      const double r = sqrt(d);
      const double q = x[t] / r;
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

// y = R^{-1} (column layout) for the upper triangle of R held in LDS,
// row-major with stride ld (only entries on and above the diagonal are
// read): back substitution R X = I, one column of X per lane, four partial
// sums per dot product.
__device__ __forceinline__ void wave_inv_upper32(const double* sR, int ld, double (&y)[W32],
                                                 int nb) {
  const int lane = threadIdx.x & 63;
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < W32; ++i) y[i] = 0.0;
#pragma unroll
  for (int i = W32 - 1; i >= 0; --i) {
    if (i < nb) {
      double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int l = i + 1; l < W32; ++l) s[l & 3] = fma(sR[i * ld + l], y[l], s[l & 3]);
      const double rii = sR[i * ld + i];
      const double sum = (s[0] + s[1]) + (s[2] + s[3]);
      y[i] = (lane == i) ? 1.0 / rii : ((lane > i && lane < nb) ? -sum / rii : 0.0);
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
#pragma unroll
  for (int i = 0; i < W32; ++i) {
    if (i < nb) {
      double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int l = 0; l < i; ++l) s[l & 3] = fma(sL[i * ld + l], y[l], s[l & 3]);
      const double sum = (s[0] + s[1]) + (s[2] + s[3]);
      y[i] = (lane == i) ? 1.0 : ((lane < i) ? -sum : 0.0);
    } else {
      y[i] = 0.0;
    }
  }
}

// LU without pivoting with the sign modification of the Householder
// reconstruction (row layout, in place): at step t, D_t = -sgn(M(t,t))
// (sgn(0) = +1), the pivot becomes M(t,t) - D_t, the column below it is
// divided by the pivot and the trailing block updated.  Lane 0 stores D_t to
// dj[t].  sb: 64 doubles of LDS owned by the calling wave.
__device__ __forceinline__ void wave_lu32_signmod_row(double (&x)[W32], int nb, double* dj,
                                                      double* sb) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < W32; ++t) {
    if (t < nb) {
      const double a = rdlane(x[t], t);
      const double d = (a >= 0.0) ? -1.0 : 1.0;
      const double piv = a - d;
      if (lane == 0) dj[t] = d;
      const double q = x[t] / piv;
      x[t] = (lane == t) ? piv : ((lane > t) ? q : x[t]);
      // row t of U, from lane t, to every lane
      if (lane == t) {
#pragma unroll
        for (int c = t + 1; c < W32; ++c) sb[c] = x[c];
      }
      wave_lds_sync();
      const double l = (lane > t) ? x[t] : 0.0;  // rows at and above t keep their values
#pragma unroll
      for (int c = t + 1; c < W32; ++c) x[c] = fma(-l, sb[c], x[c]);
      wave_lds_sync();
    }
  }
}

}  // namespace qrcp
