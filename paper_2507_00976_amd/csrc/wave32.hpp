// Register-resident factorizations of a 32 x 32 block by one 64-lane wave.
//
// A block lives in 32 registers per lane, in one of two layouts:
//   column layout: lane c holds column c, x[r] = M(r, c);
//   row layout:    lane r holds row r,    x[c] = M(r, c).
// Lanes 32..63 carry zeros and results there are ignored.  Every loop index
// is a compile-time constant after unrolling, so an entry of another lane is
// read with v_readlane into a scalar register (rdlane), and each elimination
// step costs one division per lane plus one readlane and one FMA per updated
// entry, with no LDS traffic and no barriers.
#pragma once

#include <hip/hip_runtime.h>

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
// x[r] = R(r, c) for r <= c.  Returns the first column t whose pivot is not
// positive (breakdown), else nb; columns from the breakdown on are left as
// they were at that point.
__device__ __forceinline__ int wave_potrf32_col(double (&x)[W32], int nb) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < W32; ++t) {
    if (t < nb) {
      const double d = rdlane(x[t], t);
      if (!(d > 0.0)) return t;
      const double r = sqrt(d);
      if (lane == t) x[t] = r;
      else if (lane > t) x[t] = x[t] / r;
#pragma unroll
      for (int rr = t + 1; rr < W32; ++rr) {
        if (rr < nb) {
          const double s = rdlane(x[t], rr);
          if (lane >= rr) x[rr] -= s * x[t];
        }
      }
    }
  }
  return nb;
}

// Inverse of the upper triangle R (column layout) into y (column layout):
// back substitution R X = I, one column of X per lane.
__device__ __forceinline__ void wave_inv_upper32_col(const double (&x)[W32], double (&y)[W32],
                                                     int nb) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < W32; ++i) y[i] = 0.0;
#pragma unroll
  for (int i = W32 - 1; i >= 0; --i) {
    if (i < nb) {
      double s = 0.0;
#pragma unroll
      for (int l = i + 1; l < W32; ++l)
        if (l < nb) s += rdlane(x[i], l) * y[l];
      const double rii = rdlane(x[i], i);
      y[i] = (lane == i) ? 1.0 / rii : ((lane > i && lane < nb) ? -s / rii : 0.0);
    }
  }
}

// Inverse of the upper triangle U given in row layout (lane r: x[c] = U(r,c))
// into y, column layout.
__device__ __forceinline__ void wave_inv_upper32_row(const double (&x)[W32], double (&y)[W32],
                                                     int nb) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < W32; ++i) y[i] = 0.0;
#pragma unroll
  for (int i = W32 - 1; i >= 0; --i) {
    if (i < nb) {
      double s = 0.0;
#pragma unroll
      for (int l = i + 1; l < W32; ++l)
        if (l < nb) s += rdlane(x[l], i) * y[l];
      const double uii = rdlane(x[i], i);
      y[i] = (lane == i) ? 1.0 / uii : ((lane > i && lane < nb) ? -s / uii : 0.0);
    }
  }
}

// Inverse of the unit lower triangle L given in row layout (lane r:
// x[c] = L(r,c), c < r) into y, column layout (forward substitution).
__device__ __forceinline__ void wave_inv_unit_lower32_row(const double (&x)[W32],
                                                          double (&y)[W32], int nb) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < W32; ++i) {
    if (i < nb) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < i; ++l) s += rdlane(x[l], i) * y[l];
      y[i] = (lane == i) ? 1.0 : ((lane < i) ? -s : 0.0);
    } else {
      y[i] = 0.0;
    }
  }
}

// LU without pivoting with the sign modification of the Householder
// reconstruction (row layout, in place): at step t, D_t = -sgn(M(t,t))
// (sgn(0) = +1), the pivot becomes M(t,t) - D_t, the column below it is
// divided by the pivot and the trailing block updated.  Lane 0 stores D_t to
// dj[t].
__device__ __forceinline__ void wave_lu32_signmod_row(double (&x)[W32], int nb, double* dj) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < W32; ++t) {
    if (t < nb) {
      const double a = rdlane(x[t], t);
      const double d = (a >= 0.0) ? -1.0 : 1.0;
      const double piv = a - d;
      if (lane == 0) dj[t] = d;
      if (lane == t) x[t] = piv;
      else if (lane > t) x[t] = x[t] / piv;
#pragma unroll
      for (int c = t + 1; c < W32; ++c) {
        if (c < nb) {
          const double u = rdlane(x[c], t);
          if (lane > t) x[c] -= x[t] * u;
        }
      }
    }
  }
}

}  // namespace qrcp
