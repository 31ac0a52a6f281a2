// Householder factorization of a tall narrow leaf (mi x ib, ib <= 32) for the
// unpivoted blocked QR baseline (GEQRF semantics, LAPACK DLARFG convention).
//
// One cooperative kernel: the mi rows are spread over G workgroups, one row per
// thread with its ib values in registers.  Column j needs, from all rows below
// j, the sum of squares of x_j and the dot products of x_j with the later
// columns; those ib partial sums (plus row j itself, from its owner) are
// exchanged through sentinel-initialised record slots, one slot per (column,
// workgroup), exactly as in the pivot-selection kernel.  With
// v = [1; x/(alpha - beta)] the reflector's action on column c follows from
// the exchanged sums: v^T a_c = a_c(j) + (x^T a_c)/(alpha - beta).
#include "common.hpp"
#include "kernels.hpp"
#include "wave32.hpp"

namespace qrcp {

namespace {
constexpr int IB = 32;
constexpr int NT = 256;
constexpr int RWH = 2 * IB;
constexpr uint64_t SENT = 0xFFF0DEADBEEFCAFEull;
constexpr int kMaxLeafGroups = 256;  // workgroups of one leaf (rows / 256)

struct LeafArgs {
  double* A;
  long lda;
  long mi;
  int ib;
  double* tau;
  uint64_t* rec;
  int* status;
  double* tout;  // may be null: T of the leaf's compact WY form (ib x ib, ld ldt)
  long ldt;
};

__device__ __forceinline__ uint64_t poll_w(uint64_t* p, bool& to) {
  if (to) return 0;
  uint64_t v = load_agent(p);
  long spins = 0;
  while (v == SENT) {
    if (++spins > kSpinLimit) { to = true; return 0; }
    __builtin_amdgcn_s_sleep(1);
    v = load_agent(p);
  }
  return v;
}

__global__ __launch_bounds__(NT) void hh_leaf_kernel(Gate gt, LeafArgs a) {
  QRCP_GATE(gt);
  __shared__ double sRed[NT / 64][64][IB + 1];  // per-wave rows -> reduced per wave below
  __shared__ double sSum[8][IB];
  __shared__ double sAll[8][IB];
  __shared__ double sTot[IB];
  __shared__ double sRow[IB];
  __shared__ double sF[IB];  // tau (v^T a_c) of the column's reflector, per later column c
  __shared__ double sGm[IB][IB + 1];  // V^T V (strict upper triangle), then the UT matrix
  __shared__ double sTauL[IB];
  __shared__ int sflag;
  const int g = blockIdx.x, G = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long R = (a.mi + G - 1) / G;
  const long r = (long)g * R + tid;
  const bool mine = tid < R && r < a.mi;
  const int ib = a.ib;
  double x[IB];
#pragma unroll
  for (int c = 0; c < IB; ++c) x[c] = (mine && c < ib) ? a.A[r + (long)c * a.lda] : 0.0;
  bool to = false;
  if (tid == 0) sflag = 0;
  __syncthreads();

  // The column loop is not unrolled (its body is long); the row's values stay
  // in registers because every access below names its column at compile time
  // (the pivot column is picked by a select over the unrolled columns), so
  // nothing is indexed by the loop counter.
  for (int j = 0; j < ib; ++j) {
    {
      double xj = 0.0;
#pragma unroll
      for (int c = 0; c < IB; ++c) xj = (c == j) ? x[c] : xj;
      // ---- partial sums of my row: slot j = x_j^2, slot c > j = x_j x_c, and
      // slot c < j = x_j v_c (v_c, the earlier reflectors, for the Gram) ----
      const bool below = mine && r > j;
#pragma unroll
      for (int c = 0; c < IB; ++c) sRed[wv][lane][c] = below ? xj * x[c] : 0.0;
      __syncthreads();
      {
        // 256 threads: column c = tid % 32, part = tid / 32 (8 parts x 32 rows)
        const int c = tid % IB, part = tid / IB;
        double s = 0.0;
        for (int q = 0; q < 32; ++q) {
          const int rr = part * 32 + q;
          s += sRed[rr >> 6][rr & 63][c];
        }
        sSum[part][c] = s;
      }
      __syncthreads();
      uint64_t* myrec = a.rec + ((long)j * G + g) * RWH;
      if (tid < IB) {
        double s = 0.0;
        for (int p = 0; p < 8; ++p) s += sSum[p][tid];
        store_agent(myrec + tid, dbits(s));
      }
      if (mine && r == j) {
#pragma unroll
        for (int c = 0; c < IB; ++c) store_agent(myrec + IB + c, dbits(x[c]));
      }
      // ---- combine all workgroups ----
      // Every record word this thread sums is requested before the first
      // wait (one memory round trip whatever G is); only words that had not
      // landed yet are polled again.  The sum runs in workgroup order.
      {
        const int c = tid % IB, part = tid / IB;
        const int owner = (int)(j / R);
        uint64_t rowv = 0;
        if (tid < IB && tid < ib && !to) rowv = load_agent(a.rec + ((long)j * G + owner) * RWH + IB + tid);
        double s = 0.0;
        if (c < ib) {
          uint64_t v[kMaxLeafGroups / 8];
#pragma unroll
          for (int q = 0; q < kMaxLeafGroups / 8; ++q) {
            const int gg = part + 8 * q;
            v[q] = (gg < G && !to) ? load_agent(a.rec + ((long)j * G + gg) * RWH + c) : 0;
          }
#pragma unroll
          for (int q = 0; q < kMaxLeafGroups / 8; ++q) {
            const int gg = part + 8 * q;
            if (gg < G) {
              uint64_t w = v[q];
              if (w == SENT) w = poll_w(a.rec + ((long)j * G + gg) * RWH + c, to);
              s += bitsd(w);
            }
          }
        }
        sAll[part][c] = s;
        if (tid < IB && tid < ib) {
          if (rowv == SENT) rowv = poll_w(a.rec + ((long)j * G + owner) * RWH + IB + tid, to);
          sRow[tid] = bitsd(rowv);
        }
      }
      __syncthreads();
      if (tid < IB) {
        double s = 0.0;
        for (int p = 0; p < 8; ++p) s += sAll[p][tid];
        sTot[tid] = s;
      }
      if (to) sflag = 1;
      __syncthreads();
      if (sflag) {
        if (tid == 0) store_agent_i32(a.status, QRCP_ERR_TIMEOUT);
        return;
      }
      const double alpha = sRow[j], xx = sTot[j];
      double beta = alpha, tau = 0.0, inv = 1.0;
      if (xx != 0.0) {
        const double nrm = sqrt(alpha * alpha + xx);
        beta = (alpha < 0.0) ? nrm : -nrm;
        tau = (beta - alpha) / beta;
        inv = alpha - beta;
      }
      if (g == 0 && tid == 0) a.tau[j] = tau;
      // V^T V of the leaf: v_c^T v_j = v_c(j) + (sum over rows below j of
      // v_c x_j) / (alpha - beta), for c < j (v_c(j) is the owner's row)
      if (tid < j) sGm[tid][j] = sRow[tid] + sTot[tid] / inv;
      if (tid == 0) sTauL[j] = tau;
      // the reflector's action on each later column, formed once per column
      if (tid < IB) sF[tid] = (tid > j && tid < ib) ? tau * (sRow[tid] + sTot[tid] / inv) : 0.0;
      __syncthreads();
      if (mine && r >= j) {
        const double v = (r == j) ? 1.0 : (xx != 0.0 ? xj / inv : 0.0);
        if (tau != 0.0) {
#pragma unroll
          for (int c = 0; c < IB; ++c)
            if (c > j && c < ib) x[c] -= sF[c] * v;
        }
        const double xn = (r == j) ? beta : v;
#pragma unroll
        for (int c = 0; c < IB; ++c) x[c] = (c == j) ? xn : x[c];
      }
      __syncthreads();
    }
  }
  if (mine) {
#pragma unroll
    for (int c = 0; c < IB; ++c)
      if (c < ib) a.A[r + (long)c * a.lda] = x[c];
  }
  // T of the leaf by the UT transform, T^{-1} = diag(1/tau) + striu(V^T V)
  // (a zero tau decouples its index: its row and column of T are zero), by
  // one wave of workgroup 0
  if (a.tout && g == 0 && tid < 64) {
    if (lane < IB) {
#pragma unroll
      for (int rr = 0; rr < IB; ++rr) {
        double v = 0.0;
        if (lane < ib && rr < ib && rr <= lane) {
          const double tr = sTauL[rr], tc = sTauL[lane];
          if (tr == 0.0 || tc == 0.0) v = (rr == lane) ? 1.0 : 0.0;
          else if (rr == lane) v = 1.0 / tc;
          else v = sGm[rr][lane];
        }
        sGm[rr][lane] = v;
      }
    }
    double ty[W32];
    wave_inv_upper32(&sGm[0][0], IB + 1, ty, ib);
    if (lane < ib) {
#pragma unroll
      for (int rr = 0; rr < IB; ++rr) {
        if (rr < ib) {
          const double v = (rr == lane && sTauL[lane] == 0.0) ? 0.0 : ty[rr];
          a.tout[rr + (long)lane * a.ldt] = v;
        }
      }
    }
  }
}

int leaf_groups(long mi) {
  long G = (mi + NT - 1) / NT;
  if (G < 1) G = 1;
  return (int)G;
}

}  // namespace

size_t hh_leaf_records_bytes(i64 mi) {
  return (size_t)IB * leaf_groups(mi) * RWH * sizeof(uint64_t);
}

int launch_hh_leaf(double* A, i64 lda, i64 mi, int ib, double* tau, uint64_t* rec,
                   size_t rec_bytes, int* status, hipStream_t st, double* tout, i64 ldt) {
  if (mi <= 0 || ib <= 0) return QRCP_OK;
  if (ib > IB) return QRCP_ERR_UNSUPPORTED;
  const int G = leaf_groups(mi);
  if (G > kMaxLeafGroups) return QRCP_ERR_UNSUPPORTED;
  const size_t need = hh_leaf_records_bytes(mi);
  if (need > rec_bytes) return QRCP_ERR_WORKSPACE;
  QRCP_TRY(launch_fill_u64(rec, (i64)(need / 8), SENT, st));
  LeafArgs args{A, (long)lda, (long)mi, ib, tau, rec, status, tout, (long)ldt};
  Gate gt = current_gate();
  void* params[] = {&gt, &args};
  QRCP_TRY(launch_resident((const void*)hh_leaf_kernel, dim3(G), dim3(NT), params, 0, st));
  return QRCP_OK;
}

}  // namespace qrcp
