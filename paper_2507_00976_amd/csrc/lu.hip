// Pivot selection of the wide sketch (Alg. 2): GETRF with partial pivoting on
// X = (M^sk)^T, computed as one cooperative kernel.
//
// Layout: the d x ni column-major sketch *is* X stored row-major (row t of X =
// sketch column t, d contiguous doubles), so the transpose of Alg. 2 costs
// nothing.  The ni rows are spread over G co-resident workgroups (R rows each,
// TPR threads per row); the current 32-column panel of every row sits in
// registers, the trailing columns in a working copy in HBM.
//
// One pivot step = one cross-workgroup exchange: every workgroup publishes its
// best candidate (|x|, position, row id) and that row's panel values into a
// record slot owned by (step, workgroup); every workgroup then reads all
// headers, agrees on the winner (largest |x|, ties to the smallest current
// position, as IDAMAX), reads the winner's panel values and applies the
// rank-1 update to its own rows.  Record slots are never reused within a call
// and are reset to a sentinel bit pattern beforehand, so each 64-bit word is
// valid as soon as it differs from the sentinel: no flags or fences are needed
// for the exchange itself.  Row swaps are never performed: each row carries its
// current position, and the row sitting at position j takes the pivot's
// position when the pivot leaves (the swap of GETRF).
//
// After each panel the trailing columns are updated in the blocked form:
// U12 = L11^{-1} X(piv, trail), X(r, trail) -= L(r, panel) U12.
#include <climits>

#include "common.hpp"
#include "kernels.hpp"

namespace qrcp {

namespace {
constexpr int NB = 32;            // panel width
constexpr int NT = 256;           // threads per workgroup
constexpr int RW = 2 + NB;        // words per record
constexpr int TCH = 256;          // trailing columns per chunk
constexpr uint64_t SENT = 0xFFF0DEADBEEFCAFEull;
constexpr uint64_t NOCAND = 0x7FFFFFFF00000000ull;
constexpr uint64_t BADKEY = 0x7FFFFFFE00000000ull;
constexpr int kMaxGroups = 256;

struct LuArgs {
  const double* msk;
  long ld;
  int d;
  long ni;
  double* xw;        // d x ni working copy (ld = d)
  uint64_t* rec;     // steps x G x RW words, sentinel-filled
  long* ipiv;
  long* jsk;
  int* status;
};

__device__ __forceinline__ bool better(double va, uint64_t ka, double vb, uint64_t kb) {
  return va > vb || (va == vb && ka < kb);
}

__device__ __forceinline__ uint64_t poll(uint64_t* p, bool& timed_out) {
  if (timed_out) return 0;
  uint64_t v = load_agent(p);
  long spins = 0;
  while (v == SENT) {
    if (++spins > kSpinLimit) {
      timed_out = true;
      return 0;
    }
    __builtin_amdgcn_s_sleep(1);
    v = load_agent(p);
  }
  return v;
}

// Workgroup argmax of (v, key): every thread gets the result.
__device__ __forceinline__ void wg_argmax(double& v, uint64_t& key, double* sv, uint64_t* sk) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const uint64_t ok = ((uint64_t)(uint32_t)__shfl_xor((int)(key >> 32), o, 64) << 32) |
                        (uint32_t)__shfl_xor((int)(uint32_t)key, o, 64);
    if (better(ov, ok, v, key)) { v = ov; key = ok; }
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { sv[w] = v; sk[w] = key; }
  __syncthreads();
  v = sv[0];
  key = sk[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i)
    if (better(sv[i], sk[i], v, key)) { v = sv[i]; key = sk[i]; }
}

__device__ __forceinline__ double canon(double x) { return isnan(x) ? __longlong_as_double(0x7FF8000000000000ll) : x; }

template <int TPR>
__global__ __launch_bounds__(NT) void lu_pivots_kernel(LuArgs a) {
  constexpr int R = NT / TPR;
  constexpr int CPT = NB / TPR;
  __shared__ double sU[NB][TCH];
  __shared__ double sLr[R][NB + 1];
  __shared__ double sL11[NB][NB + 1];
  __shared__ int sWin[NB];
  __shared__ double sPiv[NB];
  __shared__ long sRow[NB];
  __shared__ double sv[NT / 64];
  __shared__ uint64_t sk[NT / 64];
  __shared__ int sflag;

  const int g = blockIdx.x, G = gridDim.x;
  const int tid = threadIdx.x, rl = tid / TPR, part = tid % TPR;
  const int lane = tid & 63;
  const int d = a.d;
  const long ni = a.ni;
  const long row = (long)g * R + rl;
  const bool valid = row < ni;
  const int steps = (int)min((long)d, ni);
  long pos = valid ? row : LONG_MAX;
  bool active = valid;
  double* xw = a.xw + row * (long)d;

  // working copy of this workgroup's rows + non-finite check
  bool bad = false;
  if (valid) {
    const double* src = a.msk + row * a.ld;
    for (int c = part; c < d; c += TPR) {
      const double v = src[c];
      bad |= !isfinite(v);
      xw[c] = v;
    }
  }
  if (tid == 0) sflag = 0;
  __syncthreads();
  if (bad) sflag = 1;
  __syncthreads();
  const bool wg_bad = sflag != 0;
  __threadfence();

  double pv[CPT];
  bool timed_out = false;

  for (int p0 = 0; p0 < steps; p0 += NB) {
    // this panel's columns of my row
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int c = p0 + part * CPT + q;
      pv[q] = (active && c < d) ? xw[c] : 0.0;
    }
#pragma unroll
    for (int jl = 0; jl < NB; ++jl) {
      const int jg = p0 + jl;
      if (jg < steps) {  // uniform
        const int qj = jl / CPT, sj = jl % CPT;
        // ---- local candidate ----
        double cv = -1.0;
        uint64_t ck = NOCAND;
        if (active && part == qj) {
          const double x = pv[sj];
          cv = isnan(x) ? -0.5 : fabs(x);
          ck = ((uint64_t)pos << 32) | (uint64_t)row;
        }
        wg_argmax(cv, ck, sv, sk);
        // ---- publish ----
        uint64_t* myrec = a.rec + ((long)jg * G + g) * RW;
        if (cv >= -0.5 && (long)(ck & 0xFFFFFFFFull) == row && row < ni && valid) {
#pragma unroll
          for (int q = 0; q < CPT; ++q) store_agent(myrec + 2 + part * CPT + q, dbits(canon(pv[q])));
        }
        if (tid == 0) {
          if (jg == 0 && wg_bad) {
            store_agent(myrec + 1, BADKEY);
          } else {
            store_agent(myrec + 1, ck);
          }
          store_agent(myrec, dbits(cv));
        }
        // ---- gather headers, agree on the winner ----
        double gv = -2.0;
        uint64_t gk = NOCAND;
        if (tid < G) {
          // both header words are requested together: one round trip when ready
          uint64_t* r = a.rec + ((long)jg * G + tid) * RW;
          uint64_t key = load_agent(r + 1);
          uint64_t vb = load_agent(r);
          long spins = 0;
          while (key == SENT || vb == SENT) {
            if (++spins > kSpinLimit) { timed_out = true; break; }
            __builtin_amdgcn_s_sleep(1);
            if (key == SENT) key = load_agent(r + 1);
            if (vb == SENT) vb = load_agent(r);
          }
          if (!timed_out) {
            if (key == BADKEY) {
              sflag = 2;
            } else if (key != NOCAND) {
              gv = bitsd(vb);
              gk = key;
            }
          }
          if (timed_out) sflag = 3;
        }
        wg_argmax(gv, gk, sv, sk);  // contains __syncthreads: sflag visible after it
        if (sflag >= 2) {
          if (tid == 0) store_agent_i32(a.status, sflag == 2 ? QRCP_ERR_NONFINITE : QRCP_ERR_TIMEOUT);
          return;  // uniform
        }
        const long wrow = (long)(gk & 0xFFFFFFFFull);
        const long wpos = (long)(gk >> 32);
        const int wg = (int)(wrow / R);
        uint64_t* wrec = a.rec + ((long)jg * G + wg) * RW;
        // the winner's panel row: NB threads fetch one word each into LDS
        if (tid < NB) sPiv[tid] = bitsd(poll(wrec + 2 + tid, timed_out));
        __syncthreads();
        double piv[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) piv[q] = sPiv[part * CPT + q];
        const double pj = sPiv[jl];
        if (tid == 0) {
          sWin[jl] = wg;
          sRow[jl] = wrow;
          if (g == 0) {
            a.ipiv[jg] = wpos;
            a.jsk[jg] = wrow;
          }
        }
        // ---- swap bookkeeping and elimination ----
        const double xj = __shfl(pv[sj], (lane & ~(TPR - 1)) + qj, 64);
        if (active && row == wrow) {
          active = false;
        } else if (active) {
          if (pos == jg) pos = wpos;
          const double l = (pj != 0.0) ? xj / pj : 0.0;
#pragma unroll
          for (int q = 0; q < CPT; ++q) {
            const int c = part * CPT + q;
            if (c > jl) pv[q] -= l * piv[q];
          }
          if (part == qj) pv[sj] = l;
        }
      }
    }
    // uniform timeout check
    __syncthreads();
    if (timed_out) sflag = 3;
    __syncthreads();
    if (sflag == 3) {
      if (tid == 0) store_agent_i32(a.status, QRCP_ERR_TIMEOUT);
      return;
    }
    const int pend = min(p0 + NB, steps);
    if (pend >= steps) break;   // no later pivot step needs the trailing columns
    // ---- blocked trailing update of columns p0+NB .. d ----
    // multipliers of my rows (pivot rows are no longer updated)
#pragma unroll
    for (int q = 0; q < CPT; ++q) sLr[rl][part * CPT + q] = pv[q];
    // L11 from the winners' records
    for (int e = tid; e < NB * NB; e += NT) {
      const int ar = e / NB, t = e % NB;
      double v = 0.0;
      if (t < ar) {
        uint64_t* wrec = a.rec + ((long)(p0 + ar) * G + sWin[ar]) * RW;
        v = bitsd(load_agent(wrec + 2 + t));
      }
      sL11[ar][t] = v;
    }
    __threadfence();  // acquire: pivot rows' trailing values written by their owners
    for (int c0 = p0 + NB; c0 < d; c0 += TCH) {
      const int cw = min(TCH, d - c0);
      __syncthreads();
      for (int e = tid; e < NB * cw; e += NT) {
        const int ar = e / cw, c = e % cw;
        sU[ar][c] = a.xw[sRow[ar] * (long)d + c0 + c];
      }
      __syncthreads();
      // U12 = L11^{-1} X(piv, chunk): one column per thread
      for (int c = tid; c < cw; c += NT) {
        for (int ar = 1; ar < NB; ++ar) {
          double s = sU[ar][c];
          for (int t = 0; t < ar; ++t) s -= sL11[ar][t] * sU[t][c];
          sU[ar][c] = s;
        }
      }
      __syncthreads();
      if (active) {
        for (int c = part; c < cw; c += TPR) {
          double x = xw[c0 + c];
#pragma unroll 8
          for (int t = 0; t < NB; ++t) x -= sLr[rl][t] * sU[t][c];
          xw[c0 + c] = x;
        }
      }
    }
    __threadfence();  // release: my trailing values before the next records
    __syncthreads();
  }
  // positions of the rows that were never pivots
  if (valid && active && part == 0 && pos < ni) a.jsk[pos] = row;
}

int pick_tpr(long ni) {
  if ((ni + 63) / 64 <= kMaxGroups) return 4;
  if ((ni + 127) / 128 <= kMaxGroups) return 2;
  if ((ni + 255) / 256 <= kMaxGroups) return 1;
  return 0;
}

}  // namespace

size_t lu_records_bytes(int d, i64 ni) {
  const int tpr = pick_tpr(ni);
  if (!tpr) return 0;
  const long G = (ni + (NT / tpr) - 1) / (NT / tpr);
  const long steps = std::min((long)d, (long)ni);
  return (size_t)steps * G * RW * sizeof(uint64_t);
}

int launch_lu_pivots(const double* Msk, int d, i64 ni, i64 ld, double* Xw, uint64_t* rec,
                     size_t rec_bytes, i64* ipiv, i64* jsk, int* status_dev, hipStream_t st) {
  if (ni <= 0 || d <= 0) return QRCP_OK;
  const int tpr = pick_tpr(ni);
  if (!tpr) return QRCP_ERR_UNSUPPORTED;
  const size_t need = lu_records_bytes(d, ni);
  if (need > rec_bytes) return QRCP_ERR_WORKSPACE;
  const int R = NT / tpr;
  const int G = (int)((ni + R - 1) / R);
  QRCP_TRY(launch_fill_u64(rec, (i64)(need / sizeof(uint64_t)), SENT, st));
  LuArgs args{Msk, (long)ld, d, (long)ni, Xw, rec, (long*)ipiv, (long*)jsk, status_dev};
  void* params[] = {&args};
  const void* fn = tpr == 4 ? (const void*)lu_pivots_kernel<4>
                 : tpr == 2 ? (const void*)lu_pivots_kernel<2>
                            : (const void*)lu_pivots_kernel<1>;
  QRCP_TRY(launch_resident(fn, dim3(G), dim3(NT), params, 0, st));
  return QRCP_OK;
}

}  // namespace qrcp
