// Householder QR of the permuted wide sketch (Alg. 2 last step, GEQRF with the
// LAPACK DLARFG sign convention).
//
// Head (the first dh = min(d, ni) columns, the only sequential part): one
// cooperative kernel, workgroup w owning head columns [w PW, (w+1) PW) in LDS.
// Workgroup p factors its columns once the reflectors of panels 0..p-1 have
// been applied to them, publishes its reflectors V_p and their compact-WY
// factor T_p, and raises flag p; workgroups w > p wait for the flag and apply
// (I - V_p T_p V_p^T)^T to their own columns.  The panel factorization itself
// is a column-by-column DLARFG + rank-1 update inside LDS.  V, T (and the
// block columns of the full T) cross workgroups through device-coherent
// stores and loads, and a flag goes up only after its data's stores have
// completed, so no hand-off needs a cache-wide writeback or invalidation
// (an agent-scope fence), which would also disturb whatever runs beside.
//
// Tail (the remaining ni - dh columns): R_tail = Q^T B_tail with the explicit
// d x d Q = I - V T V^T, T from the UT transform of V^T V, all on the GEMM
// kernels.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "wave32.hpp"

namespace qrcp {

int launch_ut_zero_diag(double* T, i64 ldt, const double* tau, int n, hipStream_t st);
int launch_set_identity(double* dst, i64 ld, i64 n, hipStream_t st);

namespace {
constexpr int NT = 256;
constexpr int VCH = 64;  // rows of V_p staged per pass when applying
constexpr int VLD = VCH + 1;  // their LDS stride (odd: no bank conflicts)

struct HeadArgs {
  const double* B;
  long ldb;
  int d, dh, pw;
  double* R;
  long ldr;
  double* V;      // d x dh, clean unit lower trapezoidal
  double* tau;    // dh
  double* T;      // npanels x pw x pw
  int* flags;     // npanels, zero on entry
  int* status;
  double* Tfull;  // may be null: dh x dh T of all panels (ld dh), by the block recursion
  int* tflags;    // npanels, zero on entry: block column w of Tfull is final
};

typedef double hv4 __attribute__((ext_vector_type(4)));
typedef double dv4 __attribute__((ext_vector_type(4)));

// W(32 x 32) = V_p^T C over rows [p0, d): V_p staged from global in row chunks,
// C in LDS.  Wave w owns the 16 x 16 block (w & 1, w >> 1) of W; FP64 MFMA.
// Then C -= V_p W' with W' = T_p^T W.  PW = 32 only (the MFMA path).
__device__ void apply_panel_mfma(double* sC, int d, int ldc, const double* V, int p0, int pc,
                                 const double* Tg,
                                 double* sV, double* sW, double* sT, double* sW2) {
  constexpr int PW = 32;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < PW * PW; e += NT) sT[e] = load_agent_d(Tg + e);
  hv4 acc = {0.0, 0.0, 0.0, 0.0};
  const int bi = w & 1, bj = w >> 1;
  for (int r0 = p0; r0 < d; r0 += VCH) {
    const int rows = min(VCH, d - r0);
    __syncthreads();
    for (int e = tid; e < VCH * PW; e += NT) {
      const int rr = e % VCH, aa = e / VCH;
      sV[aa * VLD + rr] = (rr < rows && aa < pc) ? load_agent_d(V + (r0 + rr) + (long)(p0 + aa) * d) : 0.0;
    }
    __syncthreads();
    for (int k0 = 0; k0 < rows; k0 += 4) {
      const int kr = k0 + (lane >> 4);
      // src0 = A(i, k) = V(r0 + k, 16 bi + i); src1 = B(k, j) = C(r0 + k, 16 bj + j)
      const double a = (kr < rows) ? sV[(16 * bi + (lane & 15)) * VLD + kr] : 0.0;
      const double b = (kr < rows) ? sC[(16 * bj + (lane & 15)) * ldc + r0 + kr] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
  // D(i, j): lane l, reg r -> i = 4 r + l/16, j = l % 16
#pragma unroll
  for (int r = 0; r < 4; ++r) sW[(16 * bi + 4 * r + (lane >> 4)) * PW + 16 * bj + (lane & 15)] = acc[r];
  __syncthreads();
  // W' = T^T W (T upper): W'(a, c) = sum_{t <= a} T(t, a) W(t, c)
  for (int e = tid; e < PW * PW; e += NT) {
    const int aa = e / PW, c = e % PW;
    double s = 0.0;
    for (int t = 0; t <= aa; ++t) s += sT[t + aa * PW] * sW[t * PW + c];
    sW2[aa * PW + c] = s;
  }
  // C -= V W' over row chunks; 16 x 16 output blocks spread over the waves
  for (int r0 = p0; r0 < d; r0 += VCH) {
    const int rows = min(VCH, d - r0);
    __syncthreads();
    for (int e = tid; e < VCH * PW; e += NT) {
      const int rr = e % VCH, aa = e / VCH;
      sV[aa * VLD + rr] = (rr < rows && aa < pc) ? load_agent_d(V + (r0 + rr) + (long)(p0 + aa) * d) : 0.0;
    }
    __syncthreads();
    const int nrb = (rows + 15) / 16;
    for (int blk = w; blk < nrb * 2; blk += NT / 64) {
      const int rb = blk >> 1, cb = blk & 1;
      hv4 c4 = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < PW; k0 += 4) {
        const int kr = k0 + (lane >> 4);
        // src0 = A(i, k) = V(r0 + 16 rb + i, k), src1 = B(k, j) = W'(k, 16 cb + j)
        const double a = sV[kr * VLD + 16 * rb + (lane & 15)];
        const double b = sW2[kr * PW + 16 * cb + (lane & 15)];
        c4 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c4, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * rb + 4 * r + (lane >> 4), j = 16 * cb + (lane & 15);
        if (i < rows) sC[j * ldc + r0 + i] -= c4[r];
      }
    }
  }
  __syncthreads();
}

template <int PW>
__global__ __launch_bounds__(NT) void sketch_head_kernel(Gate gt, HeadArgs a) {
  QRCP_GATE(gt);
  extern __shared__ double smem[];
  const int d = a.d, dh = a.dh;
  const int ldc = d + 1;                   // odd column stride: no LDS bank conflicts across columns
  double* sC = smem;                       // PW columns x d rows
  double* sV = sC + (long)PW * ldc;        // VCH x PW staging
  double* sW = sV + VLD * PW;              // PW x PW
  double* sT = sW + PW * PW;               // PW x PW
  double* sPart = sT + PW * PW;            // max(PW x PW, NT) scratch
  __shared__ double sTau[PW];
  __shared__ double sInv[PW];
  __shared__ int sbad;

  const int w = blockIdx.x;
  const int tid = threadIdx.x;
  const int c0 = w * PW;
  const int ncol = min(PW, dh - c0);
  constexpr int RG = NT / PW;  // row groups
  const int cg = tid % PW, rg = tid / PW;

  for (int e = tid; e < PW * d; e += NT) {
    const int c = e / d, r = e % d;
    sC[c * ldc + r] = (c < ncol) ? a.B[r + (long)(c0 + c) * a.ldb] : 0.0;
  }
  if (tid == 0) sbad = 0;
  __syncthreads();

  // ---- apply the reflectors of the panels before mine ----
  for (int p = 0; p < w; ++p) {
    const int p0 = p * PW;
    const int pc = min(PW, dh - p0);
    if (tid == 0) {
      long spins = 0;
      while (load_agent_i32(a.flags + p) == 0) {
        if (++spins > kSpinLimit) { sbad = 1; break; }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __syncthreads();
    if (sbad) {
      if (tid == 0) store_agent_i32(a.status, QRCP_ERR_TIMEOUT);
      return;
    }
    // V_p and T_p are read with device-coherent loads: no fence needed
    if constexpr (PW == 32) {
      apply_panel_mfma(sC, d, ldc, a.V, p0, pc, a.T + (long)p * PW * PW, sV, sW, sT, sPart);
    } else {
      for (int e = tid; e < PW * PW; e += NT) sT[e] = load_agent_d(a.T + (long)p * PW * PW + e);
      for (int e = tid; e < PW * PW; e += NT) sW[e] = 0.0;
      __syncthreads();
      for (int r0 = p0; r0 < d; r0 += VCH) {
        const int rows = min(VCH, d - r0);
        for (int e = tid; e < VCH * PW; e += NT) {
          const int rr = e % VCH, aa = e / VCH;
          sV[aa * VLD + rr] = (rr < rows && aa < pc) ? load_agent_d(a.V + (r0 + rr) + (long)(p0 + aa) * d) : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < PW * PW; e += NT) {
          const int aa = e / PW, c = e % PW;
          double s = 0.0;
          for (int rr = 0; rr < rows; ++rr) s += sV[aa * VLD + rr] * sC[c * ldc + r0 + rr];
          sW[aa * PW + c] += s;
        }
        __syncthreads();
      }
      for (int e = tid; e < PW * PW; e += NT) {
        const int aa = e / PW, c = e % PW;
        double s = 0.0;
        for (int t = 0; t <= aa; ++t) s += sT[t + aa * PW] * sW[t * PW + c];
        sPart[aa * PW + c] = s;
      }
      __syncthreads();
      for (int r0 = p0; r0 < d; r0 += VCH) {
        const int rows = min(VCH, d - r0);
        for (int e = tid; e < VCH * PW; e += NT) {
          const int rr = e % VCH, aa = e / VCH;
          sV[aa * VLD + rr] = (rr < rows && aa < pc) ? load_agent_d(a.V + (r0 + rr) + (long)(p0 + aa) * d) : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < VCH * PW; e += NT) {
          const int rr = e % VCH, c = e / VCH;
          if (rr < rows) {
            double s = 0.0;
            for (int aa = 0; aa < pc; ++aa) s += sV[aa * VLD + rr] * sPart[aa * PW + c];
            sC[c * ldc + r0 + rr] -= s;
          }
        }
        __syncthreads();
      }
    }
  }

  // ---- factor my panel: one fused reduction per column ----
  // For column jj (diagonal row rj) every thread (rg, c) sums x_r(jj) x_r(c)
  // over its rows r > rj; slot c = jj is ||x||^2.  With v = x / (alpha - beta)
  // the reflector acts on column c through w_c = x_rj(c) + s_c / (alpha - beta).
  // Column jj itself is scaled to v when the panel is published.
  for (int jj = 0; jj < ncol; ++jj) {
    const int rj = c0 + jj;
    const double* xj = sC + jj * ldc;
    {
      double s = 0.0;
      if (cg >= jj && cg < ncol)
        for (int r = rj + 1 + rg; r < d; r += RG) s += xj[r] * sC[cg * ldc + r];
      sPart[rg * PW + cg] = s;
    }
    __syncthreads();
    if (tid < PW) {
      double t = 0.0;
      for (int q = 0; q < RG; ++q) t += sPart[q * PW + tid];
      sW[tid] = t;
    }
    __syncthreads();
    const double xx = sW[jj];
    const double alpha = xj[rj];
    double beta = alpha, tau = 0.0, inv = 1.0;
    if (xx != 0.0) {
      const double nrm = sqrt(alpha * alpha + xx);
      beta = (alpha < 0.0) ? nrm : -nrm;
      tau = (beta - alpha) / beta;
      inv = alpha - beta;
    }
    // Every thread of column cg reads x_rj(cg) here; the entry itself is
    // updated only after the barrier below (threads of several waves share a
    // column, so an earlier write would race with their reads).
    double f = 0.0;
    const bool upd = tau != 0.0 && cg > jj && cg < ncol;
    if (upd) {
      const double wc = sC[cg * ldc + rj] + sW[cg] / inv;
      f = tau * wc;
      const double fv = f / inv;
      for (int r = rj + 1 + rg; r < d; r += RG) sC[cg * ldc + r] -= fv * xj[r];
    }
    if (tid == 0) {
      sTau[jj] = tau;
      sInv[jj] = (xx != 0.0) ? inv : 0.0;
      a.tau[rj] = tau;
      a.R[rj + (long)rj * a.ldr] = beta;
    }
    __syncthreads();
    // row rj is read again only by the publication below
    if (upd && rg == 0) sC[cg * ldc + rj] -= f;
  }
  __syncthreads();

  // ---- publish V_p (clean), R part above the diagonal, and T_p ----
  for (int e = tid; e < PW * d; e += NT) {
    const int c = e / d, r = e % d;
    if (c < ncol) {
      const int rc = c0 + c;
      double v = sC[c * ldc + r];
      if (r > rc) v = (sInv[c] != 0.0) ? v / sInv[c] : 0.0;
      sC[c * ldc + r] = (r == rc) ? 1.0 : v;   // keep the scaled vector for T below
      store_agent_d(a.V + r + (long)rc * d, (r < rc) ? 0.0 : (r == rc ? 1.0 : v));
      if (r < rc) a.R[r + (long)rc * a.ldr] = v;
      else if (r > rc) a.R[r + (long)rc * a.ldr] = 0.0;
    }
  }
  __syncthreads();
  // T_p by the LARFT recurrence (robust to tau = 0): G = V^T V first
  for (int e = tid; e < PW * PW; e += NT) {
    const int i = e / PW, j = e % PW;
    double s = 0.0;
    if (i < j && j < ncol) {
      const int rjj = c0 + j;
      // V(:, i)^T V(:, j): rows >= rjj (V(r, j) = 0 above rjj, 1 at rjj)
      s = sC[i * ldc + rjj];
      for (int r = rjj + 1; r < d; ++r) s += sC[i * ldc + r] * sC[j * ldc + r];
    }
    sW[i * PW + j] = s;  // G(i, j) for i < j
  }
  __syncthreads();
  if (tid < 64) {
    // sequential over columns j, parallel over rows i < j (one wave)
    for (int j = 0; j < PW; ++j) {
      const double tj = (j < ncol) ? sTau[j] : 0.0;
      double val = 0.0;
      const int i = tid;
      if (i < j) {
        for (int t = i; t < j; ++t) val += sT[i + t * PW] * sW[t * PW + j];
        val = -tj * val;
      }
      __builtin_amdgcn_wave_barrier();
      if (i < j) sT[i + j * PW] = val;
      if (i == j) sT[j + j * PW] = tj;
      if (i > j && i < PW) sT[i + j * PW] = 0.0;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int e = tid; e < PW * PW; e += NT) store_agent_d(a.T + (long)w * PW * PW + e, sT[e]);
  __builtin_amdgcn_s_waitcnt(0);  // V and T (device-coherent stores) are in memory
  __syncthreads();
  if (tid == 0) store_agent_i32(a.flags + w, 1);
}

// ---------------------------------------------------------------------------
// Register-resident variant for d <= 320.  Wave s (0..3), lane j + 16 kk of
// the 256 threads holds panel columns j and 16 + j in rows 16 i + 4 s + kk
// (i < NR2, rows past d are zero).  In this layout a lane's register is the
// matrix-core operand B(k = kk, j) of a 4-row slab, so applying a previous
// panel, C -= V_q (T_q^T (V_q^T C)), runs on the FP64 matrix cores straight
// from registers (V_q staged in LDS).  One Householder column costs one
// workgroup barrier: the column is broadcast inside each wave through LDS
// (the rows a wave needs are the rows it holds), one fused reduction gives,
// for every panel column c, x_j . x_c over the rows below the diagonal (the
// reflector's action for c > j, the squared norm for c = j, the Gram entry
// v_c^T v_j for c < j, from which the panel's T follows by the UT transform).
// ---------------------------------------------------------------------------
constexpr int PWR = 32;  // panel width
constexpr int LDP = 33;  // padded LDS row stride

template <int NR2>
__global__ __launch_bounds__(NT) void sketch_head_reg_kernel(Gate gt, HeadArgs a) {
  QRCP_GATE(gt);
  static_assert(NR2 % 4 == 0, "row slabs come in groups of four");
  extern __shared__ double smem[];
  constexpr int DP = 16 * NR2;             // rows held (>= d); rows d.. are zero
  const int d = a.d, dh = a.dh;
  double* sV = smem;                       // DP x LDP: V_q of the panel being applied
  double* sWp = sV + (size_t)DP * LDP;     // 4 x PWR x LDP: per-wave partial V_q^T C
  double* sW = sWp + 4 * PWR * LDP;        // PWR x LDP: W = V_q^T C
  double* sW2 = sW + PWR * LDP;            // PWR x LDP: T_q^T W (then the Gram entries G)
  double* sG = sW2;
  double* sT = sW2 + PWR * LDP;            // PWR x LDP: T (applied panel's, then own)
  double* sXb = sT + PWR * LDP;            // DP: broadcast column
  double* sRed = sXb + DP;                 // 2 x 4 x PWR: per-wave column sums
  double* sRowJ = sRed + 2 * 4 * PWR;      // 2 x PWR: row rj of the panel
  double* sTau = sRowJ + 2 * PWR;          // PWR
  double* sInv = sTau + PWR;               // PWR: 1 / (alpha_j - beta_j) (1 when tau_j = 0)
  __shared__ int sbad;

  const int w = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, ws = tid >> 6;
  const int j = lane & 15, kk = lane >> 4;
  const int c0 = w * PWR;
  const int ncol = min(PWR, dh - c0);
  const int rbase = 4 * ws + kk;           // my rows: rbase + 16 i

  double x0[NR2], x1[NR2];                 // columns j and 16 + j
#pragma unroll
  for (int i = 0; i < NR2; ++i) {
    const int r = rbase + 16 * i;
    x0[i] = (j < ncol && r < d) ? a.B[r + (long)(c0 + j) * a.ldb] : 0.0;
    x1[i] = (16 + j < ncol && r < d) ? a.B[r + (long)(c0 + 16 + j) * a.ldb] : 0.0;
  }
  if (tid == 0) sbad = 0;

  // ---- apply the reflectors of the panels before mine ----
  for (int p = 0; p < w; ++p) {
    const int p0 = p * PWR;
    const int pc = min(PWR, dh - p0);
    // panel flag: 1 = V_p published, 2 = T_p published as well
    auto wait_flag = [&](int v) -> bool {
      if (tid == 0) {
        long spins = 0;
        while (load_agent_i32(a.flags + p) < v) {
          if (++spins > kSpinLimit) { sbad = 1; break; }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      __syncthreads();
      if (sbad) {
        if (tid == 0) store_agent_i32(a.status, QRCP_ERR_TIMEOUT);
        return false;
      }
      // V_p and T_p are read with device-coherent loads: no fence needed
      return true;
    };
    if (!wait_flag(1)) return;
    {
      // V_p: every load requested before the first LDS store (one memory
      // latency), consecutive threads on consecutive rows of a column
      constexpr int QV = DP * PWR / NT;
      double vr[QV];
#pragma unroll
      for (int q = 0; q < QV; ++q) {
        const int e = tid + NT * q, rr = e % DP, aa = e / DP;
        vr[q] = (aa < pc && rr >= p0 && rr < d) ? load_agent_d(a.V + rr + (long)(p0 + aa) * d) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < QV; ++q) {
        const int e = tid + NT * q, rr = e % DP, aa = e / DP;
        sV[rr * LDP + aa] = vr[q];
      }
    }
    __syncthreads();
    // partial W(aa, c) over my rows: D = A B with A(aa, k) = V(row k, aa), B(k, c) = C(row k, c)
    dv4 acc[2][2];
#pragma unroll
    for (int ab = 0; ab < 2; ++ab)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[ab][cb] = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < NR2; ++i) {
      const double* vr = sV + (rbase + 16 * i) * LDP;
      const double a0 = vr[j], a1 = vr[16 + j];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x0[i], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x1[i], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x0[i], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x1[i], acc[1][1], 0, 0, 0);
    }
    // D(aa, c) sits in lane c + 16 (aa % 4), register aa / 4
#pragma unroll
    for (int ab = 0; ab < 2; ++ab)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          sWp[(ws * PWR + 16 * ab + 4 * rr + kk) * LDP + 16 * cb + j] = acc[ab][cb][rr];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + NT * q, aa = e / PWR, c = e % PWR;
      sW[aa * LDP + c] = (sWp[aa * LDP + c] + sWp[(PWR + aa) * LDP + c]) +
                         (sWp[(2 * PWR + aa) * LDP + c] + sWp[(3 * PWR + aa) * LDP + c]);
    }
    // T_p (published after V_p, while this workgroup formed W)
    if (!wait_flag(2)) return;
    {
      constexpr int QT = PWR * PWR / NT;
      double tr[QT];
#pragma unroll
      for (int q = 0; q < QT; ++q) tr[q] = load_agent_d(a.T + (long)p * PWR * PWR + tid + NT * q);
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        const int e = tid + NT * q;
        sT[(e % PWR) * LDP + e / PWR] = tr[q];  // T(i, j) at i + PWR j
      }
    }
    __syncthreads();
    // W' = T^T W: wave ws computes block (ws & 1, ws >> 1)
    {
      const int ab = ws & 1, cb = ws >> 1;
      dv4 t4 = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k0 = 0; k0 < PWR; k0 += 4)
        t4 = __builtin_amdgcn_mfma_f64_16x16x4f64(sT[(k0 + kk) * LDP + 16 * ab + j],
                                                  sW[(k0 + kk) * LDP + 16 * cb + j], t4, 0, 0, 0);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) sW2[(16 * ab + 4 * rr + kk) * LDP + 16 * cb + j] = t4[rr];
    }
    __syncthreads();
    // C -= V W': output rows 16 (i0 + rr) + rbase land in register i0 + rr of this lane
#pragma unroll
    for (int i0 = 0; i0 < NR2; i0 += 4) {
      dv4 u0 = dv4{0.0, 0.0, 0.0, 0.0}, u1 = dv4{0.0, 0.0, 0.0, 0.0};
      const double* vr = sV + (16 * (i0 + (j >> 2)) + 4 * ws + (j & 3)) * LDP;
#pragma unroll
      for (int k0 = 0; k0 < PWR; k0 += 4) {
        const double av = vr[k0 + kk];
        u0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sW2[(k0 + kk) * LDP + j], u0, 0, 0, 0);
        u1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sW2[(k0 + kk) * LDP + 16 + j], u1, 0, 0, 0);
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        x0[i0 + rr] -= u0[rr];
        x1[i0 + rr] -= u1[rr];
      }
    }
    __syncthreads();
  }

  // ---- factor my panel ----
  // Columns stay unscaled while the panel is factored (x_j below row rj; the
  // reflector is v_j = x_j / (alpha_j - beta_j)).  Register i holds row group
  // sh + i (rows 16 (sh + i) + rbase).  Groups above the pivot row are final:
  // they are written out (R on and above the diagonal, the scaled reflectors
  // below it) and shifted away, so the pivot row's group is always register 0
  // and, with the panel's two 16-column halves as compile-time cases, every
  // row and column selection below is resolved at compile time.
  int sh = 0;
  auto emit = [&](int i, double v0, double v1) {
    const int r = 16 * (sh + i) + rbase;
    if (r >= d) return;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cl = 16 * h + j;
      if (cl < ncol) {
        const int rc = c0 + cl;
        const double v = h ? v1 : v0;
        store_agent_d(a.V + r + (long)rc * d, (r < rc) ? 0.0 : (r == rc ? 1.0 : v * sInv[cl]));
        a.R[r + (long)rc * a.ldr] = (r <= rc) ? v : 0.0;
      }
    }
  };
  auto shift1 = [&]() {
#pragma unroll
    for (int i = 0; i + 1 < NR2; ++i) {
      x0[i] = x0[i + 1];
      x1[i] = x1[i + 1];
    }
    x0[NR2 - 1] = 0.0;
    x1[NR2 - 1] = 0.0;
    ++sh;
  };
  // rows above the panel: final after the apply phase
  for (int g = 0; g < (c0 >> 4); ++g) {
    emit(0, x0[0], x1[0]);
    shift1();
  }
  auto col_step = [&](auto hic, int jc) {
    constexpr bool HI = decltype(hic)::value;
    double(&xc)[NR2] = HI ? x1 : x0;  // the half holding column jc
    const int rj = c0 + jc;
    const int jl = jc & 15;          // pivot row within its group (register 0)
    const int buf = jc & 1;
    const bool holder = (rbase == jl);  // my lane holds row rj
    if (j == jl) {
#pragma unroll
      for (int i = 0; i < NR2; ++i) sXb[rbase + 16 * i] = xc[i];
    }
    wave_lds_sync();
    double xj[NR2];
    double s0a = 0.0, s0b = 0.0, s1a = 0.0, s1b = 0.0;
#pragma unroll
    for (int i = 0; i < NR2; ++i) {
      const double v = sXb[rbase + 16 * i];
      xj[i] = (i > 0 || rbase > jl) ? v : 0.0;  // rows below rj only
      if (i & 1) {
        s0b = fma(xj[i], x0[i], s0b);
        s1b = fma(xj[i], x1[i], s1b);
      } else {
        s0a = fma(xj[i], x0[i], s0a);
        s1a = fma(xj[i], x1[i], s1a);
      }
    }
    double s0 = s0a + s0b, s1 = s1a + s1b;
    s0 = xsum_lanes16(s0);
    s1 = xsum_lanes16(s1);
    s0 = xsum_lanes32(s0);
    s1 = xsum_lanes32(s1);
    wave_lds_sync();  // this step's reads of sXb before the next step's writes
    if (kk == 0) {
      sRed[(buf * 4 + ws) * PWR + j] = s0;
      sRed[(buf * 4 + ws) * PWR + 16 + j] = s1;
    }
    if (holder) {
      sRowJ[buf * PWR + j] = x0[0];
      sRowJ[buf * PWR + 16 + j] = x1[0];
    }
    __syncthreads();
    const double* red = sRed + buf * 4 * PWR;
    const double S0 = (red[j] + red[PWR + j]) + (red[2 * PWR + j] + red[3 * PWR + j]);
    const double S1 = (red[16 + j] + red[PWR + 16 + j]) + (red[2 * PWR + 16 + j] + red[3 * PWR + 16 + j]);
    const double xx = (red[jc] + red[PWR + jc]) + (red[2 * PWR + jc] + red[3 * PWR + jc]);
    const double alpha = sRowJ[buf * PWR + jc];
    // DLARFG: v = x / (alpha - beta) is formed, as LAPACK does, with the
    // reciprocal rinv = 1 / (alpha - beta)
    double beta = alpha, tau = 0.0, rinv = 1.0;
    if (xx != 0.0) {
      const double nrm = sqrt(alpha * alpha + xx);
      beta = (alpha < 0.0) ? nrm : -nrm;
      tau = (beta - alpha) / beta;
      rinv = 1.0 / (alpha - beta);
    }
    if (tau != 0.0) {
      // the reflector acts on my columns to the right of jc
      const bool u0c = j > jc && j < ncol, u1c = 16 + j > jc && 16 + j < ncol;
      const double f0 = u0c ? tau * (sRowJ[buf * PWR + j] + S0 * rinv) : 0.0;
      const double f1 = u1c ? tau * (sRowJ[buf * PWR + 16 + j] + S1 * rinv) : 0.0;
      const double fv0 = f0 * rinv, fv1 = f1 * rinv;
      x0[0] -= fv0 * xj[0] + (holder ? f0 : 0.0);
      x1[0] -= fv1 * xj[0] + (holder ? f1 : 0.0);
#pragma unroll
      for (int i = 1; i < NR2; ++i) {
        x0[i] -= fv0 * xj[i];
        x1[i] -= fv1 * xj[i];
      }
    }
    if (holder && j == jl) xc[0] = beta;
    // G(i, jc) = v_i^T v_jc = (x_i(rj) + S_i rinv_jc) rinv_i for i < jc
    if (tid < PWR) {
      const int i = tid;
      if (i < jc) {
        const double Si = (red[i] + red[PWR + i]) + (red[2 * PWR + i] + red[3 * PWR + i]);
        sG[i * LDP + jc] = (sRowJ[buf * PWR + i] + Si * rinv) * sInv[i];
      }
      if (i == 0) {
        sTau[jc] = tau;
        sInv[jc] = rinv;
        a.tau[rj] = tau;
      }
    }
  };
  for (int jc = 0; jc < min(ncol, 16); ++jc) col_step(std::false_type{}, jc);
  if (ncol > 16) {
    __syncthreads();  // sInv of the first half
    emit(0, x0[0], x1[0]);  // rows c0 .. c0+15: final for the whole panel
    shift1();
    for (int jc = 16; jc < ncol; ++jc) col_step(std::true_type{}, jc);
  }
  __syncthreads();

  // ---- publish V (clean, scaled) and R of the remaining rows: the next
  // workgroups start forming V^T C while T is computed ----
#pragma unroll
  for (int i = 0; i < NR2; ++i) emit(i, x0[i], x1[i]);
  __builtin_amdgcn_s_waitcnt(0);  // V (device-coherent stores) is in memory
  __syncthreads();
  if (tid == 0) store_agent_i32(a.flags + w, 1);

  // ---- T of the panel: invert diag(1/tau) + striu(G) (a zero tau decouples
  // its index: its row and column of T are zero) ----
  if (tid < 64) {
    if (lane < PWR) {
#pragma unroll
      for (int r = 0; r < W32; ++r) {
        double v = 0.0;
        if (lane < ncol && r < ncol && r <= lane) {
          const double tr = sTau[r], tc = sTau[lane];
          if (tr == 0.0 || tc == 0.0) v = (r == lane) ? 1.0 : 0.0;
          else if (r == lane) v = 1.0 / tc;
          else v = sG[r * LDP + lane];
        }
        sG[r * LDP + lane] = v;
      }
    }
    double ty[W32];
    wave_inv_upper32(sG, LDP, ty, ncol);
    if (lane < PWR) {
#pragma unroll
      for (int r = 0; r < W32; ++r) {
        double v = (lane < ncol && r < ncol) ? ty[r] : 0.0;
        if (lane < ncol && r == lane && sTau[lane] == 0.0) v = 0.0;
        sT[r * LDP + lane] = v;
      }
    }
  }
  __syncthreads();

  for (int e = tid; e < PWR * PWR; e += NT) {
    const int i = e % PWR, jj = e / PWR;
    store_agent_d(a.T + (long)w * PWR * PWR + e, (i < ncol && jj < ncol) ? sT[i * LDP + jj] : 0.0);
  }
  __builtin_amdgcn_s_waitcnt(0);  // T (device-coherent stores) is in memory
  __syncthreads();
  if (tid == 0) store_agent_i32(a.flags + w, 2);

  // ---- block column w of the T of all panels (LARFT block recursion):
  // T(0:c0, c0:c0+32) = -T(0:c0, 0:c0) (V(:, 0:c0)^T V_w) T_w, T_w on the
  // diagonal.  Done here, on this workgroup's own compute unit while the next
  // panel is factored, so the tail needs no Gram product or triangular
  // inverse.  Columns of earlier panels come from their workgroups (tflags).
  if (a.Tfull) {
    const long ldt = dh;
    const int qi = ws & 1, qj = ws >> 1;
    const int li = lane & 15, lk = lane >> 4;
    for (int e = tid; e < PWR * PWR; e += NT) {
      const int i = e % PWR, jj = e / PWR;
      if (i < ncol && jj < ncol) store_agent_d(a.Tfull + (c0 + i) + (long)(c0 + jj) * ldt, sT[i * LDP + jj]);
    }
    // T is upper triangular: zero below the diagonal block
    const int below = dh - c0 - ncol;
    for (int e = tid; e < below * ncol; e += NT)
      store_agent_d(a.Tfull + (c0 + ncol + e % below) + (long)(c0 + e / below) * ldt, 0.0);
    if (w > 0) {
      // V_w, rows c0 .. d-1 (zero above), to LDS as [k][j], k = row - c0
      const int K = d - c0;
      for (int e = tid; e < K * PWR; e += NT) {
        const int k = e % K, jj = e / K;
        sV[k * LDP + jj] = (jj < ncol) ? load_agent_d(a.V + (c0 + k) + (long)(c0 + jj) * d) : 0.0;
      }
      __syncthreads();
      for (int I = 0; I < w; ++I) {
        // Y_I = V_I^T V_w over rows c0 .. d-1: A(i, k) = V(c0 + k, 32 I + i)
        const double* vcol = a.V + (long)(PWR * I + 16 * qi + li) * d + c0;  // device-coherent loads
        dv4 acc = dv4{0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < K; k0 += 32) {
          double av[8];
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const int k = k0 + 4 * b + lk;
            av[b] = (k < K) ? load_agent_d(vcol + k) : 0.0;
          }
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const int k = k0 + 4 * b + lk;
            const double bv = (k < K) ? sV[k * LDP + 16 * qj + li] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bv, av[b], acc, 0, 0, 0);
          }
        }
        // acc[r] = Y_I(16 qi + li, 16 qj + 4 r + lk)
#pragma unroll
        for (int r = 0; r < 4; ++r) sW[(16 * qi + li) * LDP + 16 * qj + 4 * r + lk] = acc[r];
        __syncthreads();
        // Y'_I = Y_I T_w, parked in T(32 I .., c0 ..) until Z overwrites it
        dv4 acc2 = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = 4 * s + lk;
          acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(sT[k * LDP + 16 * qj + li],
                                                      sW[(16 * qi + li) * LDP + k], acc2, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int jj = 16 * qj + 4 * r + lk;
          if (jj < ncol) store_agent_d(a.Tfull + (PWR * I + 16 * qi + li) + (long)(c0 + jj) * ldt, acc2[r]);
        }
        __syncthreads();
      }
      // columns 0 .. c0 of T, published by the earlier workgroups
      if (tid == 0) {
        for (int q = 0; q < w && !sbad; ++q) {
          long spins = 0;
          while (load_agent_i32(a.tflags + q) == 0) {
            if (++spins > kSpinLimit) { sbad = 1; break; }
            __builtin_amdgcn_s_sleep(2);
          }
        }
      }
      __syncthreads();
      if (sbad) {
        if (tid == 0) store_agent_i32(a.status, QRCP_ERR_TIMEOUT);
        return;
      }
      // earlier block columns are read with device-coherent loads: no fence needed
      // Z_I = -sum_{J=I}^{w-1} T(I, J) Y'_J for I = 0 .. w-1, written over Y'_I
      for (int I = 0; I < w; ++I) {
        dv4 acc = dv4{0.0, 0.0, 0.0, 0.0};
        for (int J = I; J < w; ++J) {
          double av[8], bv[8];
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int k = 4 * s + lk;
            av[s] = load_agent_d(a.Tfull + (PWR * I + 16 * qi + li) + (long)(PWR * J + k) * ldt);
            const int jj = 16 * qj + li;
            bv[s] = (jj < ncol) ? load_agent_d(a.Tfull + (PWR * J + k) + (long)(c0 + jj) * ldt) : 0.0;
          }
#pragma unroll
          for (int s = 0; s < 8; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[s], av[s], acc, 0, 0, 0);
        }
        __syncthreads();  // every wave has read Y'_I
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int jj = 16 * qj + 4 * r + lk;
          if (jj < ncol) store_agent_d(a.Tfull + (PWR * I + 16 * qi + li) + (long)(c0 + jj) * ldt, -acc[r]);
        }
        __syncthreads();
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this block column is in memory
    __syncthreads();
    if (tid == 0) store_agent_i32(a.tflags + w, 1);
  }
}

}  // namespace

static int head_pw(int d) { return d <= 320 ? 32 : (d <= 640 ? 16 : 8); }

int sketch_head_groups(int d, i64 ni) {
  const int dh = (int)std::min((i64)d, ni);
  const int pw = head_pw(d);
  return (dh + pw - 1) / pw;
}

size_t sketch_qr_ws_bytes(int d, i64 ni) {
  const int dh = (int)std::min((i64)d, ni);
  const int pw = head_pw(d);
  const int np = (dh + pw - 1) / pw;
  size_t b = 0;
  b += (size_t)d * dh * 8;          // V
  b += (size_t)dh * 8;              // tau
  b += (size_t)np * pw * pw * 8;    // T panels
  b += (size_t)dh * dh * 8;         // V^T V -> T full
  b += (size_t)dh * dh * 8;         // T full
  b += (size_t)dh * d * 8;          // X = T V^T
  b += (size_t)d * d * 8;           // Q
  b += (size_t)(np + 1) * 8 + 256;  // panel flags, T column flags
  b += gemm_splitk_bytes(dh, dh, 64);
  return b + 8 * 64;
}

int run_sketch_qr(const double* B, int d, i64 ni, i64 ldb, double* R, i64 ldr, void* ws,
                  size_t ws_bytes, int* status_dev, hipStream_t st) {
  if (d <= 0 || ni <= 0) return QRCP_OK;
  if (d > 1024) return QRCP_ERR_UNSUPPORTED;  // the tail inverts a dh x dh triangle
  if (ws_bytes < sketch_qr_ws_bytes(d, ni)) return QRCP_ERR_WORKSPACE;
  const int dh = (int)std::min((i64)d, ni);
  const int pw = head_pw(d);
  const int np = (dh + pw - 1) / pw;
  char* p = (char*)ws;
  auto take = [&](size_t bytes) { char* q = p; p += (bytes + 255) / 256 * 256; return q; };
  double* V = (double*)take((size_t)d * dh * 8);
  double* tau = (double*)take((size_t)dh * 8);
  double* Tp = (double*)take((size_t)np * pw * pw * 8);
  double* G = (double*)take((size_t)dh * dh * 8);
  double* T = (double*)take((size_t)dh * dh * 8);
  double* X = (double*)take((size_t)dh * d * 8);
  double* Q = (double*)take((size_t)d * d * 8);
  int* flags = (int*)take((size_t)(np + 1) * 8);  // panel flags, then the T column flags
  double* split = (double*)take(gemm_splitk_bytes(dh, dh, 64));
  const size_t split_bytes = gemm_splitk_bytes(dh, dh, 64);

  QRCP_TRY(launch_fill_u64((uint64_t*)flags, np + 1, 0ull, st));
  const bool tfull = d <= 320;  // the register head builds T of all panels
  HeadArgs args{B, (long)ldb, d, dh, pw, R, (long)ldr, V, tau, Tp, flags, status_dev,
                tfull ? T : nullptr, flags + np};
  Gate gt = current_gate();
  void* params[] = {&gt, &args};
  if (d <= 320) {
    const int nr2 = d <= 128 ? 8 : (d <= 192 ? 12 : 20);
    const size_t dp = (size_t)16 * nr2;
    const size_t smem_r = (dp * LDP + 4 * PWR * LDP + 3 * PWR * LDP + dp + 8 * PWR + 2 * PWR +
                           2 * PWR) * 8;
    const void* fr = nr2 == 8 ? (const void*)sketch_head_reg_kernel<8>
                   : nr2 == 12 ? (const void*)sketch_head_reg_kernel<12>
                               : (const void*)sketch_head_reg_kernel<20>;
    QRCP_HIP(hipFuncSetAttribute(fr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_r));
    QRCP_TRY(launch_resident(fr, dim3(np), dim3(NT), params, smem_r, st));
  } else {
  const size_t smem = ((size_t)pw * (d + 1) + VLD * pw + 2 * pw * pw + std::max<size_t>((size_t)pw * pw, NT)) * 8;
  const void* fn = pw == 32 ? (const void*)sketch_head_kernel<32>
                 : pw == 16 ? (const void*)sketch_head_kernel<16>
                            : (const void*)sketch_head_kernel<8>;
  QRCP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  QRCP_TRY(launch_resident(fn, dim3(np), dim3(NT), params, smem, st));
  }

  if (ni > dh) {
    if (!tfull) {
      // T = (diag(1/tau) + striu(V^T V))^{-1}
      GemmArgs g;
      g.M = dh; g.N = dh; g.K = d; g.A = V; g.lda = d; g.B = V; g.ldb = d; g.C = G; g.ldc = dh;
      QRCP_TRY(gemm(true, false, Prec::F64, g, split, split_bytes, st));
      QRCP_TRY(launch_ut_tinv(G, dh, tau, dh, st));
      QRCP_TRY(launch_trinv_upper(G, dh, dh, T, dh, st, true));  // runs beside the deferred update
      QRCP_TRY(launch_ut_zero_diag(T, dh, tau, dh, st));
    }
    // X = T V^T (dh x d)
    GemmArgs x;
    x.M = dh; x.N = d; x.K = dh; x.A = T; x.lda = dh; x.B = V; x.ldb = d; x.C = X; x.ldc = dh;
    QRCP_TRY(gemm(false, true, Prec::F64, x, nullptr, 0, st));
    // Q = I - V X
    QRCP_TRY(launch_set_identity(Q, d, d, st));
    GemmArgs q;
    q.M = d; q.N = d; q.K = dh; q.alpha = -1.0; q.beta = 1.0;
    q.A = V; q.lda = d; q.B = X; q.ldb = dh; q.C = Q; q.ldc = d;
    QRCP_TRY(gemm(false, false, Prec::F64, q, nullptr, 0, st));
    // R_tail = Q^T B_tail
    GemmArgs r;
    r.M = d; r.N = (int)(ni - dh); r.K = d;
    r.A = Q; r.lda = d; r.B = B + (long)dh * ldb; r.ldb = ldb; r.C = R + (long)dh * ldr; r.ldc = ldr;
    QRCP_TRY(gemm(true, false, Prec::F64, r, nullptr, 0, st));
  }
  return QRCP_OK;
}

}  // namespace qrcp
