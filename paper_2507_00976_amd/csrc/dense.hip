// Sketching operator and the small dense kernels of the panel (triangular
// inverses, Cholesky, the sign-modified LU of the reconstruction, copies).
#include "common.hpp"
#include "kernels.hpp"
#include "wave32.hpp"

namespace qrcp {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply/xor S-box on the 4-word counter, the 2-word key advanced by the
// Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                   (uint32_t)p0);
  }
  return c;
}

__global__ void philox_kernel(Gate gt, const uint32_t* ctr, long count, uint32_t k0, uint32_t k1,
                              uint32_t* out) {
  QRCP_GATE(gt);
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
  c = philox4x32_10(c, k0, k1);
  out[4 * i] = c.x;
  out[4 * i + 1] = c.y;
  out[4 * i + 2] = c.z;
  out[4 * i + 3] = c.w;
}

// S^T (m x d, ld): S(2p, j), S(2p+1, j) from block (j, p, 0, 0) by Box-Muller.
// BITS: the entries as BF16 bits (the FP64 value rounded to FP32, then to BF16)
// in an array of 16-bit words, for the BF16 sketch product.
template <bool BITS>
__global__ void sketch_operator_kernel(Gate gt, void* out, long m, int d, long ld, uint32_t k0,
                                       uint32_t k1) {
  QRCP_GATE(gt);
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (j >= m) return;
  const uint4 x = philox4x32_10(make_uint4((uint32_t)j, (uint32_t)p, 0u, 0u), k0, k1);
  const uint64_t w01 = ((uint64_t)x.y << 32) | x.x;
  const uint64_t w23 = ((uint64_t)x.w << 32) | x.z;
  const double u1 = ((double)(w01 >> 12) * 2.0 + 1.0) * 0x1p-53;
  const double u2 = (double)(w23 >> 11) * 0x1p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = (2.0 * 3.141592653589793) * u2;
  const double s0 = rad * cos(ang);
  const double s1 = rad * sin(ang);
  if (BITS) {
    unsigned short* St = static_cast<unsigned short*>(out);
    St[j + (long)(2 * p) * ld] = to_bf16_bits(s0);
    if (2 * p + 1 < d) St[j + (long)(2 * p + 1) * ld] = to_bf16_bits(s1);
  } else {
    double* St = static_cast<double*>(out);
    St[j + (long)(2 * p) * ld] = s0;
    if (2 * p + 1 < d) St[j + (long)(2 * p + 1) * ld] = s1;
  }
}

int launch_sketch_operator(double* St, i64 m, int d, i64 ldst, uint64_t seed, hipStream_t st) {
  if (m <= 0 || d <= 0) return QRCP_OK;
  dim3 grid((m + 255) / 256, (d + 1) / 2);
  hipLaunchKernelGGL(sketch_operator_kernel<false>, grid, dim3(256), 0, st, current_gate(), (void*)St, m, d,
                     ldst, (uint32_t)seed, (uint32_t)(seed >> 32));
  QRCP_LAUNCHED("sketch_operator");
  return QRCP_OK;
}

int launch_sketch_operator_bf16(unsigned short* St, i64 m, int d, i64 ldst, uint64_t seed, hipStream_t st) {
  if (m <= 0 || d <= 0) return QRCP_OK;
  dim3 grid((m + 255) / 256, (d + 1) / 2);
  hipLaunchKernelGGL(sketch_operator_kernel<true>, grid, dim3(256), 0, st, current_gate(), (void*)St, m, d,
                     ldst, (uint32_t)seed, (uint32_t)(seed >> 32));
  QRCP_LAUNCHED("sketch_operator_bf16");
  return QRCP_OK;
}

int launch_philox(const uint32_t* ctr, i64 count, uint32_t k0, uint32_t k1, uint32_t* out,
                  hipStream_t st) {
  if (count <= 0) return QRCP_OK;
  hipLaunchKernelGGL(philox_kernel, dim3((count + 255) / 256), dim3(256), 0, st, current_gate(), ctr, count, k0,
                     k1, out);
  QRCP_LAUNCHED("philox");
  return QRCP_OK;
}

// ---------------------------------------------------------------------------
// Compact WY factor from Y^T Y and tau (UT transform: T^{-1} = diag(1/tau) +
// strictly-upper(Y^T Y)).  A zero tau (H_j = I) decouples index j: its row and
// column are cleared and T(j,j) = 0 afterwards.
// ---------------------------------------------------------------------------
__global__ void ut_prepare_kernel(Gate gt, double* G, long ldg, const double* tau, int n) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)n * n) return;
  const int i = idx % n, j = idx / n;
  double* g = G + i + (long)j * ldg;
  if (i > j) { *g = 0.0; return; }
  if (tau[i] == 0.0 || tau[j] == 0.0) { *g = (i == j) ? 1.0 : 0.0; return; }
  if (i == j) *g = 1.0 / tau[i];
}

__global__ void ut_zero_diag_kernel(Gate gt, double* T, long ldt, const double* tau, int n) {
  QRCP_GATE(gt);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n && tau[j] == 0.0) T[j + (long)j * ldt] = 0.0;
}

int launch_ut_tinv(double* G, i64 ldg, const double* tau, int n, hipStream_t st) {
  if (n <= 0) return QRCP_OK;
  hipLaunchKernelGGL(ut_prepare_kernel, dim3(((long)n * n + 255) / 256), dim3(256), 0, st, current_gate(), G, ldg,
                     tau, n);
  QRCP_LAUNCHED("ut_prepare");
  return QRCP_OK;
}

int launch_ut_zero_diag(double* T, i64 ldt, const double* tau, int n, hipStream_t st) {
  hipLaunchKernelGGL(ut_zero_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, st, current_gate(), T, ldt, tau, n);
  QRCP_LAUNCHED("ut_zero_diag");
  return QRCP_OK;
}

// ---------------------------------------------------------------------------
// LDS-staged 64 x 64 output tiles on the FP64 matrix cores, used by the
// single-workgroup factorizations below (256 threads = 4 waves, each wave a
// 32 x 32 quarter of the tile).
// ---------------------------------------------------------------------------
constexpr int SB = 32;  // diagonal block
constexpr int TT = 64;  // output tile

typedef double dv4 __attribute__((ext_vector_type(4)));

// C(0:M, 0:N) (-)= A B for one tile: A is M x kk staged as sA[t][i], B is
// kk x N staged as sB[t][j] (kk <= 32, M, N <= 64).  assign: C = A B, else
// C -= A B; the C values are read before the products so that their latency
// overlaps the matrix-core work.
constexpr int TTP = TT + 1;  // LDS row stride of the staged operands

__device__ __forceinline__ void tile_mm(double* C, long ldc, int M, int N, int kk,
                                        const double (*sA)[TTP], const double (*sB)[TTP],
                                        bool assign) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w & 1, wn = w >> 1;
  double old[2][2][4];
  if (!assign) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = wm * 32 + a * 16 + (lane & 15);
          const int j = wn * 32 + b * 16 + 4 * r + (lane >> 4);
          old[a][b][r] = (i < M && j < N) ? C[i + (long)j * ldc] : 0.0;
        }
  }
  dv4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dv4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kk; k0 += 4) {
    const int kr = k0 + (lane >> 4);
    double af[2], bf[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) af[a] = (kr < kk) ? sA[kr][wm * 32 + a * 16 + (lane & 15)] : 0.0;
#pragma unroll
    for (int b = 0; b < 2; ++b) bf[b] = (kr < kk) ? sB[kr][wn * 32 + b * 16 + (lane & 15)] : 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[b], af[a], acc[a][b], 0, 0, 0);
  }
  // block of C^T: lane holds C(i = lane%16, j = 4 r + lane/16)
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int i = wm * 32 + a * 16 + (lane & 15);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = wn * 32 + b * 16 + 4 * r + (lane >> 4);
        if (i < M && j < N) C[i + (long)j * ldc] = assign ? acc[a][b][r] : old[a][b][r] - acc[a][b][r];
      }
  }
}

// C (-)= A B over a rows x cols output in 64 x 64 tiles, with A(i, t) and
// B(t, j) read through accessors (t < kk <= 32).  upper_only skips tiles
// strictly below the diagonal.  The operands of the next tile are loaded
// into registers while the current tile is multiplied, so the operands must
// not overlap the output.  AT / BT: the operand is contiguous in memory along
// t (consecutive threads then take consecutive t, so that the loads
// coalesce); otherwise along i / j.  blockDim.x must be 256.
template <bool AT, bool BT, typename FA, typename FB>
__device__ __forceinline__ void tiled_mm(double* C, long ldc, int rows, int cols, int kk,
                                         bool upper_only, bool assign, FA fa, FB fb,
                                         double (*sA)[TTP], double (*sB)[TTP]) {
  constexpr int PER = SB * TT / 256;
  const int tid = threadIdx.x;
  const int ntr = (rows + TT - 1) / TT, ntc = (cols + TT - 1) / TT, nt = ntr * ntc;
  auto advance = [&](int ti) {
    while (ti < nt && upper_only && (ti % ntr) > (ti / ntr)) ++ti;
    return ti;
  };
  double ra[PER], rb[PER];
  auto load = [&](int ti) {
    const int r0 = (ti % ntr) * TT, c0 = (ti / ntr) * TT;
    const int M = min(TT, rows - r0), N = min(TT, cols - c0);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * 256;
      const int ta = AT ? e % SB : e / TT, xa = AT ? e / SB : e % TT;
      const int tb = BT ? e % SB : e / TT, xb = BT ? e / SB : e % TT;
      ra[q] = (ta < kk && xa < M) ? fa(r0 + xa, ta) : 0.0;
      rb[q] = (tb < kk && xb < N) ? fb(tb, c0 + xb) : 0.0;
    }
  };
  int ti = advance(0);
  if (ti < nt) load(ti);
  while (ti < nt) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * 256;
      sA[AT ? e % SB : e / TT][AT ? e / SB : e % TT] = ra[q];
      sB[BT ? e % SB : e / TT][BT ? e / SB : e % TT] = rb[q];
    }
    __syncthreads();
    const int tn = advance(ti + 1);
    if (tn < nt) load(tn);
    const int r0 = (ti % ntr) * TT, c0 = (ti / ntr) * TT;
    tile_mm(C + r0 + (long)c0 * ldc, ldc, min(TT, rows - r0), min(TT, cols - c0), kk, sA, sB,
            assign);
    ti = tn;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// X = R^{-1}, R upper triangular n x n (only its upper triangle is read).
// Blocked by 32: the diagonal blocks are inverted in registers, one wave per
// block (trinv_diag_kernel); then each block column J of X is finished by one
// workgroup going up the block rows, X_IJ = -X_II sum_{K=I+1..J} R_IK X_KJ,
// on the FP64 matrix cores with the finished blocks of the column kept in LDS
// (trinv_offdiag_kernel).  Orders above 512 use one wave per column.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void trinv_diag_kernel(Gate gt, const double* R, long ldr, int n,
                                                         double* X, long ldx) {
  QRCP_GATE(gt);
  __shared__ double sR[W32][W32 + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int p0 = blockIdx.x * W32, nb = min(W32, n - p0);
  for (int e = tid; e < W32 * W32; e += blockDim.x) {
    const int r = e % W32, c = e / W32;
    sR[r][c] = (r < nb && c < nb && r <= c) ? R[(p0 + r) + (long)(p0 + c) * ldr] : 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    double y[W32];
    wave_inv_upper32(&sR[0][0], W32 + 1, y, nb);
    if (lane < nb) {
#pragma unroll
      for (int r = 0; r < W32; ++r)
        if (r < nb) X[(p0 + r) + (long)(p0 + lane) * ldx] = y[r];
    }
  }
  // strictly lower part of this block column
  const long below = n - p0 - nb;
  for (long e = tid; e < below * nb; e += blockDim.x)
    X[(p0 + nb + e % below) + (long)(p0 + e / below) * ldx] = 0.0;
}

template <int NBLK>
__global__ __launch_bounds__(256) void trinv_offdiag_kernel(Gate gt, const double* R, long ldr, int n,
                                                            double* X, long ldx) {
  QRCP_GATE(gt);
  __shared__ double sCol[NBLK][W32][W32 + 1];  // finished X_KJ of this column, [row][col]
  __shared__ double sS[W32][W32 + 1];
  __shared__ double sXd[W32][W32 + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;  // this wave's 16 x 16 quarter of a 32 x 32 block
  const int i16 = lane & 15, k4 = lane >> 4;
  const int J = blockIdx.x + 1, pJ = J * W32, nbJ = min(W32, n - pJ);
  for (int e = tid; e < W32 * W32; e += 256) {
    const int r = e % W32, c = e / W32;
    sCol[J][r][c] = (r < nbJ && c < nbJ) ? X[(pJ + r) + (long)(pJ + c) * ldx] : 0.0;
  }
  __syncthreads();
  for (int I = J - 1; I >= 0; --I) {
    const int pI = I * W32;
    double xd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      xd[q] = X[(pI + e % W32) + (long)(pI + e / W32) * ldx];
    }
    // S = sum_K R_IK X_KJ; A(i, k) = R(pI + 16 wm + i, pK + k) straight from
    // memory: the whole block row I (blocks K = I+1 .. J) is requested before
    // the first product, so a block row costs one memory latency
    const double* arow = R + (pI + 16 * wm + i16);
    double a[NBLK - 1][8];
#pragma unroll
    for (int q = 0; q < NBLK - 1; ++q) {
      const int K = I + 1 + q;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int col = K * W32 + 4 * s + k4;
        a[q][s] = (K <= J && col < n) ? arow[(long)col * ldr] : 0.0;
      }
    }
    dv4 acc = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NBLK - 1; ++q) {
      const int K = I + 1 + q;
      if (K <= J) {
#pragma unroll
        for (int s = 0; s < 8; ++s)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][s], sCol[K][4 * s + k4][16 * wn + i16],
                                                     acc, 0, 0, 0);
      }
    }
    // D(i, j) sits in lane j + 16 (i % 4), register i / 4
#pragma unroll
    for (int r = 0; r < 4; ++r) sS[16 * wm + 4 * r + k4][16 * wn + i16] = acc[r];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      sXd[e % W32][e / W32] = xd[q];
    }
    __syncthreads();
    dv4 acc2 = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s)
      acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(sXd[16 * wm + i16][4 * s + k4],
                                                  sS[4 * s + k4][16 * wn + i16], acc2, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * wm + 4 * r + k4, j = 16 * wn + i16;
      const double v = -acc2[r];
      sCol[I][i][j] = v;
      if (j < nbJ) X[(pI + i) + (long)(pJ + j) * ldx] = v;
    }
    __syncthreads();
  }
}

// The same block-column chain with the finished blocks X_KJ read back from X
// (written by this workgroup, L2 resident) instead of kept in LDS: 17 KB of
// LDS, so its workgroups find room on compute units shared with a concurrent
// GEMM.  Operands are requested CH blocks at a time; the products run in the
// same order as above (bitwise the same X).
__global__ __launch_bounds__(256) void trinv_offdiag_gl_kernel(Gate gt, const double* R, long ldr, int n,
                                                               double* X, long ldx) {
  QRCP_GATE(gt);
  constexpr int CH = 3;
  __shared__ double sS[W32][W32 + 1];
  __shared__ double sXd[W32][W32 + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int i16 = lane & 15, k4 = lane >> 4;
  const int J = blockIdx.x + 1, pJ = J * W32, nbJ = min(W32, n - pJ);
  const int jcol = 16 * wn + i16;  // this lane's column of X_KJ (B operand)
  for (int I = J - 1; I >= 0; --I) {
    const int pI = I * W32;
    double xd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      xd[q] = X[(pI + e % W32) + (long)(pI + e / W32) * ldx];
    }
    const double* arow = R + (pI + 16 * wm + i16);
    dv4 acc = dv4{0.0, 0.0, 0.0, 0.0};
    for (int K0 = I + 1; K0 <= J; K0 += CH) {
      double a[CH][8], b[CH][8];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int K = K0 + c;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int kr = K * W32 + 4 * s + k4;  // row of X_KJ / column of R_IK
          const bool ok = K <= J && kr < n;
          a[c][s] = ok ? arow[(long)kr * ldr] : 0.0;
          b[c][s] = (ok && jcol < nbJ) ? X[kr + (long)(pJ + jcol) * ldx] : 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        if (K0 + c <= J) {
#pragma unroll
          for (int s = 0; s < 8; ++s)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][s], b[c][s], acc, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) sS[16 * wm + 4 * r + k4][16 * wn + i16] = acc[r];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      sXd[e % W32][e / W32] = xd[q];
    }
    __syncthreads();
    dv4 acc2 = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s)
      acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(sXd[16 * wm + i16][4 * s + k4],
                                                  sS[4 * s + k4][16 * wn + i16], acc2, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * wm + 4 * r + k4, j = 16 * wn + i16;
      if (j < nbJ) X[(pI + i) + (long)(pJ + j) * ldx] = -acc2[r];
    }
    __syncthreads();  // X_IJ visible to the whole workgroup before block row I - 1
  }
}

template <int NR>
__global__ __launch_bounds__(256) void trinv_upper_kernel(Gate gt, const double* R, long ldr, int n,
                                                          double* X, long ldx) {
  QRCP_GATE(gt);
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  double x[NR];
#pragma unroll
  for (int s = 0; s < NR; ++s) x[s] = (s * 64 + lane == j) ? 1.0 : 0.0;
  for (int i = j; i >= 0; --i) {
    const int si = i >> 6, li = i & 63;
    double xi = 0.0;
#pragma unroll
    for (int s = 0; s < NR; ++s)
      if (s == si) xi = __shfl(x[s], li, 64);
    xi = xi / R[i + (long)i * ldr];
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      const int r = s * 64 + lane;
      if (r == i) x[s] = xi;
      else if (r < i) x[s] -= xi * R[r + (long)i * ldr];
    }
  }
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int r = s * 64 + lane;
    if (r < n) X[r + (long)j * ldx] = (r <= j) ? x[s] : 0.0;
  }
}

int launch_trinv_upper(const double* R, i64 ldr, int n, double* X, i64 ldx, hipStream_t st,
                       bool low_lds) {
  if (n <= 0) return QRCP_OK;
  if (n > 1024) return QRCP_ERR_UNSUPPORTED;
  if (n > 512) {
    hipLaunchKernelGGL(trinv_upper_kernel<16>, dim3((n + 3) / 4), dim3(256), 0, st, current_gate(), R, ldr, n, X,
                       ldx);
    QRCP_LAUNCHED("trinv_upper");
    return QRCP_OK;
  }
  const int nblk = (n + W32 - 1) / W32;
  hipLaunchKernelGGL(trinv_diag_kernel, dim3(nblk), dim3(256), 0, st, current_gate(), R, ldr, n, X, ldx);
  QRCP_LAUNCHED("trinv_diag");
  if (nblk > 1) {
    const dim3 g(nblk - 1), b(256);
    if (low_lds) hipLaunchKernelGGL(trinv_offdiag_gl_kernel, g, b, 0, st, current_gate(), R, ldr, n, X, ldx);
    else if (nblk <= 8) hipLaunchKernelGGL(trinv_offdiag_kernel<8>, g, b, 0, st, current_gate(), R, ldr, n, X, ldx);
    else if (nblk <= 10) hipLaunchKernelGGL(trinv_offdiag_kernel<10>, g, b, 0, st, current_gate(), R, ldr, n, X, ldx);
    else hipLaunchKernelGGL(trinv_offdiag_kernel<16>, g, b, 0, st, current_gate(), R, ldr, n, X, ldx);
    QRCP_LAUNCHED("trinv_offdiag");
  }
  return QRCP_OK;
}

// ---------------------------------------------------------------------------
// Blocked right-looking factorizations of a small square matrix (n <= 1024) by
// one 256-thread workgroup.  Per 32-column step the diagonal block is factored
// and inverted in the registers of one wave, the off-diagonal panels and the
// trailing block are updated in 64 x 64 tiles on the FP64 matrix cores.
// ---------------------------------------------------------------------------

// Cholesky G = R^T R, upper.  *info = columns factored (n if no breakdown).
__global__ __launch_bounds__(256) void potrf_upper_kernel(Gate gt, double* G, long ldg, int n, int* info) {
  QRCP_GATE(gt);
  __shared__ double sD[SB][SB + 1];
  __shared__ double sX[SB][SB + 1];
  __shared__ double sA[SB][TTP];
  __shared__ double sB[SB][TTP];
  __shared__ int brk, sflag;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid == 0) brk = -1;
  for (int p0 = 0; p0 < n; p0 += SB) {
    const int nb = min(SB, n - p0), rest = n - p0 - nb;
    __syncthreads();
    for (int e = tid; e < SB * SB; e += blockDim.x) {
      const int tr = e % SB, tc = e / SB;
      sD[tr][tc] = (tr < nb && tc < nb && tr <= tc) ? G[(p0 + tr) + (long)(p0 + tc) * ldg] : 0.0;
    }
    if (tid == 0) sflag = 0;
    __syncthreads();
    // wave 0 factors (rows of R published to sA), wave 1 builds the inverse
    // into sX row by row behind it
    if (tid < 64) {
      double x[W32];
#pragma unroll
      for (int r = 0; r < W32; ++r) x[r] = (lane < SB) ? sD[r][lane] : 0.0;
      const int t = wave_potrf32_col_pub(x, nb, &sA[0][0], TTP, &sflag);
      if (lane < SB) {
#pragma unroll
        for (int r = 0; r < W32; ++r) sD[r][lane] = (r <= lane) ? x[r] : 0.0;
      }
      if (t < nb && lane == 0) brk = p0 + t;
    } else if (tid < 128 && rest > 0) {
      wave_inv_upper32_follow(&sA[0][0], TTP, &sX[0][0], SB + 1, nb, &sflag);
    }
    __syncthreads();
    for (int e = tid; e < SB * SB; e += blockDim.x) {
      const int tr = e % SB, tc = e / SB;
      if (tr < nb && tc < nb && tr <= tc) G[(p0 + tr) + (long)(p0 + tc) * ldg] = sD[tr][tc];
    }
    if (brk >= 0) break;
    if (rest > 0) {
      // row panel R12 = R11^{-T} G12 (in place): A(i, t) = R11^{-1}(t, i)
      double* g12 = G + p0 + (long)(p0 + nb) * ldg;
      tiled_mm<false, true>(g12, ldg, nb, rest, nb, false, true,
               [&](int i, int t) { return sX[t][i]; },
               [&](int t, int j) { return g12[t + (long)j * ldg]; }, sA, sB);
      // trailing update of the upper triangle: G22 -= R12^T R12
      tiled_mm<true, true>(G + (p0 + nb) + (long)(p0 + nb) * ldg, ldg, rest, rest, nb, true, false,
               [&](int i, int t) { return g12[t + (long)i * ldg]; },
               [&](int t, int j) { return g12[t + (long)j * ldg]; }, sA, sB);
    }
  }
  __syncthreads();
  const int done = (brk >= 0) ? brk : n;
  for (long e = tid; e < (long)n * n; e += blockDim.x) {
    const int r = e % n, c = e / n;
    if (r > c) G[r + (long)c * ldg] = 0.0;
  }
  if (tid == 0) *info = done;
}

int launch_potrf_upper(double* G, i64 ldg, int n, int* info_dev, hipStream_t st) {
  hipLaunchKernelGGL(potrf_upper_kernel, dim3(1), dim3(256), 0, st, current_gate(), G, ldg, n, info_dev);
  QRCP_LAUNCHED("potrf_upper");
  return QRCP_OK;
}

// Sign-modified LU without pivoting of Q(0:k, 0:k) (Householder reconstruction):
// at step j, D_j = -sgn(Q(j,j)) (sgn(0) = +1), Q(j,j) -= D_j, the column below
// is divided by the new pivot and the trailing block updated.
__global__ __launch_bounds__(256) void headlu_kernel(Gate gt, double* Q, long ldq, int k, double* dsig) {
  QRCP_GATE(gt);
  __shared__ double sD[SB][SB + 1];
  __shared__ double sXu[SB][SB + 1];
  __shared__ double sXl[SB][SB + 1];
  __shared__ double sA[SB][TTP];
  __shared__ double sB[SB][TTP];
  __shared__ double sBc[64];
  const int tid = threadIdx.x, lane = tid & 63;
  for (int p0 = 0; p0 < k; p0 += SB) {
    const int nb = min(SB, k - p0), rest = k - p0 - nb;
    __syncthreads();
    for (int e = tid; e < SB * SB; e += blockDim.x) {
      const int tr = e % SB, tc = e / SB;
      sD[tr][tc] = (tr < nb && tc < nb) ? Q[(p0 + tr) + (long)(p0 + tc) * ldq] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      double x[W32];
#pragma unroll
      for (int c = 0; c < W32; ++c) x[c] = (lane < SB) ? sD[lane][c] : 0.0;
      wave_lu32_signmod_row(x, nb, dsig + p0, sBc);
      if (lane < SB) {
#pragma unroll
        for (int c = 0; c < W32; ++c) sD[lane][c] = x[c];
      }
      if (rest > 0) {
        double y[W32];
        wave_inv_upper32(&sD[0][0], SB + 1, y, nb);
        if (lane < SB) {
#pragma unroll
          for (int r = 0; r < W32; ++r) sXu[r][lane] = y[r];
        }
        wave_inv_unit_lower32(&sD[0][0], SB + 1, y, nb);
        if (lane < SB) {
#pragma unroll
          for (int r = 0; r < W32; ++r) sXl[r][lane] = y[r];
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < SB * SB; e += blockDim.x) {
      const int tr = e % SB, tc = e / SB;
      if (tr < nb && tc < nb) Q[(p0 + tr) + (long)(p0 + tc) * ldq] = sD[tr][tc];
    }
    if (rest > 0) {
      double* a21 = Q + (p0 + nb) + (long)p0 * ldq;   // rows below the block
      double* a12 = Q + p0 + (long)(p0 + nb) * ldq;   // columns right of the block
      // L21 = A21 U11^{-1}
      tiled_mm<false, false>(a21, ldq, rest, nb, nb, false, true,
               [&](int i, int t) { return a21[i + (long)t * ldq]; },
               [&](int t, int j) { return sXu[t][j]; }, sA, sB);
      // U12 = L11^{-1} A12
      tiled_mm<false, true>(a12, ldq, nb, rest, nb, false, true,
               [&](int i, int t) { return sXl[i][t]; },
               [&](int t, int j) { return a12[t + (long)j * ldq]; }, sA, sB);
      // A22 -= L21 U12
      tiled_mm<false, true>(Q + (p0 + nb) + (long)(p0 + nb) * ldq, ldq, rest, rest, nb, false, false,
               [&](int i, int t) { return a21[i + (long)t * ldq]; },
               [&](int t, int j) { return a12[t + (long)j * ldq]; }, sA, sB);
    }
  }
}

int launch_headlu(double* Q, i64 ldq, int k, double* dsig, hipStream_t st) {
  if (k <= 0) return QRCP_OK;
  hipLaunchKernelGGL(headlu_kernel, dim3(1), dim3(256), 0, st, current_gate(), Q, ldq, k, dsig);
  QRCP_LAUNCHED("headlu");
  return QRCP_OK;
}

__global__ void tau_from_u_kernel(Gate gt, const double* Q, long ldq, int k, const double* dsig,
                                  double* tau) {
  QRCP_GATE(gt);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) tau[j] = -dsig[j] * Q[j + (long)j * ldq];
}

int launch_tau_from_u(const double* Q, i64 ldq, int k, const double* dsig, double* tau,
                      hipStream_t st) {
  if (k <= 0) return QRCP_OK;
  hipLaunchKernelGGL(tau_from_u_kernel, dim3((k + 255) / 256), dim3(256), 0, st, current_gate(), Q, ldq, k, dsig,
                     tau);
  QRCP_LAUNCHED("tau_from_u");
  return QRCP_OK;
}

__global__ void write_r11_kernel(Gate gt, const double* P, long ldp, int k, const double* dsig, double* A,
                                 long lda) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)k * k) return;
  const int i = idx % k, j = idx / k;
  if (i <= j) A[i + (long)j * lda] = dsig[i] * P[i + (long)j * ldp];
}

int launch_write_r11(const double* P, i64 ldp, int k, const double* dsig, double* A, i64 lda,
                     hipStream_t st) {
  if (k <= 0) return QRCP_OK;
  hipLaunchKernelGGL(write_r11_kernel, dim3(((long)k * k + 255) / 256), dim3(256), 0, st, current_gate(), P, ldp,
                     k, dsig, A, lda);
  QRCP_LAUNCHED("write_r11");
  return QRCP_OK;
}

// ---------------------------------------------------------------------------
// Copies and fills (2D, column-major).  One thread per element, rows fastest.
// ---------------------------------------------------------------------------
// X = triu(S) diag(dvec) (n x n, column-major): the upper triangle of S with
// column j scaled by dvec(j), zeros below the diagonal.
__global__ void scale_upper_cols_kernel(Gate gt, const double* S, long lds, const double* dvec, int n,
                                        double* X, long ldx) {
  QRCP_GATE(gt);
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const long i = e % n, j = e / n;
  X[i + j * ldx] = (i <= j) ? S[i + j * lds] * dvec[j] : 0.0;
}

int launch_scale_upper_cols(const double* S, i64 lds, const double* dvec, int n, double* X,
                            i64 ldx, hipStream_t st) {
  if (n <= 0) return QRCP_OK;
  const long total = (long)n * n;
  hipLaunchKernelGGL(scale_upper_cols_kernel, dim3((total + 255) / 256), dim3(256), 0, st, current_gate(), S,
                     (long)lds, dvec, n, X, (long)ldx);
  QRCP_LAUNCHED("scale_upper_cols");
  return QRCP_OK;
}

__global__ void copy2d_kernel(Gate gt, const double* src, long lds, double* dst, long ldd, long rows,
                              long cols, int mode) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const long i = idx % rows, j = idx / rows;
  double v = src[i + j * lds];
  if (mode == 1 && i > j) v = 0.0;  // upper trapezoid only
  dst[i + j * ldd] = v;
}

int launch_copy2d(const double* src, i64 lds, double* dst, i64 ldd, i64 rows, i64 cols,
                  hipStream_t st) {
  if (rows <= 0 || cols <= 0) return QRCP_OK;
  hipLaunchKernelGGL(copy2d_kernel, dim3((rows * cols + 255) / 256), dim3(256), 0, st, current_gate(), src, lds,
                     dst, ldd, rows, cols, 0);
  QRCP_LAUNCHED("copy2d");
  return QRCP_OK;
}

int launch_triu_copy(const double* src, i64 lds, double* dst, i64 ldd, i64 rows, i64 cols,
                     hipStream_t st) {
  if (rows <= 0 || cols <= 0) return QRCP_OK;
  hipLaunchKernelGGL(copy2d_kernel, dim3((rows * cols + 255) / 256), dim3(256), 0, st, current_gate(), src, lds,
                     dst, ldd, rows, cols, 1);
  QRCP_LAUNCHED("triu_copy");
  return QRCP_OK;
}

__global__ void fill_kernel(Gate gt, double* dst, long ld, long rows, long cols, double v) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  dst[idx % rows + (idx / rows) * ld] = v;
}

int launch_fill(double* dst, i64 ld, i64 rows, i64 cols, double v, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return QRCP_OK;
  hipLaunchKernelGGL(fill_kernel, dim3((rows * cols + 255) / 256), dim3(256), 0, st, current_gate(), dst, ld, rows,
                     cols, v);
  QRCP_LAUNCHED("fill");
  return QRCP_OK;
}

__global__ void fill_u64_kernel(Gate gt, uint64_t* dst, long count, uint64_t v) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx < count) dst[idx] = v;
}

int launch_fill_u64(uint64_t* dst, i64 count, uint64_t v, hipStream_t st) {
  if (count <= 0) return QRCP_OK;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((count + 255) / 256), dim3(256), 0, st, current_gate(), dst, count, v);
  QRCP_LAUNCHED("fill_u64");
  return QRCP_OK;
}

// identity diagonal: dst(i,i) = 1 for a square n x n already zero-filled
__global__ void set_diag_kernel(Gate gt, double* dst, long ld, long n, double v) {
  QRCP_GATE(gt);
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) dst[i + i * ld] = v;
}

int launch_set_identity(double* dst, i64 ld, i64 n, hipStream_t st) {
  QRCP_TRY(launch_fill(dst, ld, n, n, 0.0, st));
  hipLaunchKernelGGL(set_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, st, current_gate(), dst, ld, n, 1.0);
  QRCP_LAUNCHED("set_diag");
  return QRCP_OK;
}

__global__ void any_nonfinite_kernel(Gate gt, const double* X, long ld, long rows, long cols, int* flag) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  bool bad = false;
  if (idx < rows * cols) bad = !isfinite(X[idx % rows + (idx / rows) * ld]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

int launch_any_nonfinite(const double* X, i64 ld, i64 rows, i64 cols, int* flag, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return QRCP_OK;
  hipLaunchKernelGGL(any_nonfinite_kernel, dim3((rows * cols + 255) / 256), dim3(256), 0, st, current_gate(), X,
                     ld, rows, cols, flag);
  QRCP_LAUNCHED("any_nonfinite");
  return QRCP_OK;
}

}  // namespace qrcp
