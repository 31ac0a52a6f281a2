// Tiled matrix-core GEMMs for gfx950.
//
//   C(M x N) = alpha * op(A) op(B) + beta * C        (column-major everywhere)
//
// op(A) is M x K: A stored M x K (TA = false) or K x M (TA = true).
// op(B) is K x N: B stored K x N (TB = false) or N x K (TB = true).
// Options used by the QRCP loop:
//  * `bcol`: column indirection of op(B) (TB = false only) -- used to read R12
//    in logical column order from physically unmoved columns.
//  * split-K with a fixed-order reduction (deterministic results).
//
// Compute types: FP64 (v_mfma_f64_16x16x4f64), FP32 (v_mfma_f32_16x16x4f32,
// operands rounded from FP64 on load), and BF16 operands with FP32
// accumulation (v_mfma_f32_16x16x16bf16_1k) for the reduced-precision sketch.
//
// Tile: BM x BN per 256-thread workgroup = 2 x 2 waves, each wave owns a
// (BM/2) x (BN/2) block of 16 x 16 MFMA tiles.  The MFMA is issued with the
// operands swapped (it computes the 16x16 block of C^T), so each lane's four
// results are four *columns* of one row group and 16 consecutive lanes hold
// 16 consecutive rows of a column: the stores are 128-byte contiguous.
#include <cstdlib>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace qrcp {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  using acc_t = d4v;
  static constexpr int KS = 4;  // k per instruction
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // result r of lane l is row 4 r + l/16, column l%16 of the 16x16 block
  __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

template <>
struct Mfma<float> {
  using acc_t = f4v;
  static constexpr int KS = 4;
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // result r of lane l is row 4 (l/16) + r, column l%16 of the 16x16 block
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T>
__device__ __forceinline__ T cvt(double x) {
  return (T)x;
}

template <int BM, int BN, int WGM, int WGN, int BK, bool TA, bool TB, typename T>
__device__ __forceinline__ void gemm_body(const GemmArgs& g) {
  constexpr int NTH = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LA = BM * BK / NTH, LB = BN * BK / NTH;
  using MF = Mfma<T>;
  using acc_t = typename MF::acc_t;

  // double-buffered operand tiles, padded against bank conflicts of the
  // transposed stores
  __shared__ T sA[2][BK][BM + 1];
  __shared__ T sB[2][BK][BN + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  // Tile order.  Workgroups are dispatched round-robin over the 8 XCDs, each
  // with its own L2: consecutive dispatch slots go to the same XCD's
  // contiguous range of tiles, and inside a range tiles run in groups of 8
  // tile rows, so the tiles that are in flight together share their rows of
  // op(A) and columns of op(B) in one L2.  A permutation of the tiles: the
  // result does not depend on it.
  int ti, tj;
  {
    const int tn = gridDim.x, tm = gridDim.y, nt = tn * tm;
    const int b = blockIdx.y * tn + blockIdx.x;
    const int per = nt / 8;
    const int L = (b < 8 * per) ? (b % 8) * per + b / 8 : b;
    constexpr int GM = 8;
    const int grp = L / (GM * tn), first = grp * GM, rows = min(GM, tm - first);
    const int in = L - grp * GM * tn;
    ti = first + in % rows;
    tj = in / rows;
  }
  const int i0 = ti * BM, j0 = tj * BN;
  const int M = g.M, N = g.N;
  const long kbeg = (long)blockIdx.z * g.kchunk;
  const long kend = min((long)g.K, kbeg + g.kchunk);

  // Per-thread load slots: fixed (row or column, k offset) per slot, so only
  // the k offset advances between chunks.
  const double* pa[LA];
  const double* pb[LB];
  int ka[LA], kb[LB];
  bool va[LA], vb[LB];
#pragma unroll
  for (int q = 0; q < LA; ++q) {
    const int idx = tid + NTH * q;
    int i, kk;
    if (TA) { kk = idx % BK; i = idx / BK; } else { i = idx % BM; kk = idx / BM; }
    const long gi = i0 + i;
    va[q] = gi < M;
    ka[q] = kk;
    pa[q] = TA ? g.A + (va[q] ? gi : 0) * g.lda + kbeg + kk : g.A + (va[q] ? gi : 0) + (kbeg + kk) * g.lda;
  }
#pragma unroll
  for (int q = 0; q < LB; ++q) {
    const int idx = tid + NTH * q;
    int j, kk;
    if (TB) { j = idx % BN; kk = idx / BN; } else { kk = idx % BK; j = idx / BK; }
    const long gj = j0 + j;
    vb[q] = gj < N;
    kb[q] = kk;
    const long cj = vb[q] ? (g.bcol ? g.bcol[gj] : gj) : 0;
    pb[q] = TB ? g.B + cj + (kbeg + kk) * g.ldb : g.B + cj * g.ldb + kbeg + kk;
  }
  const long sa = TA ? BK : (long)BK * g.lda;   // pointer step per chunk
  const long sbk = TB ? (long)BK * g.ldb : BK;

  // C += op(A) op(B) in FP64 (the rank-k trailing update) starts the
  // accumulators from the C tile: its loads are issued before the k loop, so
  // their latency hides behind the operand loads, and the epilogue only stores.
  bool cinit = false;
  if constexpr (std::is_same<T, double>::value) cinit = !g.partial && g.alpha == 1.0 && g.beta == 1.0;
  acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const long gi = i0 + wm * WM + a * 16 + (lane & 15);
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      acc[a][b] = MF::zero();
      if (cinit) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long gj = j0 + wn * WN + b * 16 + MF::row(lane, r);
          if (gi < M && gj < N) acc[a][b][r] = (T)g.C[gi + gj * g.ldc];
        }
      }
    }
  }

  double ra[LA], rb[LB];
  auto load_tiles = [&](long k0) {
    const long rem = kend - k0;
#pragma unroll
    for (int q = 0; q < LA; ++q) ra[q] = (va[q] && ka[q] < rem) ? *pa[q] : 0.0;
#pragma unroll
    for (int q = 0; q < LB; ++q) rb[q] = (vb[q] && kb[q] < rem) ? *pb[q] : 0.0;
#pragma unroll
    for (int q = 0; q < LA; ++q) pa[q] += sa;
#pragma unroll
    for (int q = 0; q < LB; ++q) pb[q] += sbk;
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int idx = tid + NTH * q;
      int i, kk;
      if (TA) { kk = idx % BK; i = idx / BK; } else { i = idx % BM; kk = idx / BM; }
      sA[buf][kk][i] = cvt<T>(ra[q]);
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int idx = tid + NTH * q;
      int j, kk;
      if (TB) { j = idx % BN; kk = idx / BN; } else { kk = idx % BK; j = idx / BK; }
      sB[buf][kk][j] = cvt<T>(rb[q]);
    }
  };

  if (kbeg < kend) {
    load_tiles(kbeg);
    store_tiles(0);
    __syncthreads();
    int buf = 0;
    for (long k0 = kbeg; k0 < kend; k0 += BK) {
      const bool more = k0 + BK < kend;
      if (more) load_tiles(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += MF::KS) {
        T af[FM], bf[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) af[a] = sA[buf][kk + (lane >> 4)][wm * WM + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < FN; ++b) bf[b] = sB[buf][kk + (lane >> 4)][wn * WN + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) acc[a][b] = MF::run(bf[b], af[a], acc[a][b]);
      }
      if (more) store_tiles(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // epilogue: the block computed is C^T, so lane holds C(i = base_i + lane%16,
  // j = base_j + MF::row(lane, r))
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const long gi = i0 + wm * WM + a * 16 + (lane & 15);
#pragma unroll
    for (int b = 0; b < FN; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long gj = j0 + wn * WN + b * 16 + MF::row(lane, r);
        if (gi < M && gj < N) {
          const double v = (double)acc[a][b][r];
          if (g.partial) {
            g.partial[(long)blockIdx.z * M * N + gi + gj * M] = v;
          } else {
            double* c = g.C + gi + gj * g.ldc;
            *c = cinit ? v : ((g.beta == 0.0) ? g.alpha * v : g.alpha * v + g.beta * (*c));
          }
        }
      }
    }
  }
}

// FP64 variant with 16-byte operand loads for even shapes (M, N, K, leading
// dimensions even, 16-byte aligned operands, no column indirection): each
// thread moves pairs of doubles along the operand's contiguous dimension, so a
// chunk takes half the load instructions and one base pointer per operand
// (slots differ by compile-time multiples of the leading dimension).  Same
// tile order, MFMA issue and epilogue as gemm_body, and the same sums in the
// same order per output element (the chunking of K is identical), so the
// results are bitwise those of gemm_body.
template <int BM, int BN, int WGM, int WGN, int BK, bool TA, bool TB>
__device__ __forceinline__ void gemm_vec_body(const GemmArgs& g) {
  constexpr int NTH = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  using MF = Mfma<double>;
  // op(A)(i, k) is contiguous along i when A is stored M x K (TA = false);
  // op(B)(k, j) is contiguous along j when B is stored N x K (TB = true)
  constexpr bool AR = !TA, BR = TB;
  constexpr int PA = BM * BK / 2 / NTH, PB = BN * BK / 2 / NTH;
  static_assert(PA >= 1 && PB >= 1, "tile too small for the thread count");
  static_assert(NTH % (BM / 2) == 0 && NTH % (BN / 2) == 0 && NTH % (BK / 2) == 0, "slot layout");
  __shared__ __align__(16) double sA[2][BK][BM + 2];
  __shared__ __align__(16) double sB[2][BK][BN + 2];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  int ti, tj;
  {
    const int tn = gridDim.x, tm = gridDim.y, nt = tn * tm;
    const int b = blockIdx.y * tn + blockIdx.x;
    const int per = nt / 8;
    const int L = (b < 8 * per) ? (b % 8) * per + b / 8 : b;
    constexpr int GM = 8;
    const int grp = L / (GM * tn), first = grp * GM, rows = min(GM, tm - first);
    const int in = L - grp * GM * tn;
    ti = first + in % rows;
    tj = in / rows;
  }
  const int i0 = ti * BM, j0 = tj * BN;
  const int M = g.M, N = g.N;
  const long kbeg = (long)blockIdx.z * g.kchunk;
  const long kend = min((long)g.K, kbeg + g.kchunk);

  // slot q of operand A covers op(A)(ar0 + q ARS, ak0 + q AKS) and the next
  // element along its contiguous dimension
  const int ar0 = AR ? (tid % (BM / 2)) * 2 : tid / (BK / 2);
  const int ak0 = AR ? tid / (BM / 2) : (tid % (BK / 2)) * 2;
  constexpr int ARS = AR ? 0 : NTH / (BK / 2), AKS = AR ? NTH / (BM / 2) : 0;
  const int br0 = BR ? (tid % (BN / 2)) * 2 : tid / (BK / 2);
  const int bk0 = BR ? tid / (BN / 2) : (tid % (BK / 2)) * 2;
  constexpr int BRS = BR ? 0 : NTH / (BK / 2), BKS = BR ? NTH / (BN / 2) : 0;
  const long aRs = TA ? g.lda : 1, aKs = TA ? 1 : g.lda;   // strides along i and k
  const long bRs = TB ? 1 : g.ldb, bKs = TB ? g.ldb : 1;   // strides along j and k
  const double* pa = g.A + (long)(i0 + ar0) * aRs + (kbeg + ak0) * aKs;
  const double* pb = g.B + (long)(j0 + br0) * bRs + (kbeg + bk0) * bKs;
  const long qa = ARS * aRs + AKS * aKs, qb = BRS * bRs + BKS * bKs;

  bool cinit = !g.partial && g.alpha == 1.0 && g.beta == 1.0;
  // a tile inside C: its loads and stores need no bounds checks (the loads of
  // the C tile then all go out before the first wait)
  const bool interior = i0 + BM <= M && j0 + BN <= N;
  d4v acc[FM][FN];
  if (cinit && interior) {
    const double* cb = g.C + (i0 + wm * WM + (lane & 15)) + (long)(j0 + wn * WN) * g.ldc;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[a][b][r] = cb[a * 16 + (long)(b * 16 + MF::row(lane, r)) * g.ldc];
  } else {
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const long gi = i0 + wm * WM + a * 16 + (lane & 15);
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        acc[a][b] = MF::zero();
        if (cinit) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const long gj = j0 + wn * WN + b * 16 + MF::row(lane, r);
            if (gi < M && gj < N) acc[a][b][r] = g.C[gi + gj * g.ldc];
          }
        }
      }
    }
  }

  double2 ra[PA], rb[PB];
  // an interior tile whose K range is whole chunks loads without checks
  const bool full = interior && (kend - kbeg) % BK == 0;
  auto load_tiles = [&](long k0) {
    const long rem = kend - k0;
    if (full) {
#pragma unroll
      for (int q = 0; q < PA; ++q) ra[q] = *reinterpret_cast<const double2*>(pa + q * qa);
#pragma unroll
      for (int q = 0; q < PB; ++q) rb[q] = *reinterpret_cast<const double2*>(pb + q * qb);
    } else {
#pragma unroll
      for (int q = 0; q < PA; ++q) {
        const bool ok = (i0 + ar0 + q * ARS) < M && (ak0 + q * AKS) < rem;
        ra[q] = ok ? *reinterpret_cast<const double2*>(pa + q * qa) : double2{0.0, 0.0};
      }
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const bool ok = (j0 + br0 + q * BRS) < N && (bk0 + q * BKS) < rem;
        rb[q] = ok ? *reinterpret_cast<const double2*>(pb + q * qb) : double2{0.0, 0.0};
      }
    }
    pa += BK * aKs;
    pb += BK * bKs;
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int r = ar0 + q * ARS, k = ak0 + q * AKS;
      if (AR) {
        *reinterpret_cast<double2*>(&sA[buf][k][r]) = ra[q];
      } else {
        sA[buf][k][r] = ra[q].x;
        sA[buf][k + 1][r] = ra[q].y;
      }
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int r = br0 + q * BRS, k = bk0 + q * BKS;
      if (BR) {
        *reinterpret_cast<double2*>(&sB[buf][k][r]) = rb[q];
      } else {
        sB[buf][k][r] = rb[q].x;
        sB[buf][k + 1][r] = rb[q].y;
      }
    }
  };

  if (kbeg < kend) {
    load_tiles(kbeg);
    store_tiles(0);
    __syncthreads();
    int buf = 0;
    for (long k0 = kbeg; k0 < kend; k0 += BK) {
      const bool more = k0 + BK < kend;
      if (more) load_tiles(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += MF::KS) {
        double af[FM], bf[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) af[a] = sA[buf][kk + (lane >> 4)][wm * WM + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < FN; ++b) bf[b] = sB[buf][kk + (lane >> 4)][wn * WN + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) acc[a][b] = MF::run(bf[b], af[a], acc[a][b]);
      }
      if (more) store_tiles(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  if (interior && (g.partial || cinit || g.beta == 0.0)) {
    // a split-K partial, an accumulated C, or C = alpha A B: plain stores
    const long ld = g.partial ? (long)M : g.ldc;
    const double sc = (g.partial || cinit) ? 1.0 : g.alpha;
    double* cb = (g.partial ? g.partial + (long)blockIdx.z * M * N : g.C) + (i0 + wm * WM + (lane & 15)) +
                 (long)(j0 + wn * WN) * ld;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) cb[a * 16 + (long)(b * 16 + MF::row(lane, r)) * ld] = sc * acc[a][b][r];
    return;
  }
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const long gi = i0 + wm * WM + a * 16 + (lane & 15);
#pragma unroll
    for (int b = 0; b < FN; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long gj = j0 + wn * WN + b * 16 + MF::row(lane, r);
        if (gi < M && gj < N) {
          const double v = acc[a][b][r];
          if (g.partial) {
            g.partial[(long)blockIdx.z * M * N + gi + gj * M] = v;
          } else {
            double* c = g.C + gi + gj * g.ldc;
            *c = cinit ? v : ((g.beta == 0.0) ? g.alpha * v : g.alpha * v + g.beta * (*c));
          }
        }
      }
    }
  }
}

// Named instances: the trailing update's two big products and the sketch get
// their own kernel symbols so that profiles attribute time to them.
#define QRCP_GEMM_KERNEL(NAME)                                                              \
  template <int BM, int BN, int WGM, int WGN, int BK, bool TA, bool TB, typename T, bool VEC> \
  __global__ __launch_bounds__(64 * WGM * WGN) void NAME(Gate gt, GemmArgs g) {               \
    QRCP_GATE(gt);                                                                             \
    if constexpr (VEC) gemm_vec_body<BM, BN, WGM, WGN, BK, TA, TB>(g);                        \
    else gemm_body<BM, BN, WGM, WGN, BK, TA, TB, T>(g);                                       \
  }
QRCP_GEMM_KERNEL(gemm_kernel)
QRCP_GEMM_KERNEL(trailing_update_kernel)
QRCP_GEMM_KERNEL(trailing_w_kernel)
QRCP_GEMM_KERNEL(sketch_gemm_kernel)
#undef QRCP_GEMM_KERNEL

// BF16 x BF16 -> FP32 sketch kernel: op(A) = S (from S^T stored K x M, TA),
// op(B) = the FP64 matrix (K x N).  BK = 32, two k-steps of 16 per chunk.
__global__ __launch_bounds__(256) void gemm_bf16_tn_kernel(Gate gt, GemmArgs g) {
  QRCP_GATE(gt);
  constexpr int BM = 64, BN = 64, BK = 32;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  __shared__ unsigned short sA[BM][BK + 4];
  __shared__ unsigned short sB[BN][BK + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
  const int M = g.M, N = g.N;
  const long kbeg = (long)blockIdx.z * g.kchunk;
  const long kend = min((long)g.K, kbeg + g.kchunk);
  f4v acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
  for (long k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < BM * BK / 256; ++q) {
      const int idx = tid + 256 * q, kk = idx % BK, i = idx / BK;
      const long gi = i0 + i, gk = k0 + kk;
      sA[i][kk] = (gi < M && gk < kend) ? to_bf16_bits(g.A[gk + gi * g.lda]) : (unsigned short)0;
    }
#pragma unroll
    for (int q = 0; q < BN * BK / 256; ++q) {
      const int idx = tid + 256 * q, kk = idx % BK, j = idx / BK;
      const long gj = j0 + j, gk = k0 + kk;
      sB[j][kk] = (gj < N && gk < kend) ? to_bf16_bits(g.B[gk + gj * g.ldb]) : (unsigned short)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      s4v af[FM], bf[FN];
      const int kq = kk + 4 * (lane >> 4);
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        const unsigned short* p = &sA[wm * WM + a * 16 + (lane & 15)][kq];
        af[a] = s4v{(short)p[0], (short)p[1], (short)p[2], (short)p[3]};
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const unsigned short* p = &sB[wn * WN + b * 16 + (lane & 15)][kq];
        bf[b] = s4v{(short)p[0], (short)p[1], (short)p[2], (short)p[3]};
      }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bf[b], af[a], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const long gi = i0 + wm * WM + a * 16 + (lane & 15);
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long gj = j0 + wn * WN + b * 16 + 4 * (lane >> 4) + r;
        if (gi < M && gj < N) {
          const double v = (double)acc[a][b][r];
          if (g.partial) g.partial[(long)blockIdx.z * M * N + gi + gj * M] = v;
          else g.C[gi + gj * g.ldc] = g.alpha * v;
        }
      }
  }
}

// M^sk = S A for the BF16 sketch: S arrives as BF16 bits (S^T, m x d, ld lds a
// multiple of 32, generated so), A (m x n, FP64) is rounded to BF16 on load,
// and the products accumulate in FP32 on the matrix cores.  A workgroup holds
// all d rows of a 64-column strip of M^sk, so each element of A is read once
// (the product is bound by that read); grid.y splits K, and the partials are
// summed in FP32 in a fixed order.  MB row blocks of 16 cover d; wave w owns
// the strip's columns 16 w .. 16 w + 15.
template <int MB>
__global__ __launch_bounds__(256) void sketch_bf16_kernel(Gate gt, const unsigned short* S, long lds,
                                                          const double* A, long lda, int d, int n, long m,
                                                          long kchunk, double* P, double* C, long ldc) {
  QRCP_GATE(gt);
  constexpr int BK = 32, LK = BK + 8, RS = MB * 16;
  constexpr int SQ = (RS * 4 + 255) / 256;  // 16-byte pieces of the S chunk per thread
  __shared__ __align__(16) unsigned short sS[RS][LK];
  __shared__ __align__(16) unsigned short sA[64][LK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const long j0 = (long)blockIdx.x * 64;
  const long kbeg = (long)blockIdx.y * kchunk;
  const long kend = min(m, kbeg + kchunk);
  f4v acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) acc[mb] = f4v{0.f, 0.f, 0.f, 0.f};
  uint4 rs[SQ];
  double ra[8];
  const int aj = tid >> 2, ak = (tid & 3) * 8;  // A: column j0 + aj, k = k0 + ak .. k0 + ak + 7
  const bool jok = j0 + aj < n;
  // the chunk at k0 into registers (S rows past d read as zero; S words past
  // kend are masked when stored, A words past kend are not read)
  auto load = [&](long k0) {
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const int seg = tid + 256 * q, row = seg >> 2, part = seg & 3;
      rs[q] = (seg < RS * 4 && row < d)
                  ? *reinterpret_cast<const uint4*>(S + (long)row * lds + k0 + part * 8)
                  : uint4{0u, 0u, 0u, 0u};
    }
    const double* ap = A + (j0 + aj) * lda + k0 + ak;
#pragma unroll
    for (int e = 0; e < 8; ++e) ra[e] = (jok && k0 + ak + e < kend) ? ap[e] : 0.0;
  };
  auto store = [&](long k0) {
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const int seg = tid + 256 * q, row = seg >> 2, part = seg & 3;
      if (seg < RS * 4) {
        uint4 v = rs[q];
        const long kk = k0 + part * 8;
        if (kk + 8 > kend) {
          unsigned* u = reinterpret_cast<unsigned*>(&v);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const unsigned lo = (kk + 2 * e < kend) ? (u[e] & 0xFFFFu) : 0u;
            const unsigned hi = (kk + 2 * e + 1 < kend) ? (u[e] & 0xFFFF0000u) : 0u;
            u[e] = lo | hi;
          }
        }
        *reinterpret_cast<uint4*>(&sS[row][part * 8]) = v;
      }
    }
    unsigned h[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      h[e] = (unsigned)to_bf16_bits(ra[2 * e]) | ((unsigned)to_bf16_bits(ra[2 * e + 1]) << 16);
    *reinterpret_cast<uint4*>(&sA[aj][ak]) = uint4{h[0], h[1], h[2], h[3]};
  };
  if (kbeg < kend) {
    load(kbeg);
    for (long k0 = kbeg; k0 < kend; k0 += BK) {
      __syncthreads();  // the previous chunk's LDS reads are done
      store(k0);
      __syncthreads();
      if (k0 + BK < kend) load(k0 + BK);  // in flight during this chunk's products
#pragma unroll
      for (int ks = 0; ks < BK; ks += 16) {
        const int kq = ks + 4 * (lane >> 4);
        const unsigned short* pb = &sA[w * 16 + (lane & 15)][kq];
        const s4v bf = s4v{(short)pb[0], (short)pb[1], (short)pb[2], (short)pb[3]};
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const unsigned short* pa = &sS[mb * 16 + (lane & 15)][kq];
          const s4v af = s4v{(short)pa[0], (short)pa[1], (short)pa[2], (short)pa[3]};
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bf, af, acc[mb], 0, 0, 0);
        }
      }
    }
  }
  // D(i, j): row 16 mb + lane % 16 of M^sk, column 16 w + 4 (lane / 16) + r of the strip
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int gi = mb * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long gj = j0 + w * 16 + 4 * (lane >> 4) + r;
      if (gi < d && gj < n) {
        const double v = (double)acc[mb][r];
        if (P) P[(long)blockIdx.y * d * n + gi + gj * d] = v;
        else C[gi + gj * ldc] = v;
      }
    }
  }
}

// Fixed-order reduction of split-K partials: C = alpha * sum_z P_z + beta * C.
// For the BF16 path (fp32_sum) the partials are summed in FP32 so the whole
// accumulation stays FP32.
__global__ void splitk_reduce_kernel(Gate gt, const double* P, int splits, int M, int N, double alpha,
                                     double beta, double* C, long ldc, int fp32_sum) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long MN = (long)M * N;
  if (idx >= MN) return;
  const long i = idx % M, j = idx / M;
  double v;
  if (fp32_sum) {
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += (float)P[z * MN + idx];
    v = (double)s;
  } else {
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += P[z * MN + idx];
    v = s;
  }
  double* c = C + i + j * ldc;
  *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
}

__global__ void scale_kernel(Gate gt, double* C, long ldc, int M, int N, double beta) {
  QRCP_GATE(gt);
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)M * N) return;
  double* c = C + idx % M + (idx / M) * ldc;
  *c = (beta == 0.0) ? 0.0 : beta * (*c);
}

template <int BM, int BN, int WGM, int WGN, int BK, bool TA, bool TB, typename T, bool VEC = false>
static void launch_tile(const GemmArgs& g, int splits, hipStream_t st) {
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, splits);
  dim3 block(64 * WGM * WGN);
  switch (g.kind) {
    case GemmKind::TrailingUpdate:
      hipLaunchKernelGGL((trailing_update_kernel<BM, BN, WGM, WGN, BK, TA, TB, T, VEC>), grid, block, 0, st, current_gate(), g);
      break;
    case GemmKind::TrailingW:
      hipLaunchKernelGGL((trailing_w_kernel<BM, BN, WGM, WGN, BK, TA, TB, T, VEC>), grid, block, 0, st, current_gate(), g);
      break;
    case GemmKind::Sketch:
      hipLaunchKernelGGL((sketch_gemm_kernel<BM, BN, WGM, WGN, BK, TA, TB, T, VEC>), grid, block, 0, st, current_gate(), g);
      break;
    default:
      hipLaunchKernelGGL((gemm_kernel<BM, BN, WGM, WGN, BK, TA, TB, T, VEC>), grid, block, 0, st, current_gate(), g);
  }
}

// 16-byte operand loads apply: FP64, even sizes and leading dimensions,
// 16-byte aligned operands, no column indirection of op(B)
static bool vec_ok(const GemmArgs& g) {
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  return !g.bcol && ((g.M | g.N | g.K) & 1) == 0 && ((g.lda | g.ldb) & 1) == 0 && al(g.A) && al(g.B);
}

// Tile configuration: 0 = automatic; 1 = 64x64 (4 waves); 2 = 128x128 (4 waves);
// 3 = 128x128 (8 waves); 4 = 128x64 (4 waves); 5 = 128x128 (8 waves, k chunk
// 32); 6 = 256x128 (8 waves); 7 = 128x256 (8 waves); 8 = 64x64 (4 waves, k
// chunk 32).  QRCP_GEMM_TILE overrides
// the automatic choice (used for tuning sweeps).
static int tile_override() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("QRCP_GEMM_TILE");
    v = e ? atoi(e) : 0;
  }
  return v;
}

// The tile configuration of a product: 0 = 64x64 (4 waves), or the override.
// FP64 products with even sizes take the 16-byte-load tiles: 128 x 128 over 8
// waves (each a 64 x 32 block) -- measured at 16384^2, b = 256: rank-k update
// 55 vs 47 TFLOP/s, W = Y^T C 56 vs 52 TFLOP/s -- unless their 128 x 128
// tiles fill less than one wave of the device's resident slots (two per
// compute unit) and K is too short to split, or the output is at most 64
// wide (or the product is the sketch, d = 320 rows, whose third 128-row tile
// row would be a sixth empty): those take the 64 x 64 tiles with 16-byte
// loads.  Both compute the same
// per-element sums, so the results do not depend on the choice.
static int pick_cfg(const GemmArgs& g, bool f64) {
  int cfg = tile_override();
  if (f64 && cfg == 0 && vec_ok(g)) {
    const long tiles = (long)((g.M + 127) / 128) * ((g.N + 127) / 128);
    const bool small = tiles < 2L * 256 && g.K < 512;
    // an output at most 64 wide would leave most of a 128-wide tile empty
    const bool skinny = g.M <= 64 || g.N <= 64;
    cfg = (g.kind == GemmKind::Sketch || small || skinny) ? 9 : 12;
  }
  return cfg;
}

template <bool TA, bool TB, typename T>
static void launch_shape(const GemmArgs& g, int cfg, int splits, hipStream_t st) {
  if constexpr (std::is_same<T, double>::value) {
    if (cfg >= 9 && vec_ok(g)) {
      switch (cfg) {
        case 9: launch_tile<64, 64, 2, 2, 16, TA, TB, T, true>(g, splits, st); return;
        case 10: launch_tile<128, 128, 2, 2, 16, TA, TB, T, true>(g, splits, st); return;
        case 11: launch_tile<128, 64, 2, 2, 16, TA, TB, T, true>(g, splits, st); return;
        case 12: launch_tile<128, 128, 2, 4, 16, TA, TB, T, true>(g, splits, st); return;
        case 13: launch_tile<128, 128, 4, 2, 16, TA, TB, T, true>(g, splits, st); return;
        case 14: launch_tile<256, 128, 2, 4, 16, TA, TB, T, true>(g, splits, st); return;
        case 15: launch_tile<128, 256, 2, 4, 16, TA, TB, T, true>(g, splits, st); return;
        case 16: launch_tile<128, 128, 2, 4, 32, TA, TB, T, true>(g, splits, st); return;
        case 17: launch_tile<128, 64, 2, 2, 32, TA, TB, T, true>(g, splits, st); return;
        default: break;
      }
    }
  }
  // otherwise 64 x 64 tiles (4 waves, four workgroups per CU; measured on
  // MI355X at 16384^2, b = 256, they beat the 128 x 128 tiles of this form on
  // the rank-k update (49 vs 42 TFLOP/s), on W = Y^T C (55 vs 54) and on the
  // sketch (49 vs 39))
  switch (cfg) {
    case 2: launch_tile<128, 128, 2, 2, 16, TA, TB, T>(g, splits, st); break;
    case 3: launch_tile<128, 128, 2, 4, 16, TA, TB, T>(g, splits, st); break;
    case 4: launch_tile<128, 64, 2, 2, 16, TA, TB, T>(g, splits, st); break;
    case 5: launch_tile<128, 128, 2, 4, 32, TA, TB, T>(g, splits, st); break;
    case 6: launch_tile<256, 128, 2, 4, 16, TA, TB, T>(g, splits, st); break;
    case 7: launch_tile<128, 256, 2, 4, 16, TA, TB, T>(g, splits, st); break;
    case 8: launch_tile<64, 64, 2, 2, 32, TA, TB, T>(g, splits, st); break;
    default: launch_tile<64, 64, 2, 2, 16, TA, TB, T>(g, splits, st); break;
  }
}

size_t gemm_splitk_bytes(long M, long N, int splits) { return (size_t)M * N * splits * sizeof(double); }

int launch_sketch_bf16(const double* A, i64 m, i64 n, i64 lda, int d, uint64_t seed, double* Msk, i64 ldmsk,
                       void* sbuf, size_t sbuf_bytes, double* split, size_t split_bytes, hipStream_t st) {
  if (d < 1 || d > 320 || m <= 0 || n <= 0) return QRCP_ERR_UNSUPPORTED;
  const long lds = (m + 31) / 32 * 32;  // whole 32-row chunks of S^T stay inside the buffer
  if ((size_t)lds * d * sizeof(unsigned short) > sbuf_bytes) return QRCP_ERR_UNSUPPORTED;
  QRCP_TRY(launch_sketch_operator_bf16(static_cast<unsigned short*>(sbuf), m, d, lds, seed, st));
  // about four workgroups per compute unit, at least 256 rows of K per split,
  // and the partials within the split area
  const long nstrips = (n + 63) / 64;
  long splits = std::max<long>(1, (1024 + nstrips - 1) / nstrips);
  splits = std::min<long>(splits, std::max<long>(1, m / 256));
  splits = std::min<long>(splits, 64);
  while (splits > 1 && (size_t)splits * d * n * sizeof(double) > split_bytes) --splits;
  const long kchunk = ((m + splits - 1) / splits + 31) / 32 * 32;
  splits = (m + kchunk - 1) / kchunk;
  double* P = splits > 1 ? split : nullptr;
  const dim3 grid((unsigned)nstrips, (unsigned)splits);
  const int mb = (d + 15) / 16;
  const unsigned short* S = static_cast<const unsigned short*>(sbuf);
  if (mb <= 5)
    hipLaunchKernelGGL(sketch_bf16_kernel<5>, grid, dim3(256), 0, st, current_gate(), S, lds, A, (long)lda, d,
                       (int)n, (long)m, kchunk, P, Msk, (long)ldmsk);
  else if (mb <= 10)
    hipLaunchKernelGGL(sketch_bf16_kernel<10>, grid, dim3(256), 0, st, current_gate(), S, lds, A, (long)lda, d,
                       (int)n, (long)m, kchunk, P, Msk, (long)ldmsk);
  else
    hipLaunchKernelGGL(sketch_bf16_kernel<20>, grid, dim3(256), 0, st, current_gate(), S, lds, A, (long)lda, d,
                       (int)n, (long)m, kchunk, P, Msk, (long)ldmsk);
  QRCP_LAUNCHED("sketch_bf16");
  if (P) {
    const long dn = (long)d * n;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((dn + 255) / 256), dim3(256), 0, st, current_gate(), P,
                       (int)splits, d, (int)n, 1.0, 0.0, Msk, (long)ldmsk, 1);
    QRCP_LAUNCHED("splitk_reduce");
  }
  return QRCP_OK;
}

// Chooses a split of K when the output has too few tiles to fill the GPU:
// about `target` workgroups (512 by default; the W = Y^T C product of the
// trailing update, whose tiles each run the whole long K, asks for 4096, so
// that every product below 2048 tiles is split, within the partials area).
int gemm_pick_splits(long M, long N, long K, long target) {
  const long tiles = ((M + 63) / 64) * ((N + 63) / 64);
  if (2 * tiles >= target || K < 512) return 1;
  long s = (target + tiles - 1) / tiles;
  const long kmax = K / 256;  // keep >= 256 per split
  if (s > kmax) s = kmax;
  if (s > 64) s = 64;
  return s < 1 ? 1 : (int)s;
}

// Split of K for the 128 x 128 tiles of the FP64 default, chosen so that the
// workgroups fill whole waves of the resident slots (two per compute unit):
// a grid of 1.5 waves leaves half the device idle in its second wave.  Each
// split keeps at least 256 of K, and the partials must fit the area.
static int vec_pick_splits(long M, long N, long K, size_t ws_bytes) {
  const long tiles = ((M + 127) / 128) * ((N + 127) / 128);
  const long slots = 2L * 256;
  if (tiles >= 4 * slots || K < 512) return 1;
  const long smax = std::min<long>(64, K / 256);
  int best = 1;
  double best_eff = (double)tiles / (double)(((tiles + slots - 1) / slots) * slots);
  for (long sp = 2; sp <= smax; ++sp) {
    if (gemm_splitk_bytes(M, N, (int)sp) > ws_bytes) break;
    const long t = tiles * sp;
    const double eff = (double)t / (double)(((t + slots - 1) / slots) * slots);
    if (eff > best_eff + 0.02) {
      best = (int)sp;
      best_eff = eff;
    }
  }
  return best;
}

int gemm(bool ta, bool tb, Prec prec, GemmArgs g, double* split_ws, size_t split_ws_bytes,
         hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return QRCP_OK;
  if (g.K <= 0) {
    // empty product: C = beta * C
    if (g.beta == 1.0) return QRCP_OK;
    hipLaunchKernelGGL(scale_kernel, dim3((g.M * (long)g.N + 255) / 256), dim3(256), 0, st, current_gate(), g.C,
                       g.ldc, g.M, g.N, g.beta);
    QRCP_LAUNCHED("gemm scale");
    return QRCP_OK;
  }
  int splits = 1;
  const int cfg = pick_cfg(g, prec == Prec::F64);
  const bool vec_default = prec == Prec::F64 && cfg == 12 && vec_ok(g);
  if (split_ws && !g.bcol && vec_default)
    splits = vec_pick_splits(g.M, g.N, g.K, split_ws_bytes);
  else if (split_ws && !g.bcol)
    splits = gemm_pick_splits(g.M, g.N, g.K, g.kind == GemmKind::TrailingW ? 4096 : 512);
  if (splits > 1 && gemm_splitk_bytes(g.M, g.N, splits) > split_ws_bytes)
    splits = (int)std::max<size_t>(1, split_ws_bytes / gemm_splitk_bytes(g.M, g.N, 1));
  const long BKc = 32;
  long chunk = (g.K + splits - 1) / splits;
  chunk = (chunk + BKc - 1) / BKc * BKc;
  splits = (int)((g.K + chunk - 1) / chunk);
  g.kchunk = (int)chunk;
  const double alpha = g.alpha, beta = g.beta;
  double* C = g.C;
  const long ldc = g.ldc;
  g.partial = (splits > 1) ? split_ws : nullptr;
  if (prec == Prec::BF16) {
    if (!ta || tb) return QRCP_ERR_UNSUPPORTED;
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
    if (splits == 1) g.partial = nullptr;
    hipLaunchKernelGGL(gemm_bf16_tn_kernel, grid, dim3(256), 0, st, current_gate(), g);
  } else if (prec == Prec::F32) {
    if (ta && !tb) launch_shape<true, false, float>(g, cfg, splits, st);
    else if (!ta && !tb) launch_shape<false, false, float>(g, cfg, splits, st);
    else if (!ta && tb) launch_shape<false, true, float>(g, cfg, splits, st);
    else launch_shape<true, true, float>(g, cfg, splits, st);
  } else {
    if (ta && !tb) launch_shape<true, false, double>(g, cfg, splits, st);
    else if (!ta && !tb) launch_shape<false, false, double>(g, cfg, splits, st);
    else if (!ta && tb) launch_shape<false, true, double>(g, cfg, splits, st);
    else launch_shape<true, true, double>(g, cfg, splits, st);
  }
  QRCP_LAUNCHED("gemm");
  if (splits > 1) {
    const long MN = (long)g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((MN + 255) / 256), dim3(256), 0, st, current_gate(), split_ws,
                       splits, g.M, g.N, alpha, beta, C, ldc, prec != Prec::F64 ? 1 : 0);
    QRCP_LAUNCHED("splitk_reduce");
  }
  return QRCP_OK;
}

}  // namespace qrcp
