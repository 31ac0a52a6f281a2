// Cholesky factorization (Alg. 3, CholQR) and the sign-modified LU of the
// Householder reconstruction (Alg. 3, Sec. 2.3) of matrices up to 256 x 256,
// spread over resident workgroups: one workgroup per 32 x 32 block, holding
// its block in LDS for the whole factorization.
//
// Right-looking block steps p = 0, 1, ...: the owner of diagonal block (p, p)
// factors it in registers (one wave) and publishes the inverses of its
// triangular factors; the owners of the row (and, for the LU, column) panel
// blocks form their panel block from those inverses and publish it; every
// other owner applies the rank-32 update of step p to its block as soon as
// the two panel blocks it needs are published.  Publications go through a
// scratch area (32 x 32 row-major slots) and per-slot flags (relaxed agent-
// scope atomics after a device fence; the reader fences after the flag), so
// the critical path of a step is one diagonal factorization plus two flag
// hand-offs, and the trailing updates of a step run in parallel.
//
// The arithmetic is that of the single-workgroup kernels in dense.hip,
// product by product (the same matrix-core instructions over k in the same
// order), so both give bitwise the same factors.  Every wait is bounded by
// kSpinLimit; a timeout is reported through info (< 0) or the status word.
#include <climits>
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"
#include "wave32.hpp"

namespace qrcp {
namespace {

constexpr int BS = 32;        // block order
constexpr int LDB = BS + 1;   // LDS row stride
constexpr int NT = 256;       // threads per workgroup (4 waves)
constexpr int kMaxNb = 8;     // blocks per side: orders up to 256
constexpr int SLOT = BS * BS; // doubles per published block

typedef double dv4 __attribute__((ext_vector_type(4)));

// C = op(A) B for 32 x 32 blocks in LDS (row-major, stride LDB) on the FP64
// matrix cores: wave w computes the 16 x 16 quadrant (w & 1, w >> 1); lane l
// gets C(16 (w & 1) + l % 16, 16 (w >> 1) + 4 r + l / 16) in register r.
// op(A)(i, k) = TA ? A(k, i) : A(i, k).
template <bool TA>
__device__ __forceinline__ dv4 blk_mm(const double (*sA)[LDB], const double (*sB)[LDB]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = 16 * (w & 1) + (lane & 15), j = 16 * (w >> 1) + (lane & 15);
  dv4 acc = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < BS; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const double af = TA ? sA[k][i] : sA[i][k];
    const double bf = sB[k][j];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bf, af, acc, 0, 0, 0);
  }
  return acc;
}

// (row, column) of result register r of this lane in blk_mm
__device__ __forceinline__ int mm_row() { return 16 * ((threadIdx.x >> 6) & 1) + (threadIdx.x & 15); }
__device__ __forceinline__ int mm_col(int r) {
  return 16 * (threadIdx.x >> 7) + 4 * r + ((threadIdx.x & 63) >> 4);
}

// Published blocks are written with device-coherent stores and read with
// device-coherent loads, so a hand-off needs no cache-wide writeback or
// invalidation (an agent-scope fence): the stores are complete before the
// flag goes up, and the loads come after the flag was seen.
__device__ __forceinline__ void slot_load(double (*dst)[LDB], double* src) {
  for (int e = threadIdx.x; e < SLOT; e += NT) dst[e / BS][e % BS] = load_agent_d(src + e);
}

// Stores the LDS block to a slot and raises its flag to v.
__device__ __forceinline__ void publish(double* slot, const double (*src)[LDB], int* flag, int v) {
  for (int e = threadIdx.x; e < SLOT; e += NT) store_agent_d(slot + e, src[e / BS][e % BS]);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) store_agent_i32(flag, v);
}

// Waits until both flags are nonzero (1 = published).  A flag value of 2, or
// an abort word (may be null) naming a step at or before `step`, means the
// value never comes.  Returns 1 (ready), 0 (abandoned) or -1 (timeout); uniform over the
// workgroup.
__device__ int wait_flags(int* f1, int* f2, int* abort_word, int step, int* sres) {
  if (threadIdx.x == 0) {
    int res = 1;
    long spins = 0;
    for (;;) {
      const int a = load_agent_i32(f1), b = load_agent_i32(f2);
      if (a == 2 || b == 2) { res = 0; break; }
      if (a != 0 && b != 0) break;
      const int ab = abort_word ? load_agent_i32(abort_word) : 0;
      if (ab != 0 && step >= ab - 1) { res = 0; break; }
      if (++spins > kSpinLimit) { res = -1; break; }
      __builtin_amdgcn_s_sleep(1);
    }
    *sres = res;
  }
  __syncthreads();
  return *sres;
}

__device__ __forceinline__ void atomic_min_agent(int* p, int v) {
  __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Cholesky of the upper triangle of G (n x n, n <= 256): G = R^T R, R upper
// triangular in place, strictly lower part zeroed.  info = n, or the first
// column whose pivot is not positive (then R(0:info, 0:info) is valid), or
// -1 after a timeout.  One workgroup per upper block (bi <= bj).
// flags: nb*nb slot flags + abort word, zero on entry; info: INT_MAX on entry.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void potrf_mw_kernel(Gate gt, double* G, long ldg, int n, int nb, int* info,
                                                      double* pub, int* flags) {
  QRCP_GATE(gt);
  __shared__ double sBlk[BS][LDB];
  __shared__ double sP[BS][LDB];
  __shared__ double sQ[BS][LDB];
  __shared__ int sres, sbrk, sflag;
  int bi = 0, bj = 0;
  {
    int idx = blockIdx.x;
    for (int r = 0; r < nb; ++r) {
      if (idx < nb - r) { bi = r; bj = r + idx; break; }
      idx -= nb - r;
    }
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int r0 = bi * BS, c0 = bj * BS;
  const int nr = min(BS, n - r0), nc = min(BS, n - c0);
  int* abort_word = flags + nb * nb;
  auto fl = [&](int p, int j) { return flags + p * nb + j; };
  auto sl = [&](int p, int j) { return pub + (long)(p * nb + j) * SLOT; };

  for (int e = tid; e < SLOT; e += NT) {
    const int r = e % BS, c = e / BS;
    sBlk[r][c] = (r < nr && c < nc && (bi != bj || r <= c)) ? G[(r0 + r) + (long)(c0 + c) * ldg] : 0.0;
  }
  if (tid == 0) {
    sbrk = -1;
    sflag = 0;
  }
  __syncthreads();
  bool stop = false;
  // trailing updates of steps p < bi: G_ij -= R_pi^T R_pj
  for (int p = 0; p < bi; ++p) {
    const int ok = wait_flags(fl(p, bi), fl(p, bj), abort_word, p, &sres);
    if (ok <= 0) {
      if (ok < 0 && tid == 0) atomic_min_agent(info, -1);
      stop = true;
      break;
    }
    slot_load(sP, sl(p, bi));
    slot_load(sQ, sl(p, bj));
    __syncthreads();
    const dv4 acc = blk_mm<true>(sP, sQ);
    const int i = mm_row();
#pragma unroll
    for (int r = 0; r < 4; ++r) sBlk[i][mm_col(r)] -= acc[r];
    __syncthreads();
  }
  if (!stop && bi == bj) {
    // wave 0 factors (rows of R published to sQ), wave 1 builds the inverse
    // into sP row by row behind it
    if (tid < 64) {
      double x[W32];
#pragma unroll
      for (int r = 0; r < W32; ++r) x[r] = (lane < BS) ? sBlk[r][lane] : 0.0;
      const int t = wave_potrf32_col_pub(x, nr, &sQ[0][0], LDB, &sflag);
      if (lane < BS) {
#pragma unroll
        for (int r = 0; r < W32; ++r) sBlk[r][lane] = (r <= lane) ? x[r] : 0.0;
      }
      if (t < nr && lane == 0) sbrk = t;
    } else if (tid < 128 && bi + 1 < nb) {
      wave_inv_upper32_follow(&sQ[0][0], LDB, &sP[0][0], LDB, nr, &sflag);
    }
    __syncthreads();
    if (sbrk >= 0) {
      if (tid == 0) {
        atomic_min_agent(info, r0 + sbrk);
        store_agent_i32(abort_word, bi + 1);
        store_agent_i32(fl(bi, bi), 2);
      }
      stop = true;
    } else if (bi + 1 < nb) {
      publish(sl(bi, bi), sP, fl(bi, bi), 1);
    } else if (tid == 0) {
      atomic_min_agent(info, n);
    }
  } else if (!stop) {
    // row panel block R_ij = R_ii^{-T} G_ij
    const int ok = wait_flags(fl(bi, bi), fl(bi, bi), abort_word, bi, &sres);
    if (ok <= 0) {
      if (ok < 0 && tid == 0) atomic_min_agent(info, -1);
      stop = true;
    } else {
      slot_load(sP, sl(bi, bi));
      __syncthreads();
      const dv4 acc = blk_mm<true>(sP, sBlk);
      __syncthreads();
      const int i = mm_row();
#pragma unroll
      for (int r = 0; r < 4; ++r) sBlk[i][mm_col(r)] = acc[r];
      __syncthreads();
      publish(sl(bi, bj), sBlk, fl(bi, bj), 1);
    }
  }
  __syncthreads();
  // the block back to G (diagonal: upper triangle), the mirrored lower block zeroed
  for (int e = tid; e < SLOT; e += NT) {
    const int r = e % BS, c = e / BS;
    if (r < nr && c < nc) {
      if (bi == bj) {
        G[(r0 + r) + (long)(c0 + c) * ldg] = (r <= c) ? sBlk[r][c] : 0.0;
      } else {
        G[(r0 + r) + (long)(c0 + c) * ldg] = sBlk[r][c];
        G[(c0 + c) + (long)(r0 + r) * ldg] = 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Sign-modified LU without pivoting of Q(0:k, 0:k), k <= 256 (in place: unit
// lower L below the diagonal, U on and above; dsig(j) = D_j), as the
// single-workgroup headlu kernel.  One workgroup per block (bi, bj).
// Slots: (p, j), j > p: U_pj; (i, p), i > p: L_ip; (p, p): U_pp^{-1};
// nb*nb + p: L_pp^{-1}.  flags: nb*nb, zero on entry.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void headlu_mw_kernel(Gate gt, double* Q, long ldq, int k, int nb,
                                                       double* dsig, double* pub, int* flags,
                                                       int* status) {
  QRCP_GATE(gt);
  __shared__ double sBlk[BS][LDB];
  __shared__ double sP[BS][LDB];
  __shared__ double sQ[BS][LDB];
  __shared__ double sBc[64];
  __shared__ int sres;
  const int bi = blockIdx.x / nb, bj = blockIdx.x % nb;
  const int tid = threadIdx.x, lane = tid & 63;
  const int r0 = bi * BS, c0 = bj * BS;
  const int nr = min(BS, k - r0), nc = min(BS, k - c0);
  auto fl = [&](int i, int j) { return flags + i * nb + j; };
  auto sl = [&](int i, int j) { return pub + (long)(i * nb + j) * SLOT; };
  auto sl_linv = [&](int p) { return pub + (long)(nb * nb + p) * SLOT; };

  for (int e = tid; e < SLOT; e += NT) {
    const int r = e % BS, c = e / BS;
    sBlk[r][c] = (r < nr && c < nc) ? Q[(r0 + r) + (long)(c0 + c) * ldq] : 0.0;
  }
  __syncthreads();
  bool stop = false;
  const int pm = min(bi, bj);
  // trailing updates of steps p < min(bi, bj): A_ij -= L_ip U_pj
  for (int p = 0; p < pm; ++p) {
    const int ok = wait_flags(fl(bi, p), fl(p, bj), nullptr, p, &sres);
    if (ok <= 0) {
      stop = true;
      break;
    }
    slot_load(sP, sl(bi, p));
    slot_load(sQ, sl(p, bj));
    __syncthreads();
    const dv4 acc = blk_mm<false>(sP, sQ);
    const int i = mm_row();
#pragma unroll
    for (int r = 0; r < 4; ++r) sBlk[i][mm_col(r)] -= acc[r];
    __syncthreads();
  }
  if (!stop && bi == bj) {
    if (tid < 64) {
      double x[W32];
#pragma unroll
      for (int c = 0; c < W32; ++c) x[c] = (lane < BS) ? sBlk[lane][c] : 0.0;
      wave_lu32_signmod_row(x, nr, dsig + r0, sBc);
      if (lane < BS) {
#pragma unroll
        for (int c = 0; c < W32; ++c) sBlk[lane][c] = x[c];
      }
    }
    __syncthreads();
    if (bi + 1 < nb && tid < 128) {
      // the two triangular inverses side by side: wave 0 U^{-1}, wave 1 L^{-1}
      double y[W32];
      if (tid < 64) {
        wave_inv_upper32(&sBlk[0][0], LDB, y, nr);
        if (lane < BS) {
#pragma unroll
          for (int r = 0; r < W32; ++r) sP[r][lane] = y[r];
        }
      } else {
        wave_inv_unit_lower32(&sBlk[0][0], LDB, y, nr);
        if (lane < BS) {
#pragma unroll
          for (int r = 0; r < W32; ++r) sQ[r][lane] = y[r];
        }
      }
    }
    __syncthreads();
    if (bi + 1 < nb) {
      for (int e = tid; e < SLOT; e += NT) store_agent_d(sl_linv(bi) + e, sQ[e / BS][e % BS]);
      publish(sl(bi, bi), sP, fl(bi, bi), 1);  // its store wait also covers L^{-1}
    }
  } else if (!stop) {
    const int p = pm;  // the diagonal block this panel block hangs off
    const int ok = wait_flags(fl(p, p), fl(p, p), nullptr, p, &sres);
    if (ok <= 0) {
      stop = true;
    } else {
      dv4 acc;
      if (bi < bj) {
        // U_ij = L_ii^{-1} A_ij
        slot_load(sP, sl_linv(p));
        __syncthreads();
        acc = blk_mm<false>(sP, sBlk);
      } else {
        // L_ij = A_ij U_jj^{-1}
        slot_load(sQ, sl(p, p));
        __syncthreads();
        acc = blk_mm<false>(sBlk, sQ);
      }
      __syncthreads();
      const int i = mm_row();
#pragma unroll
      for (int r = 0; r < 4; ++r) sBlk[i][mm_col(r)] = acc[r];
      __syncthreads();
      publish(sl(bi, bj), sBlk, fl(bi, bj), 1);
    }
  }
  if (stop && tid == 0 && status) store_agent_i32(status, QRCP_ERR_TIMEOUT);
  __syncthreads();
  for (int e = tid; e < SLOT; e += NT) {
    const int r = e % BS, c = e / BS;
    if (r < nr && c < nc) Q[(r0 + r) + (long)(c0 + c) * ldq] = sBlk[r][c];
  }
}

__global__ void mw_reset_kernel(Gate gt, int* flags, int nflags, int* info) {
  QRCP_GATE(gt);
  for (int e = threadIdx.x; e < nflags; e += blockDim.x) flags[e] = 0;
  if (info && threadIdx.x == 0) *info = INT_MAX;
}

bool single_forced() {
  const char* e = getenv("QRCP_SMALLFACT");
  return e && e[0] == 's';
}

}  // namespace

size_t blockfact_scratch_bytes() {
  // slots: nb*nb + nb of 32 x 32 doubles; flags: nb*nb + 1 ints
  return (size_t)(kMaxNb * kMaxNb + kMaxNb) * SLOT * sizeof(double) + 4096;
}

int blockfact_groups(int n) {
  if (n <= 0 || n > kMaxNb * BS) return 0;
  const int nb = (n + BS - 1) / BS;
  return nb * nb;
}

int launch_potrf_mw(double* G, i64 ldg, int n, int* info_dev, void* scratch, size_t scratch_bytes,
                    hipStream_t st) {
  if (n <= 0 || n > kMaxNb * BS || !scratch || scratch_bytes < blockfact_scratch_bytes() ||
      single_forced())
    return launch_potrf_upper(G, ldg, n, info_dev, st);
  const int nb = (n + BS - 1) / BS;
  double* pub = (double*)scratch;
  int* flags = (int*)((char*)scratch + (size_t)(kMaxNb * kMaxNb + kMaxNb) * SLOT * sizeof(double));
  hipLaunchKernelGGL(mw_reset_kernel, dim3(1), dim3(256), 0, st, current_gate(), flags, nb * nb + 1, info_dev);
  QRCP_LAUNCHED("potrf reset");
  long ld = (long)ldg;
  int nbv = nb;
  Gate gt = current_gate();
  void* params[] = {&gt, &G, &ld, &n, &nbv, &info_dev, &pub, &flags};
  return launch_resident((const void*)potrf_mw_kernel, dim3(nb * (nb + 1) / 2), dim3(NT), params, 0,
                         st);
}

int launch_headlu_mw(double* Q, i64 ldq, int k, double* dsig, void* scratch, size_t scratch_bytes,
                     int* status, hipStream_t st) {
  if (k <= 0) return QRCP_OK;
  if (k > kMaxNb * BS || !scratch || scratch_bytes < blockfact_scratch_bytes() || single_forced())
    return launch_headlu(Q, ldq, k, dsig, st);
  int nb = (k + BS - 1) / BS;
  double* pub = (double*)scratch;
  int* flags = (int*)((char*)scratch + (size_t)(kMaxNb * kMaxNb + kMaxNb) * SLOT * sizeof(double));
  int* none = nullptr;
  hipLaunchKernelGGL(mw_reset_kernel, dim3(1), dim3(256), 0, st, current_gate(), flags, nb * nb, none);
  QRCP_LAUNCHED("headlu reset");
  long ld = (long)ldq;
  Gate gt = current_gate();
  void* params[] = {&gt, &Q, &ld, &k, &nb, &dsig, &pub, &flags, &status};
  return launch_resident((const void*)headlu_mw_kernel, dim3(nb * nb), dim3(NT), params, 0, st);
}

}  // namespace qrcp
