// Shared device/host helpers of the gfx950 QRCP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qrcp.h"

namespace qrcp {

using i64 = int64_t;

// Records the HIP error text for qrcp_last_error().
void note_hip_error(hipError_t e, const char* what);

#define QRCP_HIP(call)                                  \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) {                             \
      ::qrcp::note_hip_error(e_, #call);                \
      return QRCP_ERR_HIP;                              \
    }                                                   \
  } while (0)

#define QRCP_LAUNCHED(what)                             \
  do {                                                  \
    hipError_t e_ = hipGetLastError();                  \
    if (e_ != hipSuccess) {                             \
      ::qrcp::note_hip_error(e_, what);                 \
      return QRCP_ERR_HIP;                              \
    }                                                   \
  } while (0)

#define QRCP_TRY(expr)              \
  do {                              \
    int rc_ = (expr);               \
    if (rc_ != QRCP_OK) return rc_; \
  } while (0)

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide sum for blockDim.x = NT (multiple of 64).  `red` needs NT/64
// doubles of shared memory.  Every thread gets the result.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// Ordering point for data one lane of a wave writes to LDS and other lanes of
// the same wave read afterwards: a wave's LDS operations execute in order, and
// this keeps the compiler from moving the accesses across it (without it a
// load may be hoisted above the store, the writing lane's value forwarded).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bit-level access for the cross-workgroup record exchange.
__device__ __forceinline__ uint64_t dbits(double x) { return __double_as_longlong(x); }
__device__ __forceinline__ double bitsd(uint64_t x) { return __longlong_as_double((long long)x); }

// FP64 -> FP32 (RNE) -> BF16 (RNE) bits.
__device__ __forceinline__ unsigned short to_bf16_bits(double x) {
  float f = (float)x;
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ void store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_agent(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// v(lane) + v(lane ^ 16) and v(lane) + v(lane ^ 32) for a double, with the
// gfx950 row-swap moves (v_permlane16_swap / v_permlane32_swap, one VALU
// instruction per 32-bit half) instead of an LDS-routed shuffle.  With both
// operands equal, the swap returns the even-row (lower-half) copy in the
// first result and the odd-row (upper-half) copy in the second, in every
// lane; their sum is the same in both partner lanes.
__device__ __forceinline__ double xsum_lanes16(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double e = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double o = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return e + o;
}
__device__ __forceinline__ double xsum_lanes32(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double e = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double o = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return e + o;
}

__device__ __forceinline__ void store_agent_d(double* p, double v) {
  store_agent(reinterpret_cast<uint64_t*>(p), dbits(v));
}
__device__ __forceinline__ double load_agent_d(const double* p) {
  return bitsd(load_agent(reinterpret_cast<uint64_t*>(const_cast<double*>(p))));
}
__device__ __forceinline__ void store_agent_i32(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_agent_i32(int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Launches a kernel whose workgroups wait on each other: checks that the whole
// grid fits on the device at once (occupancy x compute units) and launches it
// with an ordinary launch.  Every wait in such a kernel is bounded by
// kSpinLimit, so a grid that is not resident ends in QRCP_ERR_TIMEOUT.
int launch_resident(const void* fn, dim3 grid, dim3 block, void** params, size_t smem,
                    hipStream_t st);

// Spin limit of every cross-workgroup wait: far above any legitimate wait,
// it turns a lost partner into QRCP_ERR_TIMEOUT instead of a hung GPU.
constexpr long kSpinLimit = 1L << 22;

// ---------------------------------------------------------------------------
// Launch gates of the device-driven block loop.  The host enqueues every block
// of the factorization up front; a control record in device memory says how
// far the loop got, and every kernel of block `blk` returns at once when its
// gate is closed:
//   kGateRun   closed once the loop has stopped before block blk;
//   kGateExit  open only in the block at which the loop stops, and only when
//              that block's panel is short of its full width (the work that
//              finishes a block of reduced rank);
//   kGateGoOn  open only in blocks the loop continues past (the sketch update).
// The record is written by one-thread kernels earlier in the same stream, so
// every kernel reads a settled value.  ctl == nullptr: always open.
// ---------------------------------------------------------------------------
struct LoopCtl {
  int nblk;       // blocks that run (INT_MAX until the loop stops)
  int exit_blk;   // the block at which the loop stops (-1 while it runs)
  int k;          // effective width of the current block's panel
  int status;     // QRCP_OK or the first error
  long long ell;  // columns factored so far (the rank at the end)
  long long perms;  // column-map updates done (parity selects the live map)
  int kmax;       // full width of the current block's panel
  int pad;
};

// rank and status of a factorization call, in device memory
struct CallResult {
  long long rank;
  int status;
  int pad;
};

enum : int { kGateRun = 0, kGateExit = 1, kGateGoOn = 2 };

struct Gate {
  const LoopCtl* ctl;
  int blk;
  int mode;
};

__device__ __forceinline__ bool gate_closed(const Gate& g) {
  if (!g.ctl) return false;
  const int nblk = g.ctl->nblk, ex = g.ctl->exit_blk;
  if (g.blk >= nblk) return true;
  if (g.mode == kGateExit) return g.blk != ex || g.ctl->k >= g.ctl->kmax;
  if (g.mode == kGateGoOn) return g.blk == ex;
  return false;
}

#define QRCP_GATE(g)                        \
  do {                                      \
    if (::qrcp::gate_closed(g)) return;     \
  } while (0)

// The gate that launches on the calling host thread pass to their kernels
// (open by default); set by the block loop.
Gate& current_gate();

struct GateScope {
  Gate saved;
  explicit GateScope(Gate g) : saved(current_gate()) { current_gate() = g; }
  ~GateScope() { current_gate() = saved; }
};

}  // namespace qrcp
