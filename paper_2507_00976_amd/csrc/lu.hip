// Pivot selection of the wide sketch (Alg. 2): GETRF with partial pivoting on
// X = (M^sk)^T, computed as one kernel whose workgroups are all resident.
//
// Layout: the d x ni column-major sketch *is* X stored row-major (row t of X =
// sketch column t, d contiguous doubles), so the transpose of Alg. 2 costs
// nothing.  The ni rows are spread over G workgroups of 256 threads, 64*RPT
// rows each, with a working copy of the rows in HBM.
//
// Pivot steps run panel by panel (32 columns).  During the steps of a panel
// wave 0 of each workgroup runs the steps: lane l holds the panel part of rows
// l, l+64, ... in registers, shifted left by one column after each step so
// that the current column is always register 0.  The blocked trailing update
//   U12 = L11^{-1} X(piv, trail),  X(r, trail) -= L(r, panel) U12
// (forward substitution in registers, then the product on the FP64 matrix
// cores) is split in two: right after the panel all four waves update the
// next panel's 32 columns, and the remaining columns are updated by waves 1-3
// while wave 0 already runs the next panel's steps (panel state in LDS is
// double-buffered for this).  A workgroup publishes its last header of a panel
// only after that background update is in memory, so a workgroup that has
// read every header of the panel may read any pivot row's trailing values.
// Rows that other workgroups read (the working copy and the background
// update's results) are written with device-coherent stores and the pivot
// rows are read with device-coherent loads, so no cache-wide writeback or
// invalidation (an agent-scope fence) is needed anywhere in the loop.
//
// One pivot step costs one cross-workgroup round trip.  Every workgroup
// publishes a record for its best candidate: a header (|x|, key = current
// position and row id, x, the candidate's multiplier for the previous pivot,
// its value in the next column) and a payload (its panel row).  Every
// workgroup reads all headers and agrees on the winner (largest |x|, ties to
// the smallest current position, as IDAMAX).  A step's headers are stored
// word-major (word w of every workgroup contiguous), so a wave reading the
// headers of 64 workgroups touches 8 cache lines per word instead of 64.  The header alone is enough to
// eliminate in the next column at once; the previous pivot's contribution to
// the remaining panel columns is applied one step late, from the previous
// winner's payload, which was fetched while the current headers travelled
// (pivot row j = payload_j - lambda_j * pivot row j-1).  Record slots are
// never reused within a call and are reset to a sentinel bit pattern
// beforehand, so each 64-bit word is valid as soon as it differs from the
// sentinel; every wait is bounded by kSpinLimit.  Row swaps are never
// performed: each row carries its current position, and the row sitting at
// position j takes the pivot's position when the pivot leaves (the swap of
// GETRF).
#include <climits>
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace qrcp {

namespace {
constexpr int NB = 32;    // panel width
constexpr int NT = 256;   // threads per workgroup
constexpr int HW = 5;     // header words
constexpr int TCH = 256;  // trailing columns per chunk
constexpr uint64_t SENT = 0xFFF0DEADBEEFCAFEull;
constexpr uint64_t NOCAND = 0x7FFFFFFF00000000ull;
constexpr uint64_t BADKEY = 0x7FFFFFFE00000000ull;
constexpr int kMaxGroups = 256;
constexpr int GQ = kMaxGroups / 64;  // records read per lane
constexpr int LRBG = 2;  // row blocks per request group of the update beside the steps
constexpr int LUB = 8;   // pivot-row loads per request group of that update

typedef double dv4 __attribute__((ext_vector_type(4)));

struct LuArgs {
  const double* msk;
  long ld;
  int d;
  long ni;
  int steps;         // elimination steps: at most min(d, ni)
  double* xw;        // ni x d row-major working copy
  uint64_t* rec;     // steps x step_words(G) words, sentinel-filled
  long* ipiv;
  long* jsk;
  int* status;
};

// Records of one step: HW header words of each of G workgroups, word-major
// with rows of gpad(G) words (64-byte lines), then G payloads of NB words.
__host__ __device__ constexpr long gpad(int G) { return (G + 7) & ~7; }
__host__ __device__ constexpr long step_words(int G) { return HW * gpad(G) + (long)G * NB; }
__device__ __forceinline__ uint64_t* hdr_at(uint64_t* rec, long j, int G, int g) {
  return rec + j * step_words(G) + g;  // word w at + w * gpad(G)
}
__device__ __forceinline__ uint64_t* pay_at(uint64_t* rec, long j, int G, int g) {
  return rec + j * step_words(G) + HW * gpad(G) + (long)g * NB;
}

__device__ __forceinline__ bool better(double va, uint64_t ka, double vb, uint64_t kb) {
  return va > vb || (va == vb && ka < kb);
}

__device__ __forceinline__ double rdlane_d(double v, int l);
__device__ __forceinline__ uint64_t rdlane_u64(uint64_t v, int l) {
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xFFFFFFFFull), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
}

// Wave-wide argmax of (v, key), v never NaN; every lane gets the result.  The
// maximum value is reduced with DPP moves inside rows of 16 lanes (lane^1,
// lane^2, mirrored lane of the half row, of the row) and scalar reads of the
// four rows; the key is the smallest among the lanes that hold the maximum
// (one lane in the common case).
__device__ __forceinline__ void wave_argmax(double& v, uint64_t& key) {
  double m = v;
  m = fmax(m, dpp_d<0xB1>(m));   // quad_perm [1,0,3,2]
  m = fmax(m, dpp_d<0x4E>(m));   // quad_perm [2,3,0,1]
  m = fmax(m, dpp_d<0x141>(m));  // row_half_mirror
  m = fmax(m, dpp_d<0x140>(m));  // row_mirror
  const double mx = fmax(fmax(rdlane_d(m, 0), rdlane_d(m, 16)), fmax(rdlane_d(m, 32), rdlane_d(m, 48)));
  uint64_t tie = __ballot(v == mx);
  uint64_t best = ~0ull;
  while (tie) {
    const int l = __ffsll((unsigned long long)tie) - 1;
    tie &= tie - 1;
    const uint64_t k = rdlane_u64(key, l);
    if (k < best) best = k;
  }
  v = mx;
  key = best;
}

__device__ __forceinline__ double rdlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ uint64_t canon(double x) {
  return isnan(x) ? 0x7FF8000000000000ull : dbits(x);
}

__device__ __forceinline__ double cand_value(double x) { return isnan(x) ? -0.5 : fabs(x); }

// X(r, col) -= L(r, panel) U12(panel, col) for the row blocks rb0 .. rb0+NRBX
// of a workgroup (16 x 16 blocks on the FP64 matrix cores; D(i, j) sits in
// lane j + 16 (i % 4)).  `col` is this lane's matrix column, `uc` its column
// of the U12 staging array; rows that are no longer active are left alone.
// Row blocks go RBG at a time, each group's loads and stores completed before
// the next group's are issued: the update that runs beside the pivot steps
// keeps few requests in the compute unit's memory queue, where the steps'
// record loads would wait behind them.
template <int NRBX, int RBG, int LS, int US>
__device__ __forceinline__ void lu_tile_update(double* xw, long row0, int d, int col, int rb0,
                                               const double (*L)[LS], const double (*U)[US],
                                               int uc, const int* act, int i16, int k4) {
  static_assert(NRBX % RBG == 0, "row-block groups");
#pragma unroll
  for (int g0 = 0; g0 < NRBX; g0 += RBG) {
    double old[RBG][4];
#pragma unroll
    for (int rb = 0; rb < RBG; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = (rb0 + g0 + rb) * 16 + 4 * r + k4;
        old[rb][r] = (act[lr] && col < d) ? xw[(row0 + lr) * d + col] : 0.0;
      }
#pragma unroll
    for (int rb = 0; rb < RBG; ++rb) {
      dv4 acc = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < NB / 4; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(L[(rb0 + g0 + rb) * 16 + i16][4 * s + k4],
                                                   U[4 * s + k4][uc], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = (rb0 + g0 + rb) * 16 + 4 * r + k4;
        if (act[lr] && col < d) store_agent_d(xw + (row0 + lr) * d + col, old[rb][r] - acc[r]);
      }
    }
    if (RBG < NRBX) {
      __builtin_amdgcn_s_waitcnt(0);  // this group's requests retired
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// u := L11^{-1} u for the unit lower triangular L11 of a panel (rows 16-byte
// aligned in LDS, read two multipliers at a time by every lane at once).  Row
// t + 1 is requested before row t is applied, so each LDS round trip overlaps
// a row of arithmetic; each row's sum runs in four interleaved partial sums,
// so its dependency chain is a quarter of the row long.
__device__ __forceinline__ void lu_forward_subst(double (&u)[NB], const double (*L)[NB + 2]) {
  double2 cur[NB / 2], nxt[NB / 2];
  nxt[0] = reinterpret_cast<const double2*>(L[1])[0];
#pragma unroll
  for (int t = 1; t < NB; ++t) {
#pragma unroll
    for (int s2 = 0; 2 * s2 < t; ++s2) cur[s2] = nxt[s2];
    if (t + 1 < NB) {
#pragma unroll
      for (int s2 = 0; 2 * s2 < t + 1; ++s2)
        nxt[s2] = reinterpret_cast<const double2*>(L[t + 1])[s2];
    }
    double acc[4] = {u[t], 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < t; ++s) {
      const double l = (s & 1) ? cur[s >> 1].y : cur[s >> 1].x;
      acc[s & 3] -= l * u[s];
    }
    u[t] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
}

template <int RPT>
__global__ __launch_bounds__(NT) void lu_pivots_kernel(Gate gt, LuArgs a) {
  QRCP_GATE(gt);
  constexpr int R = 64 * RPT;
  // row strides padded so that the matrix-core operand reads are free of bank conflicts
  // Panel state is double-buffered by panel parity: waves 1-3 update the
  // trailing columns with panel p's multipliers while wave 0 runs the steps
  // of panel p + 1.
  __shared__ double sU[NB][TCH + 16];    // U12 chunk (trail_b: one slice per wave)
  __shared__ double sLr[2][R][NB + 2];   // multipliers of this workgroup's rows
  __shared__ __align__(16) double sL11[2][NB][NB + 2];  // multipliers of the panel's pivot rows
  __shared__ long sRow[2][NB];           // the panel's pivot rows
  __shared__ double sPs[64];             // previous pivot row, shifted to the current column
  __shared__ double sCand[NB];           // panel row of the published candidate
  __shared__ int sAct[2][R];
  __shared__ int sBad, sErr, sTrailCnt;

  const int g = blockIdx.x, G = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  const int d = a.d;
  const long ni = a.ni;
  const int steps = a.steps;
  const long row0 = (long)g * R;
  const long hs = gpad(G);  // stride between a step's header words

  // working copy of this workgroup's rows + non-finite check
  if (tid == 0) {
    sBad = 0;
    sErr = 0;
    sTrailCnt = 0;
  }
  __syncthreads();
  {
    bool bad = false;
    const long nrow = min((long)R, ni - row0);
    for (long e = tid; e < nrow * d; e += NT) {
      const long r = e / d;
      const int c = (int)(e % d);
      const double v = a.msk[(row0 + r) * a.ld + c];
      bad |= !isfinite(v);
      store_agent_d(a.xw + (row0 + r) * d + c, v);
    }
    if (bad) sBad = 1;
  }
  __builtin_amdgcn_s_waitcnt(0);  // the copy is in memory before any header goes out
  __syncthreads();
  const bool wg_bad = sBad != 0;

  // row state (meaningful in wave 0)
  long row[RPT], pos[RPT];
  bool act[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    row[q] = row0 + lane + 64 * q;
    act[q] = row[q] < ni;
    pos[q] = act[q] ? row[q] : LONG_MAX;
  }

  constexpr int NRB = R / 16;
  for (int p0 = 0, pi = 0; p0 < steps; p0 += NB, ++pi) {
    const int ns = min(NB, steps - p0);
    const int par = pi & 1;
    if (wv == 0) {
      double x[RPT][NB];
#pragma unroll
      for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int t = 0; t < NB; ++t)
          x[q][t] = (act[q] && p0 + t < d) ? a.xw[row[q] * d + p0 + t] : 0.0;
      double lprev[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) lprev[q] = 0.0;
      double pprev = 0.0;      // pivot row j-2, panel column `lane`, completed
      double lam_prev = 0.0;   // previous winner's multiplier for the pivot before it
      uint64_t pay = 0;        // payload word `lane` of the previous winner (in flight)
      uint64_t* prev_rec = a.rec;
      bool to = false;
      // The trailing update of the previous panel (waves 1-3) must be in
      // memory before this workgroup's last header of the panel: whoever
      // reads that header reads the updated rows afterwards.
      auto wait_trail = [&]() {
        if (pi == 0) return;
        long spins = 0;
        while (__hip_atomic_load(&sTrailCnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <
               3 * pi) {
          if (++spins > kSpinLimit) {
            to = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      };

      // Publishes the candidate of step j (column 0 of x; column 1 gives the
      // next-column value): the five header words go out in one store
      // instruction.  Returns the candidate's local row, -1 if there is none.
      auto publish_header = [&](int j, const double (&lnew)[RPT]) -> int {
        double cv = -1.0;
        uint64_t ck = NOCAND;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (act[q]) {
            const double v = cand_value(x[q][0]);
            const uint64_t k = ((uint64_t)pos[q] << 32) | (uint64_t)row[q];
            if (better(v, k, cv, ck)) {
              cv = v;
              ck = k;
            }
          }
        }
        wave_argmax(cv, ck);
        int olr = -1;
        uint64_t w2 = 0, w3 = 0, w4 = 0;
        if (ck != NOCAND) {
          olr = (int)((long)(ck & 0xFFFFFFFFull) - row0);
          const int ol = olr & 63, oq = olr >> 6;
          double h0 = x[0][0], h1 = lnew[0], h2 = x[0][1];
#pragma unroll
          for (int q = 1; q < RPT; ++q)
            if (oq == q) {
              h0 = x[q][0];
              h1 = lnew[q];
              h2 = x[q][1];
            }
          w2 = canon(rdlane_d(h0, ol));
          w3 = canon(rdlane_d(h1, ol));
          w4 = canon(rdlane_d(h2, ol));
        }
        if (lane < HW) {
          uint64_t word = dbits(cv);
          if (lane == 1) word = (j == 0 && wg_bad) ? BADKEY : ck;
          if (lane == 2) word = w2;
          if (lane == 3) word = w3;
          if (lane == 4) word = w4;
          store_agent(hdr_at(a.rec, j, G, g) + lane * gpad(G), word);
        }
        return olr;
      };
      // Payload of the candidate published for step j (local row olr):
      // multipliers for the panel columns before j, current values from j on,
      // staged through LDS so that one store instruction writes it.
      auto publish_payload = [&](int j, int olr) {
        if (olr < 0) return;
        const int jl = j - p0, ol = olr & 63, oq = olr >> 6;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (q == oq && lane == ol) {
#pragma unroll
            for (int t = 0; t < NB; ++t) sCand[t] = x[q][t];
          }
        }
        wave_lds_sync();
        if (lane < NB) {
          const double v = (lane < jl) ? sLr[par][olr][lane] : sCand[lane - jl];
          store_agent(pay_at(a.rec, j, G, g) + lane, canon(v));
        }
      };

      if (ns == 1) wait_trail();
      publish_payload(p0, publish_header(p0, lprev));
      for (int jl = 0; jl < ns; ++jl) {
        const int j = p0 + jl;
        // ---- headers of step j ----
        double bv = -2.0;
        uint64_t bk = NOCAND;
        double hx[GQ], hl[GQ], hr[GQ];
        bool badseen = false;
        // every record this lane reads is requested before the first wait, so
        // the headers cost one memory round trip whatever G is
        uint64_t hdr[GQ][HW];
#pragma unroll
        for (int qq = 0; qq < GQ; ++qq) {
          const int gg = lane + 64 * qq;
          if (gg < G && !to) {
            uint64_t* r = hdr_at(a.rec, j, G, gg);
#pragma unroll
            for (int i = 0; i < HW; ++i) hdr[qq][i] = load_agent(r + i * hs);
          }
        }
#pragma unroll
        for (int qq = 0; qq < GQ; ++qq) {
          hx[qq] = 0.0;
          hl[qq] = 0.0;
          hr[qq] = 0.0;
          const int gg = lane + 64 * qq;
          if (gg < G && !to) {
            uint64_t* r = hdr_at(a.rec, j, G, gg);
            uint64_t (&w)[HW] = hdr[qq];
            bool miss = false;
#pragma unroll
            for (int i = 0; i < HW; ++i) miss |= (w[i] == SENT);
            if (miss) {
              // two polls in flight, started ~500 cycles apart: each check
              // consumes the older one while the younger travels, so a word
              // that lands just after one poll is seen by the other (words
              // never change once written, so the copies merge)
              uint64_t pa[HW], pb[HW];
#pragma unroll
              for (int i = 0; i < HW; ++i) pa[i] = load_agent(r + i * hs);
              __builtin_amdgcn_s_sleep(8);
#pragma unroll
              for (int i = 0; i < HW; ++i) pb[i] = load_agent(r + i * hs);
              long spins = 0;
              for (;;) {
                miss = false;
#pragma unroll
                for (int i = 0; i < HW; ++i) {
                  w[i] = (w[i] == SENT) ? pa[i] : w[i];
                  miss |= (w[i] == SENT);
                }
                if (!miss) break;
#pragma unroll
                for (int i = 0; i < HW; ++i) pa[i] = load_agent(r + i * hs);
                miss = false;
#pragma unroll
                for (int i = 0; i < HW; ++i) {
                  w[i] = (w[i] == SENT) ? pb[i] : w[i];
                  miss |= (w[i] == SENT);
                }
                if (!miss) break;
#pragma unroll
                for (int i = 0; i < HW; ++i) pb[i] = load_agent(r + i * hs);
                if (++spins > kSpinLimit) {
                  to = true;
                  break;
                }
              }
            }
            if (!to) {
              if (w[1] == BADKEY) {
                badseen = true;
              } else if (w[1] != NOCAND) {
                const double v = bitsd(w[0]);
                if (better(v, w[1], bv, bk)) {
                  bv = v;
                  bk = w[1];
                }
              }
              hx[qq] = bitsd(w[2]);
              hl[qq] = bitsd(w[3]);
              hr[qq] = bitsd(w[4]);
            }
          }
        }
        wave_argmax(bv, bk);
        if (__any(to) || __any(badseen)) {
          if (lane == 0) {
            store_agent_i32(a.status, __any(to) ? QRCP_ERR_TIMEOUT : QRCP_ERR_NONFINITE);
            sErr = 1;
          }
          break;
        }
        const long wrow = (long)(bk & 0xFFFFFFFFull);
        const long wpos = (long)(bk >> 32);
        const int wg = (int)(wrow / R), wl = wg & 63, wq = wg >> 6;
        double sx = hx[0], sl = hl[0], sr = hr[0];
#pragma unroll
        for (int qq = 1; qq < GQ; ++qq)
          if (qq == wq) {
            sx = hx[qq];
            sl = hl[qq];
            sr = hr[qq];
          }
        const double pjj = rdlane_d(sx, wl), lam = rdlane_d(sl, wl), r1 = rdlane_d(sr, wl);

        // ---- pivot row j-1, completed from its payload ----
        double pcur = 0.0;
        if (jl > 0) {
          if (lane < NB) {
            long spins = 0;
            while (pay == SENT) {
              if (++spins > kSpinLimit) {
                to = true;
                break;
              }
              __builtin_amdgcn_s_sleep(1);
              pay = load_agent(prev_rec + lane);
            }
          }
          if (__any(to)) {
            if (lane == 0) {
              store_agent_i32(a.status, QRCP_ERR_TIMEOUT);
              sErr = 1;
            }
            break;
          }
          const double raw = bitsd(pay);
          if (lane < jl - 1) sL11[par][jl - 1][lane] = raw;
          pcur = (lane >= jl && lane < NB) ? raw - lam_prev * pprev : 0.0;
        }
        // broadcast copy: sPs[t] = pivot row j-1 in panel column jl+1+t (0 past the panel)
        if (lane >= jl + 1) sPs[lane - jl - 1] = pcur;
        wave_lds_sync();
        // this winner's payload: requested now, used at the next step
        uint64_t* wrec = pay_at(a.rec, j, G, wg);
        pay = (lane < NB) ? load_agent(wrec + lane) : 0;
        prev_rec = wrec;
        if (lane == 0) {
          sRow[par][jl] = wrow;
          if (g == 0) {
            a.ipiv[j] = wpos;
            a.jsk[j] = wrow;
          }
        }

        // ---- elimination: next column now, the rest after the header ----
        const double s1 = sPs[0], s2 = sPs[1];
        const double pj1 = r1 - lam * s1;   // U(j, j+1)
        double lnew[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (act[q] && row[q] == wrow) act[q] = false;
          if (act[q] && pos[q] == j) pos[q] = wpos;
          const double l = (act[q] && pjj != 0.0) ? x[q][0] / pjj : 0.0;
          x[q][1] = (x[q][1] - lprev[q] * s1) - l * pj1;
          x[q][2] -= lprev[q] * s2;
          lnew[q] = l;
          sLr[par][lane + 64 * q][jl] = l;
        }
        // shift: column j+1 becomes register 0
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
#pragma unroll
          for (int t = 0; t < NB - 1; ++t) x[q][t] = x[q][t + 1];
          x[q][NB - 1] = 0.0;
        }
        if (jl + 2 == ns) wait_trail();
        const int olr = (jl + 1 < ns) ? publish_header(j + 1, lnew) : -1;
        // previous pivot's contribution to the remaining panel columns
#pragma unroll
        for (int t = 2; t < NB - 1; ++t) {
          const double sv = sPs[t];
#pragma unroll
          for (int q = 0; q < RPT; ++q) x[q][t] -= lprev[q] * sv;
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q) lprev[q] = lnew[q];
        pprev = pcur;
        lam_prev = lam;
        publish_payload(j + 1, olr);
        wave_lds_sync();  // this step's LDS reads before the next step's writes
      }
      // the last pivot row's multipliers (row ns-1 of L11)
      if (!sErr) {
        if (lane < NB) {
          long spins = 0;
          while (pay == SENT) {
            if (++spins > kSpinLimit) {
              to = true;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            pay = load_agent(prev_rec + lane);
          }
        }
        if (__any(to)) {
          if (lane == 0) {
            store_agent_i32(a.status, QRCP_ERR_TIMEOUT);
            sErr = 1;
          }
        } else if (lane < ns - 1) {
          sL11[par][ns - 1][lane] = bitsd(pay);
        }
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) sAct[par][lane + 64 * q] = act[q] ? 1 : 0;
    } else if (pi > 0) {
      // ---- previous panel's update of columns p0 + NB .. d (waves 1-3) ----
      // Each wave takes 64-column groups with its own slice of sU, so the
      // three waves never wait for each other, and none waits for wave 0.
      const int pb = par ^ 1, uc0 = 64 * (wv - 1);
      for (int c0 = p0 + NB + uc0; c0 < d; c0 += 192) {
        const int cw = min(64, d - c0);
        if (lane < cw) {
          double u[NB];
#pragma unroll
          for (int t0 = 0; t0 < NB; t0 += LUB) {
#pragma unroll
            for (int t = t0; t < t0 + LUB; ++t) u[t] = load_agent_d(a.xw + sRow[pb][t] * (long)d + c0 + lane);
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_sched_barrier(0);
          }
          lu_forward_subst(u, sL11[pb]);
#pragma unroll
          for (int t = 0; t < NB; ++t) sU[t][uc0 + lane] = u[t];
        }
        wave_lds_sync();
        const int ncb = (cw + 15) / 16;
        for (int cb = 0; cb < ncb; ++cb)
          lu_tile_update<NRB, LRBG>(a.xw, row0, d, c0 + cb * 16 + i16, 0, sLr[pb], sU,
                              uc0 + cb * 16 + i16, sAct[pb], i16, k4);
        wave_lds_sync();
      }
      __builtin_amdgcn_s_waitcnt(0);  // the updated rows are in memory before wave 0's last header
      if (lane == 0)
        __hip_atomic_fetch_add(&sTrailCnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    if (sErr) return;  // uniform
    const int pend = p0 + ns;
    if (pend >= steps) break;  // no later pivot step needs the trailing columns

    // ---- this panel's update of the next panel's columns (all waves) ----
    // The rest of the trailing columns is updated by waves 1-3 during the
    // next panel's pivot steps.
    {
      constexpr int HRB = NRB / 2;
      const int cw = min(NB, d - pend);
      const int cb = wv & 1, rb0 = (wv >> 1) * HRB;
      const int col = pend + cb * 16 + i16;
      // this wave's block of own rows, requested before the substitution
      double old[HRB][4];
#pragma unroll
      for (int rb = 0; rb < HRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int lr = (rb0 + rb) * 16 + 4 * r + k4;
          old[rb][r] = (sAct[par][lr] && col < pend + cw) ? a.xw[(row0 + lr) * d + col] : 0.0;
        }
      if (tid < cw) {
        double u[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) u[t] = load_agent_d(a.xw + sRow[par][t] * (long)d + pend + tid);
        lu_forward_subst(u, sL11[par]);
#pragma unroll
        for (int t = 0; t < NB; ++t) sU[t][tid] = u[t];
      }
      __syncthreads();
      if (cb * 16 < cw) {
#pragma unroll
        for (int rb = 0; rb < HRB; ++rb) {
          dv4 acc = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int s = 0; s < NB / 4; ++s)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sLr[par][(rb0 + rb) * 16 + i16][4 * s + k4],
                                                       sU[4 * s + k4][cb * 16 + i16], acc, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int lr = (rb0 + rb) * 16 + 4 * r + k4;
            if (sAct[par][lr] && col < pend + cw) a.xw[(row0 + lr) * d + col] = old[rb][r] - acc[r];
          }
        }
      }
    }
    // Only this workgroup's wave 0 reads these columns (its next panel); the
    // rows other workgroups read were released by waves 1-3.
    __syncthreads();  // the next panel's columns before wave 0 loads them
  }
  // positions of the rows that were never pivots
  if (wv == 0) {
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (act[q] && pos[q] < ni) a.jsk[pos[q]] = row[q];
  }
}

int pick_rpt(long ni) {
  static const int forced = [] {
    const char* e = getenv("QRCP_LU_RPT");
    return e ? atoi(e) : 0;
  }();
  if ((forced == 1 || forced == 2) && (ni + 64L * forced - 1) / (64L * forced) <= kMaxGroups)
    return forced;
  if (ni <= 64L * 64) return 1;
  if ((ni + 127) / 128 <= kMaxGroups) return 2;
  return 0;
}

}  // namespace

int lu_resident_groups(i64 ni) {
  const int rpt = pick_rpt(ni);
  return rpt ? (int)((ni + 64L * rpt - 1) / (64L * rpt)) : 0;
}

size_t lu_records_bytes(int d, i64 ni, int max_steps) {
  const int rpt = pick_rpt(ni);
  if (!rpt) return 0;
  const long G = (ni + 64L * rpt - 1) / (64L * rpt);
  long steps = std::min((long)d, (long)ni);
  if (max_steps > 0) steps = std::min(steps, (long)max_steps);
  return (size_t)steps * step_words((int)G) * sizeof(uint64_t);
}

size_t lu_records_bytes_upto(int d, i64 n) {
  // records grow with n_i within each rows-per-lane regime, but the switch to
  // two rows per lane above 64 x 64 rows halves the group count, so the
  // largest need is at n itself or at the top of the one-row regime
  return std::max(lu_records_bytes(d, n), lu_records_bytes(d, std::min<i64>(n, 64L * 64)));
}

int launch_lu_pivots(const double* Msk, int d, i64 ni, i64 ld, double* Xw, uint64_t* rec,
                     size_t rec_bytes, i64* ipiv, i64* jsk, int* status_dev, hipStream_t st,
                     int max_steps) {
  if (ni <= 0 || d <= 0) return QRCP_OK;
  const int rpt = pick_rpt(ni);
  if (!rpt) return QRCP_ERR_UNSUPPORTED;
  const size_t need = lu_records_bytes(d, ni, max_steps);
  if (need > rec_bytes) return QRCP_ERR_WORKSPACE;
  const int G = (int)((ni + 64L * rpt - 1) / (64L * rpt));
  int steps = (int)std::min((long)d, (long)ni);
  if (max_steps > 0) steps = std::min(steps, max_steps);
  QRCP_TRY(launch_fill_u64(rec, (i64)(need / sizeof(uint64_t)), SENT, st));
  LuArgs args{Msk, (long)ld, d, (long)ni, steps, Xw, rec, (long*)ipiv, (long*)jsk, status_dev};
  Gate gt = current_gate();
  void* params[] = {&gt, &args};
  const void* fn = rpt == 1 ? (const void*)lu_pivots_kernel<1> : (const void*)lu_pivots_kernel<2>;
  QRCP_TRY(launch_resident(fn, dim3(G), dim3(NT), params, 0, st));
  return QRCP_OK;
}

}  // namespace qrcp
