// Internal launch interface between the host driver and the kernels.
#pragma once

#include "common.hpp"

namespace qrcp {

enum class Prec { F64, F32, BF16 };
enum class GemmKind { Generic, TrailingUpdate, TrailingW, Sketch };

struct GemmArgs {
  int M = 0, N = 0, K = 0;
  double alpha = 1.0, beta = 0.0;
  const double* A = nullptr;
  i64 lda = 0;
  const double* B = nullptr;
  i64 ldb = 0;
  const i64* bcol = nullptr;  // optional column indirection of op(B) (TB = false)
  double* C = nullptr;
  i64 ldc = 0;
  int kchunk = 0;        // set by gemm()
  double* partial = nullptr;
  GemmKind kind = GemmKind::Generic;  // selects a named kernel symbol (profiling)
};

// C = alpha op(A) op(B) + beta C.  split_ws (may be null) enables split-K.
int gemm(bool ta, bool tb, Prec prec, GemmArgs g, double* split_ws, size_t split_ws_bytes,
         hipStream_t st);
size_t gemm_splitk_bytes(long M, long N, int splits);
int gemm_pick_splits(long M, long N, long K, long target = 512);

// ---- sketch operator ----
int launch_sketch_operator(double* St, i64 m, int d, i64 ldst, uint64_t seed, hipStream_t st);
int launch_sketch_operator_bf16(unsigned short* St, i64 m, int d, i64 ldst, uint64_t seed, hipStream_t st);
// M^sk = S A with S in BF16 (generated into sbuf) and FP32 accumulation, for
// d <= 320; QRCP_ERR_UNSUPPORTED (nothing launched) otherwise, or when sbuf is
// too small, so that the caller takes the general BF16 product.
int launch_sketch_bf16(const double* A, i64 m, i64 n, i64 lda, int d, uint64_t seed, double* Msk, i64 ldmsk,
                       void* sbuf, size_t sbuf_bytes, double* split, size_t split_bytes, hipStream_t st);
int launch_philox(const uint32_t* ctr, i64 count, uint32_t k0, uint32_t k1, uint32_t* out,
                  hipStream_t st);

// ---- small dense kernels ----
// X = R^{-1} for an upper triangular n x n R (X zero below the diagonal).
// low_lds: a variant whose workgroups need little LDS (for launches that run
// beside a GEMM occupying the compute units).
int launch_trinv_upper(const double* R, i64 ldr, int n, double* X, i64 ldx, hipStream_t st,
                       bool low_lds = false);
// T^{-1} = diag(1/tau) + strictly-upper(G) formed in place in G (n x n), then
// T = inverse into T (the compact WY factor from Y^T Y and tau).
int launch_ut_tinv(double* G, i64 ldg, const double* tau, int n, hipStream_t st);
// Cholesky G = R^T R (upper, n x n) in place in G's upper triangle (lower part
// zeroed); *info_dev = number of columns factored (n when no breakdown).
int launch_potrf_upper(double* G, i64 ldg, int n, int* info_dev, hipStream_t st);
// Sign-modified LU without pivoting of the k x k head of Q (reconstruction):
// overwrites Q(0:k,0:k) with Y1 (strict lower) and U (upper); dsig[k].
int launch_headlu(double* Q, i64 ldq, int k, double* dsig, hipStream_t st);
// The same two factorizations over resident workgroups (one per 32 x 32
// block) for orders up to 256, given blockfact_scratch_bytes() of scratch;
// otherwise (or with QRCP_SMALLFACT=single) the single-workgroup kernels.
// potrf: info < 0 after a timeout; headlu: *status = QRCP_ERR_TIMEOUT.
size_t blockfact_scratch_bytes();
int blockfact_groups(int n);
int launch_potrf_mw(double* G, i64 ldg, int n, int* info_dev, void* scratch, size_t scratch_bytes,
                    hipStream_t st);
int launch_headlu_mw(double* Q, i64 ldq, int k, double* dsig, void* scratch, size_t scratch_bytes,
                     int* status, hipStream_t st);
// tau_j = -dsig_j U(j,j)
int launch_tau_from_u(const double* Q, i64 ldq, int k, const double* dsig, double* tau,
                      hipStream_t st);
// R11 = diag(dsig) * P (P = Rc Rsk11, k x k, full storage) written to the upper
// triangle of A (lda); the strictly lower part of A is left as is.
int launch_write_r11(const double* P, i64 ldp, int k, const double* dsig, double* A, i64 lda,
                     hipStream_t st);
// generic helpers
// X = triu(S) diag(dvec), n x n
int launch_scale_upper_cols(const double* S, i64 lds, const double* dvec, int n, double* X,
                            i64 ldx, hipStream_t st);
int launch_copy2d(const double* src, i64 lds, double* dst, i64 ldd, i64 rows, i64 cols,
                  hipStream_t st);
int launch_fill(double* dst, i64 ld, i64 rows, i64 cols, double v, hipStream_t st);
int launch_fill_u64(uint64_t* dst, i64 count, uint64_t v, hipStream_t st);
int launch_triu_copy(const double* src, i64 lds, double* dst, i64 ldd, i64 rows, i64 cols,
                     hipStream_t st);
int launch_scale_cols_lower_copy(double* dst, i64 ldd, const double* src, i64 lds, i64 rows,
                                 int k, hipStream_t st);
int launch_any_nonfinite(const double* X, i64 ld, i64 rows, i64 cols, int* flag, hipStream_t st);

// ---- pivot selection (cooperative GETRF pivots) ----
// max_steps > 0 stops the elimination after that many steps (ipiv[0:steps] and
// the positions they imply); 0 runs all min(d, ni) steps.
size_t lu_records_bytes(int d, i64 ni, int max_steps = 0);
// the largest lu_records_bytes(d, n_i) over 1 <= n_i <= n (a factorization's blocks)
size_t lu_records_bytes_upto(int d, i64 n);
int launch_lu_pivots(const double* Msk, int d, i64 ni, i64 ld, double* Xw, uint64_t* rec,
                     size_t rec_bytes, i64* ipiv, i64* jsk, int* status_dev, hipStream_t st,
                     int max_steps = 0);

// ---- sketch QR (cooperative head + explicit Q^T for the tail) ----
size_t sketch_qr_ws_bytes(int d, i64 ni);
int run_sketch_qr(const double* B, int d, i64 ni, i64 ldb, double* R, i64 ldr, void* ws,
                  size_t ws_bytes, int* status_dev, hipStream_t st);

// ---- column-pivoted QR of the sketch (GEQP3; the alternative wide QRCP) ----
// Msk d x ni (ld) -> jsk (pivot order), R (upper trapezoid, zeros below; may
// alias Msk); X is a d x ni work copy (ld d); only the first psteps steps pivot.
size_t sketch_geqp3_ws_bytes(int d);
int launch_sketch_geqp3(const double* Msk, int d, i64 ni, i64 ld, int psteps, double* X,
                        double* R, i64 ldr, i64* jsk, void* ws, size_t ws_bytes, int* status,
                        hipStream_t st);

// ---- column bookkeeping ----
// jsk -> new logical maps (ping-pong arrays) + the placement plan
int launch_perm_plan(const i64* jsk, i64 s, i64 n, int kmax, const i64* J0, i64* J1,
                     const i64* phys0, i64* phys1, i64* inv, i64* plan, hipStream_t st);
int launch_sketch_permute(const double* src, double* dst, int d, i64 ld, i64 ni,
                          const i64* jsk, hipStream_t st);
int launch_place_columns(double* A, i64 lda, i64 m, i64 s, int kmax, const i64* plan,
                         double* tmp, i64 ldt, hipStream_t st);
int launch_final_permute(double* A, i64 lda, i64 m, i64 l, i64 n, const i64* phys, double* tmp,
                         hipStream_t st);
int launch_jpiv_out(const i64* J, i64 n, i64 base, i64* out, hipStream_t st);
int launch_iota(i64* x, i64 n, hipStream_t st);

// Workgroups of the kernels whose workgroups wait on each other (all must be
// resident at once): pivot selection on n_i sketch columns, sketch-QR head.
int lu_resident_groups(i64 ni);
int sketch_head_groups(int d, i64 ni);

// qrcp_factor for the request server's workers: every launch on the worker's
// own stream (the concurrent requests keep the device busy, a second stream
// per worker would only share the hardware queues with other workers')
int factor_served(double* A, int64_t m, int64_t n, int64_t lda, int64_t block_size,
                  double sketch_factor, uint64_t seed, double tol, int64_t* jpiv, double* tau,
                  int64_t* rank, const qrcp_opts* opts, void* workspace, size_t workspace_bytes,
                  void* stream);

}  // namespace qrcp
