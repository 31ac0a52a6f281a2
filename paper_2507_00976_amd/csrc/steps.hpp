// Launchers of the small per-block kernels (steps.hip) and of the extra
// dense helpers shared by the host driver.
#pragma once

#include "common.hpp"

namespace qrcp {

int launch_sketch_ref(const double* X, i64 ld, int rows, i64 cols, double* colss, double* ref,
                      hipStream_t st);
int launch_trirank(const double* R, i64 ldr, int kmax, double tol, const double* ref, int* kdev,
                   hipStream_t st);
int launch_mask_k(double* X, i64 ld, int n, const int* kdev, hipStream_t st);
int launch_unit_lower(const double* H, i64 ldh, int k, double* Y, i64 ldy, hipStream_t st);
int launch_ut_zero_diag(double* T, i64 ldt, const double* tau, int n, hipStream_t st);
int launch_set_identity(double* dst, i64 ld, i64 n, hipStream_t st);

// ---- control of the device-driven block loop (LoopCtl) ----
int launch_loop_init(LoopCtl* ctl, hipStream_t st);
// status/kdev: the block's error word and effective width (second: a second
// Cholesky pass, which may only shrink the width); host_nblk (device address
// of a pinned host word, may be null) receives the block count once the loop
// stops
int launch_loop_decide(LoopCtl* ctl, const int* status, const int* kdev, int blk, int kmax, i64 s,
                       i64 c, i64 lim, bool second, int* host_nblk, hipStream_t st);
int launch_pad_identity(double* X, i64 ld, int n, const int* kdev, hipStream_t st);
int launch_zero_tail(double* v, int n, const int* kdev, hipStream_t st);
int launch_copy_cols_from(const double* src, i64 lds, double* dst, i64 ldd, i64 rows, int cols,
                          const int* kdev, hipStream_t st);
// after the loop: the live maps into slot 0
int launch_loop_pick(const LoopCtl* ctl, i64* J0, const i64* J1, i64* P0, const i64* P1, i64 n,
                     hipStream_t st);
// then tau(ell:) = 0, the unplaced columns ell.. in logical order (tmp: m x n
// doubles; jpiv is written by the caller from J0); rank and status into the
// caller's device words
int launch_loop_final(const LoopCtl* ctl, double* A, i64 lda, i64 m, i64 n, const i64* P0,
                      double* tau, i64 mn, double* tmp, const int* status, i64* rank_dev,
                      int* status_dev, hipStream_t st);
// rank 0 and QRCP_OK into the caller's device words (an empty matrix)
int launch_set_result(i64* rank_dev, int* status_dev, hipStream_t st);
int launch_copy_result(const i64* rank_dev, const int* status_dev, CallResult* out, hipStream_t st);

}  // namespace qrcp
