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

}  // namespace qrcp
