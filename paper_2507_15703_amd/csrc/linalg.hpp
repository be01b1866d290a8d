// Internal interface of the FP64 linear algebra of the covariance test (linalg.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmbx {

constexpr int kCholPanel = 64;  // panel width of the blocked factorisation and solve

// A (n x n, leading dimension lda) <- its lower Cholesky factor of A + shift I, in place
// (lower triangle only). *info (device, may be NULL) <- 0, or the 1-based column of the
// first non-positive pivot.
hipError_t launch_cholesky(double* A, int64_t n, int64_t lda, double shift, int64_t* info, hipStream_t s);
// B (nrhs x n, leading dimension ldb: one right-hand side per row) <- B L^-T for the lower
// triangular L (n x n, leading dimension ldl), i.e. every row b becomes L^-1 b.
hipError_t launch_trsm_rows(const double* L, int64_t n, int64_t ldl, double* B, int64_t nrhs, int64_t ldb,
                            hipStream_t s);
// C (m x n) -= A (m x K) B (n x K)^T, K <= kCholPanel; lower: only entries with column <= row.
hipError_t launch_gemm_nt_sub(int64_t m, int64_t n, int K, const double* A, int64_t lda, const double* B,
                              int64_t ldb, double* C, int64_t ldc, int lower, hipStream_t s);

}  // namespace cmbx
