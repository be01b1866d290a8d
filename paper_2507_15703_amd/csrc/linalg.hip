// FP64 dense linear algebra of the covariance test (Sec. III B): Cholesky factor of the
// pixel covariance Gamma + s^2 I and the triangular solve that whitens maps, for gfx950.
//
// Blocked right-looking Cholesky on 64-wide panels: the diagonal block is factored in LDS
// by one workgroup; the panel below it is solved against that block row by row
// (L21 = A21 L11^-T); the trailing lower triangle is updated, A22 -= L21 L21^T, by a
// matrix-core kernel (v_mfma_f64_16x16x4f64, FP64 in and out). The whitening solve
// X = B L^-T (the rows of B are maps) runs panel by panel the same way: the panel's
// columns solved against the diagonal block, the rest updated by the same product kernel.
//
// Matrices are row-major FP64 with a leading dimension; only the lower triangle of the
// factored matrix is read or written.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "linalg.hpp"

namespace cmbx {
namespace {

constexpr int kNB = kCholPanel;  // panel width
constexpr int kPad = kNB + 1;    // LDS row stride (doubles): rows fall on different banks

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Diagonal block (nb x nb, lower) of A factored in place: for each column j the pivot
// d = A_jj (already reduced by the earlier columns) must be positive; L_jj = sqrt(d), the
// column below is divided by it and the trailing lower triangle of the block updated. A
// non-positive (or NaN) pivot records column j0 + j + 1 in *info (the first one only) and
// the factorisation goes on with NaN.
__global__ __launch_bounds__(256) void k_potrf_diag(double* __restrict__ A, int64_t lda, int nb, int64_t j0,
                                                    int64_t* __restrict__ info) {
  __shared__ double S[kNB][kPad];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, k = e % nb;
    if (k <= i) S[i][k] = A[(int64_t)i * lda + k];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      const double d = S[j][j];
      if (!(d > 0.0) && info && *info == 0) *info = j0 + j + 1;
      S[j][j] = sqrt(d);
    }
    __syncthreads();
    const double piv = S[j][j];
    for (int i = j + 1 + tid; i < nb; i += 256) S[i][j] = S[i][j] / piv;
    __syncthreads();
    const int m = nb - j - 1;  // trailing block: rows and columns j + 1 .. nb - 1, lower part
    for (int e = tid; e < m * m; e += 256) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) S[i][k] = S[i][k] - S[i][j] * S[k][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, k = e % nb;
    if (k <= i) A[(int64_t)i * lda + k] = S[i][k];
  }
}

// Each row x of X (rows x nb, leading dimension ldx) becomes x L^-T for the lower
// triangular L (nb x nb, leading dimension ldl): forward substitution
// x_j = (x_j - sum_{k < j} x_k L_jk) / L_jj, one thread per row, L in LDS.
__global__ __launch_bounds__(256) void k_row_solve(double* __restrict__ X, int64_t ldx, int64_t rows,
                                                   const double* __restrict__ L, int64_t ldl, int nb) {
  __shared__ double S[kNB][kPad];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, k = e % nb;
    S[i][k] = k <= i ? L[(int64_t)i * ldl + k] : 0.0;
  }
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  double* x = X + r * ldx;
  double v[kNB];
#pragma unroll
  for (int j = 0; j < kNB; ++j) v[j] = j < nb ? x[j] : 0.0;
#pragma unroll
  for (int j = 0; j < kNB; ++j) {
    if (j < nb) {
      double s = v[j];
#pragma unroll
      for (int k = 0; k < j; ++k) s -= v[k] * S[j][k];
      v[j] = s / S[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < kNB; ++j)
    if (j < nb) x[j] = v[j];
}

// C -= A B^T for C m x n, A m x K, B n x K (K <= 64), all row-major. Workgroup = one 64 x 64
// tile of C, four waves of 32 x 32 (2 x 2 blocks of 16 x 16); A and B tiles staged in LDS
// (zero beyond the edges and beyond K), products on the matrix cores in steps of 4 along K.
// Operand layout of v_mfma_f64_16x16x4f64 (wave64, measured on gfx950 with one-hot
// operands): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator v of lane
// l is D[l / 16 + 4 v][l % 16]. With `lower`
// only the tiles and entries on or below the diagonal are written.
__global__ __launch_bounds__(256) void k_gemm_nt_sub(int64_t m, int64_t n, int K, const double* __restrict__ A,
                                                     int64_t lda, const double* __restrict__ B, int64_t ldb,
                                                     double* __restrict__ C, int64_t ldc, int lower) {
  const int64_t row0 = (int64_t)blockIdx.y * 64, col0 = (int64_t)blockIdx.x * 64;
  if (lower && col0 > row0) return;  // the whole tile lies above the diagonal
  __shared__ double As[64][kPad], Bs[64][kPad];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e / 64, k = e % 64;
    As[r][k] = (row0 + r < m && k < K) ? A[(row0 + r) * lda + k] : 0.0;
    Bs[r][k] = (col0 + r < n && k < K) ? B[(col0 + r) * ldb + k] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 4) {
    double a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = As[wr + 16 * t + li][k0 + lk];  // A block: row li, k = lk
      b[t] = Bs[wc + 16 * t + li][k0 + lk];  // B^T block: k = lk, column li
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + wr + 16 * bi + lk + 4 * v;
        const int64_t c = col0 + wc + 16 * bj + li;
        if (r < m && c < n && (!lower || c <= r)) C[r * ldc + c] -= acc[bi][bj][v];
      }
}

__global__ __launch_bounds__(256) void k_add_diag(double* __restrict__ A, int64_t lda, int64_t n, double s) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) A[i * lda + i] += s;
}

__global__ void k_zero_info(int64_t* info) { *info = 0; }

dim3 grid1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t launch_gemm_nt_sub(int64_t m, int64_t n, int K, const double* A, int64_t lda, const double* B,
                              int64_t ldb, double* C, int64_t ldc, int lower, hipStream_t s) {
  if (m < 1 || n < 1) return hipSuccess;
  if (K < 1 || K > kNB) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
  hipLaunchKernelGGL(k_gemm_nt_sub, grid, dim3(256), 0, s, m, n, K, A, lda, B, ldb, C, ldc, lower);
  return hipGetLastError();
}

hipError_t launch_cholesky(double* A, int64_t n, int64_t lda, double shift, int64_t* info, hipStream_t s) {
  if (info) hipLaunchKernelGGL(k_zero_info, dim3(1), dim3(1), 0, s, info);
  if (shift != 0.0) hipLaunchKernelGGL(k_add_diag, grid1(n), dim3(256), 0, s, A, lda, n, shift);
  for (int64_t j0 = 0; j0 < n; j0 += kNB) {
    const int nb = (int)(n - j0 < kNB ? n - j0 : kNB);
    double* a11 = A + j0 * lda + j0;
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, a11, lda, nb, j0, info);
    const int64_t rest = n - j0 - nb;
    if (rest > 0) {
      double* a21 = a11 + nb * lda;
      hipLaunchKernelGGL(k_row_solve, grid1(rest), dim3(256), 0, s, a21, lda, rest, (const double*)a11, lda, nb);
      const hipError_t e = launch_gemm_nt_sub(rest, rest, nb, a21, lda, a21, lda, a21 + nb, lda, 1, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t launch_trsm_rows(const double* L, int64_t n, int64_t ldl, double* B, int64_t nrhs, int64_t ldb,
                            hipStream_t s) {
  for (int64_t j0 = 0; j0 < n; j0 += kNB) {
    const int nb = (int)(n - j0 < kNB ? n - j0 : kNB);
    hipLaunchKernelGGL(k_row_solve, grid1(nrhs), dim3(256), 0, s, B + j0, ldb, nrhs, L + j0 * ldl + j0, ldl, nb);
    const int64_t rest = n - j0 - nb;
    if (rest > 0) {
      const hipError_t e = launch_gemm_nt_sub(nrhs, rest, nb, B + j0, ldb, L + (j0 + nb) * ldl + j0, ldl, B + j0 + nb, ldb,
                                              0, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

}  // namespace cmbx
