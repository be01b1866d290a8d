// Pixel covariance of a sky map with angular power spectrum C_l (Sec. III B uses it to test
// the maps; eq. harmonics gives it for every pixel pair):
//
//   Gamma_ij = sum_{l=0}^{lmax} (2l + 1) C_l P_l(x_ij) / (4 pi),  x_ij = n_i . n_j in [-1, 1].
//
// Two entries per thread (columns j and j + 16: the LDS reads of each l serve both, and
// the two recurrences are independent), 16 x 32 entries per workgroup, all in FP64. P_l
// runs by the three-term recurrence P_{l+1} = a_l x P_l - b_l P_{l-1},
// a_l = (2l + 1)/(l + 1), b_l = l/(l + 1); the per-l factors w_l = (2l + 1) C_l / (4 pi),
// a_l and b_l are staged in LDS a chunk at a time, so each entry costs two multiply-adds
// and two multiplies per l. The work is FP64 vector arithmetic: n^2 (lmax + 1) x 4
// operations per launch.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace cmbx {
namespace {

constexpr int kCovTile = 16;
constexpr int kCovChunk = 512;

__global__ __launch_bounds__(kCovTile* kCovTile) void k_pixel_cov(const double* __restrict__ dirs, int64_t n,
                                                                   const double* __restrict__ cl, int lmax,
                                                                   double* __restrict__ gamma) {
  __shared__ double w[kCovChunk], a[kCovChunk], b[kCovChunk];
  const int64_t i = (int64_t)blockIdx.y * kCovTile + threadIdx.x / kCovTile;
  const int64_t j0 = (int64_t)blockIdx.x * 2 * kCovTile + threadIdx.x % kCovTile;
  const int64_t j1 = j0 + kCovTile;
  const bool on0 = i < n && j0 < n, on1 = i < n && j1 < n;
  double x0 = 0.0, x1 = 0.0;
  if (on0) {
    x0 = dirs[3 * i] * dirs[3 * j0] + dirs[3 * i + 1] * dirs[3 * j0 + 1] + dirs[3 * i + 2] * dirs[3 * j0 + 2];
    x0 = x0 > 1.0 ? 1.0 : (x0 < -1.0 ? -1.0 : x0);
  }
  if (on1) {
    x1 = dirs[3 * i] * dirs[3 * j1] + dirs[3 * i + 1] * dirs[3 * j1 + 1] + dirs[3 * i + 2] * dirs[3 * j1 + 2];
    x1 = x1 > 1.0 ? 1.0 : (x1 < -1.0 ? -1.0 : x1);
  }
  constexpr double inv4pi = 0.0795774715459476678844418816862571810;  // 1 / (4 pi)
  // P_l and P_{l-1} of both entries, and their sums
  double p0 = 1.0, pm0 = 0.0, acc0 = 0.0, p1 = 1.0, pm1 = 0.0, acc1 = 0.0;
  for (int l0 = 0; l0 <= lmax; l0 += kCovChunk) {
    const int cnt = lmax + 1 - l0 < kCovChunk ? lmax + 1 - l0 : kCovChunk;
    __syncthreads();  // the previous chunk is no longer read
    for (int t = threadIdx.x; t < cnt; t += kCovTile * kCovTile) {
      const double l = (double)(l0 + t);
      w[t] = (2.0 * l + 1.0) * cl[l0 + t] * inv4pi;
      a[t] = (2.0 * l + 1.0) / (l + 1.0);
      b[t] = l / (l + 1.0);
    }
    __syncthreads();
    for (int t = 0; t < cnt; ++t) {
      const double wt = w[t], at = a[t], bt = b[t];
      acc0 = fma(wt, p0, acc0);
      acc1 = fma(wt, p1, acc1);
      const double n0 = fma(at * x0, p0, -bt * pm0);
      const double n1 = fma(at * x1, p1, -bt * pm1);
      pm0 = p0;
      p0 = n0;
      pm1 = p1;
      p1 = n1;
    }
  }
  if (on0) gamma[i * n + j0] = acc0;
  if (on1) gamma[i * n + j1] = acc1;
}

}  // namespace

hipError_t launch_pixel_cov(const double* dirs, int64_t n, const double* cl, int lmax, double* gamma,
                            hipStream_t s) {
  const int64_t rows = (n + kCovTile - 1) / kCovTile, cols = (n + 2 * kCovTile - 1) / (2 * kCovTile);
  hipLaunchKernelGGL(k_pixel_cov, dim3((unsigned)cols, (unsigned)rows), dim3(kCovTile * kCovTile), 0, s, dirs, n, cl,
                     lmax, gamma);
  return hipGetLastError();
}

}  // namespace cmbx
