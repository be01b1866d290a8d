// Pixel covariance of a sky map with angular power spectrum C_l (Sec. III B uses it to test
// the maps; eq. harmonics gives it for every pixel pair):
//
//   Gamma_ij = sum_{l=0}^{lmax} (2l + 1) C_l P_l(x_ij) / (4 pi),  x_ij = n_i . n_j in [-1, 1].
//
// Four entries per thread (columns j, j + 16, j + 32, j + 48: the LDS reads of each l
// serve all four, and their recurrences are independent), 16 x 64 entries per workgroup,
// all in FP64. P_l
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
constexpr int kCovCols = 4;  // entries per thread, kCovTile apart along a row
constexpr int kCovChunk = 512;

__global__ __launch_bounds__(kCovTile* kCovTile) void k_pixel_cov(const double* __restrict__ dirs, int64_t n,
                                                                   const double* __restrict__ cl, int lmax,
                                                                   double* __restrict__ gamma) {
  __shared__ double w[kCovChunk], a[kCovChunk], b[kCovChunk];
  const int64_t i = (int64_t)blockIdx.y * kCovTile + threadIdx.x / kCovTile;
  const int64_t j0 = (int64_t)blockIdx.x * kCovCols * kCovTile + threadIdx.x % kCovTile;
  double x[kCovCols];
#pragma unroll
  for (int e = 0; e < kCovCols; ++e) {
    const int64_t j = j0 + e * kCovTile;
    double v = 0.0;
    if (i < n && j < n) {
      v = dirs[3 * i] * dirs[3 * j] + dirs[3 * i + 1] * dirs[3 * j + 1] + dirs[3 * i + 2] * dirs[3 * j + 2];
      v = v > 1.0 ? 1.0 : (v < -1.0 ? -1.0 : v);
    }
    x[e] = v;
  }
  constexpr double inv4pi = 0.0795774715459476678844418816862571810;  // 1 / (4 pi)
  // P_l and P_{l-1} of each entry, and their sums
  double p[kCovCols], pm[kCovCols], acc[kCovCols];
#pragma unroll
  for (int e = 0; e < kCovCols; ++e) {
    p[e] = 1.0;
    pm[e] = 0.0;
    acc[e] = 0.0;
  }
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
#pragma unroll
      for (int e = 0; e < kCovCols; ++e) {
        acc[e] = fma(wt, p[e], acc[e]);
        const double next = fma(at * x[e], p[e], -bt * pm[e]);
        pm[e] = p[e];
        p[e] = next;
      }
    }
  }
  if (i < n) {
#pragma unroll
    for (int e = 0; e < kCovCols; ++e) {
      const int64_t j = j0 + e * kCovTile;
      if (j < n) gamma[i * n + j] = acc[e];
    }
  }
}

}  // namespace

hipError_t launch_pixel_cov(const double* dirs, int64_t n, const double* cl, int lmax, double* gamma,
                            hipStream_t s) {
  const int64_t rows = (n + kCovTile - 1) / kCovTile;
  const int64_t cols = (n + kCovCols * kCovTile - 1) / (kCovCols * kCovTile);
  hipLaunchKernelGGL(k_pixel_cov, dim3((unsigned)cols, (unsigned)rows), dim3(kCovTile * kCovTile), 0, s, dirs, n, cl,
                     lmax, gamma);
  return hipGetLastError();
}

}  // namespace cmbx
