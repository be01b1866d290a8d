// Pixel covariance of a sky map with angular power spectrum C_l (Sec. III B uses it to test
// the maps; eq. harmonics gives it for every pixel pair):
//
//   Gamma_ij = sum_{l=0}^{lmax} (2l + 1) C_l P_l(x_ij) / (4 pi),  x_ij = n_i . n_j in [-1, 1].
//
// One thread per entry, 16 x 16 entries per workgroup, all in FP64. P_l runs by the
// three-term recurrence P_{l+1} = a_l x P_l - b_l P_{l-1}, a_l = (2l + 1)/(l + 1),
// b_l = l/(l + 1); the per-l factors w_l = (2l + 1) C_l / (4 pi), a_l and b_l are staged in
// LDS a chunk at a time, so the loop is two multiply-adds and a multiply per l. The work is
// FP64 vector arithmetic: n^2 (lmax + 1) x 4 operations per launch.
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
  const int64_t j = (int64_t)blockIdx.x * kCovTile + threadIdx.x % kCovTile;
  const bool on = i < n && j < n;
  double x = 0.0;
  if (on) {
    x = dirs[3 * i] * dirs[3 * j] + dirs[3 * i + 1] * dirs[3 * j + 1] + dirs[3 * i + 2] * dirs[3 * j + 2];
    x = x > 1.0 ? 1.0 : (x < -1.0 ? -1.0 : x);
  }
  constexpr double inv4pi = 0.0795774715459476678844418816862571810;  // 1 / (4 pi)
  double p = 1.0, pm = 0.0, acc = 0.0;  // P_l and P_{l-1}
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
      acc = fma(w[t], p, acc);
      const double next = fma(a[t] * x, p, -b[t] * pm);
      pm = p;
      p = next;
    }
  }
  if (on) gamma[i * n + j] = acc;
}

}  // namespace

hipError_t launch_pixel_cov(const double* dirs, int64_t n, const double* cl, int lmax, double* gamma,
                            hipStream_t s) {
  const int64_t t = (n + kCovTile - 1) / kCovTile;
  hipLaunchKernelGGL(k_pixel_cov, dim3((unsigned)t, (unsigned)t), dim3(kCovTile * kCovTile), 0, s, dirs, n, cl,
                     lmax, gamma);
  return hipGetLastError();
}

}  // namespace cmbx
