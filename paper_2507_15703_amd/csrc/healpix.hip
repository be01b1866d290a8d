// HEALPix RING pixel centres of the cap centred on the pole (Sec. II D 1: the cap's sky
// pixels are the leading pixels of a RING-ordered HEALPix map). Pixelization of Gorski et
// al., ApJ 622 (2005) 759, Sec. 4: for n = Nside, 12 n^2 pixels on rings i = 1 .. 4n - 1
// from the north pole; polar rings (i < n) hold 4i pixels at z = 1 - i^2/(3n^2) and
// longitudes (j + 1/2) pi / (2i); equatorial rings (n <= i <= 3n) hold 4n pixels at
// z = 4/3 - 2i/(3n) and longitudes (j + s) pi / (2n), s = 1/2 for i + n even and 0 for
// odd; south rings mirror the north ones in z. RING order goes ring by ring, north to
// south, each in increasing longitude.
//
// Each ring's z is one correctly rounded quotient of exact integers, so the cap (every
// ring with z >= z_min) is decided the same way on the host and anywhere else.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"

namespace cmbx {
namespace {

// Largest i >= 1 with 2 i (i - 1) <= q: the polar ring of pixel q counted from its pole.
__host__ __device__ inline int64_t polar_ring(int64_t q) {
  int64_t i = (int64_t)((1.0 + sqrt(1.0 + 2.0 * (double)q)) * 0.5);
  if (i < 1) i = 1;
  while (i > 1 && 2 * i * (i - 1) > q) --i;
  while (2 * (i + 1) * i <= q) ++i;
  return i;
}

__host__ __device__ inline double polar_z(int64_t n, int64_t i) {
  return (double)(3 * n * n - i * i) / (double)(3 * n * n);
}

__host__ __device__ inline double belt_z(int64_t n, int64_t i) {
  return (double)(4 * n - 2 * i) / (double)(3 * n);
}

constexpr double kPi = 3.141592653589793238462643383279502884;

__global__ __launch_bounds__(256) void k_healpix_cap(double* __restrict__ dirs, int64_t n, int64_t count) {
  const int64_t npix = 12 * n * n, ncap = 2 * n * (n - 1);
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count;
       p += (int64_t)gridDim.x * blockDim.x) {
    double z, phi;
    if (p < ncap) {
      const int64_t i = polar_ring(p), j = p - 2 * i * (i - 1);
      z = polar_z(n, i);
      phi = ((double)j + 0.5) * (kPi / (double)(2 * i));
    } else if (p < npix - ncap) {
      const int64_t ip = p - ncap, i = ip / (4 * n) + n, j = ip % (4 * n);
      z = belt_z(n, i);
      phi = ((double)j + ((i + n) % 2 == 0 ? 0.5 : 0.0)) * (kPi / (double)(2 * n));
    } else {
      // the mirror pixel q sits in north ring i at j'; this one is in ring 4n - i, which
      // lists the same longitudes in the same increasing order
      const int64_t q = npix - 1 - p, i = polar_ring(q), jm = q - 2 * i * (i - 1);
      const int64_t j = 4 * i - 1 - jm;
      z = -polar_z(n, i);
      phi = ((double)j + 0.5) * (kPi / (double)(2 * i));
    }
    const double st = sqrt((1.0 - z) * (1.0 + z));
    double s, c;
    sincos(phi, &s, &c);
    dirs[3 * p + 0] = st * c;
    dirs[3 * p + 1] = st * s;
    dirs[3 * p + 2] = z;
  }
}

}  // namespace

int64_t healpix_cap_count(int64_t n, double z_min) {
  int64_t count = 0;
  for (int64_t i = 1; i <= 4 * n - 1; ++i) {
    double z;
    int64_t ring;
    if (i < n) {
      z = polar_z(n, i);
      ring = 4 * i;
    } else if (i <= 3 * n) {
      z = belt_z(n, i);
      ring = 4 * n;
    } else {
      z = -polar_z(n, 4 * n - i);
      ring = 4 * (4 * n - i);
    }
    if (!(z >= z_min)) break;  // rings run in decreasing z
    count += ring;
  }
  return count;
}

hipError_t launch_healpix_cap(int64_t n, int64_t count, double* dirs, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_healpix_cap, dim3((unsigned)blocks), dim3(256), 0, s, dirs, n, count);
  return hipGetLastError();
}

}  // namespace cmbx
