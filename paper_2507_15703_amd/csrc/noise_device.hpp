// Counter-based noise for the box modes: Philox4x32-10 and a fixed-operation FP64
// Box-Muller transform, bit-reproducible on any IEEE-754 machine.
//
// The 3-D Fourier method fills each box mode with a complex normal of variance P_box(|k|)
// (Sec. II D 1). Mode (ix, iy, iz) of the half grid is driven by Philox4x32-10 (Salmon et
// al., SC'11) with key = the seed's two 32-bit words and counter (iz >> 1, iy, ix, 0); the
// even iz of a pair takes output words (x0, x1), the odd one (x2, x3). The first word sets
// the Box-Muller radius, the second the angle.
//
// The Box-Muller transform is written with binary64 +, -, x only (contraction disabled so
// that no product is fused into an add), exact power-of-two scalings and integer bit
// operations, in a fixed order:
//   ln u1, u1 = (a + 1) 2^-32: a + 1 = m 2^e with m in [1/sqrt2, sqrt2); ln u1 =
//     (e - 32) ln2_head + ((e - 32) ln2_tail + 2 s P(s^2)), s = (m - 1)/(m + 1) with the
//     reciprocal from five Newton steps started at 1/2, P the artanh series to s^20;
//   sqrt x: four Newton steps for 1/sqrt(x) from the integer-shift seed, times x;
//   cos, sin of 2 pi b 2^-32: quadrant from the top two bits, the rest folded to
//     t in [0, pi/4] with sin/cos swapped when folded, Taylor series to t^17 / t^18.
// Single-precision plans use a binary32 variant of the same steps (below); double
// precision plans use the binary64 one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_device.hpp"

namespace cmbx {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c.x;
    const uint64_t p1 = (uint64_t)M1 * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    k0 += W0;
    k1 += W1;
  }
  return c;
}

namespace bm {
// binary64 constants (exact bit patterns)
constexpr double kLn2Head = 0x1.62e42fefa3000p-1;  // ln 2 with 12 low mantissa bits cleared
constexpr double kLn2Tail = 0x1.3de6af278ece6p-42; // ln 2 - head, rounded
constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;
constexpr double kTwoPi2m32 = 0x1.921fb54442d18p-30;  // 2 pi / 2^32, rounded
constexpr uint64_t kRsqrtMagic = 0x5FE6EB50C7B537A9ull;

constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }  // exact up to 18!
constexpr double sgn(int k) { return (k & 1) ? -1.0 : 1.0; }
// Series coefficients, evaluated at compile time (each the correctly rounded quotient).
// kSin[k] = (-1)^k / (2k+1)!, kCos[k] = (-1)^k / (2k)!, kAtanh[k] = 1 / (2k+1).
constexpr double kSin[9] = {1.0, sgn(1) / fact(3), sgn(2) / fact(5), sgn(3) / fact(7), sgn(4) / fact(9),
                            sgn(5) / fact(11), sgn(6) / fact(13), sgn(7) / fact(15), sgn(8) / fact(17)};
constexpr double kCos[10] = {1.0, sgn(1) / fact(2), sgn(2) / fact(4), sgn(3) / fact(6), sgn(4) / fact(8),
                             sgn(5) / fact(10), sgn(6) / fact(12), sgn(7) / fact(14), sgn(8) / fact(16),
                             sgn(9) / fact(18)};
constexpr double kAtanh[11] = {1.0, 1.0 / 3.0, 1.0 / 5.0, 1.0 / 7.0, 1.0 / 9.0, 1.0 / 11.0,
                               1.0 / 13.0, 1.0 / 15.0, 1.0 / 17.0, 1.0 / 19.0, 1.0 / 21.0};
}  // namespace bm

// (g_re, g_im) = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) by the fixed sequence above.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& g_re, double& g_im) {
#pragma clang fp contract(off)
  using namespace bm;
  // ---- ln u1
  const uint64_t v = (uint64_t)a + 1ull;
  const double vf = (double)v;                                   // exact
  const int e0 = 63 - __clzll((long long)v);                      // floor(log2 v)
  const double pw = __longlong_as_double((long long)((uint64_t)(1023 - e0) << 52));
  double m = vf * pw;                                             // [1, 2), exact
  const bool big = m >= kSqrt2;
  m = big ? m * 0.5 : m;
  const int e = (big ? e0 + 1 : e0) - 32;
  const double d = m + 1.0;
  double y = 0.5;
#pragma unroll
  for (int i = 0; i < 5; ++i) y = y * (2.0 - d * y);
  const double s = (m - 1.0) * y;
  const double s2 = s * s;
  double p = kAtanh[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) p = p * s2 + kAtanh[k];
  const double lnm = (s + s) * p;
  const double ef = (double)e;
  const double lnu = ef * kLn2Head + (ef * kLn2Tail + lnm);
  // ---- sqrt(-2 ln u1)
  const double x = -(lnu + lnu);
  double r = __longlong_as_double((long long)(kRsqrtMagic - ((uint64_t)__double_as_longlong(x) >> 1)));
  const double hx = 0.5 * x;
#pragma unroll
  for (int i = 0; i < 4; ++i) r = r * (1.5 - hx * (r * r));
  const double rad = (x == 0.0) ? 0.0 : x * r;
  // ---- sin, cos of 2 pi u2
  const uint32_t q = b >> 30;
  const uint32_t rr = b & 0x3FFFFFFFu;
  const bool swap = rr >= (1u << 29);
  const uint32_t rho = swap ? (1u << 30) - rr : rr;
  const double t = (double)rho * kTwoPi2m32;
  const double t2 = t * t;
  double ps = kSin[8];
#pragma unroll
  for (int k = 7; k >= 0; --k) ps = ps * t2 + kSin[k];
  const double st = t * ps;
  double pc = kCos[9];
#pragma unroll
  for (int k = 8; k >= 0; --k) pc = pc * t2 + kCos[k];
  const double ct = pc;
  const double si = swap ? ct : st;  // in-quadrant sine and cosine
  const double ci = swap ? st : ct;
  // quadrant q: (sin, cos) = (si, ci), (ci, -si), (-si, -ci), (-ci, si) for q = 0..3,
  // formed with selects and sign flips only (no divergent branches)
  const bool odd = (q & 1u) != 0u;
  double sn = odd ? ci : si;
  double cs = odd ? si : ci;
  sn = (q & 2u) ? -sn : sn;
  cs = ((q + 1u) & 2u) ? -cs : cs;
  g_re = rad * cs;
  g_im = rad * sn;
}

namespace bmf {
// binary32 constants
constexpr float kLn2Head = 0x1.62e4p-1f;     // ln 2 with a 16-bit significand
constexpr float kLn2Tail = 0x1.7f7d1cp-20f;  // ln 2 - head, rounded to binary32
constexpr float kSqrt2 = 0x1.6a09e6p+0f;
constexpr float kTwoPi2m32 = 0x1.921fb6p-30f;
constexpr uint32_t kRsqrtMagic = 0x5F3759DFu;
// the binary64 quotients rounded to binary32
constexpr float kSin[5] = {(float)bm::kSin[0], (float)bm::kSin[1], (float)bm::kSin[2], (float)bm::kSin[3],
                           (float)bm::kSin[4]};
constexpr float kCos[6] = {(float)bm::kCos[0], (float)bm::kCos[1], (float)bm::kCos[2],
                           (float)bm::kCos[3], (float)bm::kCos[4], (float)bm::kCos[5]};
constexpr float kAtanh[5] = {(float)bm::kAtanh[0], (float)bm::kAtanh[1], (float)bm::kAtanh[2],
                             (float)bm::kAtanh[3], (float)bm::kAtanh[4]};
}  // namespace bmf

// binary32 variant for single-precision plans: the same steps in binary32 with series
// sized to it. a + 1 is cut to its leading 24 bits (m = mi 2^-23, mi in [2^23, 2^24)),
// four Newton steps for 1/(m + 1), artanh series to s^8, three Newton steps for
// 1/sqrt(x), sine series to t^9 and cosine series to t^10.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& g_re, float& g_im) {
#pragma clang fp contract(off)
  using namespace bmf;
  const uint64_t v = (uint64_t)a + 1ull;
  const int e0 = 63 - __clzll((long long)v);
  const uint32_t mi = e0 >= 23 ? (uint32_t)(v >> (e0 - 23)) : (uint32_t)(v << (23 - e0));
  float m = (float)mi * 0x1p-23f;  // [1, 2), exact
  const bool big = m >= kSqrt2;
  m = big ? m * 0.5f : m;
  const int e = (big ? e0 + 1 : e0) - 32;
  const float d = m + 1.0f;
  float y = 0.5f;
#pragma unroll
  for (int i = 0; i < 4; ++i) y = y * (2.0f - d * y);
  const float s = (m - 1.0f) * y;
  const float s2 = s * s;
  float p = kAtanh[4];
#pragma unroll
  for (int k = 3; k >= 0; --k) p = p * s2 + kAtanh[k];
  const float lnm = (s + s) * p;
  const float ef = (float)e;
  const float lnu = ef * kLn2Head + (ef * kLn2Tail + lnm);
  const float x = -(lnu + lnu);
  float r = __uint_as_float(kRsqrtMagic - (__float_as_uint(x) >> 1));
  const float hx = 0.5f * x;
#pragma unroll
  for (int i = 0; i < 3; ++i) r = r * (1.5f - hx * (r * r));
  const float rad = (x == 0.0f) ? 0.0f : x * r;
  const uint32_t q = b >> 30;
  const uint32_t rr = b & 0x3FFFFFFFu;
  const bool swap = rr >= (1u << 29);
  const uint32_t rho = swap ? (1u << 30) - rr : rr;
  const float t = (float)rho * kTwoPi2m32;
  const float t2 = t * t;
  float ps = kSin[4];
#pragma unroll
  for (int k = 3; k >= 0; --k) ps = ps * t2 + kSin[k];
  const float st = t * ps;
  float pc = kCos[5];
#pragma unroll
  for (int k = 4; k >= 0; --k) pc = pc * t2 + kCos[k];
  const float ct = pc;
  const float si = swap ? ct : st;
  const float ci = swap ? st : ct;
  const bool odd = (q & 1u) != 0u;
  float sn = odd ? ci : si;
  float cs = odd ? si : ci;
  sn = (q & 2u) ? -sn : sn;
  cs = ((q + 1u) & 2u) ? -cs : cs;
  g_re = rad * cs;
  g_im = rad * sn;
}

// Words (a, b) of mode (ix, iy, iz).
__device__ __forceinline__ uint2 mode_words(uint32_t k0, uint32_t k1, int ix, int iy, int iz) {
  const uint4 w = philox4x32_10(make_uint4((uint32_t)iz >> 1, (uint32_t)iy, (uint32_t)ix, 0u), k0, k1);
  return (iz & 1) ? make_uint2(w.z, w.w) : make_uint2(w.x, w.y);
}

// A generic mode from its words: weight x (g_re, g_im), the pair from the transform of
// the working precision T and the product formed in T.
template <typename T>
__device__ __forceinline__ cpx<T> weighted(T w, uint32_t a, uint32_t b) {
  T gr, gi;
  box_muller(a, b, gr, gi);
  return {w * gr, w * gi};
}

__device__ __forceinline__ int freq2(int i, int N) {
  const int f = i <= N - i ? i : N - i;
  return f * f;
}

// Value of half-grid mode (ix, iy, iz), including the Hermitian rule on the planes
// iz = 0 and N/2: of a pair (f, -f) the one with the smaller ix N + iy is drawn and the
// other is its conjugate; the self-conjugate modes are real, full weight x g_re.
// wh: sqrt(P_box/2) per |f|^2; wself[c]: sqrt(P_box) at |f|^2 = c (N/2)^2.
template <typename T>
__device__ __forceinline__ cpx<T> mode_value(int N, int ix, int iy, int iz, uint32_t k0, uint32_t k1,
                                             const T* __restrict__ wh, const T* __restrict__ wself) {
  const int M = N / 2;
  const int m = freq2(ix, N) + freq2(iy, N) + iz * iz;
  int sx = ix, sy = iy;  // mode whose words are drawn
  bool cj = false, self = false;
  if (iz == 0 || iz == M) {
    const int px = ix == 0 ? 0 : N - ix;
    const int py = iy == 0 ? 0 : N - iy;
    const int own = ix * N + iy, par = px * N + py;
    if (own == par) {
      self = true;
    } else if (own > par) {
      sx = px;
      sy = py;
      cj = true;
    }
  }
  const uint2 w = mode_words(k0, k1, sx, sy, iz);
  T gr, gi;
  box_muller(w.x, w.y, gr, gi);
  if (self) {
    const int c = (ix == M) + (iy == M) + (iz == M);
    return {wself[c] * gr, T(0)};
  }
  const T wv = wh[m];
  const cpx<T> v = {wv * gr, wv * gi};
  return cj ? conj(v) : v;
}

}  // namespace cmbx
