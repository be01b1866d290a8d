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
//   sqrt x: four Newton steps for 1/sqrt(x) from the integer-shift seed (the binary64
//     magic constant of Lomont, "Fast inverse square root", 2003), times x;
//   cos, sin of 2 pi b 2^-32: quadrant from the top two bits, the rest folded to
//     t in [0, pi/4] with sin/cos swapped when folded, Taylor series to t^17 / t^18.
// Single-precision plans use their own binary32 sequence with small tables (below);
// double precision plans use the binary64 one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_device.hpp"

namespace cmbx {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  // each round: two 32 x 32 -> 64-bit products and two three-input XORs (v_bitop3_b32 with
  // truth table 0x96, a ^ b ^ c, one instruction each)
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c.x;
    const uint64_t p1 = (uint64_t)M1 * c.z;
    c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96), (uint32_t)p1,
                   __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96), (uint32_t)p0);
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
constexpr uint64_t kRsqrtMagic = 0x5FE6EB50C7B537A9ull;  // Lomont (2003), binary64 seed of 1/sqrt

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
constexpr float kTwoPi2m32 = 0x1.921fb6p-30f;
constexpr float kThird = 0x1.555556p-2f;     // 1/3 rounded to binary32
constexpr float kSixth = 0x1.555556p-3f;     // 1/6 rounded to binary32
constexpr uint32_t kRsqrtMagic = 0x5F3759DFu;  // the binary32 fast-inverse-square-root seed (Lomont 2003)
constexpr uint32_t kFoldJ = 54;              // entries with c_j = 1 + j/128 >= sqrt 2 hold ln(c_j / 2)
// table layout (binary32): ln c_j (or ln(c_j / 2)) and 1 / c_j for j = 0..127, then
// sin and cos of (k + 1/2) 2 pi / 256 for k = 0..255. The device copy holds the
// reciprocals times 2^-23 (exact), see box_muller_f32.
constexpr int kTabLn = 0, kTabInv = 128, kTabSin = 256, kTabCos = 512, kTabSize = 768;
}  // namespace bmf

// binary32 sequence for single-precision plans (tab: the table above, in LDS or global):
//   ln u1: a + 1 = mi 2^(e0 - 23), mi its leading 24 bits; m = mi 2^-23 in [1, 2);
//     j = the 7 bits after mi's leading one, c_j = 1 + j/128 (exact), r = (m - c_j) / c_j
//     by the table reciprocal (m - c_j is exact), ln(1 + r) ~ r (1 + r (r/3 - 1/2));
//     ln u1 = e ln2_head + (e ln2_tail + (ln c_j + ln(1 + r))), e = e0 - 32 (+1 when the
//     entry holds ln(c_j / 2));
//   sqrt x: three Newton steps for 1/sqrt(x) from the integer-shift seed, times x; x <= 0
//     gives 0;
//   sin, cos of 2 pi b 2^-32: k = b >> 24, d = ((b & 0xFFFFFF) - 2^23) 2 pi 2^-32,
//     sin d ~ d - d (d^2/6), cos d ~ 1 - d^2/2, then the angle-sum formulas with the
//     tabulated sin and cos of the sector mid-point.
__device__ __forceinline__ void box_muller_f32(uint32_t a, uint32_t b, float& g_re, float& g_im,
                                               const float* __restrict__ tab) {
#pragma clang fp contract(off)
  using namespace bmf;
  // a + 1 in 32 bits wraps to 0 only for a = 2^32 - 1, where a + 1 = 2^32: mi = 2^23, e0 = 32
  const uint32_t v = a + 1u;
  const bool wrap = v == 0u;
  const int lz = __clz((int)v);
  const uint32_t mi = wrap ? (1u << 23) : ((v << (lz & 31)) >> 8);  // leading 24 bits, truncated
  const int e0 = wrap ? 32 : 31 - lz;
  const uint32_t j = (mi >> 16) & 127u;
  // m - c_j = (mi mod 2^16) 2^-23 exactly (c_j = 1 + j/128 is m's leading 8 bits), and the
  // device table holds 2^-23 / c_j: the product is the binary32 number (m - c_j) (1 / c_j)
  // rounded once, scaled exactly by a power of two on one side instead of the other
  const float r = (float)(mi & 0xFFFFu) * tab[kTabInv + j];
  const float q = r * kThird - 0.5f;
  const float lp = r * (q * r + 1.0f);
  const float lnm = tab[kTabLn + j] + lp;
  const int e = e0 - 32 + (j >= kFoldJ ? 1 : 0);
  const float ef = (float)e;
  const float lnu = ef * kLn2Head + (ef * kLn2Tail + lnm);
  const float x = -(lnu + lnu);
  float y = __uint_as_float(kRsqrtMagic - (__float_as_uint(x) >> 1));
  const float hx = 0.5f * x;
#pragma unroll
  for (int i = 0; i < 3; ++i) y = y * (1.5f - hx * (y * y));
  const float rad = (x <= 0.0f) ? 0.0f : x * y;
  const uint32_t k = b >> 24;
  const int low = (int)(b & 0xFFFFFFu) - (1 << 23);
  const float d = (float)low * kTwoPi2m32;         // (float)low is exact
  const float d2 = d * d;
  const float sd = d - d * (d2 * kSixth);
  const float cd = 1.0f - d2 * 0.5f;
  const float S = tab[kTabSin + k], C = tab[kTabCos + k];
  const float sn = S * cd + C * sd;
  const float cs = C * cd - S * sd;
  g_re = rad * cs;
  g_im = rad * sn;
}

// the pair of the plan precision (the binary64 sequence needs no table)
__device__ __forceinline__ void normal_pair(uint32_t a, uint32_t b, double& g_re, double& g_im, const float*) {
  box_muller(a, b, g_re, g_im);
}
__device__ __forceinline__ void normal_pair(uint32_t a, uint32_t b, float& g_re, float& g_im,
                                            const float* __restrict__ tab) {
  box_muller_f32(a, b, g_re, g_im, tab);
}

// Words (a, b) of mode (ix, iy, iz).
__device__ __forceinline__ uint2 mode_words(uint32_t k0, uint32_t k1, int ix, int iy, int iz) {
  const uint4 w = philox4x32_10(make_uint4((uint32_t)iz >> 1, (uint32_t)iy, (uint32_t)ix, 0u), k0, k1);
  return (iz & 1) ? make_uint2(w.z, w.w) : make_uint2(w.x, w.y);
}

// A generic mode from its words: weight x (g_re, g_im), the pair from the transform of
// the working precision T and the product formed in T.
// A mode of zero weight (P_box = 0) is exactly +0 whatever its normal pair.
template <typename T>
__device__ __forceinline__ cpx<T> weighted(T w, uint32_t a, uint32_t b, const float* __restrict__ tab) {
  T gr, gi;
  normal_pair(a, b, gr, gi, tab);  // drawn either way: the pair does not wait for the weight
  const bool zero = w == T(0);
  return {zero ? T(0) : w * gr, zero ? T(0) : w * gi};
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
                                             const T* __restrict__ wh, const T* __restrict__ wself,
                                             const float* __restrict__ tab) {
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
  const T wv = self ? wself[(ix == M) + (iy == M) + (iz == M)] : wh[m];
  if (wv == T(0)) {  // zero weight: +0, conjugated like any other value
    const cpx<T> z = {T(0), T(0)};
    return cj ? conj(z) : z;
  }
  const uint2 w = mode_words(k0, k1, sx, sy, iz);
  T gr, gi;
  normal_pair(w.x, w.y, gr, gi, tab);
  if (self) return {wv * gr, T(0)};
  const cpx<T> v = {wv * gr, wv * gi};
  return cj ? conj(v) : v;
}

}  // namespace cmbx
