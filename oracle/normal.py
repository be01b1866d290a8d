"""Canonical Box-Muller: two 32-bit words -> one pair of unit normals (test infrastructure only).

The paper asks only that each Fourier mode be a complex normal of the right variance
(Sec. II D 1). To make the CPU and GPU noise bit-identical, the transform is fixed here as
a sequence of IEEE-754 binary64 additions, subtractions and multiplications (each rounded
on its own, never fused), exact scalings by powers of two, and integer/bit operations. No
library log, sin, cos, sqrt or division is used, because those differ between platforms.

Given words a, b (uint32):

    u1 = (a + 1) 2^-32 in (0, 1],  u2 = b 2^-32 in [0, 1)
    R  = sqrt(-2 ln u1),  (g_re, g_im) = (R cos 2 pi u2, R sin 2 pi u2)

(Box & Muller, Ann. Math. Stat. 29 (1958) 610.) The three elementary functions are
evaluated as follows.

ln u1: write a + 1 = m 2^e with m in [1/sqrt2, sqrt2). Then ln u1 = (e - 32) ln 2 + ln m,
with ln 2 split into a short head (exact products) and a tail. ln m = 2 artanh(s),
s = (m - 1)/(m + 1), |s| <= 0.1716, summed as 2 s sum_{k=0..10} s^{2k}/(2k + 1) in Horner
form (truncation < 2.5e-17 relative). 1/(m + 1) comes from five Newton steps
y <- y (2 - d y) starting at y = 1/2.

sqrt x: Newton's iteration for 1/sqrt(x), y <- y (3/2 - (x/2) y^2), four steps from the
integer-shift seed 0x5FE6EB50C7B537A9 - (bits(x) >> 1) (relative error < 3.5 %), then
sqrt x = x y. x = 0 (a = 2^32 - 1) gives R = 0.

cos, sin of 2 pi u2: the top two bits of b give the quadrant; the remaining 30 bits are
folded to an angle t = rho (2 pi 2^-32) in [0, pi/4], rho <= 2^29 an integer, with sin and
cos swapped when folded. sin t = t sum_{k=0..8} (-1)^k t^{2k}/(2k+1)! and
cos t = sum_{k=0..9} (-1)^k t^{2k}/(2k)! (truncation < 1e-16).

Single-precision plans use their own binary32 sequence (the ``*_f32`` functions), built
for fewer operations: ln by a 128-entry table of ln(1 + j/128) and a cubic in the
remainder, sin and cos by a 256-entry table of sector mid-points and the angle-sum
formulas with a short series in the offset, sqrt as above with three Newton steps. Its
tables are binary64 values rounded once to binary32.
"""
import numpy as np

F64 = np.float64

LN2_HI = float.fromhex("0x1.62e42fefa3000p-1")   # ln 2 with the 12 low mantissa bits cleared
LN2_LO = float.fromhex("0x1.3de6af278ece6p-42")  # ln 2 - LN2_HI, rounded
SQRT2 = float.fromhex("0x1.6a09e667f3bcdp+0")
TWO_PI_2M32 = float.fromhex("0x1.921fb54442d18p-30")  # 2 pi / 2^32, rounded
RSQRT_MAGIC = np.uint64(0x5FE6EB50C7B537A9)

# Series coefficients; every factorial up to 18! is exact in binary64, so each is the
# correctly rounded quotient.
_ATANH_C = [1.0 / (2 * k + 1) for k in range(11)]
_SIN_C = [(-1.0) ** k / float(np.prod(np.arange(1, 2 * k + 2, dtype=np.float64))) for k in range(9)]
_COS_C = [(-1.0) ** k / float(np.prod(np.arange(1, 2 * k + 1, dtype=np.float64))) for k in range(10)]


def canonical_log_u1(a):
    """ln((a + 1) 2^-32) for uint32 words ``a`` (array), by the fixed operation sequence."""
    a = np.asarray(a, dtype=np.uint64)
    v = a + np.uint64(1)                                # 1 .. 2^32, exact
    vf = v.astype(F64)
    mant, ex = np.frexp(vf)                             # vf = mant 2^ex, mant in [1/2, 1), exact
    e0 = ex.astype(np.int64) - 1
    m = mant * 2.0                                      # [1, 2), exact
    big = m >= SQRT2
    m = np.where(big, m * 0.5, m)
    e = np.where(big, e0 + 1, e0) - 32                  # in [-32, 0]
    d = m + 1.0
    y = np.full_like(d, 0.5)
    for _ in range(5):
        y = y * (2.0 - d * y)
    s = (m - 1.0) * y
    s2 = s * s
    p = np.full_like(s, _ATANH_C[10])
    for k in range(9, -1, -1):
        p = p * s2 + _ATANH_C[k]
    lnm = (s + s) * p
    ef = e.astype(F64)
    return ef * LN2_HI + (ef * LN2_LO + lnm)


def canonical_sqrt(x):
    """sqrt(x) for x >= 0 (array) by the fixed Newton sequence; sqrt(0) = 0."""
    x = np.asarray(x, dtype=F64)
    bits = x.view(np.uint64)
    y = (RSQRT_MAGIC - (bits >> np.uint64(1))).view(F64)
    hx = 0.5 * x
    for _ in range(4):
        y = y * (1.5 - hx * (y * y))
    r = x * y
    return np.where(x == 0.0, 0.0, r)


def canonical_sincos_2pi(b):
    """(sin, cos) of 2 pi b 2^-32 for uint32 words ``b`` (array), fixed sequence."""
    b = np.asarray(b, dtype=np.uint64)
    q = b >> np.uint64(30)
    r = b & np.uint64(0x3FFFFFFF)
    swap = r >= np.uint64(1 << 29)
    rho = np.where(swap, np.uint64(1 << 30) - r, r)
    t = rho.astype(F64) * TWO_PI_2M32
    t2 = t * t
    ps = np.full_like(t, _SIN_C[8])
    for k in range(7, -1, -1):
        ps = ps * t2 + _SIN_C[k]
    st = t * ps
    pc = np.full_like(t, _COS_C[9])
    for k in range(8, -1, -1):
        pc = pc * t2 + _COS_C[k]
    ct = pc
    s_in = np.where(swap, ct, st)      # sine of the in-quadrant angle
    c_in = np.where(swap, st, ct)
    sin = np.select([q == 0, q == 1, q == 2], [s_in, c_in, -s_in], -c_in)
    cos = np.select([q == 0, q == 1, q == 2], [c_in, -s_in, -c_in], s_in)
    return sin, cos


def box_muller(a, b):
    """Unit normal pair (g_re, g_im) from word arrays a (radius) and b (angle)."""
    lnu = canonical_log_u1(a)
    x = -(lnu + lnu)
    rad = canonical_sqrt(x)
    sin, cos = canonical_sincos_2pi(b)
    return rad * cos, rad * sin


# ---------------------------------------------------------------------------------------
# Single-precision variant (the FP32 path's noise). Same structure, every operation an
# IEEE-754 binary32 add, subtract or multiply, shorter series sized to binary32:
#   ln u1: a + 1 = v (up to 2^32) is cut to its leading 24 bits, v = mi 2^(e - 23) with
#     mi in [2^23, 2^24), so m = mi 2^-23 in [1, 2) is exact in binary32 (relative change
#     of u1 below 2^-23); then as above with four Newton steps for 1/(m + 1) and the
#     artanh series to s^8; ln 2 split into a 16-bit head and a tail.
#   sqrt x: three Newton steps from 0x5F3759DF - (bits(x) >> 1).
#   sin t: series to t^9; cos t: series to t^10; t = rho (2 pi / 2^32), rho <= 2^29
#     rounded to binary32.
# Coefficients are the binary64 quotients rounded to binary32.
F32 = np.float32
LN2_HI_F = F32(float.fromhex("0x1.62e4p-1"))
LN2_LO_F = F32(float.fromhex("0x1.7f7d1cp-20"))
TWO_PI_2M32_F = F32(float.fromhex("0x1.921fb6p-30"))
RSQRT_MAGIC_F = np.uint32(0x5F3759DF)
THIRD_F = F32(1.0 / 3.0)
SIXTH_F = F32(1.0 / 6.0)
FOLD_J = 54   # table entries with c_j = 1 + j/128 >= sqrt 2 hold ln(c_j / 2)


def _tables_f32():
    """The binary32 tables of the single-precision sequence, each entry the binary64 value
    of its definition rounded once to binary32:
      LN[j]  = ln(c_j), or ln(c_j / 2) for j >= 54, with c_j = 1 + j/128 (j = 0..127);
      INV[j] = 1 / c_j;
      SIN[k], COS[k] = sin, cos of (k + 1/2) 2 pi / 256 (k = 0..255)."""
    c = 1.0 + np.arange(128, dtype=np.float64) / 128.0
    ln = np.where(np.arange(128) >= FOLD_J, np.log(c / 2.0), np.log(c))
    ang = (np.arange(256, dtype=np.float64) + 0.5) * (2.0 * np.pi / 256.0)
    return ln.astype(F32), (1.0 / c).astype(F32), np.sin(ang).astype(F32), np.cos(ang).astype(F32)


LN_TAB_F, INV_TAB_F, SIN_TAB_F, COS_TAB_F = _tables_f32()


def canonical_log_u1_f32(a):
    """ln((a + 1) 2^-32) in binary32 by the table sequence: a + 1 = mi 2^(e0 - 23) with
    mi the leading 24 bits, m = mi 2^-23 in [1, 2), j = the 7 bits of mi after its leading
    one, c_j = 1 + j/128 (exact), r = (m - c_j) INV[j] (the subtraction is exact),
    ln(1 + r) ~ r (1 + r (r/3 - 1/2)) (|r| < 2^-7, truncation < 1e-9), and
    ln u1 = e ln 2 + (LN[j] + ln(1 + r)) with e = e0 - 32, plus one for j >= 54."""
    a = np.asarray(a, dtype=np.uint64)
    v = a + np.uint64(1)                                 # 1 .. 2^32
    _, ex = np.frexp(v.astype(np.float64))               # exact exponent: v in [2^(ex-1), 2^ex)
    e0 = ex.astype(np.int64) - 1
    sh = e0 - 23
    mi = np.where(sh >= 0, v >> np.maximum(sh, 0).astype(np.uint64),
                  v << np.maximum(-sh, 0).astype(np.uint64))       # [2^23, 2^24)
    j = ((mi >> np.uint64(16)) & np.uint64(127)).astype(np.int64)
    m = mi.astype(F32) * F32(2.0**-23)                   # [1, 2), exact
    c = (j + 128).astype(F32) * F32(2.0**-7)             # exact
    r = (m - c) * INV_TAB_F[j]
    q = r * THIRD_F - F32(0.5)
    lp = r * (q * r + F32(1.0))
    lnm = LN_TAB_F[j] + lp
    e = e0 - 32 + (j >= FOLD_J)
    ef = e.astype(F32)
    return ef * LN2_HI_F + (ef * LN2_LO_F + lnm)


def canonical_sqrt_f32(x):
    """sqrt(x) for x >= 0 by three Newton steps for 1/sqrt from the integer-shift seed;
    x <= 0 gives 0."""
    x = np.asarray(x, dtype=F32)
    bits = np.maximum(x, F32(0.0)).view(np.uint32)
    y = (RSQRT_MAGIC_F - (bits >> np.uint32(1))).view(F32)
    hx = F32(0.5) * x
    for _ in range(3):
        y = y * (F32(1.5) - hx * (y * y))
    r = x * y
    return np.where(x <= F32(0.0), F32(0.0), r).astype(F32)


def canonical_sincos_2pi_f32(b):
    """sin, cos of 2 pi b 2^-32 in binary32 by the table sequence: k = the top 8 bits of b,
    d = (low 24 bits - 2^23) 2 pi 2^-32 (|d| <= pi/256; the integer is exact in binary32),
    sin d ~ d - d (d^2 / 6), cos d ~ 1 - d^2 / 2 (truncation < 1e-9), and the sum formulas
    sin = SIN[k] cos d + COS[k] sin d, cos = COS[k] cos d - SIN[k] sin d."""
    b = np.asarray(b, dtype=np.uint64)
    k = (b >> np.uint64(24)).astype(np.int64)
    low = (b & np.uint64(0xFFFFFF)).astype(np.int64) - (1 << 23)
    d = low.astype(F32) * TWO_PI_2M32_F
    d2 = d * d
    sd = d - d * (d2 * SIXTH_F)
    cd = F32(1.0) - d2 * F32(0.5)
    S, C = SIN_TAB_F[k], COS_TAB_F[k]
    sin = S * cd + C * sd
    cos = C * cd - S * sd
    return sin.astype(F32), cos.astype(F32)


def box_muller_f32(a, b):
    """Unit normal pair (g_re, g_im), binary32, from word arrays a and b."""
    lnu = canonical_log_u1_f32(a)
    x = -(lnu + lnu)
    rad = canonical_sqrt_f32(x)
    sin, cos = canonical_sincos_2pi_f32(b)
    return rad * cos, rad * sin
