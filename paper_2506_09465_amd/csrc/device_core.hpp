// device_core.hpp -- per-lane arithmetic of the particle step on gfx950:
// counter-based sampling and the elementary functions it needs.
//
// Everything here is written so that its result is fixed bit for bit by IEEE
// binary64 round-to-nearest semantics of + - * / sqrt (the translation unit is
// built with -ffp-contract=off and without fast-math), which is what lets the
// integer tallies of the HIP path be compared bit for bit with a CPU run.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace iugkp {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32
// Philox S-box, multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments
// 0x9E3779B9 / 0xBB67AE85 between rounds.  32-bit multiplies map to
// v_mul_lo_u32 / v_mul_hi_u32.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
    const uint32_t lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Uniform double in [0,1) with 53 random bits: 27 high bits of `a`, 26 of `b`.
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b)
{
  const uint64_t m = (static_cast<uint64_t>(a >> 5) << 26) | static_cast<uint64_t>(b >> 6);
  return static_cast<double>(m) * 0x1p-53;
}

// Two uniforms of draw `d` for particle `k` of emitter `e` in slot `slot`:
// Philox counter (d, k, e, slot) under key (key0, key1).
__device__ __forceinline__ double2 draw2(uint32_t d, uint32_t k, uint32_t e, uint32_t slot,
                                         uint32_t key0, uint32_t key1)
{
  const uint4 o = philox4x32_10(make_uint4(d, k, e, slot), key0, key1);
  return make_double2(uniform53(o.x, o.y), uniform53(o.z, o.w));
}

// ---------------------------------------------------------------------------
// ln(x), x finite normal > 0, from + - * / only.  Decompose x = m 2^e with
// m in (sqrt2/2, sqrt2], f = m - 1 (exact), s = f/(2+f).  The atanh series
// gives ln m = 2 atanh s = 2s + s R with R = 2 sum_{k=1..10} z^k/(2k+1),
// z = s^2, and 2s = f - f s, hence ln m = f - s (f - R).  ln 2 is applied as a
// Cody-Waite pair (high part with zero low bits, so e * hi is exact).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double log_own(double x)
{
  const double kLn2Hi = 6.93147180369123816490e-01;
  const double kLn2Lo = 1.90821492927058770002e-10;
  const double kSqrt2 = 1.41421356237309504880;
  const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(x));
  int ex = static_cast<int>((bits >> 52) & 0x7ffu) - 1023;
  double m = __longlong_as_double(static_cast<long long>((bits & 0x000fffffffffffffull) |
                                                         (0x3ffull << 52)));
  if (m > kSqrt2) {
    m = m * 0.5;
    ex = ex + 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double R = 2.0 / 21.0;
  R = R * z + 2.0 / 19.0;
  R = R * z + 2.0 / 17.0;
  R = R * z + 2.0 / 15.0;
  R = R * z + 2.0 / 13.0;
  R = R * z + 2.0 / 11.0;
  R = R * z + 2.0 / 9.0;
  R = R * z + 2.0 / 7.0;
  R = R * z + 2.0 / 5.0;
  R = R * z + 2.0 / 3.0;
  R = R * z;
  const double corr = s * (f - R);
  const double de = static_cast<double>(ex);
  return de * kLn2Hi + ((de * kLn2Lo - corr) + f);
}

// ---------------------------------------------------------------------------
// cos(2 pi u) for u in [0,1).  t = 4u, quadrant q = floor(t), f = t - q (both
// exact), g = min(f, 1 - f) (exact), x = (pi/2) g in [0, pi/4]; Taylor series
// of cos x to x^18 and sin x to x^19 in Horner form in z = x^2; then the
// quadrant identities cos(q pi/2 + a) = cos a, -sin a, -cos a, sin a.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cos2pi_own(double u)
{
  const double kHalfPi = 1.57079632679489661923;
  const double t = 4.0 * u;
  const int q = static_cast<int>(t);
  const double f = t - static_cast<double>(q);
  const bool folded = f > 0.5;
  const double g = folded ? 1.0 - f : f;
  const double x = kHalfPi * g;
  const double z = x * x;
  double c = -1.0 / 6402373705728000.0;
  c = c * z + 1.0 / 20922789888000.0;
  c = c * z - 1.0 / 87178291200.0;
  c = c * z + 1.0 / 479001600.0;
  c = c * z - 1.0 / 3628800.0;
  c = c * z + 1.0 / 40320.0;
  c = c * z - 1.0 / 720.0;
  c = c * z + 1.0 / 24.0;
  c = c * z - 1.0 / 2.0;
  c = c * z + 1.0;
  double s = -1.0 / 121645100408832000.0;
  s = s * z + 1.0 / 355687428096000.0;
  s = s * z - 1.0 / 1307674368000.0;
  s = s * z + 1.0 / 6227020800.0;
  s = s * z - 1.0 / 39916800.0;
  s = s * z + 1.0 / 362880.0;
  s = s * z - 1.0 / 5040.0;
  s = s * z + 1.0 / 120.0;
  s = s * z - 1.0 / 6.0;
  s = s * z + 1.0;
  s = x * s;
  const double cf = folded ? s : c;   // cos(f pi / 2)
  const double sf = folded ? c : s;   // sin(f pi / 2)
  switch (q) {
    case 0: return cf;
    case 1: return -sf;
    case 2: return -cf;
    default: return sf;
  }
}

// ---------------------------------------------------------------------------
// exp(-T), T >= 0, from + - * / and exact scaling.  T = k ln2 + r with
// k = rint(T / ln2) and r = (T - k ln2_hi) - k ln2_lo (Cody-Waite pair, the
// high part with trailing zero bits), |r| <= ln2 / 2; exp(-r) by its Taylor
// polynomial to degree 14 in Horner form, times 2^-k.  0 for T > 700.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double expm_own(double T)
{
  const double kLn2Hi = 6.93147180369123816490e-01;
  const double kLn2Lo = 1.90821492927058770002e-10;
  const double kInvLn2 = 1.44269504088896338700e+00;
  if (T > 700.0) return 0.0;
  const double kd = rint(T * kInvLn2);
  const double r = (T - kd * kLn2Hi) - kd * kLn2Lo;
  const double x = -r;
  double p = 1.0 / 87178291200.0;
  p = p * x + 1.0 / 6227020800.0;
  p = p * x + 1.0 / 479001600.0;
  p = p * x + 1.0 / 39916800.0;
  p = p * x + 1.0 / 3628800.0;
  p = p * x + 1.0 / 362880.0;
  p = p * x + 1.0 / 40320.0;
  p = p * x + 1.0 / 5040.0;
  p = p * x + 1.0 / 720.0;
  p = p * x + 1.0 / 120.0;
  p = p * x + 1.0 / 24.0;
  p = p * x + 1.0 / 6.0;
  p = p * x + 0.5;
  p = p * x + 1.0;
  p = p * x + 1.0;
  return ldexp(p, -static_cast<int>(kd));
}

// Fixed-point conversion used for emission energies: rint(ldexp(v, F)).
__device__ __forceinline__ double fixed_scale(double v, int F) { return rint(ldexp(v, F)); }

}  // namespace iugkp
