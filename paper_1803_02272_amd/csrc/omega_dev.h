// Device side of the Gaussian test matrix (shared by the G-pass operand
// kernel and the batched small-MDS kernel): Philox4x64-10 (Salmon et al.,
// SC'11) and the Box-Muller transform, see k_omega.hip.
#pragma once

#include "mds_internal.h"

namespace mds {
namespace omega {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t lo0 = kM0 * x[0], hi0 = __umul64hi(kM0, x[0]);
    const uint64_t lo1 = kM1 * x[2], hi1 = __umul64hi(kM1, x[2]);
    const uint64_t y0 = hi1 ^ x[1] ^ k0;
    const uint64_t y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
  }
}

// ln, sin and cos for Box-Muller written from the mathematics with + - * /
// and sqrt only, evaluated in a fixed order without contraction into fused
// multiply-adds, so that every value is the IEEE result of the same sequence
// of correctly rounded operations on any conforming implementation.
constexpr double kLn2Hi = 0x1.62e42ff000000p-1;   // ln 2 rounded to a 32-bit fraction (e * kLn2Hi exact)
constexpr double kLn2Lo = -0x1.718432a1b0e26p-35; // ln 2 - kLn2Hi, rounded
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
constexpr double kPi4 = 0x1.921fb54442d18p-1;     // pi / 4, rounded

// ln u for u in (0, 1]: u = m 2^e, m in [sqrt(1/2), sqrt(2)) (exact);
// ln m = 2 atanh(s), s = (m - 1) / (m + 1), odd series to s^21; ln u =
// e ln2_hi + (e ln2_lo + ln m).
__device__ __forceinline__ double ln_unit(double u) {
#pragma clang fp contract(off)
  constexpr double c[10] = {0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3,
                            0x1.c71c71c71c71cp-4, 0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4,
                            0x1.1111111111111p-4, 0x1.e1e1e1e1e1e1ep-5, 0x1.af286bca1af28p-5,
                            0x1.8618618618618p-5};  // 1 / (2j + 1), j = 1..10
  int ei = 0;
  double m = frexp(u, &ei);  // u = m 2^ei, m in [1/2, 1)
  if (m < kSqrtHalf) {
    m = m + m;
    ei -= 1;
  }
  const double e = (double)ei;
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = c[9];
#pragma unroll
  for (int j = 8; j >= 0; --j) p = p * z + c[j];
  const double t = s * (z * p);
  const double lnm = (s + t) * 2.0;
  return e * kLn2Hi + (e * kLn2Lo + lnm);
}

// (sin 2 pi v, cos 2 pi v) for v in [0, 1): exact octant reduction of the
// dyadic v, x = a pi/4 in [0, pi/4], Taylor series to x^17 (sine) and x^18
// (cosine), then the octant's symmetry (sign changes and swaps).
__device__ __forceinline__ void sincos_2pi(double v, double& sn, double& cs) {
#pragma clang fp contract(off)
  constexpr double cs_s[8] = {-0x1.5555555555555p-3, 0x1.1111111111111p-7, -0x1.a01a01a01a01ap-13,
                              0x1.71de3a556c734p-19, -0x1.ae64567f544e4p-26, 0x1.6124613a86d09p-33,
                              -0x1.ae7f3e733b81fp-41, 0x1.952c77030ad4ap-49};  // (-1)^j / (2j + 1)!
  constexpr double cs_c[9] = {-0x1.0000000000000p-1, 0x1.5555555555555p-5, -0x1.6c16c16c16c17p-10,
                              0x1.a01a01a01a01ap-16, -0x1.27e4fb7789f5cp-22, 0x1.1eed8eff8d898p-29,
                              -0x1.93974a8c07c9dp-37, 0x1.ae7f3e733b81fp-45,
                              -0x1.6827863b97d97p-53};  // (-1)^j / (2j)!
  const double t = v * 8.0;
  const double o = floor(t);
  const double f = t - o;
  const int oi = (int)o;
  const double a = (oi & 1) ? 1.0 - f : f;
  const double x = a * kPi4;
  const double z = x * x;
  double ps = cs_s[7];
#pragma unroll
  for (int j = 6; j >= 0; --j) ps = ps * z + cs_s[j];
  const double sx = x + (x * z) * ps;
  double pc = cs_c[8];
#pragma unroll
  for (int j = 7; j >= 0; --j) pc = pc * z + cs_c[j];
  const double cx = 1.0 + z * pc;
  const bool swap = oi == 1 || oi == 2 || oi == 5 || oi == 6;
  const double so = swap ? cx : sx, co = swap ? sx : cx;
  sn = oi >= 4 ? -so : so;
  cs = (oi >= 2 && oi <= 5) ? -co : co;
}

__device__ __forceinline__ void box_muller(uint64_t wa, uint64_t wb, double& z0, double& z1) {
#pragma clang fp contract(off)
  const double u = ((double)(wa >> 11) + 0.5) * 0x1p-53;
  const double v = (double)(wb >> 11) * 0x1p-53;
  const double rho = sqrt(-2.0 * ln_unit(u));
  double sn, cs;
  sincos_2pi(v, sn, cs);
  z0 = rho * cs;
  z1 = rho * sn;
}

template <typename T>
__device__ __forceinline__ T cvt(double v);
template <>
__device__ __forceinline__ double cvt<double>(double v) { return v; }
template <>
__device__ __forceinline__ float cvt<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ bf16_t cvt<bf16_t>(double v) {
  uint32_t u = __float_as_uint((float)v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

// Standard normals of Omega[i][4b .. 4b+3] (key (seed, 0), counter (i, b, 0, 0)).
__device__ __forceinline__ void omega_block(uint64_t seed, int64_t i, int64_t b, double z[4]) {
  uint64_t x[4] = {(uint64_t)i, (uint64_t)b, 0ull, 0ull};
  philox4x64_10(x, seed, 0ull);
  box_muller(x[0], x[1], z[0], z[1]);
  box_muller(x[2], x[3], z[2], z[3]);
}

}  // namespace omega
}  // namespace mds
