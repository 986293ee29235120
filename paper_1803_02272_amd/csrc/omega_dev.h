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

__device__ __forceinline__ void box_muller(uint64_t wa, uint64_t wb, double& z0, double& z1) {
#pragma clang fp contract(off)
  const double u = ((double)(wa >> 11) + 0.5) * 0x1p-53;
  const double v = (double)(wb >> 11) * 0x1p-53;
  const double rho = sqrt(-2.0 * log(u));
  const double ang = 6.283185307179586 * v;  // fl(2 pi)
  z0 = rho * cos(ang);
  z1 = rho * sin(ang);
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
