// Gaussian test matrix Omega (n x l) for the randomized range finder
// (Sec. 3.2, after Halko, Martinsson and Tropp 2011).
//
// Entry (i, j) is a function of (seed, i, j) only: the Philox4x64-10 block
// (Salmon et al., SC'11) at counter (i, j/4, 0, 0) with key (seed, 0) gives
// four 64-bit words; Box-Muller turns (w0, w1) and (w2, w3) into two pairs
// of standard normals, and column 4b + t takes the t-th of them.  The matrix
// is written transposed (l_pad x ldg) in the pass dtype, zero outside l x n;
// for the split fp32 passes, fl32(Omega) as its exact three-term bf16 split
// (per row and 32 consecutive columns: the 32 x0, then x1, then x2 terms).
#include "mds_internal.h"
#include "omega_dev.h"

namespace mds {
namespace {

using namespace omega;

template <typename T>
__global__ __launch_bounds__(256) void k_omega(uint64_t seed, int64_t n, int l, int64_t ldg,
                                               T* __restrict__ Xt) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;  // columns 4b .. 4b+3 (all < l_pad)
  if (i >= ldg) return;
  double z[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n && 4 * b < l) omega_block(seed, i, b, z);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = 4 * b + t;
    Xt[(int64_t)j * ldg + i] = cvt<T>(j < l ? z[t] : 0.0);
  }
}

// Split layout: thread (i, b) writes x_p of entries (4b + t, i), t < 4.
__global__ __launch_bounds__(256) void k_omega_split(uint64_t seed, int64_t n, int l, int64_t ldg,
                                                     uint16_t* __restrict__ X3) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= ldg) return;
  double z[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n && 4 * b < l) omega_block(seed, i, b, z);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = 4 * b + t;
    const float x = j < l ? (float)z[t] : 0.0f;
    const __bf16 v0 = (__bf16)x;
    const float r1 = x - (float)v0;
    const __bf16 v1 = (__bf16)r1;
    const float r2 = r1 - (float)v1;
    const __bf16 v2 = (__bf16)r2;
    uint16_t* dst = X3 + (int64_t)j * (3 * ldg) + (i / 32) * 96 + (i % 32);
    dst[0] = __builtin_bit_cast(uint16_t, v0);
    dst[32] = __builtin_bit_cast(uint16_t, v1);
    dst[64] = __builtin_bit_cast(uint16_t, v2);
  }
}

// Raw generator blocks: in[6 i .. 6 i + 5] = counter words 0..3, key words
// 0..1; out[4 i .. 4 i + 3] = the block.
__global__ __launch_bounds__(256) void k_philox(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  uint64_t x[4] = {in[6 * i], in[6 * i + 1], in[6 * i + 2], in[6 * i + 3]};
  philox4x64_10(x, in[6 * i + 4], in[6 * i + 5]);
#pragma unroll
  for (int t = 0; t < 4; ++t) out[4 * i + t] = x[t];
}

}  // namespace

hipError_t launch_philox(const uint64_t* in, uint64_t* out, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_philox, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, in, out, count);
  return hipGetLastError();
}

hipError_t launch_omega(uint64_t seed, int64_t n, int l, int l_pad, int64_t ldg, int xk, void* Xt,
                        hipStream_t s) {
  dim3 grid((unsigned)((ldg + 255) / 256), (unsigned)(l_pad / 4));
  switch (xk) {
    case GK_F64:
      hipLaunchKernelGGL(k_omega<double>, grid, dim3(256), 0, s, seed, n, l, ldg, (double*)Xt);
      break;
    case GK_F32:
      hipLaunchKernelGGL(k_omega<float>, grid, dim3(256), 0, s, seed, n, l, ldg, (float*)Xt);
      break;
    case GK_BF16:
      hipLaunchKernelGGL(k_omega<bf16_t>, grid, dim3(256), 0, s, seed, n, l, ldg, (bf16_t*)Xt);
      break;
    case GK_F32S:
      if (ldg % 32 != 0) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_omega_split, grid, dim3(256), 0, s, seed, n, l, ldg, (uint16_t*)Xt);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mds
