// GPU generators of synthetic distance matrices (input generation only; no
// step of the MDS method).  Exported with a C ABI for the Python wrapper in
// workloads/gpu.py.
//
//   gen_hamming_f32: D[i][j] = table[mismatches(i, j)], reads given as one
//     bit-plane per base (planes[i][b][w], 64 sites per word); mismatches =
//     L - sum_b popcount(P_i[b] & P_j[b]).  The table holds count / L as the
//     float32 rounding of the float64 quotient, so the result matches the
//     numpy recipe bit for bit.
//   gen_euclid_f32/f64: D[i][j] = sqrt(sum_k (x_ik - x_jk)^2) in float64,
//     summed over k in increasing order, then rounded to the output type.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kTile = 64;
constexpr int kMaxWords = 8;  // up to 512 sites per read

template <int WORDS>
__global__ __launch_bounds__(256) void k_hamming(const uint64_t* __restrict__ planes, int64_t n,
                                                 const float* __restrict__ table, float* __restrict__ D) {
  __shared__ uint64_t pi[kTile][4 * WORDS];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * kTile, j0 = (int64_t)blockIdx.x * kTile;
  for (int e = tid; e < kTile * 4 * WORDS; e += 256) {
    const int r = e / (4 * WORDS), w = e % (4 * WORDS);
    pi[r][w] = (i0 + r < n) ? planes[(i0 + r) * 4 * WORDS + w] : 0ull;
  }
  const int jl = tid & 63;
  const int64_t j = j0 + jl;
  uint64_t pj[4 * WORDS];
#pragma unroll
  for (int w = 0; w < 4 * WORDS; ++w) pj[w] = (j < n) ? planes[j * 4 * WORDS + w] : 0ull;
  __syncthreads();
  const int ig = tid >> 6;
#pragma unroll 4
  for (int r = ig * 16; r < ig * 16 + 16; ++r) {
    const int64_t i = i0 + r;
    if (i >= n || j >= n) continue;
    int match = 0;
#pragma unroll
    for (int w = 0; w < 4 * WORDS; ++w) match += __popcll(pi[r][w] & pj[w]);
    D[i * n + j] = table[match];
  }
}

constexpr int kEuRows = 16;

template <typename OT>
__global__ __launch_bounds__(256) void k_euclid(const double* __restrict__ X, int64_t n, int dim,
                                                OT* __restrict__ D) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const double* xj = X + j * dim;
  for (int r = 0; r < kEuRows; ++r) {
    const int64_t i = (int64_t)blockIdx.y * kEuRows + r;
    if (i >= n) return;
    const double* xi = X + i * dim;
    double acc = 0.0;
    for (int k = 0; k < dim; ++k) {
      const double d = xi[k] - xj[k];
      acc = acc + d * d;
    }
    D[i * n + j] = (OT)sqrt(acc);
  }
}

}  // namespace

extern "C" int gen_hamming_f32(const uint64_t* planes, int64_t n, int words, int length, const float* table,
                               float* D, void* stream) {
  (void)length;
  if (n <= 0 || n > 1000000 || words < 1 || words > kMaxWords) return -1;
  dim3 grid((unsigned)((n + kTile - 1) / kTile), (unsigned)((n + kTile - 1) / kTile));
  hipStream_t s = (hipStream_t)stream;
  switch (words) {
#define GEN_W(W) \
  case W: hipLaunchKernelGGL(k_hamming<W>, grid, dim3(256), 0, s, planes, n, table, D); break;
    GEN_W(1) GEN_W(2) GEN_W(3) GEN_W(4) GEN_W(5) GEN_W(6) GEN_W(7) GEN_W(8)
#undef GEN_W
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

extern "C" int gen_euclid(const double* X, int64_t n, int dim, int out_f64, void* D, void* stream) {
  if (n <= 0 || dim < 1 || n > 1000000) return -1;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)((n + kEuRows - 1) / kEuRows));
  hipStream_t s = (hipStream_t)stream;
  if (out_f64)
    hipLaunchKernelGGL(k_euclid<double>, grid, dim3(256), 0, s, X, n, dim, (double*)D);
  else
    hipLaunchKernelGGL(k_euclid<float>, grid, dim3(256), 0, s, X, n, dim, (float*)D);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
