// Double centring of the squared distance matrix (Sec. 6.2, step 1):
//   gamma_ij = -1/2 (d_ij^2 - c_j - r_i + m),
//   r_i = (1/n) sum_j d_ij^2,  c_j = (1/n) sum_i d_ij^2,  m = (1/n^2) sum_ij d_ij^2.
//
// Two HBM-streaming passes over D:
//   stats: one read of D; per 1024 x 1024 tile, each wave owns 256 rows and
//          every lane 16 columns; row partials come from a 64-lane butterfly,
//          column partials from registers and a fixed-order LDS merge of the
//          four waves.  Partials are combined in a fixed order afterwards, so
//          results are bitwise reproducible (no floating-point atomics).
//   write: one read of D and one write of G in the pass dtype (plus an fp32
//          copy for the refinement pass when requested), with ||G||_F^2 and
//          tr(G) partials.  Squares are formed in fp64 (exact for fp32 input)
//          and the equation is evaluated in fp64 in the order written above.
#include "mds_internal.h"

namespace mds {
namespace {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Four consecutive elements of a row starting at column c (c % 4 == 0),
// zero beyond n.  `vec` says the row start is 16-byte aligned.
template <typename DT>
__device__ __forceinline__ void load4(const DT* __restrict__ row, int64_t c, int64_t n, bool vec,
                                      double v[4]) {
  if (vec && c + 3 < n) {
    if constexpr (sizeof(DT) == 4) {
      const float4 f = *reinterpret_cast<const float4*>(row + c);
      v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
    } else {
      const double2 a = *reinterpret_cast<const double2*>(row + c);
      const double2 b = *reinterpret_cast<const double2*>(row + c + 2);
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = (c + t < n) ? (double)row[c + t] : 0.0;
  }
}

template <typename DT>
__device__ __forceinline__ bool row_vec_ok(bool base_ok, int64_t i, int64_t n) {
  return base_ok && (((i * n) % (int64_t)(16 / sizeof(DT))) == 0);
}

constexpr int kWaves = 4;
constexpr int kRowsPerWave = kStatsRows / kWaves;  // 256
constexpr int kRowBatch = 4;

template <typename DT>
__global__ __launch_bounds__(256) void k_stats(const DT* __restrict__ D, int64_t n, int base_vec,
                                               double* __restrict__ rowpart, double* __restrict__ colpart) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t cb = blockIdx.x, rb = blockIdx.y;
  const int64_t c0 = cb * kStatsCols;
  const int64_t r0 = rb * kStatsRows + (int64_t)wave * kRowsPerWave;
  const int64_t r1 = (r0 + kRowsPerWave < n) ? r0 + kRowsPerWave : n;
  double cacc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) cacc[t] = 0.0;

  for (int64_t i = r0; i < r1; i += kRowBatch) {
    double v[kRowBatch][16];
#pragma unroll
    for (int rr = 0; rr < kRowBatch; ++rr) {
      const int64_t ii = i + rr;
      if (ii < r1) {
        const DT* row = D + ii * n;
        const bool vec = row_vec_ok<DT>(base_vec != 0, ii, n);
#pragma unroll
        for (int g = 0; g < 4; ++g) load4<DT>(row, c0 + g * 256 + lane * 4, n, vec, &v[rr][g * 4]);
      } else {
#pragma unroll
        for (int t = 0; t < 16; ++t) v[rr][t] = 0.0;
      }
    }
#pragma unroll
    for (int rr = 0; rr < kRowBatch; ++rr) {
      double rs = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const double s = v[rr][t] * v[rr][t];
        cacc[t] += s;
        rs += s;
      }
      rs = wave_sum(rs);
      const int64_t ii = i + rr;
      if (lane == 0 && ii < r1) rowpart[cb * n + ii] = rs;
    }
  }
  __shared__ double sh[kWaves][kStatsCols];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int t = 0; t < 4; ++t) sh[wave][g * 256 + lane * 4 + t] = cacc[g * 4 + t];
  __syncthreads();
  for (int cc = threadIdx.x; cc < kStatsCols; cc += 256) {
    const int64_t c = c0 + cc;
    if (c < n) colpart[rb * n + c] = ((sh[0][cc] + sh[1][cc]) + sh[2][cc]) + sh[3][cc];
  }
}

__global__ __launch_bounds__(256) void k_stats_reduce(const double* __restrict__ rowpart,
                                                      const double* __restrict__ colpart, int64_t ncb,
                                                      int64_t nrb, int64_t n, double* __restrict__ r,
                                                      double* __restrict__ c, double* __restrict__ rsum) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t b = 0; b < ncb; ++b) s += rowpart[b * n + i];
  double t = 0.0;
  for (int64_t b = 0; b < nrb; ++b) t += colpart[b * n + i];
  rsum[i] = s;
  r[i] = s / (double)n;
  c[i] = t / (double)n;
}

__global__ __launch_bounds__(1024) void k_grand(const double* __restrict__ rsum, int64_t n,
                                                double* __restrict__ mean_all, DevStatus* st) {
#pragma clang fp contract(off)
  __shared__ double sh[1024];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s += rsum[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double S = sh[0];
    mean_all[0] = S / ((double)n * (double)n);
    st->sum_sq = S;
    if (!__builtin_isfinite(S)) st->nonfinite = 1;
  }
}

// ---- G store helpers ---------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename GT>
__device__ __forceinline__ void store4(GT* __restrict__ p, const double g[4]);

template <>
__device__ __forceinline__ void store4<double>(double* __restrict__ p, const double g[4]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(g[0], g[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(g[2], g[3]);
}
template <>
__device__ __forceinline__ void store4<float>(float* __restrict__ p, const double g[4]) {
  *reinterpret_cast<float4*>(p) = make_float4((float)g[0], (float)g[1], (float)g[2], (float)g[3]);
}
template <>
__device__ __forceinline__ void store4<bf16_t>(bf16_t* __restrict__ p, const double g[4]) {
  // fp64 -> fp32 (RNE) -> bf16 (RNE)
  const uint32_t a = f32_to_bf16_rne((float)g[0]) | ((uint32_t)f32_to_bf16_rne((float)g[1]) << 16);
  const uint32_t b = f32_to_bf16_rne((float)g[2]) | ((uint32_t)f32_to_bf16_rne((float)g[3]) << 16);
  *reinterpret_cast<uint2*>(p) = make_uint2(a, b);
}

constexpr int kWriteRows = 32;
constexpr int kWriteCols = 1024;

template <typename DT, typename GT, bool REF>
__global__ __launch_bounds__(256) void k_center_write(const DT* __restrict__ D, int64_t n, int64_t ldg,
                                                      int base_vec, const double* __restrict__ r,
                                                      const double* __restrict__ c,
                                                      const double* __restrict__ mean_all,
                                                      GT* __restrict__ G, float* __restrict__ gref,
                                                      double* __restrict__ fpart) {
#pragma clang fp contract(off)
  const int64_t j0 = (int64_t)blockIdx.x * kWriteCols + threadIdx.x * 4;
  const bool active = j0 < ldg;
  double cj[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) cj[t] = (j0 + t < n) ? c[j0 + t] : 0.0;
  const double m = mean_all[0];
  double fro = 0.0, tr = 0.0;
  for (int rr = 0; rr < kWriteRows; ++rr) {
    const int64_t i = (int64_t)blockIdx.y * kWriteRows + rr;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < n && active) {
      const double ri = r[i];
      double d[4];
      load4<DT>(D + i * n, j0, n, row_vec_ok<DT>(base_vec != 0, i, n), d);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        g[t] = (j0 + t < n) ? -0.5 * (((d[t] * d[t] - cj[t]) - ri) + m) : 0.0;
    }
    if (active) {
      store4<GT>(G + i * ldg + j0, g);
      if constexpr (REF) store4<float>(gref + i * ldg + j0, g);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        fro += g[t] * g[t];
        if (i == j0 + t) tr += g[t];
      }
    }
  }
  fro = wave_sum(fro);
  tr = wave_sum(tr);
  __shared__ double sh[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sh[0][wave] = fro; sh[1][wave] = tr; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t bid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    fpart[2 * bid] = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
    fpart[2 * bid + 1] = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
  }
}

__global__ __launch_bounds__(1024) void k_finalize_stats(const double* __restrict__ fpart, int64_t nparts,
                                                         DevStatus* st) {
#pragma clang fp contract(off)
  __shared__ double sa[1024], sb[1024];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += 1024) {
    a += fpart[2 * i];
    b += fpart[2 * i + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->frob2 = sa[0];
    st->trace = sb[0];
  }
}

template <typename DT, typename GT>
hipError_t write_dispatch(const DT* D, int64_t n, int64_t n_pad, int64_t ldg, int vec, const double* r,
                          const double* c, const double* mean_all, GT* G, float* gref, double* fpart,
                          hipStream_t s) {
  dim3 grid((unsigned)((ldg + kWriteCols - 1) / kWriteCols), (unsigned)(n_pad / kWriteRows));
  if (gref)
    hipLaunchKernelGGL((k_center_write<DT, GT, true>), grid, dim3(256), 0, s, D, n, ldg, vec, r, c, mean_all,
                       G, gref, fpart);
  else
    hipLaunchKernelGGL((k_center_write<DT, GT, false>), grid, dim3(256), 0, s, D, n, ldg, vec, r, c,
                       mean_all, G, gref, fpart);
  return hipGetLastError();
}

template <typename DT>
hipError_t write_by_g(const DT* D, int64_t n, int64_t n_pad, int64_t ldg, int vec, const double* r,
                      const double* c, const double* mean_all, int gk, void* G, float* gref, double* fpart,
                      hipStream_t s) {
  switch (gk) {
    case GK_F64:
      return write_dispatch<DT, double>(D, n, n_pad, ldg, vec, r, c, mean_all, (double*)G, gref, fpart, s);
    case GK_F32:
      return write_dispatch<DT, float>(D, n, n_pad, ldg, vec, r, c, mean_all, (float*)G, gref, fpart, s);
    case GK_BF16:
      return write_dispatch<DT, bf16_t>(D, n, n_pad, ldg, vec, r, c, mean_all, (bf16_t*)G, gref, fpart, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_center_stats(const void* D, int d_is_f64, int64_t n, double* rowpart, double* colpart,
                               double* r, double* c, double* rsum, double* mean_all, DevStatus* st,
                               hipStream_t s) {
  const int64_t ncb = (n + kStatsCols - 1) / kStatsCols;
  const int64_t nrb = (n + kStatsRows - 1) / kStatsRows;
  const int vec = ((uintptr_t)D % 16) == 0;
  dim3 grid((unsigned)ncb, (unsigned)nrb);
  if (d_is_f64)
    hipLaunchKernelGGL(k_stats<double>, grid, dim3(256), 0, s, (const double*)D, n, vec, rowpart, colpart);
  else
    hipLaunchKernelGGL(k_stats<float>, grid, dim3(256), 0, s, (const float*)D, n, vec, rowpart, colpart);
  hipLaunchKernelGGL(k_stats_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rowpart, colpart,
                     ncb, nrb, n, r, c, rsum);
  hipLaunchKernelGGL(k_grand, dim3(1), dim3(1024), 0, s, rsum, n, mean_all, st);
  return hipGetLastError();
}

int64_t center_write_blocks(int64_t n_pad, int64_t ldg) {
  return ((ldg + kWriteCols - 1) / kWriteCols) * (n_pad / kWriteRows);
}

hipError_t launch_center_write(const void* D, int d_is_f64, int64_t n, int64_t n_pad, int64_t ldg,
                               const double* r, const double* c, const double* mean_all, int gk, void* G,
                               float* gref, double* fpart, DevStatus* st, hipStream_t s) {
  const int vec = ((uintptr_t)D % 16) == 0;
  hipError_t e;
  if (d_is_f64)
    e = write_by_g<double>((const double*)D, n, n_pad, ldg, vec, r, c, mean_all, gk, G, gref, fpart, s);
  else
    e = write_by_g<float>((const float*)D, n, n_pad, ldg, vec, r, c, mean_all, gk, G, gref, fpart, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize_stats, dim3(1), dim3(1024), 0, s, fpart,
                     center_write_blocks(n_pad, ldg), st);
  return hipGetLastError();
}

hipError_t launch_finalize_stats(const double* fpart, int64_t nparts, DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_stats, dim3(1), dim3(1024), 0, s, fpart, nparts, st);
  return hipGetLastError();
}

}  // namespace mds
