// Skinny fp64 kernels around the G-passes.  All tall n x l matrices are kept
// transposed (l_pad x ldg, one contiguous row per column of the tall matrix).
//
//   gram   W = A^T B for tall A, B (l x l, fp64 MFMA 16x16x4, split over
//          column chunks, fixed-order reduction).  Used for Y^T Y in
//          CholeskyQR2 and for the projected matrix B = Q^T (G Q) of the
//          Rayleigh-Ritz step (Sec. 3.2, following Halko et al.).
//   apply  Out = In T for a small l x lt matrix T (orthonormalisation
//          Q = Y R^{-1}); fp64 with the T block staged in LDS, plus an
//          optional cast copy in the dtype of the next G-pass.
//   coords X = Q (V_k diag(sqrt(max(theta,0)))) written row-major n x k
//          (Sec. 6.2, step 3: X = U Sigma, first k columns), with the
//          per-column sign fixed by the entry of largest magnitude.
#include "mds_internal.h"

namespace mds {
namespace {

constexpr int kGramChunk = 512;  // columns of the transposed layout per gram workgroup

template <int CG>
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ A, const double* __restrict__ B,
                                              int64_t ldg, int l_pad, double* __restrict__ Wpart) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tr = blockIdx.y * 4 + wave;  // 16-row tile of W
  if (tr * 16 >= l_pad) return;          // no barriers below
  const int64_t p = blockIdx.x;
  const int64_t i0 = p * kGramChunk;
  const int64_t i1 = (i0 + kGramChunk < ldg) ? i0 + kGramChunk : ldg;
  doublex4_t acc[CG];
#pragma unroll
  for (int cg = 0; cg < CG; ++cg) acc[cg] = doublex4_t{0.0, 0.0, 0.0, 0.0};
  const double* Ar = A + (int64_t)(tr * 16 + (lane & 15)) * ldg + (lane >> 4) * 2;
  const double* Br = B + (int64_t)(lane & 15) * ldg + (lane >> 4) * 2;
  for (int64_t k = i0; k < i1; k += 8) {
    const double2 a = *reinterpret_cast<const double2*>(Ar + k);
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
      const double2 b = *reinterpret_cast<const double2*>(Br + (int64_t)cg * 16 * ldg + k);
      acc[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc[cg], 0, 0, 0);
      acc[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, acc[cg], 0, 0, 0);
    }
  }
  double* W = Wpart + p * (int64_t)l_pad * l_pad;
#pragma unroll
  for (int cg = 0; cg < CG; ++cg)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      // fp64 MFMA accumulator: register r of lane group g is row g + 4r
      W[(int64_t)(tr * 16 + (lane >> 4) + 4 * r) * l_pad + cg * 16 + (lane & 15)] = acc[cg][r];
}

__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ parts, int64_t nparts,
                                                   int64_t elems, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= elems) return;
  double s = 0.0;
  for (int64_t p = 0; p < nparts; ++p) s += parts[p * elems + e];
  out[e] = s;
}

constexpr int kJC = 16;  // output columns per LDS-staged block of T

__device__ __forceinline__ uint16_t bf16_rne(double v) {
  uint32_t u = __float_as_uint((float)v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(256) void k_apply(const double* __restrict__ In, int l, int64_t ldg,
                                               const double* __restrict__ T, int ldt, int lt, int l_pad,
                                               double* __restrict__ Out, int xk, void* __restrict__ Xc) {
  __shared__ double Ts[kMaxL * kJC];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;  // ldg % 256 == 0
  for (int j0 = 0; j0 < l_pad; j0 += kJC) {
    __syncthreads();
    for (int e = threadIdx.x; e < l * kJC; e += 256) {
      const int a = e / kJC, j = j0 + e % kJC;
      Ts[e] = (j < lt) ? T[(int64_t)a * ldt + j] : 0.0;
    }
    __syncthreads();
    double acc[kJC];
#pragma unroll
    for (int jj = 0; jj < kJC; ++jj) acc[jj] = 0.0;
#pragma unroll 4
    for (int a = 0; a < l; ++a) {
      const double y = In[(int64_t)a * ldg + i];
#pragma unroll
      for (int jj = 0; jj < kJC; ++jj) acc[jj] += Ts[a * kJC + jj] * y;
    }
#pragma unroll
    for (int jj = 0; jj < kJC; ++jj) {
      const int64_t o = (int64_t)(j0 + jj) * ldg + i;
      Out[o] = acc[jj];
      if (xk == GK_F64)
        reinterpret_cast<double*>(Xc)[o] = acc[jj];
      else if (xk == GK_F32)
        reinterpret_cast<float*>(Xc)[o] = (float)acc[jj];
      else if (xk == GK_BF16)
        reinterpret_cast<uint16_t*>(Xc)[o] = bf16_rne(acc[jj]);
    }
  }
}

// Better candidate for the column's sign anchor: larger magnitude, then lower row.
__device__ __forceinline__ bool better(double va, int64_t ia, double vb, int64_t ib) {
  const double aa = fabs(va), ab = fabs(vb);
  return aa > ab || (aa == ab && ia < ib);
}

__global__ __launch_bounds__(256) void k_coords(const double* __restrict__ Qt, int l, int64_t n, int64_t ldg,
                                                const double* __restrict__ Tc, int k,
                                                double* __restrict__ coords, double* __restrict__ vpart,
                                                int64_t* __restrict__ ipart) {
  __shared__ double Ts[kMaxL * kJC];
  __shared__ double wv[4][kJC];
  __shared__ int64_t wi[4][kJC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int j0 = 0; j0 < k; j0 += kJC) {
    __syncthreads();
    for (int e = threadIdx.x; e < l * kJC; e += 256) {
      const int a = e / kJC, j = j0 + e % kJC;
      Ts[e] = (j < k) ? Tc[(int64_t)a * k + j] : 0.0;
    }
    __syncthreads();
    double acc[kJC];
#pragma unroll
    for (int jj = 0; jj < kJC; ++jj) acc[jj] = 0.0;
    if (i < n) {
#pragma unroll 4
      for (int a = 0; a < l; ++a) {
        const double y = Qt[(int64_t)a * ldg + i];
#pragma unroll
        for (int jj = 0; jj < kJC; ++jj) acc[jj] += Ts[a * kJC + jj] * y;
      }
#pragma unroll
      for (int jj = 0; jj < kJC; ++jj)
        if (j0 + jj < k) coords[i * k + j0 + jj] = acc[jj];
    }
    // per-column anchor candidates of this block
#pragma unroll
    for (int jj = 0; jj < kJC; ++jj) {
      double v = (i < n) ? acc[jj] : 0.0;
      int64_t idx = (i < n) ? i : INT64_MAX;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int64_t oi = __shfl_xor(idx, off, 64);
        if (better(ov, oi, v, idx)) {
          v = ov;
          idx = oi;
        }
      }
      if (lane == 0) {
        wv[wave][jj] = v;
        wi[wave][jj] = idx;
      }
    }
    __syncthreads();
    if (threadIdx.x < kJC && j0 + (int)threadIdx.x < k) {
      const int jj = threadIdx.x;
      double v = wv[0][jj];
      int64_t idx = wi[0][jj];
      for (int w = 1; w < 4; ++w)
        if (better(wv[w][jj], wi[w][jj], v, idx)) {
          v = wv[w][jj];
          idx = wi[w][jj];
        }
      vpart[(int64_t)blockIdx.x * k + j0 + jj] = v;
      ipart[(int64_t)blockIdx.x * k + j0 + jj] = idx;
    }
  }
}

__global__ __launch_bounds__(256) void k_sign_anchor(const double* __restrict__ vpart,
                                                     const int64_t* __restrict__ ipart, int64_t nblk, int k,
                                                     double* __restrict__ sign) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= k) return;
  double v = vpart[j];
  int64_t idx = ipart[j];
  for (int64_t b = 1; b < nblk; ++b)
    if (better(vpart[b * k + j], ipart[b * k + j], v, idx)) {
      v = vpart[b * k + j];
      idx = ipart[b * k + j];
    }
  sign[j] = (v < 0.0) ? -1.0 : 1.0;
}

__global__ __launch_bounds__(256) void k_sign_apply(double* __restrict__ coords, int64_t total, int k,
                                                    const double* __restrict__ sign) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  coords[e] *= sign[e % k];
}

template <int CG>
void gram_one(const double* A, const double* B, int l_pad, int64_t ldg, double* Wpart, hipStream_t s) {
  dim3 grid((unsigned)((ldg + kGramChunk - 1) / kGramChunk), (unsigned)((CG + 3) / 4));
  hipLaunchKernelGGL(k_gram<CG>, grid, dim3(256), 0, s, A, B, ldg, l_pad, Wpart);
}

}  // namespace

int64_t gram_chunks(int64_t ldg) { return (ldg + kGramChunk - 1) / kGramChunk; }

hipError_t launch_gram(const double* A, const double* B, int l_pad, int64_t ldg, double* Wpart, double* W,
                       hipStream_t s) {
  switch (l_pad / 16) {
#define MDS_G(N) \
  case N: gram_one<N>(A, B, l_pad, ldg, Wpart, s); break;
    MDS_G(1) MDS_G(2) MDS_G(3) MDS_G(4) MDS_G(5) MDS_G(6) MDS_G(7) MDS_G(8)
    MDS_G(9) MDS_G(10) MDS_G(11) MDS_G(12) MDS_G(13) MDS_G(14) MDS_G(15) MDS_G(16)
#undef MDS_G
    default: return hipErrorInvalidValue;
  }
  const int64_t elems = (int64_t)l_pad * l_pad;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, s, Wpart,
                     gram_chunks(ldg), elems, W);
  return hipGetLastError();
}

hipError_t launch_apply(const double* In, int l, int64_t ldg, const double* T, int ldt, int lt, int l_pad,
                        double* Out, int xk, void* Xc, hipStream_t s) {
  if (l > kMaxL || l_pad > kMaxL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_apply, dim3((unsigned)(ldg / 256)), dim3(256), 0, s, In, l, ldg, T, ldt, lt, l_pad, Out,
                     Xc ? xk : -1, Xc);
  return hipGetLastError();
}

hipError_t launch_coords(const double* Qt, int l, int64_t n, int64_t ldg, const double* Tc, int k,
                         double* coords, double* sign_part, int64_t* idx_part, hipStream_t s) {
  if (l > kMaxL) return hipErrorInvalidValue;
  const int64_t nblk = (n + 255) / 256;
  hipLaunchKernelGGL(k_coords, dim3((unsigned)nblk), dim3(256), 0, s, Qt, l, n, ldg, Tc, k, coords, sign_part,
                     idx_part);
  double* sign = sign_part + nblk * k;
  hipLaunchKernelGGL(k_sign_anchor, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, sign_part, idx_part,
                     nblk, k, sign);
  const int64_t total = n * (int64_t)k;
  hipLaunchKernelGGL(k_sign_apply, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, coords, total, k,
                     sign);
  return hipGetLastError();
}

}  // namespace mds
