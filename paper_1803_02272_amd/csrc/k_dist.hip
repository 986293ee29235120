// Pairwise distances on the device (Sec. 2.2: the dissimilarity matrix D
// between reads, the step before the method and, in Table 1, its dominant
// cost), written as the n x n row-major D that mds_run reads.
//
// Hamming distance of reads (the stand-in for the alignment-based
// dissimilarity: substitutions only).  Reads are base codes 0..3; the number
// of matching positions of reads i and j is the inner product of their
// one-hot encodings, 4 fp4 (e2m1) values per position with 1.0 (code 0x2)
// at the base's slot: an exact GEMM on gfx950's scaled MFMA 16x16x128 with
// fp4 operands (unit scales, fp32 accumulation of integer counts <= 2048),
// 32 positions per instruction, half the instructions and half the operand
// bytes of the int8 form.  d_ij = (L - matches) / L as the fp64 quotient
// rounded to the output type, looked up in a per-workgroup table.
// A code outside 0..3 matches nothing (an unknown base counts as a mismatch,
// also against itself).  The one-hot operands are expanded from the codes
// into LDS per K-step, so the call needs no workspace and reads each code
// block once per tile.
//
// Euclidean distance of points: d_ij = sqrt(sum_k (x_ik - x_jk)^2) in fp64,
// summed over k in increasing order with separate roundings of the square
// and the sum, then rounded to the output type.  Only tiles on and above
// the diagonal are computed; each off-diagonal tile is written twice (as
// itself and transposed): (a - b)^2 = (b - a)^2 exactly, so D is exactly
// symmetric with a zero diagonal.  This kernel is bound by fp64 VALU work
// (three operations per pair and coordinate), not by its write.
#include "mds_internal.h"

namespace mds {
namespace {

typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---- Hamming ---------------------------------------------------------------
constexpr int kHI = 256;      // rows (i) per tile
constexpr int kHJ = 128;      // columns (j) per tile
constexpr int kHThreads = 512;  // 8 waves: 4 (i) x 2 (j), 64 x 64 outputs each
constexpr int kHBases = 32;   // bases per K-step: 64 bytes of fp4 one-hot per row
constexpr int kHRows = kHI + kHJ;  // code rows loaded per step

constexpr int kHStgRow = 68;  // floats per staged output row (64 + 4 of padding)
static_assert(kHThreads / 64 * 16 * kHStgRow * 4 <= 2 * kHRows * 64, "the output stage fits the one-hot buffers");

// LDS writes of this wave visible to its other lanes
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// fp4 one-hot of a code: nibble c holds 1.0 (e2m1 0x2); other codes -> 0
__device__ __forceinline__ uint32_t onehot4(uint32_t c) { return c < 4 ? (0x2u << (4 * c)) : 0u; }

// 16-byte slot of piece p (0..3) of a 64-byte operand row r: rows 4m .. 4m+3
// are rotated by m so that 16 consecutive rows at one piece fall on distinct
// banks.
__device__ __forceinline__ int hslot(int r, int p) { return r * 64 + ((p ^ ((r >> 2) & 3)) * 16); }

template <int VEC, typename OT>
__global__ __launch_bounds__(kHThreads, 1) void k_hamming(const uint8_t* __restrict__ codes, int64_t n, int L,
                                                          OT* __restrict__ D, int vec_out) {
  __shared__ __attribute__((aligned(16))) unsigned char oh[2][kHRows * 64];  // i rows, then j rows
  __shared__ OT table[kMaxHammingLength + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * kHI, j0 = (int64_t)blockIdx.x * kHJ;
  for (int m = tid; m <= L; m += kHThreads) table[m] = (OT)((double)m / (double)L);

  // code row loaded by this thread (threads past kHRows load nothing)
  const bool loader = tid < kHRows;
  const int64_t crow = tid < kHI ? i0 + tid : j0 + (tid - kHI);
  const bool crow_ok = loader && crow < n;
  const uint8_t* cp = codes + (crow_ok ? crow : 0) * (int64_t)L;
  const int steps = (L + kHBases - 1) / kHBases;
  // 32 codes of step s, 4 per word (positions past L and rows past n read as 0xFF)
  auto load_codes = [&](int s, uint32_t (&w)[8]) {
    const int p0 = s * kHBases;
    if (p0 >= L) {  // past the last step
#pragma unroll
      for (int q = 0; q < 8; ++q) w[q] = 0xFFFFFFFFu;
      return;
    }
    if (VEC == 16 && crow_ok && p0 + kHBases <= L) {
      const u32x4 v0 = *reinterpret_cast<const u32x4*>(cp + p0);
      const u32x4 v1 = *reinterpret_cast<const u32x4*>(cp + p0 + 16);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        w[q] = v0[q];
        w[4 + q] = v1[q];
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      uint32_t x = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int p = p0 + 4 * q + b;
        const uint32_t c = (crow_ok && p < L) ? (uint32_t)cp[p] : 0xFFu;
        x |= c << (8 * b);
      }
      w[q] = x;
    }
  };
  // fp4 one-hot row of the 32 codes into buffer buf: piece q (16 bytes) holds
  // positions 8q .. 8q + 7, two per word (16 bits each, the lower position in
  // the low half)
  auto store_onehot = [&](const uint32_t (&w)[8], int buf) {
    if (!loader) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u32x4 o;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const uint32_t word = w[2 * q + d / 2], sh = 16 * (d % 2);
        o[d] = onehot4((word >> sh) & 0xFFu) | (onehot4((word >> (sh + 8)) & 0xFFu) << 16);
      }
      *reinterpret_cast<u32x4*>(&oh[buf][hslot(tid, q)]) = o;
    }
  };

  // wave (wi, wj): rows i0 + 64 wi .., columns j0 + 64 wj ..
  const int wi = wave >> 1, wj = wave & 1;
  floatx4_t acc[4][4];  // [j tile][i tile]
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};

  // The codes of step s + 1 are loaded while step s runs.  (A deeper
  // register prefetch was slower: the step is bound by LDS bandwidth, the
  // operand reads of 16 MFMAs per wave, not by the load latency.)
  uint32_t w[8];
  load_codes(0, w);
  store_onehot(w, 0);
  __syncthreads();
  for (int s = 0; s < steps; ++s) {
    const int buf = s & 1;
    if (s + 1 < steps) load_codes(s + 1, w);
    const int pc = lane >> 4;  // operand piece: positions 8 pc .. 8 pc + 7 of the step
    u32x4 bi[4], aj[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ri = wi * 64 + t * 16 + (lane & 15);
      const int rj = kHI + wj * 64 + t * 16 + (lane & 15);
      bi[t] = *reinterpret_cast<const u32x4*>(&oh[buf][hslot(ri, pc)]);
      aj[t] = *reinterpret_cast<const u32x4*>(&oh[buf][hslot(rj, pc)]);
    }
    // A = j rows, B = i rows: lane l then holds matches(j = 4 (l / 16) + e,
    // i = l % 16) of each tile, four consecutive j of one row i of D.  The
    // fp4 operand is the first four words of the 8-word register (format 4 =
    // e2m1 for both, scale exponents 127 = 1.0)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const i32x8 av = {(int)aj[a][0], (int)aj[a][1], (int)aj[a][2], (int)aj[a][3], 0, 0, 0, 0};
        const i32x8 bv = {(int)bi[b][0], (int)bi[b][1], (int)bi[b][2], (int)bi[b][3], 0, 0, 0, 0};
        acc[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc[a][b], 4, 4, 0, 127, 0, 127);
      }
    if (s + 1 < steps) store_onehot(w, buf ^ 1);
    __syncthreads();
  }

  // (the last step ended with a barrier: the one-hot buffers are free)
  if constexpr (sizeof(OT) == 4) {
    // fp32 D: 16 rows of the wave's 64 x 64 block at a time are staged in
    // its share of the one-hot buffers (rows padded to 68 floats, so that
    // the 16 rows written at one column fall on distinct banks) and stored
    // as 256-byte row segments, 4 rows per instruction: whole 128-byte lines
    float* stg = reinterpret_cast<float*>(&oh[0][0]) + wave * (16 * kHStgRow);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        float4 v;
        v.x = table[L - (int)acc[a][b][0]];
        v.y = table[L - (int)acc[a][b][1]];
        v.z = table[L - (int)acc[a][b][2]];
        v.w = table[L - (int)acc[a][b][3]];
        *reinterpret_cast<float4*>(&stg[(lane & 15) * kHStgRow + a * 16 + 4 * (lane >> 4)]) = v;
      }
      wave_lds_sync();
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = (lane >> 4) + 4 * t;
        const int64_t i = i0 + wi * 64 + b * 16 + r;
        const int64_t j = j0 + wj * 64 + 4 * (lane & 15);
        const float4 v = *reinterpret_cast<const float4*>(&stg[r * kHStgRow + 4 * (lane & 15)]);
        if (i < n) {
          OT* dst = D + i * n + j;
          if (vec_out && j + 3 < n) {
            *reinterpret_cast<float4*>(dst) = v;
          } else {
            const float e4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (j + e < n) dst[e] = e4[e];
          }
        }
      }
      wave_lds_sync();  // the stage is read before the next rows are written
    }
  } else {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t i = i0 + wi * 64 + b * 16 + (lane & 15);
      if (i >= n) continue;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int64_t j = j0 + wj * 64 + a * 16 + 4 * (lane >> 4);
        OT v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = table[L - (int)acc[a][b][e]];
        OT* dst = D + i * n + j;
        if (vec_out && j + 3 < n) {
          reinterpret_cast<double2*>(dst)[0] = make_double2(v[0], v[1]);
          reinterpret_cast<double2*>(dst)[1] = make_double2(v[2], v[3]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (j + e < n) dst[e] = v[e];
        }
      }
    }
  }
}

// ---- Euclidean ---------------------------------------------------------------
constexpr int kET = 64;   // tile edge
constexpr int kEK = 32;   // coordinates per LDS chunk

template <typename OT>
__device__ __forceinline__ void store4(OT* dst, const double (&v)[4], bool vec) {
  if (vec) {
    if constexpr (sizeof(OT) == 4) {
      *reinterpret_cast<float4*>(dst) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    } else {
      reinterpret_cast<double2*>(dst)[0] = make_double2(v[0], v[1]);
      reinterpret_cast<double2*>(dst)[1] = make_double2(v[2], v[3]);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) dst[e] = (OT)v[e];
  }
}

// One tile (I, J) with I <= J of the upper triangle of 64 x 64 tiles per
// workgroup; thread t computes the 4 x 4 block rows 4 (t / 16) .., columns
// 4 (t % 16) ...
template <typename OT>
__global__ __launch_bounds__(256) void k_euclid(const double* __restrict__ X, int64_t n, int dim, int64_t nt,
                                                OT* __restrict__ D, int vec_out) {
#pragma clang fp contract(off)
  __shared__ double xi[kEK][kET + 2];  // [k][row]: 4 rows of one k are 32 contiguous bytes
  __shared__ double xj[kEK][kET + 2];
  int64_t I, J;
  upper_tile((int64_t)blockIdx.x, nt, I, J);
  const int tid = threadIdx.x;
  const int ti = tid >> 4, tj = tid & 15;
  const int64_t r0 = I * kET, c0 = J * kET;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k0 = 0; k0 < dim; k0 += kEK) {
    const int kc = dim - k0 < kEK ? dim - k0 : kEK;
    __syncthreads();
    for (int e = tid; e < kET * kEK; e += 256) {
      const int r = e / kEK, k = e % kEK;
      const int64_t gi = r0 + r, gj = c0 + r;
      xi[k][r] = (k < kc && gi < n) ? X[gi * dim + k0 + k] : 0.0;
      xj[k][r] = (k < kc && gj < n) ? X[gj * dim + k0 + k] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < kc; ++k) {  // increasing k
      double a[4], b[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[e] = xi[k][4 * ti + e];
        b[e] = xj[k][4 * tj + e];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double d = a[p] - b[q];
          const double sq = d * d;
          acc[p][q] = acc[p][q] + sq;
        }
    }
  }
  double v[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) v[p][q] = __builtin_sqrt(acc[p][q]);
  // the tile itself: rows r0 + 4 ti + p, columns c0 + 4 tj ..
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int64_t i = r0 + 4 * ti + p, j = c0 + 4 * tj;
    if (i >= n || j >= n) continue;
    double row[4] = {v[p][0], v[p][1], v[p][2], v[p][3]};
    if (j + 3 < n) {
      store4<OT>(D + i * n + j, row, vec_out != 0);
    } else {
      for (int q = 0; j + q < n; ++q) D[i * n + j + q] = (OT)row[q];
    }
  }
  if (I == J) return;
  // its transpose: rows c0 + 4 tj + q, columns r0 + 4 ti ..
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = c0 + 4 * tj + q, j = r0 + 4 * ti;
    if (i >= n || j >= n) continue;
    double col[4] = {v[0][q], v[1][q], v[2][q], v[3][q]};
    if (j + 3 < n) {
      store4<OT>(D + i * n + j, col, vec_out != 0);
    } else {
      for (int p = 0; j + p < n; ++p) D[i * n + j + p] = (OT)col[p];
    }
  }
}

}  // namespace

hipError_t launch_hamming(const uint8_t* codes, int64_t n, int L, bool f64, void* D, hipStream_t s) {
  const dim3 grid((unsigned)((n + kHJ - 1) / kHJ), (unsigned)((n + kHI - 1) / kHI));
  const bool vin = L % 16 == 0 && ((uintptr_t)codes % 16) == 0;
  const int vout = (n % 4 == 0 && ((uintptr_t)D % (f64 ? 32 : 16)) == 0) ? 1 : 0;
  if (f64) {
    if (vin)
      hipLaunchKernelGGL((k_hamming<16, double>), grid, dim3(kHThreads), 0, s, codes, n, L, (double*)D, vout);
    else
      hipLaunchKernelGGL((k_hamming<1, double>), grid, dim3(kHThreads), 0, s, codes, n, L, (double*)D, vout);
  } else {
    if (vin)
      hipLaunchKernelGGL((k_hamming<16, float>), grid, dim3(kHThreads), 0, s, codes, n, L, (float*)D, vout);
    else
      hipLaunchKernelGGL((k_hamming<1, float>), grid, dim3(kHThreads), 0, s, codes, n, L, (float*)D, vout);
  }
  return hipGetLastError();
}

hipError_t launch_euclid(const double* X, int64_t n, int dim, bool f64, void* D, hipStream_t s) {
  const int64_t nt = (n + kET - 1) / kET;
  const int64_t tiles = nt * (nt + 1) / 2;
  const int vout = (n % 4 == 0 && ((uintptr_t)D % (f64 ? 32 : 16)) == 0) ? 1 : 0;
  if (f64)
    hipLaunchKernelGGL(k_euclid<double>, dim3((unsigned)tiles), dim3(256), 0, s, X, n, dim, nt, (double*)D, vout);
  else
    hipLaunchKernelGGL(k_euclid<float>, dim3((unsigned)tiles), dim3(256), 0, s, X, n, dim, nt, (float*)D, vout);
  return hipGetLastError();
}

}  // namespace mds
