// Double centring of the squared distance matrix (Sec. 6.2, step 1):
//   gamma_ij = -1/2 (d_ij^2 - c_j - r_i + m),
//   r_i = (1/n) sum_j d_ij^2,  c_j = (1/n) sum_i d_ij^2,  m = (1/n^2) sum_ij d_ij^2.
//
// Two HBM-streaming passes over D:
//   stats: per 1024 x 1024 tile, each wave owns 256 rows and every lane 16
//          columns; row partials come from a 64-lane butterfly, column
//          partials from registers and a fixed-order LDS merge of the four
//          waves; the tiles on the diagonal also sum d_ii^2.  With a
//          symmetric D (the default) only the tiles on and above the
//          diagonal are read, half of D: an off-diagonal tile's row sums go
//          to its rows and its column sums to the mirrored rows, so
//          r_i = c_i = (1/n) (sum over tiles right of and on the diagonal
//          of row i's partials + sum over tiles above it of column i's
//          partials), and its sum of d^4 counts twice.  The full mode reads
//          all of D and keeps row and column means as written.  Partials
//          are combined in a fixed order afterwards, so results are bitwise
//          reproducible (no floating-point atomics).  A symmetric D with
//          n <= 16384 is read row by row instead (one wave per row): at those
//          sizes the tile grid would leave most of the GPU idle.
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

// D is streamed: every element is read once per pass, so its loads carry the
// nontemporal hint (measured on MI355X: 7.1 TB/s for nontemporal 16-byte
// loads against 6.3 TB/s for plain ones).  Here each wave's load covers
// whole 128-byte lines; where one instruction covers half lines (the MFMA
// operand layout of the G-passes) the hint made the passes slower.
typedef float f32v4 __attribute__((ext_vector_type(4)));
typedef double f64v2 __attribute__((ext_vector_type(2)));

template <typename V>
__device__ __forceinline__ V ld_stream(const void* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
}

// Four consecutive elements of a row starting at column c (c % 4 == 0),
// zero beyond n.  `vec` says the row start is 16-byte aligned.
template <typename DT>
__device__ __forceinline__ void load4(const DT* __restrict__ row, int64_t c, int64_t n, bool vec,
                                      double v[4]) {
  if (vec && c + 3 < n) {
    if constexpr (sizeof(DT) == 4) {
      const f32v4 f = ld_stream<f32v4>(row + c);
      v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
    } else {
      const f64v2 a = ld_stream<f64v2>(row + c);
      const f64v2 b = ld_stream<f64v2>(row + c + 2);
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
static_assert(kStatsRows == kStatsCols, "the diagonal of D lies in the tiles with cb == rb");

// One read of D per 1024 x 1024 tile.  Loads of the next batch of rows are
// issued before the current batch is reduced (raw values held in registers).
// p4part[rb * ncb + cb] = sum of d^4 over the tile; a diagonal tile (cb == rb)
// also writes p4part[np4 + rb] = sum of its d_ii^2 (np4 = ncb * nrb).  sym:
// the grid is one workgroup per tile on or above the diagonal, taken in
// row-major order of the upper triangle (np4 = nb (nb + 1) / 2, p4part
// indexed by that order); the diagonal tile writes no column partials and an
// off-diagonal tile's d^4 sum is doubled.
template <typename DT>
__global__ __launch_bounds__(256, 2) void k_stats(const DT* __restrict__ D, int64_t n, int base_vec,
                                                  double* __restrict__ rowpart, double* __restrict__ colpart,
                                                  double* __restrict__ p4part, int sym, int64_t nb) {
#pragma clang fp contract(off)
  constexpr int RB = 2;  // rows per batch
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int64_t cb = blockIdx.x, rb = blockIdx.y, p4i = rb * nb + cb, np4 = nb * nb;
  if (sym) {  // tile t of the upper triangle: row rb holds nb - rb tiles
    int64_t t = blockIdx.x;
    rb = 0;
    while (t >= nb - rb) t -= nb - rb++;
    cb = rb + t;
    p4i = blockIdx.x;
    np4 = nb * (nb + 1) / 2;
  }
  const int64_t c0 = cb * kStatsCols;
  const int64_t r0 = rb * kStatsRows + (int64_t)wave * kRowsPerWave;
  const int64_t r1 = (r0 + kRowsPerWave < n) ? r0 + kRowsPerWave : n;
  double cacc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) cacc[t] = 0.0;
  double acc4 = 0.0, accd = 0.0;
  const bool diag_tile = cb == rb;

  DT raw[RB][16], rawn[RB][16];
  auto load_batch = [&](DT (&dst)[RB][16], int64_t i) {
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int64_t ii = i + rr;
      const DT* row = D + ii * n;
      const bool rowok = ii < r1;
      const bool vec = rowok && row_vec_ok<DT>(base_vec != 0, ii, n);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t c = c0 + g * 256 + lane * 4;
        if (vec && c + 3 < n) {
          if constexpr (sizeof(DT) == 4) {
            const f32v4 f = ld_stream<f32v4>(row + c);
            dst[rr][g * 4 + 0] = f.x; dst[rr][g * 4 + 1] = f.y; dst[rr][g * 4 + 2] = f.z; dst[rr][g * 4 + 3] = f.w;
          } else {
            const f64v2 a = ld_stream<f64v2>(row + c);
            const f64v2 b = ld_stream<f64v2>(row + c + 2);
            dst[rr][g * 4 + 0] = a.x; dst[rr][g * 4 + 1] = a.y; dst[rr][g * 4 + 2] = b.x; dst[rr][g * 4 + 3] = b.y;
          }
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) dst[rr][g * 4 + t] = (rowok && c + t < n) ? row[c + t] : (DT)0;
        }
      }
    }
  };

  if (r0 < r1) load_batch(raw, r0);
  for (int64_t i = r0; i < r1; i += RB) {
    const bool more = i + RB < r1;
    if (more) load_batch(rawn, i + RB);
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      double rs = 0.0;
      const int64_t ii = i + rr;
      // column offset of d_ii from this lane's first column (diagonal tiles only)
      const int dcol = diag_tile ? (int)(ii - c0) - lane * 4 : -1;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const double d = (double)raw[rr][t];
        const double sq = d * d;
        cacc[t] += sq;
        rs += sq;
        acc4 += sq * sq;
        accd += ((t >> 2) * 256 + (t & 3) == dcol) ? sq : 0.0;
      }
      rs = wave_sum(rs);
      if (lane == 0 && ii < r1) rowpart[cb * n + ii] = rs;
    }
    if (more) {
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
#pragma unroll
        for (int t = 0; t < 16; ++t) raw[rr][t] = rawn[rr][t];
    }
  }
  __shared__ double sh[kWaves][kStatsCols];
  __shared__ double sh4[kWaves], shd[kWaves];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int t = 0; t < 4; ++t) sh[wave][g * 256 + lane * 4 + t] = cacc[g * 4 + t];
  acc4 = wave_sum(acc4);
  accd = wave_sum(accd);
  if (lane == 0) {
    sh4[wave] = acc4;
    shd[wave] = accd;
  }
  __syncthreads();
  const bool mirror_cols = !sym || cb != rb;  // sym: the diagonal tile's column sums repeat its row sums
  for (int cc = threadIdx.x; cc < kStatsCols; cc += 256) {
    const int64_t c = c0 + cc;
    if (c < n) colpart[rb * n + c] = mirror_cols ? ((sh[0][cc] + sh[1][cc]) + sh[2][cc]) + sh[3][cc] : 0.0;
  }
  if (threadIdx.x == 0) {
    const double q4 = ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
    p4part[p4i] = (sym && cb != rb) ? 2.0 * q4 : q4;
    if (diag_tile) p4part[np4 + rb] = ((shd[0] + shd[1]) + shd[2]) + shd[3];
  }
}

// r_i, c_j (means of d^2), and hc_j = fl32(c_j / 2) for the fp32 recentring
// of the G-passes (zero beyond n up to ldg).  sym: r_i = c_i from the row
// and column partials together.
__global__ __launch_bounds__(256) void k_stats_reduce(const double* __restrict__ rowpart,
                                                      const double* __restrict__ colpart, int64_t ncb,
                                                      int64_t nrb, int64_t n, int64_t ldg, double* __restrict__ r,
                                                      double* __restrict__ c, double* __restrict__ rsum,
                                                      float* __restrict__ hc, int sym) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= ldg) return;
  if (i >= n) {
    hc[i] = 0.0f;
    return;
  }
  // sym: row i's tiles right of and on the diagonal, column i's tiles above it
  const int64_t bi = i / kStatsRows;
  double s = 0.0;
#pragma unroll 8
  for (int64_t b = sym ? bi : 0; b < ncb; ++b) s += rowpart[b * n + i];
  double t = 0.0;
#pragma unroll 8
  for (int64_t b = 0; b < (sym ? bi : nrb); ++b) t += colpart[b * n + i];
  if (sym) {
    const double u = s + t;
    rsum[i] = u;
    r[i] = u / (double)n;
    c[i] = u / (double)n;
    hc[i] = (float)(0.5 * (u / (double)n));
  } else {
    rsum[i] = s;
    r[i] = s / (double)n;
    c[i] = t / (double)n;
    hc[i] = (float)(0.5 * (t / (double)n));
  }
}

// Statistics of a symmetric D up to kStatsRowModeMax points: one wave per row
// sums d_ij^2 over the whole row (twice the bytes of the tile mode, but one
// workgroup per 4 rows instead of one per 1024 x 1024 tile, which leaves
// most of the GPU idle at these sizes).  Writes r = c, rsum and hc directly;
// p4part[b] = sum of d^4 over the rows of workgroup b and p4part[nwg + b] =
// sum of their d_ii^2 (fixed-order merge of the four waves).
constexpr int64_t kStatsRowModeMax = 16384;
constexpr int kStatsRowModeRows = 4;  // rows per workgroup, one per wave
template <typename DT>
__global__ __launch_bounds__(256) void k_stats_rows(const DT* __restrict__ D, int64_t n, int base_vec, int64_t ldg,
                                                    double* __restrict__ r, double* __restrict__ c,
                                                    double* __restrict__ rsum, float* __restrict__ hc,
                                                    double* __restrict__ p4part) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * kStatsRowModeRows + wave;
  double sr = 0.0, s4 = 0.0, sd = 0.0;
  if (i < n) {
    const DT* row = D + i * n;
    const bool vec = row_vec_ok<DT>(base_vec != 0, i, n);
    int64_t c0 = lane * 4;
    for (; c0 + 768 < n; c0 += 1024) {  // four 16-byte loads in flight per lane
      double v[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) load4<DT>(row, c0 + 256 * u, n, vec, v[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double sq = v[u][t] * v[u][t];
          sr += sq;
          s4 += sq * sq;
          sd += (c0 + 256 * u + t == i) ? sq : 0.0;
        }
    }
    for (; c0 < n; c0 += 256) {
      double v[4];
      load4<DT>(row, c0, n, vec, v);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double sq = v[t] * v[t];
        sr += sq;
        s4 += sq * sq;
        sd += (c0 + t == i) ? sq : 0.0;
      }
    }
  }
  sr = wave_sum(sr);
  s4 = wave_sum(s4);
  sd = wave_sum(sd);
  if (lane == 0 && i < n) {
    rsum[i] = sr;
    r[i] = sr / (double)n;
    c[i] = sr / (double)n;
    hc[i] = (float)(0.5 * (sr / (double)n));
  }
  __shared__ double w4[kStatsRowModeRows], wd[kStatsRowModeRows];
  if (lane == 0) {
    w4[wave] = s4;
    wd[wave] = sd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    p4part[blockIdx.x] = ((w4[0] + w4[1]) + w4[2]) + w4[3];
    p4part[gridDim.x + blockIdx.x] = ((wd[0] + wd[1]) + wd[2]) + wd[3];
  }
  if (blockIdx.x == 0)
    for (int64_t j = n + threadIdx.x; j < ldg; j += 256) hc[j] = 0.0f;
}

// Grand mean m, and the by-products ||G||_F^2 and tr(G) from their closed
// forms in the centring statistics: with A = [d_ij^2] and B = J A J,
// A = B + r 1^T + 1 c^T - m 1 1^T splits into Frobenius-orthogonal parts, so
// ||B||^2 = ||A||^2 - n ||r||^2 - n ||c||^2 + n^2 m^2 and ||G||^2 = ||B||^2 / 4;
// tr G = -1/2 (sum_i d_ii^2 - n m).
__global__ __launch_bounds__(1024) void k_grand(const double* __restrict__ rsum, const double* __restrict__ r,
                                                const double* __restrict__ c, const double* __restrict__ p4part,
                                                int64_t np4, int64_t ndiag, int64_t n, double* __restrict__ mean_all,
                                                DevStatus* st) {
#pragma clang fp contract(off)
  __shared__ double sh[5][1024];
  double s = 0.0, rr = 0.0, cc = 0.0, q = 0.0, dg = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    s += rsum[i];
    rr += r[i] * r[i];
    cc += c[i] * c[i];
  }
  for (int64_t i = threadIdx.x; i < np4; i += 1024) q += p4part[i];
  for (int64_t i = threadIdx.x; i < ndiag; i += 1024) dg += p4part[np4 + i];
  sh[0][threadIdx.x] = s;
  sh[1][threadIdx.x] = rr;
  sh[2][threadIdx.x] = cc;
  sh[3][threadIdx.x] = q;
  sh[4][threadIdx.x] = dg;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double S = sh[0][0];
    const double dn = (double)n;
    const double m = S / (dn * dn);
    mean_all[0] = m;
    st->sum_sq = S;
    st->frob2 = 0.25 * (((sh[3][0] - dn * sh[1][0]) - dn * sh[2][0]) + (dn * dn) * (m * m));
    st->trace = -0.5 * (sh[4][0] - dn * m);
    if (!__builtin_isfinite(S) || !__builtin_isfinite(sh[3][0])) st->nonfinite = 1;
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
                                                      GT* __restrict__ G, float* __restrict__ gref) {
#pragma clang fp contract(off)
  const int64_t j0 = (int64_t)blockIdx.x * kWriteCols + threadIdx.x * 4;
  const bool active = j0 < ldg;
  double cj[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) cj[t] = (j0 + t < n) ? c[j0 + t] : 0.0;
  const double m = mean_all[0];
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
    }
  }
}

template <typename DT, typename GT>
hipError_t write_dispatch(const DT* D, int64_t n, int64_t n_pad, int64_t ldg, int vec, const double* r,
                          const double* c, const double* mean_all, GT* G, float* gref, hipStream_t s) {
  dim3 grid((unsigned)((ldg + kWriteCols - 1) / kWriteCols), (unsigned)(n_pad / kWriteRows));
  if (gref)
    hipLaunchKernelGGL((k_center_write<DT, GT, true>), grid, dim3(256), 0, s, D, n, ldg, vec, r, c, mean_all,
                       G, gref);
  else
    hipLaunchKernelGGL((k_center_write<DT, GT, false>), grid, dim3(256), 0, s, D, n, ldg, vec, r, c,
                       mean_all, G, gref);
  return hipGetLastError();
}

template <typename DT>
hipError_t write_by_g(const DT* D, int64_t n, int64_t n_pad, int64_t ldg, int vec, const double* r,
                      const double* c, const double* mean_all, int gk, void* G, float* gref, hipStream_t s) {
  switch (gk) {
    case GK_F64:
      return write_dispatch<DT, double>(D, n, n_pad, ldg, vec, r, c, mean_all, (double*)G, gref, s);
    case GK_F32:
      return write_dispatch<DT, float>(D, n, n_pad, ldg, vec, r, c, mean_all, (float*)G, gref, s);
    case GK_BF16:
      return write_dispatch<DT, bf16_t>(D, n, n_pad, ldg, vec, r, c, mean_all, (bf16_t*)G, gref, s);
    default:
      return hipErrorInvalidValue;
  }
}

// OCP E4M3 code of x (|x| <= 448 up to rounding, finite), nearest even,
// saturating: 1 sign, 4 exponent (bias 7) and 3 fraction bits; below 2^-6
// the subnormal multiples of 2^-9.
// E4M3 encoding (OCP, round to nearest even) of values with |x| <= 448
// (1 + 2^-23): gfx950's v_cvt_pk_fp8_f32, two values per instruction.  It was
// checked on the GPU against a bit-level software encoder (fp32 fraction
// rounded to 3 bits, ties to even; subnormals in units of 2^-9) on every fp32
// bit pattern of magnitude up to 452, both signs: no difference.
template <bool HI>
__device__ __forceinline__ int e4m3_pack2(float a, float b, int old) {
  return __builtin_amdgcn_cvt_pk_fp8_f32(a, b, old, HI);
}

constexpr int kF8Threads = 1024;  // one workgroup per 256 x 256 block, the block held in registers

// Thread t owns columns 4 (t % 64) .. +3 of its block and the 16 rows
// 16 (t / 64) .. +15: it loads and recentres its 64 entries once (float4
// loads, 16 in flight), the block maximum is reduced over the workgroup, and
// the codes are written from registers, so D is read exactly once.
template <typename DT>
__global__ __launch_bounds__(kF8Threads) void k_center_write_fp8(const DT* __restrict__ D, int64_t n, int64_t ldg,
                                                               int base_vec, const double* __restrict__ r,
                                                               const double* __restrict__ c,
                                                               const double* __restrict__ mean_all,
                                                               uint8_t* __restrict__ G8, float* __restrict__ scales,
                                                               int64_t nsb) {
#pragma clang fp contract(off)
  __shared__ float red[kF8Threads / 64];
  const int tid = threadIdx.x;
  const int64_t J = blockIdx.x, I = blockIdx.y;
  const int64_t j0 = J * kF8Block + 4 * (tid & 63);
  const int64_t ib = I * kF8Block + 16 * (tid >> 6);
  const double m = mean_all[0];
  double cj[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) cj[t] = (j0 + t < n) ? c[j0 + t] : 0.0;
  float g[16][4];
  float mx = 0.0f;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t i = ib + u;
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < n) load4<DT>(D + i * n, j0, n, row_vec_ok<DT>(base_vec != 0, i, n), d);
    const double ri = i < n ? r[i] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      g[u][t] = (i < n && j0 + t < n) ? (float)(-0.5 * (((d[t] * d[t] - cj[t]) - ri) + m)) : 0.0f;
      mx = fmaxf(mx, fabsf(g[u][t]));
    }
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = mx;
  __syncthreads();
  mx = red[0];
#pragma unroll
  for (int w = 1; w < kF8Threads / 64; ++w) mx = fmaxf(mx, red[w]);
  const float s = mx > 0.0f ? mx / 448.0f : 1.0f;
  if (tid == 0) scales[I * nsb + J] = s;
  // fl32(g / s) as fl32(g * (1 / s)) in fp64: the quotient of two fp32
  // values is never a midpoint of the fp32 grid and stays at least ~2^-48
  // (relative) away from one, while the fp64 product is within ~2^-52 of
  // g / s, so both round to the same fp32 value (no fp32 division sequence)
  const double rinv = 1.0 / (double)s;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    float q[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) q[t] = (float)((double)g[u][t] * rinv);
    int w = e4m3_pack2<false>(q[0], q[1], 0);  // bytes 0, 1
    w = e4m3_pack2<true>(q[2], q[3], w);       // bytes 2, 3
    *reinterpret_cast<int*>(G8 + (ib + u) * ldg + j0) = w;
  }
}

// ---- finite-metric check (MDS_FLAG_CHECK_INPUT) ------------------------------
// One workgroup per pair of 64 x 64 tiles (I, J), I <= J: tile (J, I) is
// staged transposed in LDS and compared entry by entry with tile (I, J);
// a diagonal tile compares its strict upper triangle with the lower one and
// tests its diagonal.  Integer counts, so the result is exact.
constexpr int kChk = 64;
template <typename DT>
__global__ __launch_bounds__(256) void k_check_input(const DT* __restrict__ D, int64_t n, DevStatus* st) {
  const int64_t I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;
  __shared__ DT t[kChk][kChk + 1];
  __shared__ unsigned int cnt[2];
  const int tid = threadIdx.x;
  if (tid < 2) cnt[tid] = 0;
  const int c = tid & 63, r0 = tid >> 6;  // lane c reads column c of 4 rows per sweep
  // stage tile (J, I): t[col][row] = D[J*64 + row][I*64 + col]
  for (int r = r0; r < kChk; r += 4) {
    const int64_t i = J * kChk + r, j = I * kChk + c;
    t[c][r] = (i < n && j < n) ? D[i * n + j] : (DT)0;
  }
  __syncthreads();
  unsigned int asym = 0, diag = 0;
  for (int r = r0; r < kChk; r += 4) {
    const int64_t i = I * kChk + r, j = J * kChk + c;
    if (i >= n || j >= n) continue;
    const DT a = D[i * n + j];
    if (I == J && r == c) {
      diag += a != (DT)0;
    } else if (I < J || r < c) {
      asym += !(a == t[r][c]);  // t[r][c] = D[j][i]; NaN counts as asymmetric
    }
  }
  if (asym) atomicAdd(&cnt[0], asym);
  if (diag) atomicAdd(&cnt[1], diag);
  __syncthreads();
  if (tid == 0 && cnt[0]) atomicAdd(&st->asym_pairs, (unsigned long long)cnt[0]);
  if (tid == 0 && cnt[1]) atomicAdd(&st->diag_nonzero, (unsigned long long)cnt[1]);
}

}  // namespace

hipError_t launch_center_write_fp8(const void* D, int d_is_f64, int64_t n, int64_t n_pad, int64_t ldg,
                                   const double* r, const double* c, const double* mean_all, uint8_t* G8,
                                   float* scales, hipStream_t s) {
  if (n_pad % kF8Block != 0 || ldg != n_pad) return hipErrorInvalidValue;
  const int64_t nsb = n_pad / kF8Block;
  const int vec = ((uintptr_t)D % 16) == 0;
  dim3 grid((unsigned)nsb, (unsigned)nsb);
  if (d_is_f64)
    hipLaunchKernelGGL(k_center_write_fp8<double>, grid, dim3(kF8Threads), 0, s, (const double*)D, n, ldg, vec, r, c,
                       mean_all, G8, scales, nsb);
  else
    hipLaunchKernelGGL(k_center_write_fp8<float>, grid, dim3(kF8Threads), 0, s, (const float*)D, n, ldg, vec, r, c,
                       mean_all, G8, scales, nsb);
  return hipGetLastError();
}

hipError_t launch_check_input(const void* D, int d_is_f64, int64_t n, DevStatus* st, hipStream_t s) {
  const int64_t tiles = (n + kChk - 1) / kChk;
  if (tiles > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tiles, (unsigned)tiles);
  if (d_is_f64)
    hipLaunchKernelGGL(k_check_input<double>, grid, dim3(256), 0, s, (const double*)D, n, st);
  else
    hipLaunchKernelGGL(k_check_input<float>, grid, dim3(256), 0, s, (const float*)D, n, st);
  return hipGetLastError();
}

int64_t stats_parts(int64_t n) {
  const int64_t nrb = (n + kStatsRows - 1) / kStatsRows;
  const int64_t tiles = ((n + kStatsCols - 1) / kStatsCols) * nrb + nrb;
  const int64_t rows = 2 * ((n + kStatsRowModeRows - 1) / kStatsRowModeRows);  // row mode
  return n <= kStatsRowModeMax && rows > tiles ? rows : tiles;
}

hipError_t launch_center_stats(const void* D, int d_is_f64, int64_t n, int64_t ldg, double* rowpart,
                               double* colpart, double* p4part, double* r, double* c, double* rsum, float* hc,
                               double* mean_all, DevStatus* st, int sym, hipStream_t s) {
  const int64_t ncb = (n + kStatsCols - 1) / kStatsCols;
  const int64_t nrb = (n + kStatsRows - 1) / kStatsRows;
  const int vec = ((uintptr_t)D % 16) == 0;
  if (sym && n <= kStatsRowModeMax) {
    const int64_t nwg = (n + kStatsRowModeRows - 1) / kStatsRowModeRows;
    if (d_is_f64)
      hipLaunchKernelGGL(k_stats_rows<double>, dim3((unsigned)nwg), dim3(256), 0, s, (const double*)D, n, vec, ldg, r,
                         c, rsum, hc, p4part);
    else
      hipLaunchKernelGGL(k_stats_rows<float>, dim3((unsigned)nwg), dim3(256), 0, s, (const float*)D, n, vec, ldg, r, c,
                         rsum, hc, p4part);
    hipLaunchKernelGGL(k_grand, dim3(1), dim3(1024), 0, s, rsum, r, c, p4part, nwg, nwg, n, mean_all, st);
    return hipGetLastError();
  }
  dim3 grid = sym ? dim3((unsigned)(ncb * (ncb + 1) / 2)) : dim3((unsigned)ncb, (unsigned)nrb);
  if (d_is_f64)
    hipLaunchKernelGGL(k_stats<double>, grid, dim3(256), 0, s, (const double*)D, n, vec, rowpart, colpart, p4part,
                       sym, ncb);
  else
    hipLaunchKernelGGL(k_stats<float>, grid, dim3(256), 0, s, (const float*)D, n, vec, rowpart, colpart, p4part,
                       sym, ncb);
  hipLaunchKernelGGL(k_stats_reduce, dim3((unsigned)((ldg + 255) / 256)), dim3(256), 0, s, rowpart, colpart, ncb,
                     nrb, n, ldg, r, c, rsum, hc, sym);
  hipLaunchKernelGGL(k_grand, dim3(1), dim3(1024), 0, s, rsum, r, c, p4part, sym ? ncb * (ncb + 1) / 2 : ncb * nrb,
                     nrb, n, mean_all, st);
  return hipGetLastError();
}

int64_t center_write_blocks(int64_t n_pad, int64_t ldg) {
  return ((ldg + kWriteCols - 1) / kWriteCols) * (n_pad / kWriteRows);
}

hipError_t launch_center_write(const void* D, int d_is_f64, int64_t n, int64_t n_pad, int64_t ldg,
                               const double* r, const double* c, const double* mean_all, int gk, void* G,
                               float* gref, hipStream_t s) {
  const int vec = ((uintptr_t)D % 16) == 0;
  if (d_is_f64) return write_by_g<double>((const double*)D, n, n_pad, ldg, vec, r, c, mean_all, gk, G, gref, s);
  return write_by_g<float>((const float*)D, n, n_pad, ldg, vec, r, c, mean_all, gk, G, gref, s);
}

}  // namespace mds
