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

__device__ __forceinline__ uint16_t bf16_rne(double v) {
  uint32_t u = __float_as_uint((float)v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

constexpr int kGramChunk = 512;   // most columns of the transposed layout per gram workgroup
constexpr int kGramStep = 32;     // columns staged in LDS per step
constexpr int kGramThreads = 512;

// Wpart[p] = A_p B_p^T over column chunk p (chunk columns, a multiple of 64):
// every workgroup stages STEP-column slices of all l_pad rows of A (and B) in
// LDS (double-buffered, 16-byte loads), and each of its 8 waves accumulates
// a share of the 16 x 16 output
// tiles with fp64 MFMA (16x16x4).  sym (A == B): only tiles on or above the
// diagonal are computed; k_sum_parts mirrors them.
template <int CG, bool SYM, int STEP>
__global__ __launch_bounds__(kGramThreads) void k_gram(const double* __restrict__ A, const double* __restrict__ B,
                                                       int64_t ldg, int l_pad, double* __restrict__ Wpart,
                                                       int64_t chunk) {
  constexpr int kGramRow = STEP + 1;  // LDS row stride (doubles)
  constexpr int NT = SYM ? CG * (CG + 1) / 2 : CG * CG;  // output tiles
  constexpr int NW = kGramThreads / 64;
  constexpr int TPW = (NT + NW - 1) / NW;  // tiles per wave (at most)
  constexpr int LP = CG * 16;
  constexpr int NB = SYM ? 1 : 2;  // staged matrices
  __shared__ double st[2][NB][LP * kGramRow];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = (i0 + chunk < ldg) ? i0 + chunk : ldg;  // ldg and chunk are multiples of 64
  // this wave's tiles (ta, tb), ta <= tb when SYM
  int ta[TPW], tb[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    int t = wave + NW * u, a = 0;
    if (t >= NT) t = NT - 1;  // duplicate of a live tile, not stored
    if constexpr (SYM) {
      while (t >= CG - a) {
        t -= CG - a;
        ++a;
      }
      ta[u] = a;
      tb[u] = a + t;
    } else {
      ta[u] = t / CG;
      tb[u] = t % CG;
    }
  }
  doublex4_t acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) acc[u] = doublex4_t{0.0, 0.0, 0.0, 0.0};
  // staging: LP rows x 32 doubles per matrix = LP * 16 pieces of 16 bytes
  constexpr int PIECES = LP * (STEP / 2);
  constexpr int PPT = (PIECES + kGramThreads - 1) / kGramThreads;
  double2 rg[NB][PPT];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int pc = tid + kGramThreads * u;
        if (PIECES % kGramThreads == 0 || pc < PIECES) {
          const int row = pc / (STEP / 2), c2 = pc % (STEP / 2);
          const double* src = (m == 0 ? A : B) + (int64_t)row * ldg + k0 + 2 * c2;
          rg[m][u] = k0 < i1 ? *reinterpret_cast<const double2*>(src) : double2{0.0, 0.0};
        }
      }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int pc = tid + kGramThreads * u;
        if (PIECES % kGramThreads == 0 || pc < PIECES) {
          const int row = pc / (STEP / 2), c2 = pc % (STEP / 2);
          st[buf][m][row * kGramRow + 2 * c2] = rg[m][u].x;
          st[buf][m][row * kGramRow + 2 * c2 + 1] = rg[m][u].y;
        }
      }
  };
  load(i0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = i0; k0 < i1; k0 += STEP) {
    const bool more = k0 + STEP < i1;
    if (more) load(k0 + STEP);
    const double* SA = st[buf][0];
    const double* SB = st[buf][NB - 1];
#pragma unroll
    for (int kg = 0; kg < STEP; kg += 4) {
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        // fp64 MFMA operands: lane supplies row l % 16 and K index l / 16
        const double av = SA[(ta[u] * 16 + (lane & 15)) * kGramRow + kg + (lane >> 4)];
        const double bv = SB[(tb[u] * 16 + (lane & 15)) * kGramRow + kg + (lane >> 4)];
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
      }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double* W = Wpart + blockIdx.x * (int64_t)l_pad * l_pad;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    if (wave + NW * u >= NT) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      // fp64 MFMA accumulator: register r of lane group g is row g + 4r
      W[(int64_t)(ta[u] * 16 + (lane >> 4) + 4 * r) * l_pad + tb[u] * 16 + (lane & 15)] = acc[u][r];
  }
}

// Register-streamed variant for l_pad > 128 (the LDS tiles of k_gram would
// need too many accumulators per wave): each wave owns half of a 16-row tile
// strip over one column chunk; SYM (A == B): only the tiles on or above the
// diagonal are computed (the strip's B loads and MFMAs left of it are
// skipped), as in k_gram.
template <int CG, bool SYM>
__global__ __launch_bounds__(256) void k_gram_wide(const double* __restrict__ A, const double* __restrict__ B,
                                              int64_t ldg, int l_pad, double* __restrict__ Wpart, int64_t chunk) {
  // each wave owns half of a 16-row tile strip (HALF tiles of 16 columns):
  // the accumulators and operand registers of half a strip let three waves
  // share a SIMD, which hides the operand loads of one another
  constexpr int HALF = (CG + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int w = blockIdx.y * 4 + wave;
  const int tr = w >> 1;              // 16-row tile of W
  const int c0 = (w & 1) * HALF;      // first 16-column tile of this half
  if (tr * 16 >= l_pad) return;       // no barriers below
  if (SYM && c0 + HALF <= tr) return;  // the half lies left of the diagonal
  const int64_t p = blockIdx.x;
  const int64_t i0 = p * chunk;
  const int64_t i1 = (i0 + chunk < ldg) ? i0 + chunk : ldg;
  doublex4_t acc[HALF];
#pragma unroll
  for (int h = 0; h < HALF; ++h) acc[h] = doublex4_t{0.0, 0.0, 0.0, 0.0};
  auto live = [&](int h) { return c0 + h < CG && (!SYM || c0 + h >= tr); };
  const double* Ar = A + (int64_t)(tr * 16 + (lane & 15)) * ldg + (lane >> 4) * 2;
  const double* Br = B + (int64_t)(c0 * 16 + (lane & 15)) * ldg + (lane >> 4) * 2;
  // software pipeline: the operands of step k+8 are loaded while step k runs
  double2 a = *reinterpret_cast<const double2*>(Ar + i0);
  double2 b[HALF];
#pragma unroll
  for (int h = 0; h < HALF; ++h)
    if (live(h)) b[h] = *reinterpret_cast<const double2*>(Br + (int64_t)h * 16 * ldg + i0);
  for (int64_t k = i0; k < i1; k += 8) {
    const bool more = k + 8 < i1;
    double2 an = a, bn[HALF];
    if (more) {
      an = *reinterpret_cast<const double2*>(Ar + k + 8);
#pragma unroll
      for (int h = 0; h < HALF; ++h)
        if (live(h)) bn[h] = *reinterpret_cast<const double2*>(Br + (int64_t)h * 16 * ldg + k + 8);
    }
#pragma unroll
    for (int h = 0; h < HALF; ++h)
      if (live(h)) {
        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b[h].x, acc[h], 0, 0, 0);
        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b[h].y, acc[h], 0, 0, 0);
      }
    if (more) {
      a = an;
#pragma unroll
      for (int h = 0; h < HALF; ++h)
        if (live(h)) b[h] = bn[h];
    }
  }
  double* W = Wpart + p * (int64_t)l_pad * l_pad;
#pragma unroll
  for (int h = 0; h < HALF; ++h)
    if (live(h))
#pragma unroll
      for (int r = 0; r < 4; ++r)
        // fp64 MFMA accumulator: register r of lane group g is row g + 4r
        W[(int64_t)(tr * 16 + (lane >> 4) + 4 * r) * l_pad + (c0 + h) * 16 + (lane & 15)] = acc[h][r];
}

// out[i][j] = sum_p parts[p][i][j]; sym: only entries of tiles on or above the
// diagonal were computed, and each such sum is also written to the mirrored
// entry.  A workgroup takes 16 entries with 16 threads each: thread slice q
// sums parts q, q + 16, ... in order, and the 16 slice sums are added in
// slice order, so the result is the same on every run (many partials, as
// with small gram chunks, no longer form one serial chain per entry).
constexpr int kSumEntries = 16, kSumSlices = 16;
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ parts, int64_t nparts,
                                                   int64_t elems, double* __restrict__ out, int l_pad, int sym) {
#pragma clang fp contract(off)
  __shared__ double sh[kSumSlices][kSumEntries];
  const int el = threadIdx.x % kSumEntries, q = threadIdx.x / kSumEntries;
  const int64_t e = (int64_t)blockIdx.x * kSumEntries + el;
  double s = 0.0;
  if (e < elems) {
#pragma unroll 4
    for (int64_t p = q; p < nparts; p += kSumSlices) s += parts[p * elems + e];
  }
  sh[q][el] = s;
  __syncthreads();
  if (q != 0 || e >= elems) return;
  const int i = (int)(e / l_pad), j = (int)(e % l_pad);
  if (sym && (j >> 4) < (i >> 4)) return;  // written by its mirror
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < kSumSlices; ++k) t += sh[k][el];
  out[e] = t;
  if (sym && (j >> 4) > (i >> 4)) out[(int64_t)j * l_pad + i] = t;
}

// Xc = cast(Out) for the next G-pass operand, 4 consecutive entries per thread.
// GK_F32S: x = fl32(Out) split exactly into x0 + x1 + x2 (bf16, each step
// rounding to nearest even); per row and 32 consecutive columns, the 32 x0,
// then the 32 x1, then the 32 x2 (the layout the split G-pass reads).
template <int XK>
__global__ __launch_bounds__(256) void k_cast(const double* __restrict__ In, int64_t elems, int64_t ldg,
                                              void* __restrict__ Xc) {
  const int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (e >= elems) return;  // elems is a multiple of 4
  const double2 a = reinterpret_cast<const double2*>(In + e)[0];
  const double2 b = reinterpret_cast<const double2*>(In + e)[1];
  if constexpr (XK == GK_F32S) {
    const float x[4] = {(float)a.x, (float)a.y, (float)b.x, (float)b.y};
    uint16_t h[3][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const __bf16 v0 = (__bf16)x[t];
      const float r1 = x[t] - (float)v0;
      const __bf16 v1 = (__bf16)r1;
      const float r2 = r1 - (float)v1;
      const __bf16 v2 = (__bf16)r2;
      h[0][t] = __builtin_bit_cast(uint16_t, v0);
      h[1][t] = __builtin_bit_cast(uint16_t, v1);
      h[2][t] = __builtin_bit_cast(uint16_t, v2);
    }
    const int64_t j = e / ldg, k = e % ldg;  // 4 | ldg: the four entries share a row and a 32-column group
    uint16_t* dst = reinterpret_cast<uint16_t*>(Xc) + j * (3 * ldg) + (k / 32) * 96 + (k % 32);
#pragma unroll
    for (int p = 0; p < 3; ++p)
      *reinterpret_cast<uint2*>(dst + 32 * p) =
          make_uint2(h[p][0] | ((uint32_t)h[p][1] << 16), h[p][2] | ((uint32_t)h[p][3] << 16));
  } else if constexpr (XK == GK_F64) {
    reinterpret_cast<double2*>(reinterpret_cast<double*>(Xc) + e)[0] = a;
    reinterpret_cast<double2*>(reinterpret_cast<double*>(Xc) + e)[1] = b;
  } else if constexpr (XK == GK_F32) {
    *reinterpret_cast<float4*>(reinterpret_cast<float*>(Xc) + e) = make_float4((float)a.x, (float)a.y, (float)b.x,
                                                                               (float)b.y);
  } else {
    const uint32_t lo = bf16_rne(a.x) | ((uint32_t)bf16_rne(a.y) << 16);
    const uint32_t hi = bf16_rne(b.x) | ((uint32_t)bf16_rne(b.y) << 16);
    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(Xc) + e) = make_uint2(lo, hi);
  }
}


// Out[j][i] = sum_a T[a][j] In[a][i] on fp64 MFMA (16x16x4): A operand = T^T
// (rows j, K = a) from an LDS block of 64 columns of T, B operand = In (K = a,
// columns i, 16 consecutive i per lane group: 128-byte loads).  A workgroup
// of NTH / 64 waves covers NN 16-column tiles per wave and 64 rows j; the l
// rows of In are padded to a multiple of 4 (In is zero beyond l).  Large n:
// 8 waves of two tiles (256 columns) keep more loads of In in flight than 4
// waves of four; when that gives fewer than 128 workgroups, 4 waves of one
// tile (64 columns) spread the work over more CUs.
constexpr int kApJ = 64;
constexpr int kApRow = kApJ + 2;  // LDS row stride (doubles)
constexpr int kApPf = 8;          // steps of In rows in flight

template <int NN, int NTH>
__global__ __launch_bounds__(NTH) void k_apply(const double* __restrict__ In, int l, int64_t ldg,
                                               const double* __restrict__ T, int ldt, int lt, int l_out,
                                               double* __restrict__ Out, int gx, int jb) {
  extern __shared__ double Ts[];  // la x kApRow
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int la = (l + 3) & ~3;
  // the jb column blocks of one strip of rows i go to one XCD (workgroup wg
  // runs on XCD wg % 8) one after another in dispatch order, so all but the
  // first read that strip of In from the XCD's L2
  const int wg = blockIdx.x, wq = wg >> 3;
  const int bx = (wq / jb) * 8 + (wg & 7), by = wq % jb;
  if (bx >= gx) return;  // uniform: the grid is padded to a multiple of 8 strips
  const int j0 = by * kApJ;
  const int64_t i0 = (int64_t)bx * ((NTH / 64) * 16 * NN) + wave * (16 * NN);
  for (int e = tid; e < la * kApJ; e += NTH) {
    const int a = e / kApJ, jj = e % kApJ, j = j0 + jj;
    Ts[a * kApRow + jj] = (a < l && j < lt) ? T[(int64_t)a * ldt + j] : 0.0;
  }
  __syncthreads();
  doublex4_t acc[NN][4];
#pragma unroll
  for (int nt = 0; nt < NN; ++nt)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[nt][t] = doublex4_t{0.0, 0.0, 0.0, 0.0};
  const double* Ib = In + (int64_t)(lane >> 4) * ldg + i0 + (lane & 15);
  const int ar = lane >> 4, jc = lane & 15;
  // software pipeline: a ring of kApPf steps of In rows in registers, step
  // a + 4 kApPf loading while step a runs (the loop is latency-bound: a step
  // is 4 NN MFMAs against a round trip to memory)
  double b[kApPf][NN];
#pragma unroll
  for (int p = 0; p < kApPf; ++p)
#pragma unroll
    for (int nt = 0; nt < NN; ++nt) b[p][nt] = Ib[(int64_t)(4 * p < la ? 4 * p : la - 4) * ldg + nt * 16];
  for (int a0 = 0; a0 < la; a0 += 4 * kApPf) {
#pragma unroll
    for (int p = 0; p < kApPf; ++p) {
      const int a = a0 + 4 * p;
      if (a >= la) break;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double av = Ts[(a + ar) * kApRow + t * 16 + jc];
#pragma unroll
        for (int nt = 0; nt < NN; ++nt)
          acc[nt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[p][nt], acc[nt][t], 0, 0, 0);
      }
      // past the end the last step is loaded again (rows < la exist): the
      // loads stay unconditional, so the compiler keeps exact wait counts
      const int an = a + 4 * kApPf < la ? a + 4 * kApPf : la - 4;
#pragma unroll
      for (int nt = 0; nt < NN; ++nt) b[p][nt] = Ib[(int64_t)an * ldg + nt * 16];
    }
  }
  // fp64 accumulator layout: register r of lane group g is row g + 4r
#pragma unroll
  for (int nt = 0; nt < NN; ++nt)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + t * 16 + (lane >> 4) + 4 * r;
        if (j < l_out) {
          const int64_t o = (int64_t)j * ldg + i0 + nt * 16 + (lane & 15);
          Out[o] = acc[nt][t][r];
        }
      }
    }
}

// Better candidate for the column's sign anchor: larger magnitude, then lower row.
__device__ __forceinline__ bool better(double va, int64_t ia, double vb, int64_t ib) {
  const double aa = fabs(va), ab = fabs(vb);
  return aa > ab || (aa == ab && ia < ib);
}

constexpr int kAnchorChunk = 4096;

// Per (column a, chunk): entry of largest magnitude of row a of Ct.
__global__ __launch_bounds__(256) void k_anchor_part(const double* __restrict__ Ct, int64_t n, int64_t ldg,
                                                     double* __restrict__ vpart, int64_t* __restrict__ ipart,
                                                     int64_t nchunks) {
  __shared__ double wv[4];
  __shared__ int64_t wi[4];
  const int a = blockIdx.y;
  const int64_t c0 = (int64_t)blockIdx.x * kAnchorChunk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v = 0.0;
  int64_t idx = INT64_MAX;
  for (int64_t i = c0 + threadIdx.x; i < c0 + kAnchorChunk && i < n; i += 256) {
    const double x = Ct[(int64_t)a * ldg + i];
    if (better(x, i, v, idx)) {
      v = x;
      idx = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int64_t oi = __shfl_xor(idx, off, 64);
    if (better(ov, oi, v, idx)) {
      v = ov;
      idx = oi;
    }
  }
  if (lane == 0) {
    wv[wave] = v;
    wi[wave] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w)
      if (better(wv[w], wi[w], v, idx)) {
        v = wv[w];
        idx = wi[w];
      }
    vpart[(int64_t)a * nchunks + blockIdx.x] = v;
    ipart[(int64_t)a * nchunks + blockIdx.x] = idx;
  }
}

__global__ __launch_bounds__(64) void k_sign_anchor(const double* __restrict__ vpart,
                                                    const int64_t* __restrict__ ipart, int64_t nchunks,
                                                    double* __restrict__ sign) {
  const int a = blockIdx.x;
  double v = 0.0;
  int64_t idx = INT64_MAX;
  for (int64_t c = threadIdx.x; c < nchunks; c += 64)
    if (better(vpart[a * nchunks + c], ipart[a * nchunks + c], v, idx)) {
      v = vpart[a * nchunks + c];
      idx = ipart[a * nchunks + c];
    }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int64_t oi = __shfl_xor(idx, off, 64);
    if (better(ov, oi, v, idx)) {
      v = ov;
      idx = oi;
    }
  }
  if (threadIdx.x == 0) sign[a] = (v < 0.0) ? -1.0 : 1.0;
}

// coords[i][a] = sign[a] * Ct[a][i], transposed through LDS (64 rows i x k).
__global__ __launch_bounds__(256) void k_coords_write(const double* __restrict__ Ct, int64_t n, int64_t ldg, int k,
                                                      const double* __restrict__ sign, double* __restrict__ coords) {
  __shared__ double tile[16][64 + 1];
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int a0 = blockIdx.y * 16;
  const int tid = threadIdx.x;
  for (int e = tid; e < 16 * 64; e += 256) {
    const int aa = e / 64, ii = e % 64;
    const int a = a0 + aa;
    tile[aa][ii] = (a < k) ? sign[a] * Ct[(int64_t)a * ldg + i0 + ii] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 16 * 64; e += 256) {
    const int ii = e / 16, aa = e % 16;
    const int64_t i = i0 + ii;
    const int a = a0 + aa;
    if (i < n && a < k) coords[i * k + a] = tile[aa][ii];
  }
}

// Columns per gram workgroup: 512 once that gives at least 128 workgroups
// (more, smaller chunks only add partial sums to reduce at n = 1e5), else
// the power of two (at least 64) that gives about 256 workgroups, so that
// small and mid-size problems still spread over the GPU.
int64_t gram_chunk_cols(int64_t ldg) {
  if (ldg >= 128 * (int64_t)kGramChunk) return kGramChunk;
  int64_t c = 64;
  while (c * 2 <= ldg / 256 && c * 2 <= kGramChunk) c *= 2;
  return c;
}

template <int CG>
void gram_one(const double* A, const double* B, int l_pad, int64_t ldg, double* Wpart, hipStream_t s) {
  const int64_t chunk = gram_chunk_cols(ldg);
  dim3 grid((unsigned)((ldg + chunk - 1) / chunk));
  if constexpr (CG > 8) {
    const dim3 wg(grid.x, (unsigned)((2 * CG + 3) / 4));  // two waves (half strips) per 16-row tile strip
    if (A == B)
      hipLaunchKernelGGL((k_gram_wide<CG, true>), wg, dim3(256), 0, s, A, B, ldg, l_pad, Wpart, chunk);
    else
      hipLaunchKernelGGL((k_gram_wide<CG, false>), wg, dim3(256), 0, s, A, B, ldg, l_pad, Wpart, chunk);
  } else if (A == B) {
    hipLaunchKernelGGL((k_gram<CG, true, kGramStep>), grid, dim3(kGramThreads), 0, s, A, B, ldg, l_pad, Wpart, chunk);
  } else {
    hipLaunchKernelGGL((k_gram<CG, false, kGramStep>), grid, dim3(kGramThreads), 0, s, A, B, ldg, l_pad, Wpart,
                       chunk);
  }
}

}  // namespace

int64_t gram_chunks(int64_t ldg) {
  const int64_t chunk = gram_chunk_cols(ldg);
  return (ldg + chunk - 1) / chunk;
}

hipError_t launch_gram(const double* A, const double* B, int l_pad, int64_t ldg, double* Wpart, double* W,
                       hipStream_t s) {
  if (ldg % kGramStep != 0) return hipErrorInvalidValue;
  switch (l_pad / 16) {
#define MDS_G(N) \
  case N: gram_one<N>(A, B, l_pad, ldg, Wpart, s); break;
    MDS_G(1) MDS_G(2) MDS_G(3) MDS_G(4) MDS_G(5) MDS_G(6) MDS_G(7) MDS_G(8)
    MDS_G(9) MDS_G(10) MDS_G(11) MDS_G(12) MDS_G(13) MDS_G(14) MDS_G(15) MDS_G(16)
#undef MDS_G
    default: return hipErrorInvalidValue;
  }
  const int64_t elems = (int64_t)l_pad * l_pad;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((elems + kSumEntries - 1) / kSumEntries)), dim3(256), 0, s, Wpart,
                     gram_chunks(ldg), elems, W, l_pad, A == B ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_apply(const double* In, int l, int64_t ldg, const double* T, int ldt, int lt, int l_pad,
                        double* Out, int xk, void* Xc, hipStream_t s) {
  constexpr int64_t kWide = 8 * 16 * 2, kNarrow = 4 * 16 * 1;  // columns i per workgroup
  if (l > kMaxL || l_pad > kMaxL || ldg % kWide != 0) return hipErrorInvalidValue;
  const int la = (l + 3) & ~3;
  const size_t shm = (size_t)la * kApRow * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    const int mx = (int)(kMaxL * kApRow * sizeof(double));
    (void)hipFuncSetAttribute((const void*)k_apply<2, 512>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)k_apply<1, 256>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    attr_set = true;
  }
  const int jb = (l_pad + kApJ - 1) / kApJ;
  const bool wide = ldg / kWide >= 128;
  const int gx = (int)(ldg / (wide ? kWide : kNarrow));
  const dim3 grid((unsigned)(((gx + 7) / 8) * 8 * jb));
  if (wide)
    hipLaunchKernelGGL((k_apply<2, 512>), grid, dim3(512), shm, s, In, l, ldg, T, ldt, lt, l_pad, Out, gx, jb);
  else
    hipLaunchKernelGGL((k_apply<1, 256>), grid, dim3(256), shm, s, In, l, ldg, T, ldt, lt, l_pad, Out, gx, jb);
  if (Xc) {
    // the cast copy in its own elementwise kernel (fewer registers in k_apply)
    const int64_t elems = (int64_t)l_pad * ldg;
    const dim3 cg((unsigned)((elems / 4 + 255) / 256));
    if (xk == GK_F64)
      hipLaunchKernelGGL(k_cast<GK_F64>, cg, dim3(256), 0, s, Out, elems, ldg, Xc);
    else if (xk == GK_F32)
      hipLaunchKernelGGL(k_cast<GK_F32>, cg, dim3(256), 0, s, Out, elems, ldg, Xc);
    else if (xk == GK_BF16)
      hipLaunchKernelGGL(k_cast<GK_BF16>, cg, dim3(256), 0, s, Out, elems, ldg, Xc);
    else if (xk == GK_F32S && ldg % 32 == 0)
      hipLaunchKernelGGL(k_cast<GK_F32S>, cg, dim3(256), 0, s, Out, elems, ldg, Xc);
    else
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int64_t coords_anchor_chunks(int64_t n) { return (n + kAnchorChunk - 1) / kAnchorChunk; }

hipError_t launch_coords(const double* Qt, int l, int64_t n, int64_t ldg, const double* Tc, int k, double* Ct,
                         double* coords, double* sign_part, int64_t* idx_part, hipStream_t s) {
  if (l > kMaxL || k > l) return hipErrorInvalidValue;
  const int k_pad = (k + 15) & ~15;
  hipError_t e = launch_apply(Qt, l, ldg, Tc, k, k, k_pad, Ct, -1, nullptr, s);
  if (e != hipSuccess) return e;
  const int64_t nch = coords_anchor_chunks(n);
  hipLaunchKernelGGL(k_anchor_part, dim3((unsigned)nch, (unsigned)k), dim3(256), 0, s, Ct, n, ldg, sign_part,
                     idx_part, nch);
  double* sign = sign_part + nch * k;
  hipLaunchKernelGGL(k_sign_anchor, dim3((unsigned)k), dim3(64), 0, s, sign_part, idx_part, nch, sign);
  hipLaunchKernelGGL(k_coords_write, dim3((unsigned)((n + 63) / 64), (unsigned)((k + 15) / 16)), dim3(256), 0, s,
                     Ct, n, ldg, k, sign, coords);
  return hipGetLastError();
}

}  // namespace mds
