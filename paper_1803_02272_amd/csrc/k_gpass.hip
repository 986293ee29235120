// G-pass: Y = G X for the randomized range finder and the projection
// (Sec. 3.2-3.3; every power iteration and the final Q^T (G Q) need one
// product of the n x n Gram matrix with an n x l tall matrix).
//
// This is the bandwidth-dominant kernel of the method: each pass streams all
// of G from HBM once while X is small and reused.  Design for gfx950:
//   * MFMA 16x16 tiles: bf16 (16x16x32, fp32 accumulate), fp32 (16x16x4),
//     fp64 (16x16x4).  Both operands are contiguous in K because G is
//     row-major and X is stored transposed (l_pad x ldg).
//   * A workgroup (4 waves) owns BM = 64 * RG rows of G and *all* l_pad
//     columns of Y, so each G byte is loaded exactly once per pass.  Each wave
//     streams its RG x 16 rows of G straight from HBM into MFMA A-operand
//     registers (16 bytes per lane, one full 128-byte line per row per step),
//     prefetching one step ahead.
//   * The X tile of a step (l_pad x 128 bytes) is shared by the four waves
//     through double-buffered LDS (rows padded to 144 bytes: conflict-free
//     ds_read_b128 for the B operand).
//   * Split-K with a deterministic fixed-order reduction (no atomics).  The
//     split index is blockIdx % split: with split a multiple of 8, every
//     workgroup on an XCD works on the same K range, so that XCD's slice of X
//     stays in its own L2 while G streams past.
//   * Symmetric mode (projection pass only, B = Q^T G Q): G is symmetric, so
//     B = S + S^T with S = Q^T Z and Z = W o G Q, where W weights the strict
//     upper triangle by 1, the diagonal by 1/2 and the lower triangle by 0.
//     Only the upper triangle of G is streamed: half the bytes and half the
//     MFMA work of a full pass.  The kernel writes 2Z (weights 2 / 1 / 0,
//     exact power-of-two scaling), so that the usual symmetrisation
//     1/2 (B + B^T) of B = Q^T (2Z) gives S + S^T.  Work item (row block,
//     K split) covers the split's K range clipped to the columns at or right
//     of the block's first row; row blocks are dealt to XCDs round-robin
//     (block mb on XCD mb % 8), which spreads the triangle evenly over the
//     XCDs, and inside an XCD the split index varies slowest so that
//     concurrently running workgroups share their slice of X in L2.
#include <type_traits>

#include "mds_internal.h"

namespace mds {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int GK>
struct Tr;

template <>
struct Tr<GK_BF16> {
  using T = bf16_t;   // stored G element
  using XT = bf16_t;  // X operand element
  using Acc = floatx4_t;
  using AccS = float;
  static constexpr int kSub = 1;  // MFMAs per 16-byte operand chunk
  static __device__ __forceinline__ void mma_sub(Acc& c, const u32x4& a, const u32x4& b, int) { mma(c, a, b); }
  static __device__ __forceinline__ void mma(Acc& c, const u32x4& a, const u32x4& b) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }
};

template <>
struct Tr<GK_F32> {
  using T = float;
  using XT = float;
  using Acc = floatx4_t;
  using AccS = float;
  // one 16-byte chunk holds 4 K-values per lane: four K=4 MFMAs, the t-th
  // taking element t of every lane group (same K pairing for A and B)
  static constexpr int kSub = 4;
  static __device__ __forceinline__ void mma_sub(Acc& c, const u32x4& a, const u32x4& b, int t) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[t]), __uint_as_float(b[t]), c, 0, 0, 0);
  }
  static __device__ __forceinline__ void mma(Acc& c, const u32x4& a, const u32x4& b) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
  }
};

template <>
struct Tr<GK_F64> {
  using T = double;
  using XT = double;
  using Acc = doublex4_t;
  using AccS = double;
  static constexpr int kSub = 2;
  static __device__ __forceinline__ void mma_sub(Acc& c, const u32x4& a, const u32x4& b, int t) {
    const double av = t == 0 ? __hiloint2double((int)a.y, (int)a.x) : __hiloint2double((int)a.w, (int)a.z);
    const double bv = t == 0 ? __hiloint2double((int)b.y, (int)b.x) : __hiloint2double((int)b.w, (int)b.z);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void mma(Acc& c, const u32x4& a, const u32x4& b) {
    const double a0 = __hiloint2double((int)a.y, (int)a.x), a1 = __hiloint2double((int)a.w, (int)a.z);
    const double b0 = __hiloint2double((int)b.y, (int)b.x), b1 = __hiloint2double((int)b.w, (int)b.z);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c, 0, 0, 0);
  }
};

// FP8: E4M3 codes, decoded and scaled into bf16 A operands (X is bf16).
template <>
struct Tr<GK_FP8> {
  using T = uint8_t;
  using XT = bf16_t;
  using Acc = floatx4_t;
  using AccS = float;
  static constexpr int kSub = 1;
  static __device__ __forceinline__ void mma_sub(Acc& c, const u32x4& a, const u32x4& b, int) { mma(c, a, b); }
  static __device__ __forceinline__ void mma(Acc& c, const u32x4& a, const u32x4& b) {
    Tr<GK_BF16>::mma(c, a, b);
  }
};

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v_t __attribute__((ext_vector_type(2)));

// Two floats rounded to nearest even into packed bf16 (one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t bf16x2_bits(f32x2 v) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v_t));
}

constexpr int kRowB = 144;  // LDS bytes per X row within a step tile

// 16-row groups per wave, chosen so accumulators + prefetched A operands fit
// the register file at two workgroups per CU without spilling.
__host__ __device__ constexpr int rg_for(int gk, int cg) {
  if (gk == GK_F64) return cg <= 3 ? 4 : (cg <= 7 ? 2 : 1);
  if (gk == GK_FP8) return cg <= 8 ? 4 : 2;  // the E4M3 decode needs a few more registers than bf16
  return cg <= 8 ? 4 : 2;
}
// Recentring passes hold raw D values and recentring terms in registers as
// well; fewer row groups keep two workgroups per CU.
__host__ __device__ constexpr int rg_fd(int gk, int cg, bool d8) {
  if (gk == GK_F64) return cg <= 3 ? 2 : 1;
  if (gk == GK_BF16) return cg <= 8 ? 2 : 1;  // fused write-and-pass: 8 raw D values per chunk
  return cg <= (d8 ? 2 : 4) ? 4 : (cg <= 8 ? 2 : 1);  // fp32; fp64 D doubles the raw values
}
__host__ __device__ constexpr int minb_for(int gk, int cg) { return (gk == GK_F64 && cg >= 12) ? 1 : 2; }

// Element type of D when the A operand is recentred on the fly (void: G is stored).
template <typename DT>
struct DLoad {
  static constexpr bool kFromD = true;
};
template <>
struct DLoad<void> {
  static constexpr bool kFromD = false;
};

template <int GK, typename DT>
__host__ __device__ constexpr int minb_of(int cg) {
  // fp64 recentring passes with l_pad > 144 need more than 256 registers
  return DLoad<DT>::kFromD ? ((GK == GK_F64 && cg >= 10) ? 1 : 2) : minb_for(GK, cg);
}

// E consecutive elements of row i of D starting at column k0 (k0 % E == 0),
// zero outside the n x n matrix; vector loads when the row start is aligned.
template <typename DT, int E>
__device__ __forceinline__ void load_d(const DT* __restrict__ D, int64_t n, int64_t i, int64_t k0, bool rowvec,
                                       DT (&v)[E]) {
  const DT* p = D + i * n + k0;
  if (i < n && rowvec && k0 + E - 1 < n) {
    if constexpr (sizeof(DT) * E == 16) {
      const u32x4 w = *reinterpret_cast<const u32x4*>(p);
      __builtin_memcpy(&v, &w, 16);
    } else if constexpr (sizeof(DT) * E == 32) {
      const u32x4 w0 = *reinterpret_cast<const u32x4*>(p);
      const u32x4 w1 = *reinterpret_cast<const u32x4*>(p + E / 2);
      __builtin_memcpy(&v, &w0, 16);
      __builtin_memcpy(reinterpret_cast<char*>(&v) + 16, &w1, 16);
    } else if constexpr (sizeof(DT) * E == 64) {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const u32x4 w = *reinterpret_cast<const u32x4*>(p + h * (E / 4));
        __builtin_memcpy(reinterpret_cast<char*>(&v) + 16 * h, &w, 16);
      }
    } else {  // 8 bytes
      const uint2 w = *reinterpret_cast<const uint2*>(p);
      __builtin_memcpy(&v, &w, 8);
    }
  } else {
#pragma unroll
    for (int t = 0; t < E; ++t) v[t] = (i < n && k0 + t < n) ? p[t] : (DT)0;
  }
}

template <int GK, int RG, int CG, typename DT, bool SYM>
__global__ __launch_bounds__(256, (minb_of<GK, DT>(CG))) void k_gpass(
    const typename Tr<GK>::T* __restrict__ G, int64_t ldg, const typename Tr<GK>::XT* __restrict__ Xt, int split,
    int64_t steps_total, int64_t steps_per_split, typename Tr<GK>::AccS* __restrict__ Ypart, GPassDSrc src,
    int64_t sym_nbx) {
  using TT = Tr<GK>;
  using T = typename TT::T;
  using XT = typename TT::XT;
  using Acc = typename TT::Acc;
  using AccS = typename TT::AccS;
  constexpr bool FD = DLoad<DT>::kFromD;
  constexpr bool F8 = GK == GK_FP8;
  using RawT = typename std::conditional<FD, DT, T>::type;
  constexpr int E = 16 / sizeof(XT);  // A elements per lane per chunk (one 16-byte B operand)
  constexpr int AB = E * sizeof(T);   // stored-G bytes per lane per chunk
  constexpr int LPAD = CG * 16;
  constexpr int PIECES = LPAD * 8;  // 16-byte pieces per X step tile
  constexpr int PPT = (PIECES + 255) / 256;
  constexpr int BK = 128 / sizeof(XT);  // K elements per step (a 128-byte row of the X tile)
  __shared__ __attribute__((aligned(16))) unsigned char xs[2][LPAD * kRowB];
  // fused write-and-pass: the step's c_k (fp64) staged with the X tile
  __shared__ __attribute__((aligned(16))) double cs[(FD && GK == GK_BF16) ? 2 : 1][(FD && GK == GK_BF16) ? BK : 1];

  static_assert(!SYM || DLoad<DT>::kFromD, "symmetric mode recentres D on the fly");
  constexpr int64_t kStepsPerBlock = (64 * RG) / BK;  // K steps spanned by one row block
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t bid = blockIdx.x;
  int s;
  int64_t mb, st0, st1;
  if constexpr (SYM) {
    const int64_t loc = bid >> 3;
    s = (int)(loc / sym_nbx);
    mb = (loc % sym_nbx) * 8 + (bid & 7);
    const int64_t diag0 = mb * kStepsPerBlock;  // first step at or right of the diagonal
    st0 = (int64_t)s * steps_per_split;
    st1 = (st0 + steps_per_split < steps_total) ? st0 + steps_per_split : steps_total;
    if (diag0 > st0) st0 = diag0;
    if (diag0 >= steps_total || st0 >= st1) return;  // empty item: no partial written (the reduce skips it)
  } else {
    s = (int)(bid % split);
    mb = bid / split;
    st0 = (int64_t)s * steps_per_split;
    st1 = (st0 + steps_per_split < steps_total) ? st0 + steps_per_split : steps_total;
  }
  const int64_t diag_end = (mb + 1) * kStepsPerBlock;  // steps below this cross the diagonal (SYM)
  const int64_t row0 = mb * (64 * RG) + (int64_t)wave * (RG * 16);

  Acc acc[RG][CG];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int cg = 0; cg < CG; ++cg)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[rg][cg][e] = 0;

  const size_t rowbytes = (size_t)ldg * sizeof(T);    // stored G
  const size_t xrowbytes = (size_t)ldg * sizeof(XT);  // X
  const unsigned char* Ab =
      reinterpret_cast<const unsigned char*>(G) + (size_t)(row0 + (lane & 15)) * rowbytes + (lane >> 4) * AB;
  const size_t rg_stride = 16 * rowbytes;
  const unsigned char* Xb = reinterpret_cast<const unsigned char*>(Xt);
  const int64_t f8_row_block = F8 ? (mb * (64 * RG)) / kF8Block : 0;

  // recentring state (only used when FD).  CT: precision of the recentring
  // terms (fp32 passes use fl32(c/2) and fl32((r - m)/2), fp64 passes and the
  // fused bf16 write-and-pass c, r, m in fp64).
  using CT = typename std::conditional<sizeof(T) == 4, float, double>::type;
  // Fused centring write: a bf16 pass from D stores the bf16 A operands it
  // computes, i.e. writes G (bf16 of fl32 of the fp64 gamma) while taking the
  // first range pass, so that pass does not read G back.
  constexpr bool WG = FD && GK == GK_BF16;
  T* Gw = const_cast<T*>(G);
  const DT* Dp = reinterpret_cast<const DT*>(src.D);
  const int64_t n = src.n;
  CT ri[RG];
  bool rowvec[RG];
  double mval = 0.0;
  if constexpr (FD) {
    mval = src.m[0];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg) {
      const int64_t i = row0 + rg * 16 + (lane & 15);
      if constexpr (sizeof(T) == 4)
        ri[rg] = (i < n) ? (float)(0.5 * (src.r[i] - mval)) : 0.0f;
      else
        ri[rg] = (i < n) ? src.r[i] : 0.0;
      rowvec[rg] = src.vec && (((i * n) % E) == 0);
    }
  }

  if (st0 < st1) {
    RawT a[RG][2][E], an[RG][2][E];
    CT cv[2][E], cvn[2][E];
    u32x4 xr[PPT];
    auto load_a = [&](RawT (&dst)[RG][2][E], CT (&cdst)[2][E], int64_t st) {
      if constexpr (FD) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int64_t k0 = st * BK + c * (BK / 2) + (lane >> 4) * E;
#pragma unroll
          for (int rg = 0; rg < RG; ++rg)
            load_d<DT, E>(Dp, n, row0 + rg * 16 + (lane & 15), k0, rowvec[rg], dst[rg][c]);
          if constexpr (sizeof(T) == 4) {
            // hc holds ldg zero-padded entries: one aligned 16-byte load
            const u32x4 w = *reinterpret_cast<const u32x4*>(src.hc + k0);
            __builtin_memcpy(&cdst[c], &w, 16);
          } else if constexpr (!WG) {
#pragma unroll
            for (int t = 0; t < E; ++t) cdst[c][t] = (k0 + t < n) ? src.c[k0 + t] : 0.0;
          }
        }
      } else {
#pragma unroll
        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const unsigned char* p = Ab + rg * rg_stride + (size_t)st * (BK * sizeof(T)) + c * (BK / 2 * sizeof(T));
            if constexpr (AB == 16) {
              const u32x4 w = *reinterpret_cast<const u32x4*>(p);
              __builtin_memcpy(&dst[rg][c], &w, 16);
            } else {
              const uint2 w = *reinterpret_cast<const uint2*>(p);
              __builtin_memcpy(&dst[rg][c], &w, 8);
            }
          }
      }
    };
    double2 xc = make_double2(0.0, 0.0);  // WG: this thread's two c_k of the step
    auto load_x = [&](int64_t st) {
      if constexpr (WG) {
        if (tid < BK / 2) {
          const int64_t k = st * BK + 2 * tid;
          xc = make_double2(k < n ? src.c[k] : 0.0, k + 1 < n ? src.c[k + 1] : 0.0);
        }
      }
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int p = tid + 256 * u;
        if (PIECES % 256 == 0 || p < PIECES)
          xr[u] = *reinterpret_cast<const u32x4*>(Xb + (size_t)(p >> 3) * xrowbytes + (size_t)st * 128 +
                                                  (p & 7) * 16);
      }
    };
    auto store_x = [&](unsigned char* buf) {
      if constexpr (WG) {
        if (tid < BK / 2) *reinterpret_cast<double2*>(&cs[buf == xs[0] ? 0 : 1][2 * tid]) = xc;
      }
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int p = tid + 256 * u;
        if (PIECES % 256 == 0 || p < PIECES)
          *reinterpret_cast<u32x4*>(buf + (p >> 3) * kRowB + (p & 7) * 16) = xr[u];
      }
    };
    // A operand of one chunk in MFMA register form.  Recentring mode, fp64:
    // gamma = -1/2 (((d^2 - c_k) - r_i) + m); fp32: gamma = fma(-1/2,
    // fl32(d^2), hc_k + hr_i) (one fma per entry instead of fp64 arithmetic).
    // Symmetric mode: 2 gamma (the same roundings scaled by 2, exactly),
    // times 1, 1/2, 0 right of, on and left of the diagonal.
    auto a_operand = [&](int rg, int c, int64_t st, const double* cl, const RawT (&a)[RG][2][E],
                         const CT (&cv)[2][E]) -> u32x4 {
      if constexpr (FD && GK == GK_BF16) {
        // fused centring write: bf16(fl32(gamma)) with gamma in fp64 (no
        // symmetric mode here), rounded two at a time
#pragma clang fp contract(off)
        const int64_t k0 = st * BK + c * (BK / 2) + (lane >> 4) * E;
        const int64_t i = row0 + rg * 16 + (lane & 15);
        float f[E];
#pragma unroll
        for (int t = 0; t < E; ++t) {
          const double d = (double)a[rg][c][t];
          const double e = ((d * d - cl[c * (BK / 2) + (lane >> 4) * E + t]) - ri[rg]) + mval;
          f[t] = (i < n && k0 + t < n) ? (float)(-0.5 * e) : 0.0f;
        }
        u32x4 w;
#pragma unroll
        for (int h = 0; h < E / 2; ++h) w[h] = bf16x2_bits(f32x2{f[2 * h], f[2 * h + 1]});
        return w;
      } else if constexpr (FD) {
#pragma clang fp contract(off)
        const int64_t k0 = st * BK + c * (BK / 2) + (lane >> 4) * E;
        const int64_t i = row0 + rg * 16 + (lane & 15);
        const bool band = SYM && st < diag_end;
        T g[E];
#pragma unroll
        for (int t = 0; t < E; ++t) {
          const bool valid = (i < n) && (k0 + t < n);
          T v;
          if constexpr (sizeof(T) == 4) {
            float d2;
            if constexpr (sizeof(DT) == 4) {
              const float d = a[rg][c][t];
              d2 = d * d;
            } else {
              const double d = a[rg][c][t];
              d2 = (float)(d * d);
            }
            const float h = cv[c][t] + ri[rg];
            v = SYM ? __builtin_fmaf(-1.0f, d2, h + h) : __builtin_fmaf(-0.5f, d2, h);
          } else {
            const double d = (double)a[rg][c][t];
            const double e = ((d * d - cv[c][t]) - ri[rg]) + mval;
            v = SYM ? -e : -0.5 * e;
          }
          if (band) {
            const int64_t j = k0 + t;
            v = j > i ? v : (j == i ? (T)0.5 * v : (T)0);
          }
          g[t] = valid ? v : (T)0;
        }
        u32x4 w;
        __builtin_memcpy(&w, &g, 16);
        return w;
      } else if constexpr (F8) {
        const float sc = src.g8_scales[f8_row_block * src.g8_nsb + (st * BK) / kF8Block];
        uint32_t cw[2];
        __builtin_memcpy(cw, &a[rg][c], 8);
        u32x4 w;
        // hardware E4M3 decode (OCP, two codes per instruction), scale in
        // fp32, round to bf16: element t of the chunk is byte t
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)cw[h], false);  // bytes 0, 1
          const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)cw[h], true);   // bytes 2, 3
          w[2 * h] = bf16x2_bits(lo * sc);
          w[2 * h + 1] = bf16x2_bits(hi * sc);
        }
        return w;
      } else {
        u32x4 w;
        __builtin_memcpy(&w, &a[rg][c], 16);
        return w;
      }
    };

    // One step: the operands of step st are in (ac, cc) and xs[buf]; the
    // loads of step st + 1 go to (an_, cn_) and the other LDS buffer.  The
    // prefetch is issued on every step (the last step re-loads step st1 - 1
    // into buffers that are not read again) and the two register sets swap
    // roles from one step to the next, so that the loads of step st + 1 stay
    // in flight during all of step st: no conditional loads or register
    // copies for the compiler's wait counts to merge.
    auto step = [&](int64_t st, int buf, RawT (&ac)[RG][2][E], CT (&cc)[2][E], RawT (&an_)[RG][2][E],
                    CT (&cn_)[2][E]) {
      const int64_t stn = st + 1 < st1 ? st + 1 : st1 - 1;
      load_x(stn);
      load_a(an_, cn_, stn);
      // keep the prefetch at the top of the step (the scheduler would sink it
      // towards its uses at the end of the step, leaving nothing in flight)
      __builtin_amdgcn_sched_barrier(0);
      const unsigned char* xb = xs[buf];
      const double* cl = cs[WG ? buf : 0];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        u32x4 av[RG];
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) av[rg] = a_operand(rg, c, st, cl, ac, cc);
        if constexpr (WG) {
#pragma unroll
          for (int rg = 0; rg < RG; ++rg)
            *reinterpret_cast<u32x4*>(Gw + (row0 + rg * 16 + (lane & 15)) * ldg + st * BK + c * (BK / 2) +
                                      (lane >> 4) * E) = av[rg];
        }
#pragma unroll
        for (int cg = 0; cg < CG; ++cg) {
          const u32x4 b =
              *reinterpret_cast<const u32x4*>(xb + (cg * 16 + (lane & 15)) * kRowB + c * 64 + (lane >> 4) * 16);
          // consecutive MFMAs go to independent accumulators (row groups)
#pragma unroll
          for (int t = 0; t < TT::kSub; ++t)
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) TT::mma_sub(acc[rg][cg], av[rg], b, t);
        }
      }
      store_x(xs[buf ^ 1]);
      __syncthreads();
    };

    load_a(a, cv, st0);
    load_x(st0);
    store_x(xs[0]);
    __syncthreads();
    for (int64_t st = st0; st < st1; st += 2) {
      step(st, 0, a, cv, an, cvn);
      if (st + 1 < st1) step(st + 1, 1, an, cvn, a, cv);
    }
  }

  // C layout of a 16x16 MFMA tile (measured on gfx950): column l%16; the
  // four accumulator registers of lane group g = l/16 hold rows 4g..4g+3 for
  // the fp32-accumulating instructions and rows g, g+4, g+8, g+12 for fp64.
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
      const int col = cg * 16 + (lane & 15);
      AccS* dst = Ypart + ((int64_t)s * LPAD + col) * ldg + row0 + rg * 16;
      if constexpr (sizeof(AccS) == 4) {
        *reinterpret_cast<float4*>(dst + 4 * (lane >> 4)) =
            make_float4(acc[rg][cg][0], acc[rg][cg][1], acc[rg][cg][2], acc[rg][cg][3]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[(lane >> 4) + 4 * r] = acc[rg][cg][r];
      }
    }
  }
}

// ---- fp32 passes on bf16 MFMA: three-term split ----------------------------
// An fp32 value a is the exact sum a0 + a1 + a2 of three bf16 values:
// a0 = bf16(a), a1 = bf16(a - a0), a2 = (a - a0) - a1, rounding to nearest
// even; both differences are exact in fp32 and a2 has at most 8 significant
// bits.  With |a1| <= 2^-8 |a| and |a2| <= 2^-16 |a| (normal range), the six
// products a_p b_q with p + q <= 2 leave out terms below 2^-22 |a b|, about
// one fp32 rounding of the product, so this pass computes the fp32 pass's
// Y = G X (fp32 operands fl32(gamma) and fl32(x), fp32 accumulation) to fp32
// accuracy.  Per 32 K-values and 16 x 16 tile: six bf16 MFMAs (16x16x32,
// 16 cycles) instead of eight fp32 ones (16x16x4, 32 cycles).
//
// X is stored split (written by the cast after the orthonormalisation): row
// j of the transposed operand holds, per 32 consecutive K-values, the 32
// bf16 a0 terms, then the a1 terms, then the a2 terms (192 bytes).  A step
// covers 32 K-values: each lane recentres 8 consecutive entries of D per row
// group (one 128-byte line per row and step), splits them in registers, and
// meets the three 16-byte B pieces of its K-group from the LDS step tile.
constexpr int kX3Step = 32;           // K-values per step
constexpr int kX3RowB = 3 * 64 + 16;  // LDS bytes per X row of a step tile: 3 planes + pad (conflict-free reads)

__host__ __device__ constexpr int rg_x3(int cg, bool d8) { return cg <= (d8 ? 6 : 8) ? 2 : 1; }

// Three-term split of 8 floats into the bf16 planes w[0..2] (element t at
// halfword t of each plane).
__device__ __forceinline__ void split3(const float (&g)[8], u32x4 (&w)[3]) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const f32x2 v = {g[2 * h], g[2 * h + 1]};
    const bf16x2v_t v0 = __builtin_convertvector(v, bf16x2v_t);
    const f32x2 r1 = v - __builtin_convertvector(v0, f32x2);
    const bf16x2v_t v1 = __builtin_convertvector(r1, bf16x2v_t);
    const f32x2 r2 = r1 - __builtin_convertvector(v1, f32x2);
    const bf16x2v_t v2 = __builtin_convertvector(r2, bf16x2v_t);
    w[0][h] = __builtin_bit_cast(uint32_t, v0);
    w[1][h] = __builtin_bit_cast(uint32_t, v1);
    w[2][h] = __builtin_bit_cast(uint32_t, v2);
  }
}

// WG: the fused centring write (fp32 D, full pass): each entry is recentred
// in fp64 as in the centring equation, g = fl32(gamma) is stored into the
// bf16 G as bf16(g) (the stored-G value of the bf16 form) and split for the
// pass, so that the first range pass takes fl32(gamma) itself.
// NT, NTB: terms of the G and X operands (3, 3: six products, fp32
// accuracy; 2, 2: three products a1 b0 + a0 b1 + a0 b0, the 16-bit sketch
// of Omega and projection; 2, 1: two products a1 b0 + a0 b0, each exact in
// fp32, the last 16-bit range pass).
template <int RG, int CG, typename DT, bool SYM, bool WG = false, int NT = 3, int NTB = 3>
__global__ __launch_bounds__(256, 2) void k_gpass_x3(const uint16_t* __restrict__ X3, int64_t ldg, int split,
                                                     int64_t steps_total, int64_t steps_per_split,
                                                     float* __restrict__ Ypart, GPassDSrc src, int64_t sym_nbx,
                                                     uint16_t* __restrict__ Gw) {
  static_assert(!WG || (!SYM && sizeof(DT) == 4), "the fused write is a full pass over fp32 D");
  constexpr int LPAD = CG * 16;
  constexpr int BK = kX3Step;
  constexpr int PIECES = LPAD * 12;  // 16-byte pieces of a step's X tile (3 planes x 4 K-groups per row)
  constexpr int PPT = (PIECES + 255) / 256;
  constexpr int64_t kStepsPerBlock = (64 * RG) / BK;
  constexpr int DV = 16 / (int)sizeof(DT);  // row alignment (elements) for 16-byte loads of D
  __shared__ __attribute__((aligned(16))) unsigned char xs[2][LPAD * kX3RowB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t bid = blockIdx.x;
  int s;
  int64_t mb, st0, st1;
  if constexpr (SYM) {  // same work items as the symmetric k_gpass
    const int64_t loc = bid >> 3;
    s = (int)(loc / sym_nbx);
    mb = (loc % sym_nbx) * 8 + (bid & 7);
    const int64_t diag0 = mb * kStepsPerBlock;
    st0 = (int64_t)s * steps_per_split;
    st1 = (st0 + steps_per_split < steps_total) ? st0 + steps_per_split : steps_total;
    if (diag0 > st0) st0 = diag0;
    if (diag0 >= steps_total || st0 >= st1) return;
  } else {
    s = (int)(bid % split);
    mb = bid / split;
    st0 = (int64_t)s * steps_per_split;
    st1 = (st0 + steps_per_split < steps_total) ? st0 + steps_per_split : steps_total;
  }
  const int64_t diag_end = (mb + 1) * kStepsPerBlock;
  const int64_t row0 = mb * (64 * RG) + (int64_t)wave * (RG * 16);

  floatx4_t acc[RG][CG];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int cg = 0; cg < CG; ++cg)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[rg][cg][e] = 0.0f;

  const DT* Dp = reinterpret_cast<const DT*>(src.D);
  const int64_t n = src.n;
  const double mval = src.m[0];
  float ri[RG];  // hr_i (symmetric mode: 2 hr_i, exact)
  double rd[RG];  // WG: (r_i - m) / 2 in fp64
  bool rowvec[RG];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) {
    const int64_t i = row0 + rg * 16 + (lane & 15);
    const float h = (i < n) ? (float)(0.5 * (src.r[i] - mval)) : 0.0f;
    ri[rg] = SYM ? h + h : h;
    rd[rg] = (WG && i < n) ? 0.5 * (src.r[i] - mval) : 0.0;
    rowvec[rg] = src.vec && (((i * n) % DV) == 0);
  }
  const size_t xrowbytes = (size_t)ldg * 6;
  const unsigned char* Xb = reinterpret_cast<const unsigned char*>(X3);
  // recentring terms per K-value: fl32(c_k / 2), or c_k in fp64 for the fused write
  using CVT = typename std::conditional<WG, double, float>::type;

  if (st0 < st1) {
    DT a[RG][8], an[RG][8];
    CVT cv[8], cvn[8];
    u32x4 xr[PPT];
    auto load_a = [&](DT (&dst)[RG][8], CVT (&cdst)[8], int64_t st) {
      const int64_t k0 = st * BK + (lane >> 4) * 8;
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) load_d<DT, 8>(Dp, n, row0 + rg * 16 + (lane & 15), k0, rowvec[rg], dst[rg]);
      if constexpr (WG) {
#pragma unroll
        for (int t = 0; t < 8; ++t) cdst[t] = (k0 + t < n) ? src.c[k0 + t] : 0.0;
      } else {
        // hc holds ldg zero-padded entries (ldg is a multiple of 32)
        const u32x4 w0 = *reinterpret_cast<const u32x4*>(src.hc + k0);
        const u32x4 w1 = *reinterpret_cast<const u32x4*>(src.hc + k0 + 4);
        __builtin_memcpy(&cdst[0], &w0, 16);
        __builtin_memcpy(&cdst[4], &w1, 16);
      }
    };
    auto load_x = [&](int64_t st) {
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int p = tid + 256 * u;
        if (PIECES % 256 == 0 || p < PIECES)
          xr[u] = *reinterpret_cast<const u32x4*>(Xb + (size_t)(p / 12) * xrowbytes + (size_t)st * 192 +
                                                  (p % 12) * 16);
      }
    };
    auto store_x = [&](unsigned char* buf) {
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int p = tid + 256 * u;
        if (PIECES % 256 == 0 || p < PIECES) *reinterpret_cast<u32x4*>(buf + (p / 12) * kX3RowB + (p % 12) * 16) = xr[u];
      }
    };
    // gamma = fma(-1/2, fl32(d^2), hc_k + hr_i) as in the fp32 pass
    // (symmetric mode: 2 gamma = fma(-1, fl32(d^2), 2 hc_k + 2 hr_i), the same
    // roundings scaled by 2, times 1, 1/2, 0 right of, on and left of the
    // diagonal), then split into three bf16 planes.  Entries outside n x n
    // need no mask: columns k >= n meet zero rows of X (the padding of Q),
    // and rows i >= n are zeroed in the output.
    auto a_split = [&](int rg, const CVT (&ch)[8], auto band_tag, int64_t st, u32x4 (&w)[3]) {
#pragma clang fp contract(off)
      constexpr bool BAND = decltype(band_tag)::value;
      float g[8];
      if constexpr (WG) {
        // gamma = 1/2 (c_k - d^2) + (r_i - m) / 2 in fp64 as two fused
        // operations (the LDS-ring kernel's expression), g = fl32(gamma),
        // zero outside n x n; bf16(g) is the stored G entry
        const int64_t k0 = st * BK + (lane >> 4) * 8;
        const int64_t i = row0 + rg * 16 + (lane & 15);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const double d = (double)a[rg][t];
          const double e = __builtin_fma(-d, d, ch[t]);
          g[t] = (i < n && k0 + t < n) ? (float)__builtin_fma(0.5, e, rd[rg]) : 0.0f;
        }
        u32x4 gw;
#pragma unroll
        for (int h = 0; h < 4; ++h) gw[h] = bf16x2_bits(f32x2{g[2 * h], g[2 * h + 1]});
        *reinterpret_cast<u32x4*>(Gw + i * ldg + k0) = gw;
        split3(g, w);
        return;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        float d2;
        if constexpr (sizeof(DT) == 4) {
          const float d = a[rg][t];
          d2 = d * d;
        } else {
          const double d = a[rg][t];
          d2 = (float)(d * d);
        }
        float v = __builtin_fmaf(SYM ? -1.0f : -0.5f, d2, ch[t] + ri[rg]);
        if constexpr (BAND) {
          const int64_t j = st * BK + (lane >> 4) * 8 + t;
          const int64_t i = row0 + rg * 16 + (lane & 15);
          v = j > i ? v : (j == i ? 0.5f * v : 0.0f);
        }
        g[t] = v;
      }
      split3(g, w);
    };

    load_a(a, cv, st0);
    load_x(st0);
    store_x(xs[0]);
    __syncthreads();
    for (int64_t st = st0; st < st1; ++st) {
      const int buf = (int)((st - st0) & 1);
      const bool more = st + 1 < st1;
      if (more) {
        load_x(st + 1);
        load_a(an, cvn, st + 1);
      }
      u32x4 w[RG][3];
      CVT ch[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) ch[t] = SYM ? cv[t] + cv[t] : cv[t];
      if (SYM && st < diag_end) {
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) a_split(rg, ch, std::true_type{}, st, w[rg]);
      } else {
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) a_split(rg, ch, std::false_type{}, st, w[rg]);
      }
      const unsigned char* xb = xs[buf];
#pragma unroll
      for (int cg0 = 0; cg0 < CG; cg0 += 2) {
        constexpr int NP = 2;
        u32x4 bb[NP][3];
#pragma unroll
        for (int h = 0; h < NP; ++h)
          if (cg0 + h < CG) {
            const unsigned char* bp = xb + ((cg0 + h) * 16 + (lane & 15)) * kX3RowB + (lane >> 4) * 16;
            bb[h][0] = *reinterpret_cast<const u32x4*>(bp);
            bb[h][1] = *reinterpret_cast<const u32x4*>(bp + 64);
            bb[h][2] = *reinterpret_cast<const u32x4*>(bp + 128);
          }
        // products smallest first: six for three terms, three or two for two
        constexpr int NPR = NT == 3 ? 6 : (NTB == 2 ? 3 : 2);
        constexpr int PA[6] = {NT == 3 ? 2 : 1, NT == 3 ? 1 : 0, 0, 1, 0, 0};
        constexpr int PB[6] = {0, NTB >= 2 ? 1 : 0, NT == 3 ? 2 : 0, 0, 1, 0};
#pragma unroll
        for (int pr = 0; pr < NPR; ++pr)
#pragma unroll
          for (int h = 0; h < NP; ++h)
            if (cg0 + h < CG)
#pragma unroll
              for (int rg = 0; rg < RG; ++rg) Tr<GK_BF16>::mma(acc[rg][cg0 + h], w[rg][PA[pr]], bb[h][PB[pr]]);
      }
      if (more) store_x(xs[buf ^ 1]);
      __syncthreads();
      if (more) {
#pragma unroll
        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
          for (int t = 0; t < 8; ++t) a[rg][t] = an[rg][t];
#pragma unroll
        for (int t = 0; t < 8; ++t) cv[t] = cvn[t];
      }
    }
  }

#pragma unroll
  for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
      const int col = cg * 16 + (lane & 15);
      float* dst = Ypart + ((int64_t)s * LPAD + col) * ldg + row0 + rg * 16;
      const int64_t i4 = row0 + rg * 16 + 4 * (lane >> 4);  // rows i4 .. i4+3 of this lane
      float4 o = make_float4(acc[rg][cg][0], acc[rg][cg][1], acc[rg][cg][2], acc[rg][cg][3]);
      if (i4 + 3 >= n) {
        o.x = i4 < n ? o.x : 0.0f;
        o.y = i4 + 1 < n ? o.y : 0.0f;
        o.z = i4 + 2 < n ? o.z : 0.0f;
        o.w = i4 + 3 < n ? o.w : 0.0f;
      }
      *reinterpret_cast<float4*>(dst + 4 * (lane >> 4)) = o;
    }
  }
}

// The split passes that stream D through LDS (fp32 D, n % 4 == 0, aligned D,
// l_pad <= 128 with three terms, <= 224 with two) run in k_split.hip: 8 waves
// of 2 row groups per workgroup.  The pass over the stored bf16 G streams
// up to l_pad = 224 as well (k_gstream).
constexpr int kDmaMaxL = 128, kDmaMaxL2 = 224;

// Symmetric mode: row block mb has partials only in the splits whose K
// range reaches its diagonal, k >= first_split(row) = (mb * bm) / cols_per_split.
template <typename AccS>
__global__ __launch_bounds__(256) void k_splitk_reduce(const AccS* __restrict__ Yp, int split, int64_t elems,
                                                       double* __restrict__ Y, int64_t ldg, int64_t sym_bm,
                                                       int64_t sym_cols_per_split) {
#pragma clang fp contract(off)
  const int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (e >= elems) return;  // elems is a multiple of 4
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int k0 = 0;
  if (sym_cols_per_split > 0) {
    const int64_t row = e % ldg;  // e..e+3 share the row block (ldg and bm are multiples of 4)
    k0 = (int)(((row / sym_bm) * sym_bm) / sym_cols_per_split);
  }
  // the four entries of a partial as one vector load (partials start on
  // 256-byte boundaries and e is a multiple of 4); four partials' loads are
  // issued before their sums, which still run in split order
  auto ld4 = [&](int k, double (&v)[4]) {
    const AccS* p = Yp + (int64_t)k * elems + e;
    if constexpr (sizeof(AccS) == 4) {
      const float4 f = *reinterpret_cast<const float4*>(p);
      v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
    } else {
      const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
  };
  int k = k0;
  for (; k + 4 <= split; k += 4) {
    double v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) ld4(k + u, v[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s0 += v[u][0];
      s1 += v[u][1];
      s2 += v[u][2];
      s3 += v[u][3];
    }
  }
  for (; k < split; ++k) {
    double v[4];
    ld4(k, v);
    s0 += v[0];
    s1 += v[1];
    s2 += v[2];
    s3 += v[3];
  }
  reinterpret_cast<double2*>(Y + e)[0] = make_double2(s0, s1);
  reinterpret_cast<double2*>(Y + e)[1] = make_double2(s2, s3);
}

template <int GK, int RG, int CG, typename DT, bool SYM>
void launch_one(const void* G, int64_t ldg, const void* Xt, const GPassCfg& cfg, int64_t n_pad, void* Yp,
                const GPassDSrc& src, hipStream_t s) {
  using T = typename Tr<GK>::T;
  using XT = typename Tr<GK>::XT;
  using AccS = typename Tr<GK>::AccS;
  const int64_t blocks = gpass_blocks(cfg, n_pad);
  hipLaunchKernelGGL((k_gpass<GK, RG, CG, DT, SYM>), dim3((unsigned)blocks), dim3(256), 0, s, (const T*)G, ldg,
                     (const XT*)Xt, cfg.split, cfg.steps_total, cfg.steps_per_split, (AccS*)Yp, src, cfg.sym_nbx);
}

template <int GK, int RG, int CG, typename DT>
void launch_fd(const void* G, int64_t ldg, const void* Xt, const GPassCfg& cfg, int64_t n_pad, void* Yp,
               const GPassDSrc& src, hipStream_t s) {
  if (cfg.sym)
    launch_one<GK, RG, CG, DT, true>(G, ldg, Xt, cfg, n_pad, Yp, src, s);
  else
    launch_one<GK, RG, CG, DT, false>(G, ldg, Xt, cfg, n_pad, Yp, src, s);
}

template <int GK, int CG>
hipError_t launch_cg(const void* G, int64_t ldg, const void* Xt, const GPassCfg& cfg, int64_t n_pad, void* Yp,
                     const GPassDSrc& src, hipStream_t s) {
  if (!src.D) {
    constexpr int RG = rg_for(GK, CG);
    if (cfg.rg != RG || cfg.sym) return hipErrorInvalidValue;
    launch_one<GK, RG, CG, void, false>(G, ldg, Xt, cfg, n_pad, Yp, src, s);
  } else if constexpr (GK == GK_FP8) {
    return hipErrorInvalidValue;  // fp8 passes read the stored G
  } else if constexpr (GK == GK_BF16) {
    // from D: the fused centring write and first range pass (fp32 D only)
    constexpr int RG = rg_fd(GK, CG, false);
    if (cfg.rg != RG || cfg.sym || src.d_is_f64 || !G) return hipErrorInvalidValue;
    launch_one<GK, RG, CG, float, false>(G, ldg, Xt, cfg, n_pad, Yp, src, s);
  } else {
    if (src.d_is_f64) {
      constexpr int RG = rg_fd(GK, CG, true);
      if (cfg.rg != RG) return hipErrorInvalidValue;
      launch_fd<GK, RG, CG, double>(G, ldg, Xt, cfg, n_pad, Yp, src, s);
    } else {
      constexpr int RG = rg_fd(GK, CG, false);
      if (cfg.rg != RG) return hipErrorInvalidValue;
      launch_fd<GK, RG, CG, float>(G, ldg, Xt, cfg, n_pad, Yp, src, s);
    }
  }
  return hipGetLastError();
}

template <int CG, typename DT, bool SYM, bool WG, int NT, int NTB>
void launch_x3_one(const void* Xt, int64_t ldg, const GPassCfg& cfg, int64_t n_pad, void* Yp, const GPassDSrc& src,
                   hipStream_t s, void* Gw = nullptr) {
  constexpr int RG = rg_x3(CG, sizeof(DT) == 8);
  hipLaunchKernelGGL((k_gpass_x3<RG, CG, DT, SYM, WG, NT, NTB>), dim3((unsigned)gpass_blocks(cfg, n_pad)), dim3(256), 0,
                     s, (const uint16_t*)Xt, ldg, cfg.split, cfg.steps_total, cfg.steps_per_split, (float*)Yp, src,
                     cfg.sym_nbx, (uint16_t*)Gw);
}

// the term combinations (G, X) of each use: (3, 3) everywhere, (2, 2) in
// every mode (the 16-bit sketch of Omega, fused with the centring write or
// not, and the 16-bit projection), (2, 1) in the full pass (the last 16-bit
// range pass)
template <int CG, int NT, int NTB>
hipError_t launch_x3_nt(const void* Xt, int64_t ldg, const GPassCfg& cfg, int64_t n_pad, void* Yp,
                        const GPassDSrc& src, hipStream_t s, void* Gw) {
  constexpr bool kWriteOk = NTB != 1, kSymOk = NTB != 1;
  if (Gw) {  // fused centring write: full pass over fp32 D
    if (!kWriteOk || cfg.sym || src.d_is_f64 || cfg.rg != rg_x3(CG, false)) return hipErrorInvalidValue;
    if constexpr (kWriteOk) launch_x3_one<CG, float, false, true, NT, NTB>(Xt, ldg, cfg, n_pad, Yp, src, s, Gw);
    return hipGetLastError();
  }
  if (cfg.rg != rg_x3(CG, src.d_is_f64 != 0) || (cfg.sym && !kSymOk)) return hipErrorInvalidValue;
  if (src.d_is_f64) {
    if constexpr (kSymOk)
      if (cfg.sym) {
        launch_x3_one<CG, double, true, false, NT, NTB>(Xt, ldg, cfg, n_pad, Yp, src, s);
        return hipGetLastError();
      }
    launch_x3_one<CG, double, false, false, NT, NTB>(Xt, ldg, cfg, n_pad, Yp, src, s);
  } else {
    if constexpr (kSymOk)
      if (cfg.sym) {
        launch_x3_one<CG, float, true, false, NT, NTB>(Xt, ldg, cfg, n_pad, Yp, src, s);
        return hipGetLastError();
      }
    launch_x3_one<CG, float, false, false, NT, NTB>(Xt, ldg, cfg, n_pad, Yp, src, s);
  }
  return hipGetLastError();
}

template <int CG>
hipError_t launch_x3_cg(int gt, int xt, const void* Xt, int64_t ldg, const GPassCfg& cfg, int64_t n_pad, void* Yp,
                        const GPassDSrc& src, hipStream_t s, void* Gw) {
  if (!src.D) return hipErrorInvalidValue;
  if (cfg.dma) return launch_split_pass(gt, xt, Xt, ldg, CG * 16, cfg, gpass_blocks(cfg, n_pad), Yp, src, Gw, s);
  if (gt == 3 && xt == 3) return launch_x3_nt<CG, 3, 3>(Xt, ldg, cfg, n_pad, Yp, src, s, Gw);
  if (gt == 2 && xt == 1) return launch_x3_nt<CG, 2, 1>(Xt, ldg, cfg, n_pad, Yp, src, s, Gw);
  if (gt == 2 && xt == 2) return launch_x3_nt<CG, 2, 2>(Xt, ldg, cfg, n_pad, Yp, src, s, Gw);
  return hipErrorInvalidValue;
}

hipError_t launch_x3(int gt, int xt, const void* Xt, int64_t ldg, int l_pad, const GPassCfg& cfg, int64_t n_pad,
                     void* Yp, const GPassDSrc& src, hipStream_t s, void* Gw) {
  switch (l_pad / 16) {
#define MDS_CG(N) \
  case N: return launch_x3_cg<N>(gt, xt, Xt, ldg, cfg, n_pad, Yp, src, s, Gw);
    MDS_CG(1) MDS_CG(2) MDS_CG(3) MDS_CG(4) MDS_CG(5) MDS_CG(6) MDS_CG(7) MDS_CG(8)
    MDS_CG(9) MDS_CG(10) MDS_CG(11) MDS_CG(12) MDS_CG(13) MDS_CG(14) MDS_CG(15) MDS_CG(16)
#undef MDS_CG
    default: return hipErrorInvalidValue;
  }
}

template <int GK>
hipError_t launch_gk(const void* G, int64_t ldg, const void* Xt, int l_pad, const GPassCfg& cfg, int64_t n_pad,
                     void* Yp, const GPassDSrc& src, hipStream_t s) {
  switch (l_pad / 16) {
#define MDS_CG(N) \
  case N: return launch_cg<GK, N>(G, ldg, Xt, cfg, n_pad, Yp, src, s);
    MDS_CG(1) MDS_CG(2) MDS_CG(3) MDS_CG(4) MDS_CG(5) MDS_CG(6) MDS_CG(7) MDS_CG(8)
    MDS_CG(9) MDS_CG(10) MDS_CG(11) MDS_CG(12) MDS_CG(13) MDS_CG(14) MDS_CG(15) MDS_CG(16)
#undef MDS_CG
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

GPassCfg gpass_config(int gk, int l_pad, int64_t n_pad, int64_t ldg, int split_hint, bool from_d, bool sym,
                      bool d8, bool dma_ok) {
  GPassCfg c{};
  c.rg = gk_split(gk) ? rg_x3(l_pad / 16, d8) : (from_d ? rg_fd(gk, l_pad / 16, d8) : rg_for(gk, l_pad / 16));
  c.bm = 64 * c.rg;
  if (gk_split(gk) && dma_ok && from_d && !d8 && l_pad <= (gk == GK_F32S ? kDmaMaxL : kDmaMaxL2) &&
      n_pad % split_pass_rows() == 0) {
    c.dma = 1;  // k_split: 8 waves of 2 row groups, row blocks dealt to XCDs (see sym_nbx)
    c.rg = 2;
    c.bm = split_pass_rows();
  }
  if (gk == GK_BF16 && !from_d && dma_ok && l_pad <= kDmaMaxL2 && n_pad % gstream_rows() == 0 && ldg == n_pad) {
    c.dma = 1;  // k_gstream: the stored bf16 G through an LDS ring, same work mapping
    c.rg = 2;
    c.bm = gstream_rows();
  }
  // bytes per K-value of a step's 128-byte row (the split pass steps 32 K-values, like fp32)
  const int64_t esize = gk == GK_F64 ? 8 : ((gk == GK_F32 || gk_split(gk)) ? 4 : 2);
  c.steps_total = ldg * esize / 128;
  const int64_t row_blocks = n_pad / c.bm;
  if (sym && from_d) {
    // 8 K splits (one slice of X per XCD-resident wave of workgroups); every
    // split index below `split` holds at least one step
    int64_t split = split_hint > 0 ? split_hint : 8;
    if (split > c.steps_total) split = c.steps_total;
    c.steps_per_split = (c.steps_total + split - 1) / split;
    c.split = (int)((c.steps_total + c.steps_per_split - 1) / c.steps_per_split);
    c.sym = 1;
    c.sym_nbx = (row_blocks + 7) / 8;
    c.sym_cols_per_split = c.steps_per_split * (128 / esize);
    return c;
  }
  int64_t split = split_hint > 0 ? split_hint : (2048 + row_blocks - 1) / row_blocks;
  int64_t max_split = c.steps_total / 16;
  if (max_split < 1) max_split = 1;
  if (split > max_split) split = max_split;
  if (split >= 8 && split_hint <= 0) split = ((split + 7) / 8) * 8;
  if (split < 1) split = 1;
  c.split = (int)split;
  c.steps_per_split = (c.steps_total + split - 1) / split;
  if (c.dma) {
    c.sym_nbx = (row_blocks + 7) / 8;  // row blocks per XCD
    // K ranges of an even number of steps (the fused write stores step
    // pairs); every split index below `split` keeps at least one step
    c.steps_per_split += c.steps_per_split % 2;
    c.split = (int)((c.steps_total + c.steps_per_split - 1) / c.steps_per_split);
  }
  return c;
}

GPassCfg gpass_config_nodma(const GPassCfg& c, int l_pad, int64_t n_pad, bool d8) {
  GPassCfg f = c;
  if (!c.dma) return f;
  f.dma = 0;
  f.rg = rg_x3(l_pad / 16, d8);
  f.bm = 64 * f.rg;
  if (f.sym) f.sym_nbx = (n_pad / f.bm + 7) / 8;
  return f;
}

hipError_t launch_gpass(int gk, const void* G, int64_t ldg, int64_t n_pad, const void* Xt, int l_pad,
                        const GPassCfg& cfg, void* Ypart, const GPassDSrc& src, hipStream_t s) {
  if (l_pad % 16 != 0 || l_pad < 16 || l_pad > kMaxL || n_pad % cfg.bm != 0) return hipErrorInvalidValue;
  switch (gk) {
    case GK_F64: return launch_gk<GK_F64>(G, ldg, Xt, l_pad, cfg, n_pad, Ypart, src, s);
    case GK_F32: return launch_gk<GK_F32>(G, ldg, Xt, l_pad, cfg, n_pad, Ypart, src, s);
    case GK_BF16:
      if (cfg.dma && !src.D) return launch_gstream(G, ldg, Xt, l_pad, cfg, src.n, gpass_blocks(cfg, n_pad), Ypart, s);
      return launch_gk<GK_BF16>(G, ldg, Xt, l_pad, cfg, n_pad, Ypart, src, s);
    case GK_FP8:
      if (!src.g8_scales || (cfg.bm > kF8Block) || (kF8Block % cfg.bm)) return hipErrorInvalidValue;
      return launch_gk<GK_FP8>(G, ldg, Xt, l_pad, cfg, n_pad, Ypart, src, s);
    case GK_F32S:
    case GK_S2:
    case GK_S2X:
      return launch_x3(gk_g_terms(gk), gk_x_terms(gk), Xt, ldg, l_pad, cfg, n_pad, Ypart, src, s,
                       const_cast<void*>(G));
    default: return hipErrorInvalidValue;
  }
}

int64_t gpass_blocks(const GPassCfg& cfg, int64_t n_pad) {
  return (cfg.sym || cfg.dma) ? 8 * cfg.sym_nbx * cfg.split : (n_pad / cfg.bm) * cfg.split;
}

hipError_t launch_splitk_reduce(int gk, const GPassCfg& cfg, const void* Ypart, int64_t ldg, int64_t elems,
                                double* Y, hipStream_t s) {
  const unsigned blocks = (unsigned)((elems / 4 + 255) / 256);
  const int64_t cps = cfg.sym ? cfg.sym_cols_per_split : 0;
  if (gk == GK_F64)
    hipLaunchKernelGGL(k_splitk_reduce<double>, dim3(blocks), dim3(256), 0, s, (const double*)Ypart, cfg.split,
                       elems, Y, ldg, (int64_t)cfg.bm, cps);
  else
    hipLaunchKernelGGL(k_splitk_reduce<float>, dim3(blocks), dim3(256), 0, s, (const float*)Ypart, cfg.split,
                       elems, Y, ldg, (int64_t)cfg.bm, cps);
  return hipGetLastError();
}

}  // namespace mds
