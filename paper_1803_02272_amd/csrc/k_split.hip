// fp32 G-passes on bf16 MFMA with the G operand as an exact bf16 expansion
// (Sec. 3.2-3.3: the products Y = G X of the range finder and of the
// projection), streamed from the fp32 distance matrix D and recentred on the
// fly (Sec. 6.2, step 1), software-pipelined for gfx950.
//
// Arithmetic (the same as k_gpass_x3): an fp32 value a is the exact sum
// a0 + a1 + a2 of three bf16 terms (each rounded to nearest even).  With
// three terms (NT = 3, the fp32 passes) both operands are split and the six
// products a_p b_q with p + q <= 2 are accumulated in fp32; the three
// dropped ones are below 2^-22 |a b|.  With two terms (NT = 2) G is carried
// as a0 + a1 (within 2^-17 of its fp32 value): the sketch of Omega and the
// projection split X into two terms as well (NTB = 2) and take a1 b0 +
// a0 b1 + a0 b0, within 2^-15 |a b| per product; the last range pass rounds
// X once (NTB = 1, b0 = bf16(x)) and takes a1 b0 + a0 b0, each product
// exact in fp32, with two thirds of those MFMAs and one plane of X.  Both
// need much less of the splitting work than three terms.  Three modes:
//   kFull  Y = G X over all of D, gamma = fma(-1/2, fl32(d^2), hc_k + hr_i)
//          with hc_k = fl32(c_k / 2), hr_i = fl32((r_i - m) / 2);
//   kSym   the projection's symmetric pass, 2 (W o G) X over the upper
//          triangle of D (W = 1 above, 1/2 on, 0 below the diagonal),
//          accumulated as (W o G) X from the kFull gamma and doubled at the
//          end (exactly the doubled terms' sum: scaling by 2 is exact);
//   kWrite the fused centring write: gamma in fp64 from the centring
//          equation, g = fl32(gamma) stored as bf16(g) into G (the padding
//          outside n x n is zeroed by a separate small kernel) and split for
//          the first range pass.
//
// Organisation (512 threads = 8 waves x 32 rows, 256 rows per workgroup,
// one workgroup per CU, steps of 32 K-values):
//   * every wave streams its own 32 rows of D into a three-stage LDS ring
//     with buffer-to-LDS loads (lane l's 16 bytes land at the instruction's
//     LDS address + 16 l), whole 128-byte lines per 8 lanes with the
//     nontemporal hint, issued three steps before the step they feed; the
//     pieces of a row are placed in XOR-swizzled slots so that the reads in
//     the MFMA operand layout are free of bank conflicts;
//   * the X tile of a step (the pass's bf16 planes, 64 bytes per row each), and with
//     it the recentring terms of the following step (c_k / 2, or c_k in
//     fp64), are loaded the same way into one of two LDS buffers shared by
//     the eight waves; K-group kg of row r sits in slot kg ^ ((r / 2) % 4),
//     so that the B-operand reads run at the LDS's full rate;
//   * the split A operands of step st + 1 are computed during step st, in
//     slices placed between the MFMAs of step st, so that the recentring
//     and splitting VALU work runs in the MFMA shadow rather than between
//     the steps;
//   * one workgroup barrier per step, without a memory fence (which would
//     also wait for the D loads in flight): after it the next X tile is
//     complete and the current one is no longer read.
// Every LDS buffer is its own __shared__ array and the step loop is unrolled
// six ways (2 X buffers x 3 ring stages), so each LDS access names a fixed
// array and the compiler's wait counts stay as precise as the explicit ones.
// Requires fp32 D, n % 4 == 0, a 16-byte aligned D and l_pad <= 128 (three
// terms) or <= 224 (two terms).
#include <type_traits>

#include "mds_internal.h"

namespace mds {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

enum SplitMode { kFull = 0, kSym = 1, kWrite = 2 };

constexpr int kWaves = 8;
constexpr int kRG = 2;                  // 16-row groups per wave
constexpr int kBK = 32;                 // K-values per step
constexpr int kBM = kWaves * kRG * 16;  // 256 rows per workgroup
constexpr int kAux = 256;               // recentring terms carried with an X tile (32 doubles)

// 16 bytes per lane from a buffer resource at byte offset voff into LDS at
// l + 16 lane (buffer_load_dwordx4 ... lds).  Offsets at or past the
// resource's size read zeros, which bounds every read by the buffer.
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t r, uint32_t voff, void* l) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t*)l, 16, voff, 0, 0, 0);
}
// The same with the nontemporal hint, for D: every byte is read once per pass
// (measured on MI355X for whole 128-byte lines per 8 lanes: 6.5 TB/s with the
// hint against 5.9 without; lanes that cover half lines reach 5.4 and lose
// more with it)
__device__ __forceinline__ void dma16_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff, void* l) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t*)l, 16, voff, 0, 0, 2);
}

constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit elements (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}

__device__ __forceinline__ uint32_t bf16x2_bits(f32x2 v) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v_t));
}

// Three-term split of 4 floats into dwords 2 half, 2 half + 1 of the planes.
__device__ __forceinline__ void split3_4(const float (&g)[4], u32x4 (&w)[3], int half) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const f32x2 v = {g[2 * h], g[2 * h + 1]};
    const bf16x2v_t v0 = __builtin_convertvector(v, bf16x2v_t);
    const f32x2 r1 = v - __builtin_convertvector(v0, f32x2);
    const bf16x2v_t v1 = __builtin_convertvector(r1, bf16x2v_t);
    const f32x2 r2 = r1 - __builtin_convertvector(v1, f32x2);
    const bf16x2v_t v2 = __builtin_convertvector(r2, bf16x2v_t);
    w[0][2 * half + h] = __builtin_bit_cast(uint32_t, v0);
    w[1][2 * half + h] = __builtin_bit_cast(uint32_t, v1);
    w[2][2 * half + h] = __builtin_bit_cast(uint32_t, v2);
  }
}

__device__ __forceinline__ void mma(floatx4_t& c, const u32x4& a, const u32x4& b) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                              0, 0, 0);
}

template <int CG, int MODE, int NT, int NTB>
__global__ __launch_bounds__(512, 1) void k_split(const uint16_t* __restrict__ X3, int64_t ldg, int split,
                                                  int64_t steps_total, int64_t steps_per_split,
                                                  float* __restrict__ Ypart, GPassDSrc src, int64_t sym_nbx,
                                                  uint16_t* __restrict__ Gw) {
  constexpr bool SYM = MODE == kSym;
  constexpr bool WG = MODE == kWrite;
  constexpr int LPAD = CG * 16;
  static_assert((NT == 3 && NTB == 3) || (NT == 2 && (NTB == 1 || NTB == 2)), "term counts");
  constexpr int XINS = CG * NTB;                        // 1 KB loads per X step tile (NTB planes)
  constexpr int XBYTES = XINS * 1024 + kAux;
  constexpr int DSTAGE = kRG * 2 * 1024;               // one wave's D stage (32 rows x 32 fp32)
  constexpr int64_t kStepsPerBlock = kBM / kBK;
  using CT = typename std::conditional<WG, double, float>::type;  // recentring term per K-value
  constexpr int kPieces = kBK * (int)sizeof(CT) / 16;              // 16-byte pieces of a step's terms
  constexpr int NCP = (CG + 1) / 2;                                // column-group pairs per step
  __shared__ __attribute__((aligned(16))) unsigned char xs0[XBYTES];
  __shared__ __attribute__((aligned(16))) unsigned char xs1[XBYTES];
  __shared__ __attribute__((aligned(16))) unsigned char ds0[kWaves * DSTAGE];
  __shared__ __attribute__((aligned(16))) unsigned char ds1[kWaves * DSTAGE];
  __shared__ __attribute__((aligned(16))) unsigned char ds2[kWaves * DSTAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t bid = blockIdx.x;
  int s;
  int64_t mb, st0, st1;
  if constexpr (SYM) {  // work item (row block, K split) clipped to the triangle
    const int64_t loc = bid >> 3;
    s = (int)(loc / sym_nbx);
    mb = (loc % sym_nbx) * 8 + (bid & 7);
    const int64_t diag0 = mb * kStepsPerBlock;
    st0 = (int64_t)s * steps_per_split;
    st1 = (st0 + steps_per_split < steps_total) ? st0 + steps_per_split : steps_total;
    if (diag0 > st0) st0 = diag0;
    if (diag0 >= steps_total || st0 >= st1) return;  // empty item: no partial written
  } else {
    // row blocks dealt to XCDs round-robin (block mb on XCD mb % 8), the split
    // index varying slowest inside an XCD: the workgroups that run together
    // on an XCD stream the same K range in step, so each X tile is fetched
    // into that XCD's L2 once and read there by all of them
    const int64_t loc = bid >> 3;
    s = (int)(loc / sym_nbx);
    mb = (loc % sym_nbx) * 8 + (bid & 7);
    st0 = (int64_t)s * steps_per_split;
    st1 = (st0 + steps_per_split < steps_total) ? st0 + steps_per_split : steps_total;
    // (the second test never holds: every split has a step.  Stating it lets
    // the compiler see a loop that runs at least once, which keeps the
    // accumulators in place instead of spilling them.)
    if (mb * kBM >= ldg || st0 >= st1) return;
  }
  const int64_t diag_end = (mb + 1) * kStepsPerBlock;
  const int64_t row0 = mb * kBM + (int64_t)wave * (kRG * 16);
  const int64_t row0s = mb * kBM + (int64_t)__builtin_amdgcn_readfirstlane(wave) * (kRG * 16);  // in SGPRs

  floatx4_t acc[kRG][CG];
#pragma unroll
  for (int rg = 0; rg < kRG; ++rg)
#pragma unroll
    for (int cg = 0; cg < CG; ++cg)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[rg][cg][e] = 0.0f;

  const float* Dp = reinterpret_cast<const float*>(src.D);
  const int64_t n = src.n;
  const double mval = src.m[0];
  float ri[kRG];   // hr_i = fl32((r_i - m) / 2)
  double rd[kRG];  // fused write: (r_i - m) / 2 in fp64
#pragma unroll
  for (int rg = 0; rg < kRG; ++rg) {
    const int64_t i = row0 + rg * 16 + (lane & 15);
    const float h = (i < n) ? (float)(0.5 * (src.r[i] - mval)) : 0.0f;
    ri[rg] = h;
    rd[rg] = (WG && i < n) ? 0.5 * (src.r[i] - mval) : 0.0;
  }
  // Buffer resources (32-bit offsets, reads past the end return zeros):
  //   this workgroup's rows of D (rows >= n read zeros; a row's columns >= n
  //   run into the next row, finite values that meet zero rows of X or are
  //   masked in the fused write), the split operand X, and the recentring
  //   terms (fl32(c_k / 2), ldg zero-padded entries, or c_k, n entries)
  const int64_t blk_rows = n - mb * kBM < kBM ? (n - mb * kBM > 0 ? n - mb * kBM : 0) : kBM;
  const __amdgpu_buffer_rsrc_t rD = make_rsrc(Dp + mb * kBM * n, blk_rows * n * 4);
  const __amdgpu_buffer_rsrc_t rX = make_rsrc(X3, (int64_t)LPAD * ldg * 6);
  const __amdgpu_buffer_rsrc_t rC =
      WG ? make_rsrc(src.c, n * 8) : make_rsrc(src.hc, ldg * 4);
  // per-lane offsets of step 0.  D: load q (0..3) of a wave covers its rows
  // 8q .. 8q + 7 as whole 128-byte lines (8 lanes per row); lane l lands at
  // LDS slot l = 8 (row % 8) + slot and brings piece (16 bytes, 4 K-values)
  // slot ^ f(row) of its row, f(r) = (r % 8) ^ ((r / 8) % 2), so that the
  // A-operand reads below (lane l: row l % 16, piece 2 (l / 16) + half) run at
  // the full rate of gfx950's 64-bank LDS (measured on MI355X: with
  // f(r) = r % 8 they take 1.6 times as long).
  uint32_t d_off[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rr = lane >> 3, piece = (lane & 7) ^ rr ^ (q & 1);
    d_off[q] = (uint32_t)((((int64_t)wave * (kRG * 16) + q * 8 + rr) * n + piece * 4) * 4);
  }
  constexpr int XPW = (XINS + kWaves - 1) / kWaves;  // X tile loads per wave
  uint32_t x_off[XPW];
#pragma unroll
  for (int u = 0; u < XPW; ++u) {
    const int q = wave + u * kWaves;
    const int S = q * 64 + lane;
    const int p = S / (LPAD * 4), rem = S % (LPAD * 4);
    const int row = rem >> 2, kg = (rem & 3) ^ ((row >> 1) & 3);
    x_off[u] = (uint32_t)((int64_t)row * ldg * 6 + p * 64 + kg * 16);
  }

  // D of step st into stage dd: this wave's 32 rows x 128 bytes
  auto dma_d = [&](int64_t st, unsigned char (&dd)[kWaves * DSTAGE]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) dma16_nt(rD, d_off[q] + (uint32_t)st * (kBK * 4), &dd[wave * DSTAGE + q * 1024]);
  };
  // recentring terms of step stc into the aux area of xd (last wave, one
  // 16-byte piece per lane)
  auto dma_aux = [&](int64_t stc, unsigned char (&xd)[XBYTES]) {
    if (wave == kWaves - 1 && lane < kPieces)
      dma16(rC, (uint32_t)(stc * kBK * (int)sizeof(CT)) + lane * 16, &xd[XINS * 1024]);
  };
  // X tile of step st: slot S = q * 64 + lane holds plane p, row, K-group kg
  // at S = p * 4 LPAD + 4 row + (kg ^ ((row >> 1) & 3)); then the terms of stc
  auto dma_x = [&](int64_t st, int64_t stc, unsigned char (&xd)[XBYTES]) {
#pragma unroll
    for (int u = 0; u < XPW; ++u) {
      const int q = wave + u * kWaves;
      if (XINS % kWaves != 0 && q >= XINS) break;
      dma16(rX, x_off[u] + (uint32_t)st * 192, &xd[q * 1024]);
    }
    dma_aux(stc, xd);
  };

  using DBuf = unsigned char[kWaves * DSTAGE];
  using XBuf = unsigned char[XBYTES];
  // A slice of the split A operands of step st: row group part / 2, K-values
  // 4 (part % 2) .. + 3 of the lane's 8, from D in stage dd and the terms in
  // the aux area of xa.  It is computed in kSliceOps small operations so that
  // the step can place them between its MFMAs.
  struct Slice {
    float dv[4];
    CT cv[4];
    float g[4];
    bf16x2v_t v[2][NT];  // planes of the two value pairs
    f32x2 r[2];
    float fd;  // symmetric mode: K-value of dv[0] minus the row index, clamped to +-64
    int rg, half;
  };
  constexpr int kSliceOps = 4 + 2 * NT - 2;  // 4 recentring + (NT - 1) split phases per value pair
  auto slice_load = [&](Slice& S, int part, int64_t st, const DBuf& dd, const XBuf& xa) {
    S.rg = part >> 1;
    S.half = part & 1;
    // this lane's row r of the wave's 32 and K-piece pc (see d_off)
    const int r = S.rg * 16 + (lane & 15), pc = 2 * (lane >> 4) + S.half;
    const u32x4 dw = *reinterpret_cast<const u32x4*>(
        &dd[wave * DSTAGE + (r >> 3) * 1024 + (r & 7) * 128 + ((pc ^ (r & 7) ^ ((r >> 3) & 1)) * 16)]);
    __builtin_memcpy(S.dv, &dw, 16);
    const int kk = (lane >> 4) * 8 + S.half * 4;  // K-value of dv[0] within the step
    __builtin_memcpy(S.cv, &xa[XINS * 1024 + kk * sizeof(CT)], 4 * sizeof(CT));
    if constexpr (SYM) {  // a wave-uniform part (scalar) and a lane part
      const int64_t u = st * kBK - (row0s + S.rg * 16);
      const int uc = u < -64 ? -64 : (u > 64 ? 64 : (int)u);
      S.fd = (float)(uc + kk - (lane & 15));
    }
  };
  // fused write: bf16 G of the lane's row and K-values 8j .. 8j + 7 (j = lane / 16)
  // of the step being split (gcur) and of the step before it (gprev)
  u32x4 gcur[kRG], gprev[kRG];
  // operation j: 0..3 recentre value j (the fused write stores the four bf16
  // entries after the last), 4..9 split the two value pairs into the planes
  auto slice_op = [&](Slice& S, int j, u32x4 (&w)[kRG][NT]) {
#pragma clang fp contract(off)
    if (j < 4) {
      const int t = j;
      if constexpr (WG) {
        // gamma = 1/2 (c_k - d^2) + (r_i - m) / 2, the centring equation
        // rearranged into two fused operations in fp64 (d^2 is exact in
        // fp64 for an fp32 d); entries outside n x n are zeroed afterwards
        // (launch_split_zero_pad), their values here are finite and meet
        // zero rows of Omega
        const double d = (double)S.dv[t];
        const double e = __builtin_fma(-d, d, S.cv[t]);
        S.g[t] = (float)__builtin_fma(0.5, e, rd[S.rg]);
        if (t == 3) {  // half h holds K-values 8j + 4h .. 8j + 4h + 3
          gcur[S.rg][2 * S.half] = bf16x2_bits(f32x2{S.g[0], S.g[1]});
          gcur[S.rg][2 * S.half + 1] = bf16x2_bits(f32x2{S.g[2], S.g[3]});
        }
      } else {
        const float d2 = S.dv[t] * S.dv[t];
        float g = __builtin_fmaf(-0.5f, d2, S.cv[t] + ri[S.rg]);
        if (SYM)  // weights 1, 1/2, 0 right of, on and left of the diagonal: clamp(k - i + 1/2, 0, 1)
          g *= __builtin_fminf(__builtin_fmaxf(S.fd + (t + 0.5f), 0.0f), 1.0f);
        S.g[t] = g;
      }
    } else {
      const int q = (j - 4) / (NT - 1), ph = (j - 4) % (NT - 1);  // value pair, phase
      if (ph == 0) {
        const f32x2 x = {S.g[2 * q], S.g[2 * q + 1]};
        S.v[q][0] = __builtin_convertvector(x, bf16x2v_t);
        S.r[q] = x - __builtin_convertvector(S.v[q][0], f32x2);
      } else if (NT == 3 && ph == 1) {
        S.v[q][1] = __builtin_convertvector(S.r[q], bf16x2v_t);
        S.r[q] = S.r[q] - __builtin_convertvector(S.v[q][1], f32x2);
      }
      if (ph == NT - 2) {  // last phase: the final term, then the planes
        S.v[q][NT - 1] = __builtin_convertvector(S.r[q], bf16x2v_t);
#pragma unroll
        for (int p = 0; p < NT; ++p) w[S.rg][p][2 * S.half + q] = __builtin_bit_cast(uint32_t, S.v[q][p]);
      }
    }
  };
  auto split_slice = [&](int part, int64_t st, const DBuf& dd, const XBuf& xa, u32x4 (&w)[kRG][NT]) {
    Slice S;
    slice_load(S, part, st, dd, xa);
#pragma unroll
    for (int j = 0; j < kSliceOps; ++j) slice_op(S, j, w);
  };

  // Fused write, K-steps sp - 1 and sp (an aligned pair: 128 bytes of each
  // row): both are staged in this wave's area of the D stage dd, whose D the
  // wave has finished reading, and read back as whole lines, so that each of
  // the four 16-byte stores covers 8 rows x 128 bytes.  Staging slot of row r,
  // 16-byte piece p: r * 128 + (p ^ (r % 8)) * 16.
  auto store_pair = [&](int64_t sp, DBuf& dd) {
    unsigned char* area = &dd[wave * DSTAGE];
#pragma unroll
    for (int rg = 0; rg < kRG; ++rg) {
      const int r = rg * 16 + (lane & 15), j = lane >> 4;
      *reinterpret_cast<u32x4*>(&area[r * 128 + ((j ^ (r & 7)) * 16)]) = gprev[rg];
      *reinterpret_cast<u32x4*>(&area[r * 128 + (((4 + j) ^ (r & 7)) * 16)]) = gcur[rg];
    }
    const int64_t col = (sp - 1) * kBK + (lane & 7) * 8;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = q * 8 + (lane >> 3);
      const u32x4 v = *reinterpret_cast<const u32x4*>(&area[r * 128 + (((lane & 7) ^ (r & 7)) * 16)]);
      __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(Gw + (row0 + r) * ldg + col));  // streamed out
    }
  };

  u32x4 wA[kRG][NT], wB[kRG][NT];
  // prologue: X(st0) with the terms of st0 + 1, D of the first three steps,
  // the terms of st0 (into the other buffer's aux area) and the split of st0
  const int64_t last = st1 - 1;
  dma_x(st0, st0 + 1 < st1 ? st0 + 1 : last, xs0);
  dma_aux(st0, xs1);
  dma_d(st0, ds0);
  dma_d(st0 + 1 < st1 ? st0 + 1 : last, ds1);
  dma_d(st0 + 2 < st1 ? st0 + 2 : last, ds2);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  __syncthreads();
#pragma unroll
  for (int part = 0; part < 4; ++part) split_slice(part, st0, ds0, xs1, wA);
  if constexpr (WG) {
#pragma unroll
    for (int rg = 0; rg < kRG; ++rg) gprev[rg] = gcur[rg];
  }
  __syncthreads();  // every wave has read the terms in xs1 before it is reloaded

  // One step: X(st) in xr (with the terms of st + 1), D(st + 1) in dn; the
  // loads of X(st + 1) (+ terms of st + 2) go to xw and D(st + 3) to dw;
  // wc holds the split of st, wn receives the split of st + 1.  The loads are
  // issued on every step (clamped to the last step at the end), so that the
  // wait counts below are the same on every path.
  auto step = [&](int64_t st, XBuf& xr, XBuf& xw, DBuf& dn, DBuf& dw, u32x4 (&wc)[kRG][NT],
                  u32x4 (&wn)[kRG][NT], bool pair_end) {
    const int64_t s1 = st + 1 < st1 ? st + 1 : last;
    const int64_t s2 = st + 2 < st1 ? st + 2 : last;
    const int64_t s3 = st + 3 < st1 ? st + 3 : last;
    dma_x(s1, s2, xw);
    dma_d(s3, dw);
    // products smallest first: a2 b0, a1 b1, a0 b2, a1 b0, a0 b1, a0 b0 (three
    // terms), a1 b0, a0 b1, a0 b0 (two and two) or a1 b0, a0 b0 (two and one)
    constexpr int NPR = NT == 3 ? 6 : (NTB == 2 ? 3 : 2);
    constexpr int PA[6] = {NT == 3 ? 2 : 1, NT == 3 ? 1 : 0, 0, 1, 0, 0};
    constexpr int PB[6] = {0, NTB >= 2 ? 1 : 0, NT == 3 ? 2 : 0, 0, 1, 0};
#pragma unroll
    for (int cp = 0; cp < NCP; ++cp) {
      // One column-group pair: its B operands and the inputs of its share of
      // the next step's split are read first; then its MFMAs are issued in a
      // fixed order, each followed by one small operation of that share, so
      // that the SIMD runs the VALU work while the MFMA executes (the two
      // are independent).  The schedule barriers keep this order.
      const int cg0 = 2 * cp;
      constexpr int kMaxSl = 4;
      const int sl0 = (cp * 4) / NCP, sl1 = ((cp + 1) * 4) / NCP;  // slices of this pair
      __builtin_amdgcn_sched_barrier(0);
      u32x4 bb[2][NTB];
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (cg0 + h < CG) {
          const int row = (cg0 + h) * 16 + (lane & 15);
          const int kgs = (lane >> 4) ^ ((row >> 1) & 3);
#pragma unroll
          for (int p = 0; p < NTB; ++p)
            bb[h][p] = *reinterpret_cast<const u32x4*>(&xr[(p * LPAD * 4 + row * 4 + kgs) * 16]);
        }
      Slice S[kMaxSl];
#pragma unroll
      for (int sl = 0; sl < kMaxSl; ++sl)
        if (sl0 + sl < sl1) slice_load(S[sl], sl0 + sl, s1, dn, xr);
      __builtin_amdgcn_sched_barrier(0);
      const int nops = (sl1 - sl0) * kSliceOps;
      auto mfmas = [&]() {
#pragma unroll
        for (int pr = 0; pr < NPR; ++pr)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (cg0 + h < CG)
#pragma unroll
              for (int rg = 0; rg < kRG; ++rg) mma(acc[rg][cg0 + h], wc[rg][PA[pr]], bb[h][PB[pr]]);
      };
      auto slices = [&]() {
#pragma unroll
        for (int op = 0; op < nops; ++op) slice_op(S[op / kSliceOps], op % kSliceOps, wn);
      };
      // The two waves of a SIMD (waves w and w + 4) take the pair's VALU and
      // MFMA work in opposite orders, so that one wave's splitting runs while
      // the other's MFMAs execute.
      if (wave & 4) {
        slices();
        __builtin_amdgcn_sched_barrier(0);
        mfmas();
      } else {
        mfmas();
        __builtin_amdgcn_sched_barrier(0);
        slices();
      }
    }
    // The fused write: the split of s1 is the second step of an aligned pair
    // when the step offset st - st0 is even (st0 and the range length are
    // even); the pair is stored, else the step is kept for the next one.  The
    // last step splits s1 = st1 - 1 again, at an odd offset: kept, not stored.
    if constexpr (WG) {
      if (pair_end) {
        store_pair(s1, dn);
      } else {
#pragma unroll
        for (int rg = 0; rg < kRG; ++rg) gprev[rg] = gcur[rg];
      }
    }
    // X(st + 1) and its terms complete; D(st + 3) and, after a stored pair,
    // the four G stores issued after it may still run (stores count in
    // vmcnt, in issue order with the loads)
    if (WG && pair_end)
      __builtin_amdgcn_s_waitcnt(0x0F70 | 8);  // vmcnt(8)
    else
      __builtin_amdgcn_s_waitcnt(0x0F70 | 4);  // vmcnt(4)
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);  // steps are scheduled one at a time (register pressure)
  };
  // X(st) in buffer (st - st0) % 2, D(st) in stage (st - st0) % 3, the split of
  // st in wA or wB by (st - st0) % 2: six steps per trip keep every array static
  for (int64_t st = st0; st < st1; st += 6) {
    step(st, xs0, xs1, ds1, ds0, wA, wB, true);
    if (st + 1 >= st1) break;
    step(st + 1, xs1, xs0, ds2, ds1, wB, wA, false);
    if (st + 2 >= st1) break;
    step(st + 2, xs0, xs1, ds0, ds2, wA, wB, true);
    if (st + 3 >= st1) break;
    step(st + 3, xs1, xs0, ds1, ds0, wB, wA, false);
    if (st + 4 >= st1) break;
    step(st + 4, xs0, xs1, ds2, ds1, wA, wB, true);
    if (st + 5 >= st1) break;
    step(st + 5, xs1, xs0, ds0, ds2, wB, wA, false);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // no load outstanding at exit

#pragma unroll
  for (int rg = 0; rg < kRG; ++rg) {
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
      const int col = cg * 16 + (lane & 15);
      float* dst = Ypart + ((int64_t)s * LPAD + col) * ldg + row0 + rg * 16;
      const int64_t i4 = row0 + rg * 16 + 4 * (lane >> 4);
      float4 o = make_float4(acc[rg][cg][0], acc[rg][cg][1], acc[rg][cg][2], acc[rg][cg][3]);
      if constexpr (SYM) o = o + o;  // 2 (W o G) X: the doubling is exact, as in every term
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

// Widest X tile per term count: the LDS holds two X buffers of CG * NTB KB
// beside the three 32 KB D stages (three-term passes up to l_pad = 128,
// two-term ones up to 224).
constexpr int kMaxCG3 = 8, kMaxCG2 = 14;

template <int CG, int MODE, int NT, int NTB>
void launch_one(const void* Xt, int64_t ldg, const GPassCfg& cfg, int64_t blocks, void* Yp, const GPassDSrc& src,
                void* Gw, hipStream_t s) {
  hipLaunchKernelGGL((k_split<CG, MODE, NT, NTB>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, s,
                     (const uint16_t*)Xt, ldg, cfg.split, cfg.steps_total, cfg.steps_per_split, (float*)Yp, src,
                     cfg.sym_nbx, (uint16_t*)(MODE == kWrite ? Gw : nullptr));
}

// term combinations per mode: the fp32 passes (3, 3) and the 16-bit sketch
// of Omega and projection (2, 2) in every mode, the last 16-bit range pass
// (2, 1) in the full pass
template <int CG>
hipError_t launch_cg(int mode, int gt, int xt, const void* Xt, int64_t ldg, const GPassCfg& cfg, int64_t blocks,
                     void* Yp, const GPassDSrc& src, void* Gw, hipStream_t s) {
  if (gt == 3 && xt == 3) {
    if constexpr (CG <= kMaxCG3) {
      if (mode == kSym) launch_one<CG, kSym, 3, 3>(Xt, ldg, cfg, blocks, Yp, src, Gw, s);
      else if (mode == kWrite) launch_one<CG, kWrite, 3, 3>(Xt, ldg, cfg, blocks, Yp, src, Gw, s);
      else launch_one<CG, kFull, 3, 3>(Xt, ldg, cfg, blocks, Yp, src, Gw, s);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (gt == 2 && xt == 2) {
    if (mode == kSym) launch_one<CG, kSym, 2, 2>(Xt, ldg, cfg, blocks, Yp, src, Gw, s);
    else if (mode == kWrite) launch_one<CG, kWrite, 2, 2>(Xt, ldg, cfg, blocks, Yp, src, Gw, s);
    else launch_one<CG, kFull, 2, 2>(Xt, ldg, cfg, blocks, Yp, src, Gw, s);
  } else if (gt == 2 && xt == 1 && mode == kFull) {
    launch_one<CG, kFull, 2, 1>(Xt, ldg, cfg, blocks, Yp, src, Gw, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Zero the entries of the bf16 G outside n x n (rows >= n, and columns >= n
// of the rows below n) after the fused centring write.
__global__ __launch_bounds__(256) void k_zero_pad(uint16_t* __restrict__ G, int64_t n, int64_t n_pad, int64_t ldg) {
  const int64_t tail = n_pad - n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t cols_part = n * tail;  // (i < n, k >= n)
  if (e < cols_part) {
    G[(e / tail) * ldg + n + e % tail] = 0;
  } else {
    const int64_t f = e - cols_part;  // rows >= n, all ldg columns
    if (f < tail * ldg) G[(n + f / ldg) * ldg + f % ldg] = 0;
  }
}

}  // namespace

hipError_t launch_split_zero_pad(void* G, int64_t n, int64_t n_pad, int64_t ldg, hipStream_t s) {
  const int64_t total = n * (n_pad - n) + (n_pad - n) * ldg;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_pad, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (uint16_t*)G, n, n_pad, ldg);
  return hipGetLastError();
}

int split_pass_rows() { return kBM; }

hipError_t launch_split_pass(int gterms, int xterms, const void* Xt, int64_t ldg, int l_pad, const GPassCfg& cfg,
                             int64_t blocks, void* Yp, const GPassDSrc& src, void* Gw, hipStream_t s) {
  if (!src.D || src.d_is_f64 || !src.vec || src.n % 4 != 0 || cfg.bm != kBM || l_pad % 16 != 0 ||
      l_pad > 16 * (gterms == 3 ? kMaxCG3 : kMaxCG2))
    return hipErrorInvalidValue;
  if (Gw && cfg.sym) return hipErrorInvalidValue;
  // the fused write stores aligned pairs of steps: every K range starts on an
  // even step and has an even length
  if (Gw && (cfg.steps_per_split % 2 != 0 || cfg.steps_total % 2 != 0)) return hipErrorInvalidValue;
  const int mode = cfg.sym ? kSym : (Gw ? kWrite : kFull);
  switch (l_pad / 16) {
#define MDS_CG(N) \
  case N: return launch_cg<N>(mode, gterms, xterms, Xt, ldg, cfg, blocks, Yp, src, Gw, s);
    MDS_CG(1) MDS_CG(2) MDS_CG(3) MDS_CG(4) MDS_CG(5) MDS_CG(6) MDS_CG(7) MDS_CG(8)
    MDS_CG(9) MDS_CG(10) MDS_CG(11) MDS_CG(12) MDS_CG(13) MDS_CG(14)
#undef MDS_CG
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mds
