// Range pass over the stored bf16 G (Sec. 3.2: Y = G X of the range finder,
// the middle passes of the bf16 form), streamed through LDS for gfx950.
//
// Y_part[s] = G[row block, K range s] X[K range s] on bf16 MFMA with fp32
// accumulation: the same arithmetic as the register-streaming k_gpass
// (products of bf16 values are exact in fp32, the sums round in fp32), only
// the data path differs.  The pass reads each entry of G once, so it is
// bound by HBM bandwidth (2 bytes per entry against 2 l_pad flops); the MFMA
// work is under half of the streaming time at l_pad = 128.
//
// Organisation (512 threads = 8 waves x 32 rows, 256 rows per workgroup,
// one workgroup per CU, steps of 64 K-values = one 128-byte line per row):
//   * every wave streams its own 32 rows of G into a three-stage LDS ring
//     with buffer-to-LDS loads (lane l's 16 bytes land at the instruction's
//     LDS address + 16 l): whole lines per 8 lanes with the nontemporal hint,
//     issued three steps ahead; a wave reads only its own rows, so the G
//     ring needs no workgroup barrier;
//   * the X tile of a step (l_pad rows of 128 bytes) is loaded the same way,
//     two steps ahead, into a three-buffer ring shared by the eight waves
//     (one barrier per step); above l_pad = 128 the ring has two buffers
//     and the tile is loaded one step ahead;
//   * 16-byte pieces of a 128-byte row r sit in slot piece ^ (r % 8): the
//     MFMA operand reads (lane l: row l % 16, piece l / 16) then run at the
//     full rate of gfx950's 64-bank LDS (measured on MI355X: with slot
//     piece ^ (r % 8) ^ ((r / 8) % 2) the same reads take 1.6 times as long).
// Requires l_pad <= 224, ldg a multiple of 256 and n_pad = ldg rows of G.
#include "mds_internal.h"

namespace mds {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_t;

constexpr int kWaves = 8;
constexpr int kRG = 2;                  // 16-row groups per wave
constexpr int kBM = kWaves * kRG * 16;  // 256 rows per workgroup
constexpr int kStage = 32 * 128;        // one wave's G stage: 32 rows x 128 bytes
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit elements (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}
// 16 bytes per lane at byte offset voff of the resource into LDS at l + 16 lane;
// aux 2 = nontemporal.  Offsets past the resource's size read zeros.
template <int AUX>
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t r, uint32_t voff, void* l) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t*)l, 16, voff, 0, 0, AUX);
}
__device__ __forceinline__ int swz(int r) { return r & 7; }

// XB: X buffers, 3 (X loaded two steps ahead) up to l_pad = 128; 2 (one
// step ahead) for the wider tiles, whose three buffers would not fit in LDS
// beside the G stages.
template <int CG, int XB>
__global__ __launch_bounds__(512, 1) void k_gstream(const uint16_t* __restrict__ G, int64_t ldg,
                                                    const uint16_t* __restrict__ Xt, int64_t steps_total,
                                                    int64_t steps_per_split, float* __restrict__ Ypart, int64_t n,
                                                    int64_t nbx) {
  constexpr int LPAD = CG * 16;
  constexpr int XINS = LPAD / 8;                       // 1 KB loads per X tile (8 rows each)
  constexpr int XPW = (XINS + kWaves - 1) / kWaves;    // per wave (the same count on every wave)
  __shared__ __attribute__((aligned(16))) unsigned char gs0[kWaves * kStage];
  __shared__ __attribute__((aligned(16))) unsigned char gs1[kWaves * kStage];
  __shared__ __attribute__((aligned(16))) unsigned char gs2[kWaves * kStage];
  __shared__ __attribute__((aligned(16))) unsigned char xs0[LPAD * 128];
  __shared__ __attribute__((aligned(16))) unsigned char xs1[LPAD * 128];
  __shared__ __attribute__((aligned(16))) unsigned char xs2[XB == 3 ? LPAD * 128 : 16];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t bid = blockIdx.x;
  // row blocks dealt to XCDs round-robin, the split index varying slowest
  // inside an XCD (the workgroups running together share their X range in L2)
  const int64_t loc = bid >> 3;
  const int s = (int)(loc / nbx);
  const int64_t mb = (loc % nbx) * 8 + (bid & 7);
  const int64_t st0 = (int64_t)s * steps_per_split;
  const int64_t st1 = (st0 + steps_per_split < steps_total) ? st0 + steps_per_split : steps_total;
  if (mb * kBM >= ldg || st0 >= st1) return;  // (every split has a step: the second test never holds)
  const int64_t row0 = mb * kBM + wave * 32;

  floatx4_t acc[kRG][CG];
#pragma unroll
  for (int rg = 0; rg < kRG; ++rg)
#pragma unroll
    for (int cg = 0; cg < CG; ++cg)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[rg][cg][e] = 0.0f;

  const __amdgpu_buffer_rsrc_t rG = make_rsrc(G + mb * kBM * ldg, (int64_t)kBM * ldg * 2);
  const __amdgpu_buffer_rsrc_t rX = make_rsrc(Xt, (int64_t)LPAD * ldg * 2);
  // G: load q (0..3) covers the wave's rows 8q .. 8q + 7; lane l lands in slot
  // l % 8 of row 8q + l / 8 and brings piece (l % 8) ^ f(row)
  uint32_t g_off[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = q * 8 + (lane >> 3);
    g_off[q] = (uint32_t)(((int64_t)(wave * 32 + r) * ldg) * 2 + ((lane & 7) ^ swz(r)) * 16);
  }
  // X: load u of this wave is tile load q = wave + 8u (rows 8q .. 8q + 7); a
  // wave past the last load repeats one (the same bytes to the same place),
  // so that every wave issues XPW loads and the wait counts are uniform
  uint32_t x_off[XPW];
  int x_lds[XPW];
#pragma unroll
  for (int u = 0; u < XPW; ++u) {
    const int q = (wave + kWaves * u) % XINS;
    const int r = q * 8 + (lane >> 3);
    x_off[u] = (uint32_t)((int64_t)r * ldg * 2 + ((lane & 7) ^ swz(r)) * 16);
    x_lds[u] = q * 1024;
  }
  using GBuf = unsigned char[kWaves * kStage];
  using XBuf = unsigned char[LPAD * 128];
  auto dma_g = [&](int64_t st, GBuf& gb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) dma16<2>(rG, g_off[q] + (uint32_t)st * 128, &gb[wave * kStage + q * 1024]);
  };
  auto dma_x = [&](int64_t st, XBuf& xb) {
#pragma unroll
    for (int u = 0; u < XPW; ++u) dma16<0>(rX, x_off[u] + (uint32_t)st * 128, &xb[x_lds[u]]);
  };

  const int64_t last = st1 - 1;
  auto clamp = [&](int64_t st) { return st < st1 ? st : last; };
  // G(st) and X(st) landed and every wave's part of X(st) visible; no wave
  // reads X(st - 1) any more.  With three X buffers, after X(st) each wave
  // issued G(st + 1), X(st + 1) and G(st + 2) (in this order: the loads of
  // step st - 1 are X(st + 1), then G(st + 2) at its end); with two, G(st + 1)
  // and G(st + 2) come before X(st), and only G(st + 3) after it.
  constexpr int kAfter = XB == 3 ? 8 + XPW : 4;  // loads allowed in flight
  auto settle = [&]() {
    __builtin_amdgcn_s_waitcnt(0x0F70 | kAfter);
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
  };
  dma_g(st0, gs0);
  dma_x(st0, xs0);
  dma_g(clamp(st0 + 1), gs1);
  if constexpr (XB == 3) {
    dma_x(clamp(st0 + 1), xs1);
    dma_g(clamp(st0 + 2), gs2);
    settle();
  } else {
    dma_g(clamp(st0 + 2), gs2);
    __builtin_amdgcn_s_waitcnt(0x0F70 | 8);  // G(st0) and X(st0)
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
  }

  // One step: G(st) in gb, X(st) in xb; X(st + XB - 1) goes to xn (which
  // held X(st - 1)) and G(st + 3) to gb once this wave has read it; then the
  // state above for st + 1 (the wait ends the step, so that the loop closes
  // after it and the compiler's own wait counts stay exact).
  auto step = [&](int64_t st, GBuf& gb, XBuf& xb, XBuf& xn) {
    dma_x(clamp(st + XB - 1), xn);
    // the X load goes out first.  (At the top of the loop the compiler adds a
    // wait for the older loads: it does not carry the ring's state across
    // the back edge.  Twelve steps per trip make that one step in twelve.)
    __builtin_amdgcn_sched_barrier(0);
    const unsigned char* ga = &gb[wave * kStage];
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {  // two MFMA K-blocks of 32 per step
      const int pc = (lane >> 4) + 4 * kh;
      u32x4 a[kRG];
#pragma unroll
      for (int rg = 0; rg < kRG; ++rg) {
        const int r = rg * 16 + (lane & 15);
        a[rg] = *reinterpret_cast<const u32x4*>(&ga[r * 128 + ((pc ^ swz(r)) * 16)]);
      }
#pragma unroll
      for (int cg = 0; cg < CG; ++cg) {
        const int r = cg * 16 + (lane & 15);
        const u32x4 b = *reinterpret_cast<const u32x4*>(&xb[r * 128 + ((pc ^ swz(r)) * 16)]);
#pragma unroll
        for (int rg = 0; rg < kRG; ++rg)
          acc[rg][cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a[rg]),
                                                                __builtin_bit_cast(bf16x8_t, b), acc[rg][cg], 0, 0, 0);
      }
    }
    // this wave's reads of G(st) are complete before its stage is reloaded
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __asm__ volatile("" ::: "memory");
    dma_g(clamp(st + 3), gb);
    settle();
  };
  if constexpr (XB == 3) {
    for (int64_t st = st0; st < st1; st += 12) {
#pragma unroll
      for (int u = 0; u < 12; u += 3) {
        if (st + u >= st1) break;
        step(st + u, gs0, xs0, xs2);
        if (st + u + 1 >= st1) break;
        step(st + u + 1, gs1, xs1, xs0);
        if (st + u + 2 >= st1) break;
        step(st + u + 2, gs2, xs2, xs1);
      }
    }
  } else {
    for (int64_t st = st0; st < st1; st += 12) {
#pragma unroll
      for (int u = 0; u < 12; u += 6) {
        if (st + u >= st1) break;
        step(st + u, gs0, xs0, xs1);
        if (st + u + 1 >= st1) break;
        step(st + u + 1, gs1, xs1, xs0);
        if (st + u + 2 >= st1) break;
        step(st + u + 2, gs2, xs0, xs1);
        if (st + u + 3 >= st1) break;
        step(st + u + 3, gs0, xs1, xs0);
        if (st + u + 4 >= st1) break;
        step(st + u + 4, gs1, xs0, xs1);
        if (st + u + 5 >= st1) break;
        step(st + u + 5, gs2, xs1, xs0);
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // no load into LDS outstanding at exit

#pragma unroll
  for (int rg = 0; rg < kRG; ++rg) {
#pragma unroll
    for (int cg = 0; cg < CG; ++cg) {
      const int col = cg * 16 + (lane & 15);
      float* dst = Ypart + ((int64_t)s * LPAD + col) * ldg + row0 + rg * 16;
      const int64_t i4 = row0 + rg * 16 + 4 * (lane >> 4);
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

}  // namespace

int gstream_rows() { return kBM; }

hipError_t launch_gstream(const void* G, int64_t ldg, const void* Xt, int l_pad, const GPassCfg& cfg, int64_t n,
                          int64_t blocks, void* Yp, hipStream_t s) {
  if (!G || !Xt || !Yp || l_pad % 16 != 0 || l_pad < 16 || l_pad > 224 || ldg % kBM != 0 || cfg.bm != kBM ||
      !cfg.dma || cfg.steps_total * 64 != ldg || blocks != 8 * cfg.sym_nbx * cfg.split)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), block(64 * kWaves);
  switch (l_pad / 16) {
#define MDS_CG(N)                                                                                           \
  case N:                                                                                                   \
    hipLaunchKernelGGL((k_gstream<N, (N <= 8 ? 3 : 2)>), grid, block, 0, s, (const uint16_t*)G, ldg,      \
                       (const uint16_t*)Xt,                                                                \
                       cfg.steps_total, cfg.steps_per_split, (float*)Yp, n, cfg.sym_nbx);                  \
    return hipGetLastError();
    MDS_CG(1) MDS_CG(2) MDS_CG(3) MDS_CG(4) MDS_CG(5) MDS_CG(6) MDS_CG(7) MDS_CG(8)
    MDS_CG(9) MDS_CG(10) MDS_CG(11) MDS_CG(12) MDS_CG(13) MDS_CG(14)
#undef MDS_CG
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mds
