// Batched small MDS: many independent instances of uneven n in one
// persistent launch, one workgroup (four waves) per instance running the
// whole method of Sec. 6.2 / 3.2-3.3 on its own:
//   centring sums (fp64) -> G in the pass dtype -> Omega (the same Philox
//   stream as the single-instance path) -> (2q+1) x [G-pass on MFMA ->
//   CholeskyQR2 in fp64] -> projection pass -> B = Q^T G Q -> cyclic Jacobi
//   -> coordinates with the sign convention of the single-instance path.
// The launch is persistent: its grid is sized to the device (as many
// workgroups as fit at once) and every workgroup takes the next instance
// from a job table in device memory through an atomic counter until the
// table is exhausted, so one launch runs any number of instances and keeps
// every CU busy while instances of uneven size finish at different times
// (the host orders the table by decreasing work).  Workgroups never wait on
// each other.  Meant for n up to a few thousand and l_pad <= 64 (the serving
// mix: k = 20, l = 30).
//
// The values of every dtype follow the single-instance path: fp64 G
// entries from the centring equation in fp64, fp32 entries as
// fma(-1/2, fl32(d^2), fl32(c_j/2) + fl32((r_i - m)/2)), bf16 entries as the
// bf16 rounding of the fp32 rounding of the fp64 entry; the bf16 form's
// first range pass and its projection multiply the fp32 entries with fp32 X,
// its last range pass with X rounded to bf16 (the single-instance path's
// 16-bit passes with fp32 in place of the two-term expansions, within 2^-17
// of them).  Sums run in a different order, so results agree with a
// single-instance run to rounding, not bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/mds.h"
#include "mds_internal.h"
#include "omega_dev.h"
#include "plan.h"
#include "small_dev.h"

namespace mds {
namespace {

using namespace small;

constexpr int kBT = 256;         // threads per instance
constexpr int kBMaxL = 64;       // largest l_pad
constexpr int kBPad = 64;        // n is padded to a multiple of this
constexpr int64_t kBMaxN = 16384;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct BJob {
  const void* D;
  double* coords;
  double* eigvals;
  char* ws;
  DevStatus* st;
  int32_t* status_out;  // optional device word: the instance's final mds_status
  int64_t n, n_pad;
  uint64_t seed;
  int k, l, l_pad, q, d_is_f64, pad_;
};

// Head of a batch workspace: per-instance status words, the job table (in
// the order the workgroups take it) and the work counter.
struct BHead {
  int64_t status, table, counter, total;
};
__host__ __device__ inline int64_t rup(int64_t v, int64_t m);
inline BHead bhead(int32_t count) {
  BHead h;
  h.status = 0;
  h.table = rup((int64_t)count * (int64_t)sizeof(DevStatus), 256);
  h.counter = h.table + rup((int64_t)count * (int64_t)sizeof(BJob), 256);
  h.total = h.counter + 256;
  return h;
}

__host__ __device__ inline int64_t rup(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Per-instance workspace (offsets in bytes from the instance base).
struct BLayout {
  int64_t r, c, hc, hr, G, X, Y, Q, total;
};

__host__ __device__ inline BLayout blayout(int64_t np, int l_pad, int form) {
  const int64_t gsz = form == MDS_FORM_FP64 ? 8 : (form == MDS_FORM_FP32 ? 4 : 2);
  const int64_t xsz = form == MDS_FORM_FP64 ? 8 : 4;  // bf16 form: bf16 range operand, fp32 projection operand
  BLayout L;
  int64_t o = 0;
  L.r = o, o += rup(np * 8, 256);
  L.c = o, o += rup(np * 8, 256);
  L.hc = o, o += rup(np * 4, 256);
  L.hr = o, o += rup(np * 4, 256);
  L.G = o, o += rup(np * np * gsz, 256);
  L.X = o, o += rup((int64_t)l_pad * np * xsz, 256);
  L.Y = o, o += rup((int64_t)l_pad * np * 8, 256);
  L.Q = o, o += rup((int64_t)l_pad * np * 8, 256);
  L.total = o;
  return L;
}

__device__ __forceinline__ bf16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
// the bf16 rounding of f as an fp32 value (X of the bf16 form's fp32 passes)
__device__ __forceinline__ float bf16_value(float f) { return __uint_as_float((uint32_t)to_bf16(f) << 16); }

// ---- centring sums with many loads in flight per thread ---------------------
constexpr int kUnroll = 16;  // independent loads issued before they are used

// c_j (column means of d^2): thread j walks down its column kUnroll rows at
// a time (each row access is coalesced over the workgroup).
template <typename DT>
__device__ void col_means(const DT* __restrict__ D, int64_t n, int64_t np, double* c) {
  for (int64_t j = threadIdx.x; j < np; j += kBT) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (j < n) {
      for (int64_t i0 = 0; i0 < n; i0 += kUnroll) {
        double d[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) d[u] = (i0 + u < n) ? (double)D[(i0 + u) * n + j] : 0.0;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) s[u & 3] += d[u] * d[u];
      }
    }
    c[j] = j < n ? ((s[0] + s[1]) + (s[2] + s[3])) / (double)n : 0.0;
  }
}

// r_i (row means of d^2), one wave per row; returns this thread's share of sum_i r_i.
template <typename DT>
__device__ double row_means(const DT* __restrict__ D, int64_t n, int64_t np, double* r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double part = 0.0;
  for (int64_t i = wave; i < np; i += kBT / 64) {
    double s = 0.0;
    if (i < n) {
      const DT* row = D + i * n;
      for (int64_t j0 = 0; j0 < n; j0 += 64 * 8) {
        double d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t j = j0 + lane + 64 * u;
          d[u] = j < n ? (double)row[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s += d[u] * d[u];
      }
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
      r[i] = i < n ? s / (double)n : 0.0;
      part += i < n ? s / (double)n : 0.0;
    }
  }
  return part;
}

// G in the pass dtype (rows and columns >= n zero), 8 entries per lane in flight.
template <int FORM, typename DT>
__device__ void write_g(const DT* __restrict__ D, int64_t n, int64_t np, const double* r, const double* c, double m,
                        const float* hc, const float* hr, void* G) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t i = wave; i < np; i += kBT / 64) {
    const double ri = i < n ? r[i] : 0.0;
    const float hri = hr[i];
    for (int64_t j0 = 0; j0 < np; j0 += 64 * 8) {
      DT d[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t j = j0 + lane + 64 * u;
        d[u] = (i < n && j < n) ? D[i * n + j] : (DT)0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t j = j0 + lane + 64 * u;
        if (j >= np) continue;
        const bool in = i < n && j < n;
        const double dd = (double)d[u];
        if constexpr (FORM == MDS_FORM_FP64) {
          ((double*)G)[i * np + j] = in ? -0.5 * (((dd * dd - c[j]) - ri) + m) : 0.0;
        } else if constexpr (FORM == MDS_FORM_FP32) {
          const float d2 = sizeof(DT) == 8 ? (float)(dd * dd) : (float)d[u] * (float)d[u];
          ((float*)G)[i * np + j] = in ? __builtin_fmaf(-0.5f, d2, hc[j] + hri) : 0.0f;
        } else {
          ((bf16_t*)G)[i * np + j] = in ? to_bf16((float)(-0.5 * (((dd * dd - c[j]) - ri) + m))) : (bf16_t)0;
        }
      }
    }
  }
}

// ---- MFMA G-pass: Yt (fp64, l_pad x np) = (G X)^T --------------------------
// GK: operand kind.  FROM_D: A entries recentred from D in fp32 (projection
// of the bf16 form), else read from the stored G.
template <int GK, bool FROM_D, int KU>
__device__ void block_gpass(const BJob& J, const void* G, const void* Xt, double* Yt, const float* hc,
                            const float* hr) {
#pragma clang fp contract(off)
  using T = typename std::conditional<GK == GK_F64, double, typename std::conditional<GK == GK_F32, float,
                                                                                          bf16_t>::type>::type;
  constexpr int E = 16 / sizeof(T);  // elements per lane per 16-byte chunk
  constexpr int KS = 4 * E;          // K per chunk (four lane groups)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t np = J.n_pad, n = J.n;
  const int CG = J.l_pad / 16;
  const T* Gp = (const T*)G;
  const T* Xp = (const T*)Xt;
  for (int64_t tr = wave; tr < np / 16; tr += 4) {
    const int64_t row = tr * 16 + (lane & 15);
    using Acc = typename std::conditional<GK == GK_F64, doublex4_t, floatx4_t>::type;
    Acc acc[kBMaxL / 16];
#pragma unroll
    for (int cg = 0; cg < kBMaxL / 16; ++cg)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[cg][e] = 0;
    // KU chunks (the K depth of the register tile) are loaded before the
    // MFMAs that use them; KU is the tile shape the autotuner picks
    for (int64_t k0 = 0; k0 < np; k0 += KU * KS) {
      u32x4 a[KU], b[KU][kBMaxL / 16];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int64_t kk = k0 + u * KS + (lane >> 4) * E;
        const bool live = k0 + u * KS < np;  // np is a multiple of 64, KS divides 64
        if constexpr (FROM_D) {
          float g[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int64_t col = kk + t;
            float v = 0.0f;
            if (live && row < n && col < n) {
              float d2;
              if (J.d_is_f64) {
                const double d = ((const double*)J.D)[row * n + col];
                d2 = (float)(d * d);
              } else {
                const float d = ((const float*)J.D)[row * n + col];
                d2 = d * d;
              }
              v = __builtin_fmaf(-0.5f, d2, hc[col] + hr[row]);
            }
            g[t] = v;
          }
          __builtin_memcpy(&a[u], g, 16);
        } else {
          a[u] = live ? *reinterpret_cast<const u32x4*>(Gp + row * np + kk) : u32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int cg = 0; cg < kBMaxL / 16; ++cg)
          b[u][cg] = (live && cg < CG) ? *reinterpret_cast<const u32x4*>(Xp + (int64_t)(cg * 16 + (lane & 15)) * np + kk)
                                       : u32x4{0, 0, 0, 0};
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
#pragma unroll
        for (int cg = 0; cg < kBMaxL / 16; ++cg) {
          if (cg >= CG) break;
          if constexpr (GK == GK_BF16) {
            acc[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[u]),
                                                              __builtin_bit_cast(bf16x8, b[u][cg]), acc[cg], 0, 0, 0);
          } else if constexpr (GK == GK_F32) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
              acc[cg] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[u][t]), __uint_as_float(b[u][cg][t]),
                                                             acc[cg], 0, 0, 0);
          } else {
            const double a0 = __hiloint2double((int)a[u].y, (int)a[u].x);
            const double a1 = __hiloint2double((int)a[u].w, (int)a[u].z);
            const double b0 = __hiloint2double((int)b[u][cg].y, (int)b[u][cg].x);
            const double b1 = __hiloint2double((int)b[u][cg].w, (int)b[u][cg].z);
            acc[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[cg], 0, 0, 0);
            acc[cg] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[cg], 0, 0, 0);
          }
        }
      }
    }
    // accumulator layout: column lane % 16; rows 4g + r (fp32 accumulate)
    // or g + 4r (fp64), g = lane / 16
#pragma unroll
    for (int cg = 0; cg < kBMaxL / 16; ++cg) {
      if (cg >= CG) break;
      double* dst = Yt + (int64_t)(cg * 16 + (lane & 15)) * np + tr * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = GK == GK_F64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        dst[rr] = (double)acc[cg][r];
      }
    }
  }
}

// M (LDS, ld ldm) = A B^T over the l_pad rows of the transposed tall
// matrices At, Bt (l_pad x np fp64), with fp64 MFMA.
__device__ void block_gram(const double* At, const double* Bt, int64_t np, int l_pad, lds_double* M, int ldm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int CG = l_pad / 16;
  for (int t = wave; t < CG * CG; t += 4) {
    const int ta = t / CG, tb = t % CG;
    doublex4_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    const double* pa = At + (int64_t)(ta * 16 + (lane & 15)) * np + (lane >> 4);
    const double* pb = Bt + (int64_t)(tb * 16 + (lane & 15)) * np + (lane >> 4);
    for (int64_t k0 = 0; k0 < np; k0 += 32) {  // np is a multiple of 64
      double xa[8], xb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        xa[u] = pa[k0 + 4 * u];
        xb[u] = pb[k0 + 4 * u];
      }
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], xb[u], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u + 1], xb[u + 1], acc1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) M[(ta * 16 + (lane >> 4) + 4 * r) * ldm + tb * 16 + (lane & 15)] = acc0[r] + acc1[r];
  }
}

// Out^T = (In T)^T: out[b][i] = sum_a T[a][b] in[a][i] (T in LDS, ld ldm),
// rows b >= l and columns i >= n zero; optional cast copy into X (kind xk).
__device__ void block_apply(const double* In, double* Out, int64_t np, int64_t n, int l, int l_pad,
                            const lds_double* Tm, int ldm, void* X, int xk) {
  for (int64_t i = threadIdx.x; i < np; i += kBT) {
    double y[kBMaxL];
#pragma unroll
    for (int a = 0; a < kBMaxL; ++a) y[a] = (a < l) ? In[(int64_t)a * np + i] : 0.0;
    for (int b = 0; b < l_pad; ++b) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < kBMaxL; ++a)
        if (a < l) acc += Tm[a * ldm + b] * y[a];
      const double v = (b < l && i < n) ? acc : 0.0;
      Out[(int64_t)b * np + i] = v;
      if (xk == GK_F64)
        ((double*)X)[(int64_t)b * np + i] = v;
      else if (xk == GK_F32)
        ((float*)X)[(int64_t)b * np + i] = (float)v;
      else if (xk == GK_S2)  // fp32 storage of bf16(fl32(v))
        ((float*)X)[(int64_t)b * np + i] = bf16_value((float)v);
      else if (xk == GK_BF16)
        ((bf16_t*)X)[(int64_t)b * np + i] = to_bf16((float)v);
    }
  }
}

struct BShared {
  JacobiShared sh;
  double M[kBMaxL * kBMaxL + kBMaxL];  // ld kBMaxL, or kBMaxL + 1 (odd) for the Jacobi
  double V[kBMaxL * kBMaxL];  // eigenvectors of B (gfx950: up to 160 KB of LDS per workgroup)
  double P[kBMaxL * kNB];
  double wdiag[kBMaxL];
  double th[kBMaxL];
  int perm[kBMaxL];
  int defl[kBMaxL];
  int dropped;
  double best_v[kBT / 64];
  int64_t best_i[kBT / 64];
};

// T with (Yt)^T T orthonormal from M = W = Y^T Y (in LDS): Cholesky and
// inverse (deflating collapsed pivots: those columns of Q are zero), or the
// first-order factor of an almost orthonormal basis.  Leaves the full T in M
// (strictly lower part zero).
__device__ void block_factor(BShared& S, int l, int l_pad, bool near_identity, DevStatus* st) {
  lds_double* M = (lds_double*)(void*)S.M;
  const int tid = threadIdx.x;
  const int ldm = kBMaxL;
  for (int i = tid; i < l; i += kBT) S.wdiag[i] = M[i * ldm + i];
  __syncthreads();
  if (near_identity) {
    double emax = 0.0;
    for (int e = tid; e < l * l; e += kBT) {
      const int i = e / l, j = e % l;
      emax = fmax(emax, fabs(M[i * ldm + j] - (i == j ? 1.0 : 0.0)));
    }
    emax = block_max<kBT>(emax, S.sh.red);
    if (emax < 1e-9) {
      for (int e = tid; e < l_pad * l_pad; e += kBT) {
        const int i = e / l_pad, j = e % l_pad;
        double t = 0.0;
        if (i < l && j < l) {
          const double x = M[i * ldm + j] - (i == j ? 1.0 : 0.0);
          t = (i == j) ? 1.0 - 0.5 * x : (j > i ? -x : 0.0);
        }
        M[i * ldm + j] = t;  // each entry depends on itself only
      }
      __syncthreads();
      return;
    }
  }
  if (tid == 0) S.dropped = 0;
  __syncthreads();
  chol_blocked<kBT>(M, ldm, l, S.wdiag, S.defl, &S.dropped);
  trinv_blocked<kBT>(M, ldm, l, S.P);
  for (int e = tid; e < l_pad * l_pad; e += kBT) {
    const int i = e / l_pad, j = e % l_pad;
    if (j < i || i >= l || j >= l || S.defl[j]) M[i * ldm + j] = 0.0;  // dropped columns: zero in Q
  }
  __syncthreads();
  if (tid == 0) {
    st->rank_deficient = S.dropped;
    if (S.dropped) atomicAdd(&st->orth_fallbacks, 1);
  }
}

// CholeskyQR2 of Yt into Qt (fp64) with a cast copy of Q into X (kind xk).
__device__ void block_orth(BShared& S, const BJob& J, double* Yt, double* Qt, void* X, int xk) {
  lds_double* M = (lds_double*)(void*)S.M;
  const int64_t np = J.n_pad;
  for (int step = 0; step < 2; ++step) {
    const double* In = step == 0 ? Yt : Qt;
    __syncthreads();
    block_gram(In, In, np, J.l_pad, M, kBMaxL);
    __syncthreads();
    block_factor(S, J.l, J.l_pad, step == 1, J.st);
    __syncthreads();
    // step 0 writes Q1 over Y (In = Yt, Out = Qt would alias in step 1), so:
    // step 0: Qt = Y T; step 1: Yt = Qt T, then the result is copied back
    block_apply(In, step == 0 ? Qt : Yt, np, J.n, J.l, J.l_pad, M, kBMaxL, step == 1 ? X : nullptr,
                step == 1 ? xk : -1);
    __syncthreads();
  }
  for (int64_t e = threadIdx.x; e < (int64_t)J.l_pad * np; e += kBT) Qt[e] = Yt[e];
  __syncthreads();
}

// Column r of the n x k row-major coords: make the entry of largest
// magnitude positive (lowest row index on ties).
__device__ void block_sign(BShared& S, double* C, int64_t n, int k, int r) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double bv = -1.0;
  int64_t bi = 0;
  for (int64_t i = tid; i < n; i += kBT) {
    const double v = fabs(C[i * k + r]);
    if (v > bv) {
      bv = v;
      bi = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int64_t oi = __shfl_xor(bi, off, 64);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    S.best_v[wave] = bv;
    S.best_i[wave] = bi;
  }
  __syncthreads();
  bv = S.best_v[0];
  bi = S.best_i[0];
  for (int w = 1; w < kBT / 64; ++w)
    if (S.best_v[w] > bv || (S.best_v[w] == bv && S.best_i[w] < bi)) {
      bv = S.best_v[w];
      bi = S.best_i[w];
    }
  const bool flip = C[bi * k + r] < 0.0;
  __syncthreads();
  if (flip)
    for (int64_t i = tid; i < n; i += kBT) C[i * k + r] = -C[i * k + r];
}

template <int FORM, int KU>
__device__ void batch_instance(const BJob& J, BShared& S);

__global__ void k_batch_reset(int* counter) { *counter = 0; }

// The job table is written by kernels from their arguments (at most
// kTableChunk jobs per launch), so enqueueing a batch copies no host memory.
constexpr int kTableChunk = 32;
struct BChunk {
  int first, count;
  BJob job[kTableChunk];
};
__global__ void k_batch_table(BChunk c, BJob* __restrict__ table) {
  if ((int)threadIdx.x < c.count) table[c.first + threadIdx.x] = c.job[threadIdx.x];
}

// Persistent launch: each workgroup takes instances from the table until it
// is exhausted (every workgroup reaches the exit; no workgroup waits on
// another).
template <int FORM, int KU>
__global__ __launch_bounds__(kBT, 1) void k_batch(const BJob* __restrict__ table, int count, int* counter) {
  __shared__ BShared S;
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int t = next;
    __syncthreads();  // every thread has read `next` before thread 0 overwrites it
    if (t >= count) return;
    const BJob job = table[t];
    batch_instance<FORM, KU>(job, S);
    __syncthreads();
  }
}

template <int FORM, int KU>
__device__ void batch_instance(const BJob& J, BShared& S) {
#pragma clang fp contract(off)
  lds_double* M = (lds_double*)(void*)S.M;
  const int tid = threadIdx.x;
  const int64_t n = J.n, np = J.n_pad;
  const int l = J.l, l_pad = J.l_pad, k = J.k;
  const BLayout Lo = blayout(np, l_pad, FORM);
  double* r = (double*)(J.ws + Lo.r);
  double* c = (double*)(J.ws + Lo.c);
  float* hc = (float*)(J.ws + Lo.hc);
  float* hr = (float*)(J.ws + Lo.hr);
  void* G = J.ws + Lo.G;
  void* X = J.ws + Lo.X;
  double* Yt = (double*)(J.ws + Lo.Y);
  double* Qt = (double*)(J.ws + Lo.Q);
  constexpr int GK = FORM == MDS_FORM_FP64 ? GK_F64 : (FORM == MDS_FORM_FP32 ? GK_F32 : GK_BF16);
  constexpr int PK = FORM == MDS_FORM_FP64 ? GK_F64 : GK_F32;  // projection operand
  // the bf16 form's first and last range passes recentre D in fp32 (like its
  // projection), the last with bf16-valued X; the passes between them read
  // the stored bf16 G
  const int passes = 2 * J.q + 1;
  auto f32_pass = [&](int it) { return FORM == MDS_FORM_BF16 && (it == 0 || it == passes - 1); };
  const bool store_g = !(FORM == MDS_FORM_BF16 && J.q == 0);

  if (tid == 0) {
    DevStatus z = {};
    *J.st = z;
  }
  // ---- centring sums (fp64): column means by thread, row means by wave ----
  double rsum_part;
  if (J.d_is_f64) {
    col_means<double>((const double*)J.D, n, np, c);
    rsum_part = row_means<double>((const double*)J.D, n, np, r);
  } else {
    col_means<float>((const float*)J.D, n, np, c);
    rsum_part = row_means<float>((const float*)J.D, n, np, r);
  }
  const double m = block_sum<kBT>(rsum_part, S.sh.red) / (double)n;
  __syncthreads();
  if (tid == 0 && !(m == m && fabs(m) <= 1.7976931348623157e308)) J.st->nonfinite = 1;
  for (int64_t j = tid; j < np; j += kBT) {
    hc[j] = j < n ? (float)(0.5 * c[j]) : 0.0f;
    hr[j] = j < n ? (float)(0.5 * (r[j] - m)) : 0.0f;
  }
  __syncthreads();
  // ---- G in the pass dtype ------------------------------------------------
  if (store_g) {
    if (J.d_is_f64)
      write_g<FORM, double>((const double*)J.D, n, np, r, c, m, hc, hr, G);
    else
      write_g<FORM, float>((const float*)J.D, n, np, r, c, m, hc, hr, G);
  }
  // ---- Omega in the first pass's operand dtype (transposed, l_pad x np) -----
  for (int64_t e = tid; e < np * (l_pad / 4); e += kBT) {
    const int64_t i = e % np, b = e / np;
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < n && 4 * b < l) omega::omega_block(J.seed, i, b, z);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t col = 4 * b + t;
      const double v = col < l ? z[t] : 0.0;
      if constexpr (GK == GK_F64)
        ((double*)X)[col * np + i] = v;
      else if constexpr (GK == GK_F32 || FORM == MDS_FORM_BF16)  // bf16: fp32 first pass
        ((float*)X)[col * np + i] = (float)v;
      else
        ((bf16_t*)X)[col * np + i] = to_bf16((float)v);
    }
  }
  __syncthreads();
  // ---- range finder ---------------------------------------------------------
  for (int it = 0; it < passes; ++it) {
    if (f32_pass(it))
      block_gpass<GK_F32, true, KU>(J, nullptr, X, Yt, hc, hr);
    else
      block_gpass<GK, false, KU>(J, G, X, Yt, hc, hr);
    const int next = it == passes - 1 ? PK : (f32_pass(it + 1) ? (int)GK_S2 : GK);
    block_orth(S, J, Yt, Qt, X, next);
  }
  // ---- projection B = Q^T G Q ------------------------------------------------
  if constexpr (FORM == MDS_FORM_BF16)
    block_gpass<GK_F32, true, KU>(J, nullptr, X, Yt, hc, hr);
  else
    block_gpass<PK, false, KU>(J, G, X, Yt, hc, hr);
  __syncthreads();
  block_gram(Qt, Yt, np, l_pad, M, kBMaxL);
  __syncthreads();
  for (int e = tid; e < kBMaxL * kBMaxL; e += kBT) {
    const int i = e / kBMaxL, j = e % kBMaxL;
    double v = 0.0;
    if (i < l && j < l) v = 0.5 * (M[i * kBMaxL + j] + M[j * kBMaxL + i]);
    S.V[e] = v;  // symmetrised B staged in V
  }
  __syncthreads();
  constexpr int ldj = kBMaxL + 1;  // odd: the Jacobi's (min, max) accesses spread over LDS banks
  for (int e = tid; e < kBMaxL * kBMaxL; e += kBT) {
    M[(e / kBMaxL) * ldj + e % kBMaxL] = S.V[e];
    S.V[e] = (e / kBMaxL == e % kBMaxL) ? 1.0 : 0.0;
  }
  __syncthreads();
  // ---- eigenpairs of B ------------------------------------------------------
  int rounds = 0;
  const int sweeps = jacobi<kBT>(M, ldj, S.V, kBMaxL, (double2*)nullptr, l + (l & 1), S.sh, &rounds);
  __syncthreads();
  for (int i = tid; i < l; i += kBT) S.th[i] = M[i * ldj + i];
  __syncthreads();
  for (int i = tid; i < l; i += kBT) S.perm[desc_rank(S.th, l, i)] = i;  // a permutation, NaN included
  __syncthreads();
  // Tc = V_k diag(sqrt(max(theta, 0))) into M (l x k, ld kBMaxL)
  for (int e = tid; e < kBMaxL * kBMaxL; e += kBT) {
    const int a = e / kBMaxL, rr = e % kBMaxL;
    double v = 0.0;
    if (a < l && rr < k) {
      const double thr = S.th[S.perm[rr]];
      v = S.V[a * kBMaxL + S.perm[rr]] * sqrt(fmax(thr, 0.0));
    }
    M[e] = v;
  }
  if (tid < k) J.eigvals[tid] = S.th[S.perm[tid]];
  if (tid == 0) {
    J.st->jacobi_sweeps = sweeps < 0 ? -sweeps : sweeps;
    if (sweeps < 0) atomicAdd(&J.st->jacobi_unconv, 1);
  }
  __syncthreads();
  // ---- coordinates X = Q Tc, signs ------------------------------------------
  for (int64_t i = tid; i < n; i += kBT) {
    double qv[kBMaxL];
#pragma unroll
    for (int a = 0; a < kBMaxL; ++a) qv[a] = (a < l) ? Qt[(int64_t)a * np + i] : 0.0;
    for (int rr = 0; rr < k; ++rr) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < kBMaxL; ++a)
        if (a < l) acc += qv[a] * M[a * kBMaxL + rr];
      J.coords[i * k + rr] = acc;
    }
  }
  __syncthreads();
  for (int rr = 0; rr < k; ++rr) block_sign(S, J.coords, n, k, rr);
  __syncthreads();
  if (tid == 0 && J.status_out) {
    const DevStatus& d = *J.st;
    *J.status_out = d.nonfinite ? MDS_ERR_NONFINITE : (d.jacobi_unconv ? MDS_ERR_NUMERICAL : MDS_OK);
  }
}

}  // namespace
}  // namespace mds

using namespace mds;

int mds::batch_max_l() { return kBMaxL; }
int64_t mds::batch_max_n() { return kBMaxN; }

namespace {

// Workgroups of the persistent launch: as many as the device holds at once
// (one per CU at this kernel's LDS and register use), never more than the
// instances.
template <int FORM, int KU>
int persistent_grid(int count) {
  static int per_device[64] = {0};  // workgroups that fit, per device
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int g = per_device[dev];
  if (g == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<FORM, KU>, kBT, 0) != hipSuccess ||
        per_cu <= 0)
      per_cu = 1;
    g = cus * per_cu;
    per_device[dev] = g;
  }
  return count < g ? count : g;
}

template <int FORM, int KU>
void launch_fk(const BJob* table, int count, int* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, counter);
  hipLaunchKernelGGL((k_batch<FORM, KU>), dim3(persistent_grid<FORM, KU>(count)), dim3(kBT), 0, s, table, count,
                     counter);
}

template <int FORM>
void launch_form(int ku, const BJob* table, int count, int* counter, hipStream_t s) {
  switch (ku) {
    case 1: launch_fk<FORM, 1>(table, count, counter, s); break;
    case 2: launch_fk<FORM, 2>(table, count, counter, s); break;
    default: launch_fk<FORM, 4>(table, count, counter, s); break;
  }
}

void launch_batch(int form, int ku, const BJob* table, int count, int* counter, hipStream_t s) {
  if (form == MDS_FORM_FP64)
    launch_form<MDS_FORM_FP64>(ku, table, count, counter, s);
  else if (form == MDS_FORM_FP32)
    launch_form<MDS_FORM_FP32>(ku, table, count, counter, s);
  else
    launch_form<MDS_FORM_BF16>(ku, table, count, counter, s);
}

// Process-wide autotuning table: (form, size class of n_pad, l_pad) -> KU.
std::mutex g_tune_mu;
std::map<uint64_t, int> g_tune;
constexpr int kDefaultKU = 4;
constexpr int kKUs[] = {1, 2, 4};

uint64_t tune_key(int form, int64_t np, int l_pad) {
  int cls = 0;
  while ((int64_t(64) << cls) < np) ++cls;  // n_pad <= 64 * 2^cls
  return ((uint64_t)form << 32) | ((uint64_t)cls << 16) | (uint64_t)l_pad;
}

int tuned_ku(int form, int64_t np, int l_pad) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(tune_key(form, np, l_pad));
  return it == g_tune.end() ? kDefaultKU : it->second;
}

// Symmetric matrix with zero diagonal and entries in [1, 2) from a hash of
// (min(i, j), max(i, j)): a full-rank G for timing the batched kernel.
__global__ void k_synth_d(float* D, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e / n, j = e % n;
  uint64_t h = (uint64_t)(i < j ? i : j) * 0x9E3779B97F4A7C15ull ^ (uint64_t)(i < j ? j : i) * 0xC2B2AE3D27D4EB4Full;
  h ^= h >> 29;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 32;
  D[e] = i == j ? 0.0f : 1.0f + (float)(h >> 40) * 0x1p-24f;
}

mds_status batch_check(const mds_batch_job* jobs, int32_t count, int32_t form) {
  if (!jobs || count < 0) return fail(MDS_ERR_INVALID_ARG, "NULL jobs or count < 0");
  if (form < MDS_FORM_FP64 || form > MDS_FORM_BF16) return fail(MDS_ERR_INVALID_ARG, "unknown form %d", form);
  for (int32_t i = 0; i < count; ++i) {
    const mds_batch_job& b = jobs[i];
    const int64_t l = (int64_t)b.k + b.oversample;
    if (b.n < 2 || b.n > kBMaxN) return fail(MDS_ERR_INVALID_ARG, "job %d: n = %lld outside [2, %lld]", i,
                                             (long long)b.n, (long long)kBMaxN);
    if (b.k < 1 || b.oversample < 0 || b.q < 0 || l > b.n || rup(l, 16) > kBMaxL)
      return fail(MDS_ERR_INVALID_ARG, "job %d: k = %d, oversample = %d, q = %d (need k + oversample <= "
                  "min(n, %d))", i, b.k, b.oversample, b.q, kBMaxL);
    if (b.d_dtype != MDS_DTYPE_F32 && b.d_dtype != MDS_DTYPE_F64)
      return fail(MDS_ERR_INVALID_ARG, "job %d: unknown D dtype %d", i, b.d_dtype);
  }
  return MDS_OK;
}

size_t job_bytes(const mds_batch_job& b, int form) {
  const int l_pad = (int)rup((int64_t)b.k + b.oversample, 16);
  return (size_t)blayout(rup(b.n, kBPad), l_pad, form).total;
}

// Enqueue a checked batch into `workspace` (a BHead followed by the
// per-instance regions): job table (ordered by decreasing work), counter
// reset and the persistent launch.  status_out: optional device array of
// count words for the final status of each instance.
mds_status enqueue_batch(const mds_batch_job* jobs, int32_t count, int32_t form, char* base, int32_t tile,
                         int32_t* status_out, hipStream_t s) {
  const BHead H = bhead(count);
  DevStatus* stat = reinterpret_cast<DevStatus*>(base + H.status);
  std::vector<BJob> table((size_t)count);
  std::vector<double> work((size_t)count);
  size_t off = (size_t)H.total;
  int64_t np_max = 0;
  int lp_max = 0;
  for (int32_t i = 0; i < count; ++i) {
    const mds_batch_job& b = jobs[i];
    BJob& J = table[i];
    J.D = b.D;
    J.coords = b.coords;
    J.eigvals = b.eigvals;
    J.ws = base + off;
    J.st = stat + i;
    J.status_out = status_out ? status_out + i : nullptr;
    J.n = b.n;
    J.n_pad = rup(b.n, kBPad);
    J.seed = b.seed;
    J.k = b.k;
    J.l = b.k + b.oversample;
    J.l_pad = (int)rup(J.l, 16);
    J.q = b.q;
    J.d_is_f64 = b.d_dtype == MDS_DTYPE_F64;
    J.pad_ = 0;
    off += job_bytes(b, form);
    work[i] = (double)J.n_pad * (double)J.n_pad * (2 * J.q + 3) * J.l_pad;
    np_max = J.n_pad > np_max ? J.n_pad : np_max;
    lp_max = J.l_pad > lp_max ? J.l_pad : lp_max;
  }
  // largest instances first: the persistent grid then ends with short ones
  std::vector<int32_t> order((size_t)count);
  for (int32_t i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
  std::vector<BJob> sorted((size_t)count);
  for (int32_t i = 0; i < count; ++i) sorted[i] = table[order[i]];
  BJob* dtable = reinterpret_cast<BJob*>(base + H.table);
  for (int32_t i0 = 0; i0 < count; i0 += kTableChunk) {
    BChunk c{};
    c.first = i0;
    c.count = count - i0 < kTableChunk ? count - i0 : kTableChunk;
    for (int t = 0; t < c.count; ++t) c.job[t] = sorted[i0 + t];
    hipLaunchKernelGGL(k_batch_table, dim3(1), dim3(kTableChunk), 0, s, c, dtable);
  }
  mds_status st = hip_check(hipGetLastError(), "batch job table");
  if (st != MDS_OK) return st;
  const int ku = tile > 0 ? tile : tuned_ku(form, np_max, lp_max);
  launch_batch(form, ku, dtable, count, reinterpret_cast<int*>(base + H.counter), s);
  return hip_check(hipGetLastError(), "k_batch launch");
}

mds_status batch_args(const mds_batch_job* jobs, int32_t count, int32_t form, int32_t tile) {
  mds_status st = batch_check(jobs, count, form);
  if (st != MDS_OK) return st;
  if (tile != 0 && tile != 1 && tile != 2 && tile != 4) return fail(MDS_ERR_INVALID_ARG, "tile = %d", tile);
  for (int32_t i = 0; i < count; ++i)
    if (!jobs[i].D || !jobs[i].coords || !jobs[i].eigvals)
      return fail(MDS_ERR_INVALID_ARG, "job %d: NULL D, coords or eigvals", i);
  return MDS_OK;
}

mds_status have_device() {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(MDS_ERR_NO_DEVICE, "no HIP device available");
  }
  return MDS_OK;
}

}  // namespace

extern "C" {

mds_status mds_batch_workspace_size(const mds_batch_job* jobs, int32_t count, int32_t form, size_t* bytes) {
  if (!bytes) return fail(MDS_ERR_INVALID_ARG, "bytes is NULL");
  const mds_status st = batch_check(jobs, count, form);
  if (st != MDS_OK) return st;
  size_t total = (size_t)bhead(count).total;
  for (int32_t i = 0; i < count; ++i) total += job_bytes(jobs[i], form);
  *bytes = total;
  return MDS_OK;
}

mds_status mds_run_batch(const mds_batch_job* jobs, int32_t count, int32_t form, void* workspace, size_t bytes,
                         int32_t tile, void* stream) {
  mds_status st = batch_args(jobs, count, form, tile);
  if (st != MDS_OK) return st;
  size_t need = 0;
  mds_batch_workspace_size(jobs, count, form, &need);
  if (!workspace || bytes < need || ((uintptr_t)workspace % 256) != 0)
    return fail(MDS_ERR_INVALID_ARG, "workspace NULL, unaligned or smaller than %zu bytes", need);
  if (count == 0) return MDS_OK;
  st = have_device();
  if (st != MDS_OK) return st;
  return enqueue_batch(jobs, count, form, static_cast<char*>(workspace), tile, nullptr, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Device memory of mds_run_batch_static: a file-scope array, one copy per
// device, held until the process ends.  Host code never passes the array's
// name to a kernel: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is used.
constexpr size_t kStaticScratchBytes = MDS_BATCH_STATIC_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Address of this device's scratch (the current device), looked up on the
// first call on the device.
mds_status static_scratch(char** out) {
  int dev = 0;
  mds_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st != MDS_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) return fail(MDS_ERR_NO_DEVICE, "device %d outside the supported range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st != MDS_OK) return st;
    if (!p || ((uintptr_t)p % 256) != 0) return fail(MDS_ERR_HIP, "scratch address %p not 256-byte aligned", p);
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return MDS_OK;
}

}  // namespace

extern "C" {

mds_status mds_run_batch_static(const mds_batch_job* jobs, int32_t count, int32_t form, int32_t tile,
                                int32_t* statuses, void* stream) {
  mds_status st = batch_args(jobs, count, form, tile);
  if (st != MDS_OK) return st;
  size_t need = 0;
  mds_batch_workspace_size(jobs, count, form, &need);
  if (need > kStaticScratchBytes)
    return fail(MDS_ERR_INVALID_ARG, "batch needs %zu bytes of workspace; the static scratch holds %zu", need,
                kStaticScratchBytes);
  if (count == 0) return MDS_OK;
  st = have_device();
  if (st != MDS_OK) return st;
  char* base = nullptr;
  st = static_scratch(&base);
  if (st != MDS_OK) return st;
  return enqueue_batch(jobs, count, form, base, tile, statuses, (hipStream_t)stream);
}

mds_status mds_autotune_batch(int32_t form, int64_t n, int32_t k, int32_t oversample, int32_t q, int32_t batch,
                              void* stream, mds_batch_tune* out) {
  if (!out || batch < 1 || batch > 4096) return fail(MDS_ERR_INVALID_ARG, "NULL out or batch outside [1, 4096]");
  mds_batch_job probe{};
  probe.D = (void*)256;
  probe.coords = (double*)256;
  probe.eigvals = (double*)256;
  probe.n = n;
  probe.k = k;
  probe.oversample = oversample;
  probe.q = q;
  mds_status st = batch_check(&probe, 1, form);
  if (st != MDS_OK) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(MDS_ERR_NO_DEVICE, "no HIP device available");
  }
  hipStream_t s = (hipStream_t)stream;
  float* D = nullptr;
  double* outs = nullptr;
  void* ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  mds_plan_t plan = nullptr;
  std::vector<mds_batch_job> jobs((size_t)batch, probe);
  size_t wsb = 0;
  const size_t per = (size_t)n * k + k;
  auto cleanup = [&](mds_status r) {
    if (plan) mds_destroy(plan);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(D);
    (void)hipFree(outs);
    (void)hipFree(ws);
    return r;
  };
  if (hipMalloc((void**)&D, (size_t)n * n * 4) != hipSuccess ||
      hipMalloc((void**)&outs, per * batch * sizeof(double)) != hipSuccess)
    return cleanup(fail(MDS_ERR_OOM, "autotune allocation failed"));
  for (int32_t b = 0; b < batch; ++b) {
    jobs[b].D = D;
    jobs[b].coords = outs + per * b;
    jobs[b].eigvals = outs + per * b + (size_t)n * k;
    jobs[b].d_dtype = MDS_DTYPE_F32;
    jobs[b].seed = (uint64_t)b;
  }
  mds_batch_workspace_size(jobs.data(), batch, form, &wsb);
  if (hipMalloc(&ws, wsb) != hipSuccess) return cleanup(fail(MDS_ERR_OOM, "autotune workspace allocation failed"));
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return cleanup(fail(MDS_ERR_HIP, "event creation failed"));
  hipLaunchKernelGGL(k_synth_d, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, D, n);
  auto time_ms = [&](auto&& run, float* ms) -> mds_status {
    mds_status r = run();  // warm-up
    if (r != MDS_OK) return r;
    float best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      (void)hipEventRecord(e0, s);
      r = run();
      if (r != MDS_OK) return r;
      (void)hipEventRecord(e1, s);
      r = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
      if (r != MDS_OK) return r;
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      best = t < best ? t : best;
    }
    *ms = best;
    return MDS_OK;
  };
  out->tile = kDefaultKU;
  float best = 1e30f;
  for (int v = 0; v < 3; ++v) {
    float ms = 0.f;
    st = time_ms([&] { return mds_run_batch(jobs.data(), batch, form, ws, wsb, kKUs[v], stream); }, &ms);
    if (st != MDS_OK) return cleanup(st);
    out->batch_ms_per_job[v] = ms / batch;
    if (ms < best) {
      best = ms;
      out->tile = kKUs[v];
    }
  }
  out->batch_ms_best = best / batch;
  // the plan path on one instance, for the batching decision
  mds_opts o = {form, MDS_DTYPE_F32, 0, 0};
  st = mds_plan_ex(&plan, n, k, oversample, q, 0, &o);
  if (st != MDS_OK) return cleanup(st);
  st = time_ms([&] { return mds_run(plan, D, outs, outs + (size_t)n * k, stream); }, &out->plan_ms);
  if (st != MDS_OK) return cleanup(st);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[tune_key(form, rup(n, kBPad), (int)rup((int64_t)k + oversample, 16))] = out->tile;
  }
  return cleanup(MDS_OK);
}

mds_status mds_batch_status(const void* workspace, int32_t count, int32_t* statuses, void* stream) {
  if (!workspace || !statuses || count < 0) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  if (count == 0) return MDS_OK;
  std::vector<DevStatus> h((size_t)count);
  mds_status st = hip_check(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
  if (st != MDS_OK) return st;
  st = hip_check(hipMemcpy(h.data(), workspace, (size_t)count * sizeof(DevStatus), hipMemcpyDeviceToHost),
                 "status copy");
  if (st != MDS_OK) return st;
  for (int32_t i = 0; i < count; ++i)
    statuses[i] = h[i].nonfinite ? MDS_ERR_NONFINITE : (h[i].jacobi_unconv ? MDS_ERR_NUMERICAL : MDS_OK);
  return MDS_OK;
}

}  // extern "C"
