// Block-level fp64 helpers shared by the small dense kernels (one workgroup
// per l x l problem) and the batched small-MDS kernel: reductions, cyclic
// Jacobi with the round-robin parallel ordering, blocked Cholesky and the
// blocked inverse of an upper triangular factor.  See k_small.hip for the
// methods.
#pragma once

#include "mds_internal.h"

namespace mds {
namespace small {

constexpr int kEigThreads = 1024;  // small_eig workgroup
constexpr int kOrthRegThreads = 1024;  // orth_factor workgroup, l_pad <= 128 (register-resident factor)
constexpr int kSmallLMax = 64;              // l_pad up to which orth_factor runs a quarter of the threads
constexpr int kOrthRegThreadsSmall = 256;   // orth_factor workgroup, l_pad <= kSmallLMax
constexpr int kRegSlots = 16;  // rows per thread of the register-resident factor
constexpr int kNB = 16;            // panel width of the blocked Cholesky / inverse
// Deflation of the orthonormalisation factor: a Cholesky pivot of W = Y^T Y
// at or below kDeflate times its column's diagonal entry of W (column j of Y
// keeps a relative residual of at most 1e-7 after the earlier columns are
// projected out), or not positive, drops column j: its row of R is e_j, no
// later column is updated with it, and T = R^{-1} gets a zero row and column
// j (column j of Q is exactly zero).  The kept columns have a condition
// number below about 1e7, inside CholeskyQR2's range (u^{-1/2}).
constexpr double kDeflate = 1e-14;
constexpr int kMaxPairs = kMaxL / 2;
constexpr int kMaxSweeps = 40;

typedef __attribute__((address_space(3))) double lds_double;

struct JacobiShared {
  int2 pq[kMaxPairs];
  double2 cs[kMaxPairs];
  double t[kMaxPairs];
  int nrot;
  double red[kEigThreads / 64];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int kThreads>
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

template <int kThreads>
__device__ double block_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < kThreads / 64; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

// Round-robin (chess tournament) pairing of le indices: in round r of a
// sweep, position t pairs index le - 1 with r (t = 0) or (r + t) with
// (r - t), modulo le - 1; returned with p < q.  Callers keep 0 <= r < le - 1
// and 0 <= t < le / 2, so one conditional subtraction or addition replaces
// each reduction modulo le - 1.
__device__ __forceinline__ void round_robin_pair(int le, int r, int t, int& p, int& q) {
  const int m = le - 1;
  if (t == 0) {
    p = m;
    q = r;
  } else {
    p = r + t;
    p -= p >= m ? m : 0;
    q = r - t;
    q += q < 0 ? m : 0;
  }
  if (p > q) {
    const int x = p;
    p = q;
    q = x;
  }
}

// Squared Frobenius norm and squared off-diagonal norm of the symmetric
// le x le matrix held in the upper triangle of M (diagonal included).
template <int kThreads, typename MT>
__device__ void upper_norms2(MT M, int ldm, int le, double& fro2, double& off2) {
  double d = 0.0, o = 0.0;
  for (int e = threadIdx.x; e < le * le; e += kThreads) {
    const int i = e / le, j = e % le;
    if (j < i) continue;
    const double v = M[i * ldm + j];
    if (i == j)
      d += v * v;
    else
      o += 2.0 * v * v;
  }
  fro2 = d + o;
  off2 = o;
}

// Offset of entry (i, j) of a symmetric matrix kept in the upper triangle.
__device__ __forceinline__ int upper_at(int i, int j, int ldm) { return i < j ? i * ldm + j : j * ldm + i; }

// 1/x and 1/sqrt(y) for normal fp64 arguments: the hardware estimate refined
// by two Newton steps (each at least doubles the correct bits), giving a
// result within about one ulp without the IEEE division and square-root
// sequences.
__device__ __forceinline__ double rcp_newton(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsqrt_newton(double y) {
  double r = __builtin_amdgcn_rsq(y);
  r = r * fma(-0.5 * y, r * r, 1.5);
  return r * fma(-0.5 * y, r * r, 1.5);
}

// Cyclic Jacobi on the symmetric le x le matrix M (ld ldm; le even, a padding
// row/column of zeros is never rotated).  Only the upper triangle of M
// (diagonal included) is read and updated: each round rotates the 2x2 blocks
// of pairs a <= b, whose entries are addressed by (min, max) index, so an
// odd ldm keeps the LDS accesses of a wave on distinct banks.  On return the
// upper triangle holds the rotated matrix (eigenvalues on the diagonal); the
// strict lower triangle is left as it was.  Either accumulates V <- V J in
// place (V != nullptr, ld ldv, identity on entry) or records (c, s) of every
// pair and round in rot (rot != nullptr).  Returns sweeps used (negative if
// the cap was hit); *rounds receives the number of rounds recorded.
template <int kThreads, typename MT>
__device__ int jacobi(MT M, int ldm, double* V, int ldv, double2* rot, int le, JacobiShared& sh, int* rounds) {
  constexpr int kMaxBlocksPerThread = ((kMaxL / 2) * (kMaxL / 2 + 1) / 2 + kThreads - 1) / kThreads;
  const int tid = threadIdx.x;
  const int np = le / 2;
  // this thread's fixed (pair a, pair b) blocks, a <= b, in row-major order
  // of the upper triangle; pairs are renamed every round but the block list
  // of a thread is the same in all rounds
  int nblk = 0;
  int blk[kMaxBlocksPerThread];
  for (int e = tid; e < np * (np + 1) / 2 && nblk < kMaxBlocksPerThread; e += kThreads) {
    int a = 0, rem = e;
    while (rem >= np - a) rem -= np - a++;
    blk[nblk++] = (a << 16) | (a + rem);
  }
  double fro2, off2;
  upper_norms2<kThreads>(M, ldm, le, fro2, off2);
  const double fro = sqrt(block_sum<kThreads>(fro2, sh.red));
  const double thr = 1e-17 * fro;
  int nr = 0;
  int sweep = 0;
  bool converged = false;
  for (; sweep < kMaxSweeps && !converged; ++sweep) {
    if (tid == 0) sh.nrot = 0;
    __syncthreads();
    for (int r = 0; r < le - 1; ++r, ++nr) {
      if (tid < np) {
        int p, q;
        round_robin_pair(le, r, tid, p, q);
        const double app = M[p * ldm + p], aqq = M[q * ldm + q], apq = M[p * ldm + q];
        double c = 1.0, s = 0.0, t = 0.0;
        if (fabs(apq) > thr) {
          // tan of the rotation angle, the root of t^2 + 2 tau t - 1 = 0 of
          // smaller magnitude; cos = 1/sqrt(1 + t^2), sin = t cos
          if (fabs(apq) > 1e-200) {
            const double tau = (aqq - app) * rcp_newton(2.0 * apq);
            const double y = fma(tau, tau, 1.0);  // finite up to |tau| ~ 1e154
            t = fabs(tau) > 1e150 ? 0.5 * rcp_newton(tau)
                                  : (tau >= 0.0 ? 1.0 : -1.0) * rcp_newton(fma(y, rsqrt_newton(y), fabs(tau)));
            c = rsqrt_newton(fma(t, t, 1.0));
          } else {  // off-diagonal near the fp64 underflow range: IEEE operations
            const double tau = (aqq - app) / (2.0 * apq);
            t = fabs(tau) > 1e150 ? 0.5 / tau : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
          }
          s = t * c;
          sh.nrot = 1;  // any rotation this sweep (all writers store the same value)
        }
        sh.pq[tid] = make_int2(p, q);
        sh.cs[tid] = make_double2(c, s);
        sh.t[tid] = t;
        if (rot) rot[(int64_t)nr * np + tid] = make_double2(c, s);
      }
      __syncthreads();
      // M <- J^T M J, one 2x2 block (pair a rows, pair b columns, a <= b) at a
      // time.  All loads of this thread's blocks are issued before any store
      // (the blocks are disjoint), so their LDS latencies overlap.
      for (int u0 = 0; u0 < nblk; u0 += 4) {
        double m[4][4];
        int idx[4][4];
        bool act[4];
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) {
          const int u = u0 + uu;
          act[uu] = false;
          if (u < nblk) {
            const int a = blk[u] >> 16, b = blk[u] & 0xffff;
            act[uu] = sh.cs[a].y != 0.0 || sh.cs[b].y != 0.0;
            const int2 pqa = sh.pq[a], pqb = sh.pq[b];
            idx[uu][0] = upper_at(pqa.x, pqb.x, ldm);
            idx[uu][1] = upper_at(pqa.x, pqb.y, ldm);
            idx[uu][2] = upper_at(pqa.y, pqb.x, ldm);  // == idx[uu][1] when a == b
            idx[uu][3] = upper_at(pqa.y, pqb.y, ldm);
            if (act[uu]) {
#pragma unroll
              for (int e = 0; e < 4; ++e) m[uu][e] = M[idx[uu][e]];
            }
          }
        }
#pragma unroll
        for (int uu = 0; uu < 4; ++uu) {
          if (!act[uu]) continue;
          const int u = u0 + uu;
          const int a = blk[u] >> 16, b = blk[u] & 0xffff;
          const double m00 = m[uu][0], m01 = m[uu][1], m10 = m[uu][2], m11 = m[uu][3];
          if (a == b) {
            const double t = sh.t[a];
            M[idx[uu][0]] = m00 - t * m01;
            M[idx[uu][3]] = m11 + t * m01;
            M[idx[uu][1]] = 0.0;
          } else {
            const double2 csa = sh.cs[a], csb = sh.cs[b];
            const double ca = csa.x, sa = csa.y, cb = csb.x, sb = csb.y;
            // rows: r_p = c x_p - s x_q, r_q = s x_p + c x_q
            const double r00 = ca * m00 - sa * m10, r01 = ca * m01 - sa * m11;
            const double r10 = sa * m00 + ca * m10, r11 = sa * m01 + ca * m11;
            // columns: y_p = c r_p - s r_q, y_q = s r_p + c r_q
            M[idx[uu][0]] = cb * r00 - sb * r01;
            M[idx[uu][1]] = sb * r00 + cb * r01;
            M[idx[uu][2]] = cb * r10 - sb * r11;
            M[idx[uu][3]] = sb * r10 + cb * r11;
          }
        }
      }
      if (V) {
        for (int i = tid / np; i < le; i += kThreads / np) {
          const int b = tid % np;
          if (tid >= (kThreads / np) * np) break;
          const double2 csb = sh.cs[b];
          if (csb.y == 0.0) continue;
          const int2 pqb = sh.pq[b];
          const double vp = V[i * ldv + pqb.x], vq = V[i * ldv + pqb.y];
          V[i * ldv + pqb.x] = csb.x * vp - csb.y * vq;
          V[i * ldv + pqb.y] = csb.y * vp + csb.x * vq;
        }
      }
      __syncthreads();
    }
    const int nrot = sh.nrot;
    upper_norms2<kThreads>(M, ldm, le, fro2, off2);
    const double off = sqrt(block_sum<kThreads>(off2, sh.red));
    converged = (nrot == 0) || (off <= 1e-15 * fro);
  }
  *rounds = nr;
  return converged ? sweep : -sweep;
}

// ---- orthonormalisation factor ----------------------------------------------
// Blocked right-looking Cholesky W = R^T R (upper R in M).  Panel rows
// [k0, k0+16) are factored by wave 0 alone (wave-synchronous, no workgroup
// barrier); the trailing update M22 -= R12^T R12 is done by all threads with
// 4x4 register tiles.  Deflates collapsed pivots (kDeflate): defl[j] = 1 for
// a dropped column (its row of R is e_j), *ndefl counts them.
template <int NT, typename MT>
__device__ void chol_blocked(MT M, int ldm, int l, const double* wdiag, int* defl, int* ndefl) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k0 = 0; k0 < l; k0 += kNB) {
    const int nb = (l - k0 < kNB) ? l - k0 : kNB;
    if (wave == 0) {
      // left-looking inside the panel: row kk of R from the finished panel
      // rows above it (loads only, then one store per entry)
      for (int kk = k0; kk < k0 + nb; ++kk) {
        const int nm = kk - k0;  // finished rows in this panel
        // loads are unconditional from in-bounds addresses (k0 + 15 < l_pad,
        // columns clamped) and masked by selects, so they issue back to back
        double col[kNB];  // R[m][kk], m = k0 .. kk-1 (same on every lane)
#pragma unroll
        for (int m = 0; m < kNB; ++m) {
          const double x = M[(k0 + m) * ldm + kk];
          col[m] = (m < nm) ? x : 0.0;
        }
        constexpr int kMaxJ = kMaxL / 64;
        double row[kMaxJ];
#pragma unroll
        for (int c = 0; c < kMaxJ; ++c) {
          const int j = kk + 1 + lane + 64 * c;
          const int jc = j < ldm ? j : ldm - 1;
          double v = M[kk * ldm + jc];
#pragma unroll
          for (int m = 0; m < kNB; ++m) v -= col[m] * M[(k0 + m) * ldm + jc];
          row[c] = v;
        }
        double piv = M[kk * ldm + kk];
#pragma unroll
        for (int m = 0; m < kNB; ++m) piv -= col[m] * col[m];
        const bool drop = !(piv > kDeflate * wdiag[kk]) || !(piv > 0.0);  // uniform within the wave
        const double rkk = drop ? 1.0 : sqrt(piv), rinv = 1.0 / rkk;
#pragma unroll
        for (int c = 0; c < kMaxJ; ++c) {
          const int j = kk + 1 + lane + 64 * c;
          if (j < l) M[kk * ldm + j] = drop ? 0.0 : row[c] * rinv;
        }
        if (lane == 0) {
          M[kk * ldm + kk] = rkk;
          defl[kk] = drop ? 1 : 0;
          if (drop) ++*ndefl;
        }
        wave_sync();
      }
    }
    __syncthreads();
    const int t0 = k0 + nb;
    if (t0 < l) {
      const int ty = tid / 16, tx = tid % 16;  // NT == 256
      for (int ib = t0; ib < l; ib += 64) {
        for (int jb = ib; jb < l; jb += 64) {
          double acc[4][4];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
          for (int kk = k0; kk < t0; ++kk) {
            double ci[4], cj[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const int i = ib + ty + 16 * a;
              const double x = M[kk * ldm + (i < ldm ? i : ldm - 1)];
              ci[a] = (i < l) ? x : 0.0;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int j = jb + tx + 16 * c;
              const double x = M[kk * ldm + (j < ldm ? j : ldm - 1)];
              cj[c] = (j < l) ? x : 0.0;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int c = 0; c < 4; ++c) acc[a][c] += ci[a] * cj[c];
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int i = ib + ty + 16 * a, j = jb + tx + 16 * c;
              if (i < l && j < l && j >= i) M[i * ldm + j] -= acc[a][c];
            }
        }
      }
    }
    __syncthreads();
  }
}

// In-place blocked inverse of the upper triangular R in M (T = R^{-1}).  For
// each 16-column block J = [k0, k0+nb):
//   P = T[0:k0, 0:k0] R[0:k0, J]   (all threads, 4x1 tiles)
//   T_JJ = R_JJ^{-1}                (wave 0, concurrently)
//   T[0:k0, J] = -P T_JJ
template <int NT, typename MT>
__device__ void trinv_blocked(MT M, int ldm, int l, double* P /* kMaxL x kNB, LDS */) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k0 = 0; k0 < l; k0 += kNB) {
    const int nb = (l - k0 < kNB) ? l - k0 : kNB;
    // P rows i < k0: thread (ty, tx) -> column jj = tx, rows ty + 16a
    {
      const int ty = tid / 16, tx = tid % 16;
      for (int ib = 0; ib < k0; ib += 64) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const int jcol = k0 + tx;
        if (tx < nb) {
          // T upper: row i uses m in [i, k0)
          const int i_lo = ib + ty;
          for (int m = i_lo; m < k0; ++m) {
            const double r = M[m * ldm + jcol];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const int i = i_lo + 16 * a;
              const double x = M[(i < ldm ? i : ldm - 1) * ldm + m];
              acc[a] += (i <= m) ? x * r : 0.0;
            }
          }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int i = ib + ty + 16 * a;
          if (i < k0 && tx < nb) P[i * kNB + tx] = acc[a];
        }
      }
    }
    if (wave == NT / 64 - 1) {
      // T_JJ = R_JJ^{-1}, column by column, by the last wave
      for (int j = 0; j < nb; ++j) {
        const int jj = k0 + j;
        const double tjj = 1.0 / M[jj * ldm + jj];
        double acc = 0.0;
        const int i = lane;  // row within the block
        if (i < j) {
#pragma unroll
          for (int m = 0; m < kNB; ++m) {
            const double x = M[(k0 + (i < kNB ? i : 0)) * ldm + (k0 + m)] * M[(k0 + m) * ldm + jj];
            acc += (m >= i && m < j) ? x : 0.0;
          }
        }
        wave_sync();
        if (i < j) M[(k0 + i) * ldm + jj] = -tjj * acc;
        if (lane == 0) M[jj * ldm + jj] = tjj;
        wave_sync();
      }
    }
    __syncthreads();
    // T[0:k0, J] = -P T_JJ
    for (int e = tid; e < k0 * kNB; e += NT) {
      const int i = e / kNB, jj = e % kNB;
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < kNB; ++m) {
        const double x = P[i * kNB + m] * M[(k0 + m) * ldm + (k0 + jj)];
        acc += (m <= jj) ? x : 0.0;
      }
      if (jj < nb) M[i * ldm + k0 + jj] = -acc;
    }
    __syncthreads();
  }
}

// ---- register-resident factor for l <= 128 --------------------------------
// Right-looking Cholesky W = L L^T (R = L^T) with NT threads.  With cw = l
// rounded up to 64 and rpc = NT / cw threads per column (cw^2 <= kRegSlots
// NT), thread (j, h) keeps A[i][j] of column j for the rows
// i = 2h + 2 rpc p + e (e = 0, 1) in static register slots 2p + e.  Step k
// reads column k from a double-buffered LDS copy (colbuf, 2 x 128) that the
// owners of column k publish at the end of step k - 1, so a step needs one
// barrier; the update A[i][j] -= A[i][k] A[j][k] / A[k][k] uses the unscaled
// column (1/A[k][k] by Newton), and each column is scaled by 1/sqrt(pivot)
// once at the end (its pivot is the value its own row held when it became
// the pivot column; later steps do not touch it).  Rows i < j of a column
// are never read back.  Writes R (upper triangle, ld ldm) into M and
// 1/R[j][j] into rdinv.  Deflates collapsed pivots as chol_blocked (the same
// test): a dropped column updates no other column, its row of R is e_j and
// rdinv[j] = 0, so that trinv_reg returns T with row and column j zero;
// *ndefl counts the dropped columns.
template <int NT, typename MT>
__device__ void chol_reg(const double* __restrict__ W, int ldw, MT M, int ldm, int l, const double* wdiag,
                         double* colbuf, double* rdinv, int* ndefl) {
  const int tid = threadIdx.x;
  const int cw = (l + 63) & ~63;
  const int rpc = NT / cw;
  const int j = tid / rpc, h = tid % rpc;
  auto row = [&](int s) { return 2 * h + 2 * rpc * (s >> 1) + (s & 1); };
  double a[kRegSlots];
#pragma unroll
  for (int s = 0; s < kRegSlots; ++s) {
    const int i = row(s);
    a[s] = (j < l && i < l && i >= j) ? W[j * ldw + i] : 0.0;  // A[i][j] = W[j][i]
  }
  if (j == 0) {
#pragma unroll
    for (int s = 0; s < kRegSlots; ++s) {
      const int i = row(s);
      if (i < l) colbuf[i] = a[s];
    }
  }
  __syncthreads();
  for (int k = 0; k < l; ++k) {
    const double* cb = colbuf + (k & 1) * kLdsMaxL;
    const double piv = cb[k], wk = wdiag[k], cj = cb[j < l ? j : 0];
    const bool drop = !(piv > kDeflate * wk) || !(piv > 0.0);  // uniform
    if (j > k && j < l) {
      if (!drop) {
        double rp = rcp_newton(piv);
        if (!(piv > 1e-290)) rp = 1.0 / piv;  // uniform; the estimate is for normal arguments
        const double ajk = cj * rp;
#pragma unroll
        for (int p = 0; p < kRegSlots / 2; ++p) {  // rows of this thread in 16-byte pairs
          const int i0 = 2 * h + 2 * rpc * p;
          const double2 v = *(const double2*)(cb + (i0 < kLdsMaxL - 2 ? i0 : kLdsMaxL - 2));
          if (i0 >= j && i0 < l) a[2 * p] -= v.x * ajk;
          if (i0 + 1 >= j && i0 + 1 < l) a[2 * p + 1] -= v.y * ajk;
        }
      }
      if (j == k + 1) {  // publish the finished column k + 1
        double* nb = colbuf + ((k + 1) & 1) * kLdsMaxL;
#pragma unroll
        for (int s = 0; s < kRegSlots; ++s) {
          const int i = row(s);
          if (i >= j && i < l) nb[i] = a[s];
        }
      }
    }
    __syncthreads();
  }
  double pj = 0.0;  // the pivot of column j, held by one lane of the column
#pragma unroll
  for (int s = 0; s < kRegSlots; ++s) pj = (row(s) == j) ? a[s] : pj;
  for (int o = 1; o < rpc; o <<= 1) pj += __shfl_xor(pj, o, 64);
  // the same pivot and test as at step j
  const bool dropj = j < l && (!(pj > kDeflate * wdiag[j]) || !(pj > 0.0));
  const double rs = (j < l && !dropj) ? 1.0 / sqrt(pj) : 0.0;
#pragma unroll
  for (int s = 0; s < kRegSlots; ++s) {
    const int i = row(s);
    if (j < l && i < l && i >= j) M[j * ldm + i] = dropj ? (i == j ? 1.0 : 0.0) : ((i == j) ? pj * rs : a[s] * rs);
  }
  if (j < l && h == 0) {
    rdinv[j] = rs;
    if (dropj) atomicAdd(ndefl, 1);
  }
  __syncthreads();
}

// T = R^{-1} for the upper R in M (ld ldm) with 1/R[m][m] in rdinv, written
// to T (row-major, ld ldt; zero below the diagonal and in rows/columns
// l..ldt-1).  Column j of T solves R t = e_j upwards; thread (j, h) keeps
// the entries of rows i = h + rpc s in static slots.  The steps m run
// downwards in slot order, so the owner of t_m holds it in a static slot and
// hands it to the other lanes of its column (same wave) with a shuffle; R
// is only read, so the columns need no barrier.  A wave stops once every one
// of its columns is finished.
template <int NT, typename MT>
__device__ void trinv_reg(MT M, int ldm, int l, const double* rdinv, double* __restrict__ T, int ldt) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int cw = (l + 63) & ~63;
  const int rpc = NT / cw;
  const int j = tid / rpc, h = tid % rpc;
  double b[kRegSlots], rdv[kRegSlots];
#pragma unroll
  for (int s = 0; s < kRegSlots; ++s) {
    const int i = h + rpc * s;
    b[s] = (i == j) ? 1.0 : 0.0;
    rdv[s] = rdinv[i < l ? i : 0];
  }
  const int jmax = __builtin_amdgcn_readfirstlane((tid | 63) / rpc);  // last column of this wave
#pragma unroll
  for (int sp = kRegSlots - 1; sp >= 0; --sp) {
    for (int hp = rpc - 1; hp >= 0; --hp) {
      const int m = hp + rpc * sp;
      if (m >= l || m > jmax) continue;  // uniform
      double r[kRegSlots];
#pragma unroll
      for (int s = 0; s <= sp; ++s) {
        const int i = h + rpc * s;
        r[s] = M[(i < m ? i : 0) * ldm + m];
      }
      const double own = b[sp] * rdv[sp];  // t_m in the lane that owns row m
      const double tsh = __shfl(own, (lane & ~(rpc - 1)) | hp, 64);
      const double t = (m <= j) ? tsh : 0.0;
      if (h == hp) b[sp] = t;
#pragma unroll
      for (int s = 0; s <= sp; ++s) {
        const int i = h + rpc * s;
        if (i < m) b[s] -= r[s] * t;
      }
    }
  }
  if (j < ldt) {
#pragma unroll
    for (int s = 0; s < kRegSlots; ++s) {
      const int i = h + rpc * s;
      if (i < ldt) T[i * ldt + j] = (j < l && i <= j) ? b[s] : 0.0;
    }
  }
}

// Position of th[i] in descending order: a total order on (value, index)
// with NaN below every number, so the ranks of th[0..l) are always a
// permutation of 0..l-1 (ties go to the lower index).
__device__ __forceinline__ int desc_rank(const double* th, int l, int i) {
  const double v = th[i] != th[i] ? -__builtin_inf() : th[i];
  int rank = 0;
  for (int j = 0; j < l; ++j) {
    const double w = th[j] != th[j] ? -__builtin_inf() : th[j];
    rank += (w > v || (w == v && j < i)) ? 1 : 0;
  }
  return rank;
}

}  // namespace small
}  // namespace mds
