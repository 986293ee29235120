// Small dense kernels (fp64, one workgroup per l x l problem):
//
//   orth_factor  From W = Y^T Y build T with Y T orthonormal.  First choice is
//                Cholesky W = R^T R and T = R^{-1} (one CholeskyQR step;
//                applied twice this is CholeskyQR2, Fukaya et al. 2014).  In
//                the second step W is I + E with tiny E; when max|E| < 1e-9
//                the factor is I - triu(E) (diagonal E/2), exact to O(E^2).  A
//                pivot that collapses (a column of Y within 1e-7 of the span
//                of the earlier ones: rank-deficient or too ill-conditioned
//                Y) deflates its column, which becomes exactly zero in Q, and
//                the factorization goes on (no eigen fallback: a rank-
//                deficient Y costs no more than a full-rank one).  For l_pad <= 128 the
//                Cholesky and the inverse keep the matrix in registers of a
//                1024-thread workgroup, 256 threads for l_pad <= 64
//                (right-looking, one barrier per column; then barrier-free
//                back substitution per column of R^{-1}); larger l factor
//                two diagonal blocks of at most 128 that way and join them
//                with the Schur complement (k_blk_schur).
//   small_eig    Rayleigh-Ritz on B = Q^T G Q (symmetrised): eigenpairs in
//                algebraic descending order (Sec. 6.2, step 2 on the projected
//                matrix), eigenvalues keep their sign (G need not be PSD,
//                Sec. 6.3), and Tc = V_k diag(sqrt(max(theta, 0))) for the
//                coordinates X = Q Tc (Sec. 6.2, step 3).
//
// The symmetric eigensolver is cyclic Jacobi with the round-robin parallel
// ordering: every round rotates l/2 disjoint pairs at once, each thread
// updating whole 2x2 blocks J_p^T M_pq J_q of the upper triangle (pairs
// p <= q only, half the LDS traffic of the full matrix), so a round needs
// two barriers.
// A rotation is skipped when |m_pq| <= 1e-17 ||M||_F; the iteration stops
// after the first sweep that ends with off(M) <= 1e-15 ||M||_F or that
// rotated nothing (cap 40 sweeps).  In small_eig the rotations are recorded
// (c, s per pair and round) and the eigenvector matrix is accumulated
// afterwards by k_rot_apply, one workgroup per row of V, so the sweep loop
// touches only LDS.  This is the solver for l_pad <= 128, where the working
// matrix lives in LDS; larger l reduce the matrix to tridiagonal form and
// run implicit QL (k_tri_reduce, k_tri_ql, k_ql_vectors).
#include <type_traits>

#include "mds_internal.h"
#include "small_dev.h"

namespace mds {
namespace {

using namespace small;

// the register-resident factor holds cw^2 / NT rows per thread (cw = l rounded
// up to 64) in kRegSlots registers: every l_pad <= kLdsMaxL must fit
static_assert(kLdsMaxL * kLdsMaxL <= kRegSlots * kOrthRegThreads, "register slots of chol_reg / trinv_reg");
static_assert(kSmallLMax * kSmallLMax <= kRegSlots * kOrthRegThreadsSmall, "register slots at l_pad <= kSmallLMax");
static_assert(kSmallLMax % 64 == 0 && (kOrthRegThreadsSmall / kSmallLMax) * kSmallLMax == kOrthRegThreadsSmall,
              "the lanes of one column share a wave (small l)");
static_assert(kOrthRegThreads / kLdsMaxL <= 64 && (kOrthRegThreads / kLdsMaxL) * kLdsMaxL == kOrthRegThreads,
              "the lanes of one column share a wave");

// Cholesky factor and its inverse of the l x l matrix W (ld ldw, l <= 128,
// l_pad = l rounded up to 16) into T (ld ldt): the register-resident
// chol_reg and trinv_reg.  The deflation test compares each pivot with the
// diagonal of wd (ld ldd), W itself when wd is null.  accumulate: add the
// dropped columns to a count made by an earlier call (the second diagonal
// block of a blocked factor).  skip: a flag in device memory that, when set,
// leaves the call with nothing to do (the second CholeskyQR step once its W
// was found near the identity).
template <int NT>
__global__ __launch_bounds__(NT) void k_orth_factor(const double* __restrict__ W, int l, int l_pad, int ldw,
                                                     double* __restrict__ T, int ldt, const double* __restrict__ wd,
                                                     int ldd,
                                                     DevStatus* st, int near_identity, int accumulate,
                                                     const int* __restrict__ skip) {
  __shared__ JacobiShared sh;
  __shared__ double Ml[kLdsMaxL * (kLdsMaxL + 1)];  // ld l_pad + 1 (R)
  __shared__ double wdiag[kMaxL];
  __shared__ __attribute__((aligned(16))) double colbuf[2 * kLdsMaxL];
  __shared__ double rdinv[kMaxL];
  __shared__ int ndefl;
  if (skip && *skip) return;  // uniform
  lds_double* M = (lds_double*)(void*)Ml;
  const int tid = threadIdx.x;
  const int ldm = l_pad + 1;  // odd: column reads of R spread over banks

  for (int i = tid; i < l; i += NT) wdiag[i] = wd ? wd[i * ldd + i] : W[i * ldw + i];
  if (tid == 0) ndefl = 0;
  __syncthreads();

  if (near_identity) {
    // Second CholeskyQR step: W = Q1^T Q1 = I + E.  If max|E| < 1e-9, then
    // chol(I + E) = I + U + O(|E|^2) with U = triu(E), diag(E)/2 on the
    // diagonal, and R^{-1} = I - U + O(|E|^2): no factorization needed.
    double emax = 0.0;
    for (int i = tid / 64; i < l; i += NT / 64)
      for (int j = tid % 64; j < l; j += 64) emax = fmax(emax, fabs(W[i * ldw + j] - (i == j ? 1.0 : 0.0)));
    emax = block_max<NT>(emax, sh.red);
    if (emax < 1e-9) {
      for (int i = tid / 64; i < l_pad; i += NT / 64)
        for (int j = tid % 64; j < l_pad; j += 64) {
          double t = 0.0;
          if (i < l && j < l) {
            const double e = W[i * ldw + j] - (i == j ? 1.0 : 0.0);
            t = (i == j) ? 1.0 - 0.5 * e : (j > i ? -e : 0.0);
          }
          T[i * ldt + j] = t;
        }
      if (tid == 0) st->rank_deficient = 0;
      return;
    }
  }

  chol_reg<NT>(W, ldw, M, ldm, l, wdiag, colbuf, rdinv, &ndefl);
  trinv_reg<NT>(M, ldm, l, rdinv, T, ldt);  // zero rows and columns of the dropped
  __syncthreads();
  if (tid == 0) {
    const int before = accumulate ? st->rank_deficient : 0;
    st->rank_deficient = before + ndefl;
    if (ndefl && before == 0) atomicAdd(&st->orth_fallbacks, 1);
  }
}

// ---- orthonormalisation factor for 128 < l <= 256: two diagonal blocks ------
// With W = [W11 W12; W21 W22] (W11 of size l1 = ceil(l / 2), W22 of l2 =
// l - l1, both <= 128) and W = R^T R, R = [R11 R12; 0 R22]:
//   R11 = chol(W11), T11 = R11^{-1};  L21 = R12^T = W21 T11;
//   S = W22 - L21 L21^T,  R22 = chol(S),  T22 = R22^{-1};
//   T = R^{-1} = [T11, -T11 L21^T T22; 0, T22].
// Both diagonal factors are the register kernels above (one barrier per
// column); a column dropped in the first block has a zero column of T11 and
// so of L21, i.e. it updates no later column, as in the unblocked factor,
// and the second block's pivots are tested against the diagonal of W22.
// The blocks live in a scratch area of four 128 x 128 fp64 matrices (T11,
// S then T11 L21^T, T22, L21) and a flag.
constexpr int kBlk = 128;            // ld of the scratch blocks
constexpr int kBlkThreads = 1024;

__device__ __forceinline__ int blk_split(int l) { return (l + 1) / 2; }

// The second CholeskyQR step's test on the whole W: near the identity, T is
// written directly (as in k_orth_factor) and the flag tells the block kernels
// to skip.
__global__ __launch_bounds__(kBlkThreads) void k_orth_near_identity(const double* __restrict__ W, int l, int l_pad,
                                                                     double* __restrict__ T, DevStatus* st,
                                                                     int* __restrict__ flag) {
  __shared__ double red[kBlkThreads / 64];
  const int tid = threadIdx.x;
  double emax = 0.0;
  for (int e = tid; e < l * l; e += kBlkThreads) {
    const int i = e / l, j = e % l;
    emax = fmax(emax, fabs(W[i * l_pad + j] - (i == j ? 1.0 : 0.0)));
  }
  emax = block_max<kBlkThreads>(emax, red);
  const bool near = emax < 1e-9;
  if (near) {
    for (int e = tid; e < l_pad * l_pad; e += kBlkThreads) {
      const int i = e / l_pad, j = e % l_pad;
      double t = 0.0;
      if (i < l && j < l) {
        const double x = W[i * l_pad + j] - (i == j ? 1.0 : 0.0);
        t = (i == j) ? 1.0 - 0.5 * x : (j > i ? -x : 0.0);
      }
      T[e] = t;
    }
  }
  if (tid == 0) {
    *flag = near ? 1 : 0;
    if (near) st->rank_deficient = 0;
  }
}

// C = beta Cin + alpha op(A) op(B) for M, N, K <= 128 by the whole workgroup
// (kBlkThreads: a 4 x 4 tile of C per thread), K in chunks of 16 staged in
// LDS.  op(A)(i, k) = A[k * lda + i] if ta else A[i * lda + k], likewise B.
__device__ void blk_gemm(int M, int N, int K, double alpha, const double* __restrict__ A, int lda, bool ta,
                         const double* __restrict__ B, int ldb, bool tb, double beta,
                         const double* __restrict__ Cin, int ldci, double* __restrict__ C, int ldc,
                         double (*As)[kBlk + 1], double (*Bs)[kBlk + 1]) {
  const int tid = threadIdx.x;
  const int ti = tid / 32, tj = tid % 32;  // rows 4 ti .., columns 4 tj ..
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    __syncthreads();
    for (int e = tid; e < 16 * kBlk; e += kBlkThreads) {
      // A chunk: As[kk][i]; the layout of the loads follows the contiguous index
      const int kk = ta ? e / kBlk : e % 16, i = ta ? e % kBlk : e / 16;
      const int kb = kk, ib = i;
      double va = 0.0;
      if (ib < M && k0 + kb < K) va = ta ? A[(size_t)(k0 + kb) * lda + ib] : A[(size_t)ib * lda + k0 + kb];
      As[kb][ib] = va;
      const int kk2 = tb ? e % 16 : e / kBlk, j = tb ? e / 16 : e % kBlk;
      double vbv = 0.0;
      if (j < N && k0 + kk2 < K) vbv = tb ? B[(size_t)j * ldb + k0 + kk2] : B[(size_t)(k0 + kk2) * ldb + j];
      Bs[kk2][j] = vbv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][4 * ti + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][4 * tj + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = 4 * ti + r, j = 4 * tj + c;
      if (i < M && j < N) {
        double v = alpha * acc[r][c];
        if (beta != 0.0) v += beta * Cin[(size_t)i * ldci + j];
        C[(size_t)i * ldc + j] = v;
      }
    }
  __syncthreads();
}

// L21 = W21 T11 (l2 x l1, T11 upper with zeros below), then
// S = W22 - L21 L21^T (l2 x l2).
__global__ __launch_bounds__(kBlkThreads) void k_blk_schur(const double* __restrict__ W, int l, int l_pad,
                                                            const double* __restrict__ T11, double* __restrict__ L21,
                                                            double* __restrict__ S, const int* __restrict__ skip) {
  __shared__ double As[16][kBlk + 1], Bs[16][kBlk + 1];
  if (skip && *skip) return;
  const int l1 = blk_split(l), l2 = l - l1;
  blk_gemm(l2, l1, l1, 1.0, W + (size_t)l1 * l_pad, l_pad, false, T11, kBlk, false, 0.0, nullptr, 0, L21, kBlk, As,
           Bs);
  blk_gemm(l2, l2, l1, -1.0, L21, kBlk, false, L21, kBlk, true, 1.0, W + (size_t)l1 * l_pad + l1, l_pad, S, kBlk, As,
           Bs);
}

// M1 = T11 L21^T (l1 x l2), then T = [T11, -M1 T22; 0, T22] with its padding.
__global__ __launch_bounds__(kBlkThreads) void k_blk_assemble(int l, int l_pad, const double* __restrict__ T11,
                                                               const double* __restrict__ L21,
                                                               const double* __restrict__ T22,
                                                               double* __restrict__ M1, double* __restrict__ T,
                                                               const int* __restrict__ skip) {
  __shared__ double As[16][kBlk + 1], Bs[16][kBlk + 1];
  if (skip && *skip) return;
  const int tid = threadIdx.x;
  const int l1 = blk_split(l);
  const int l2 = l - l1;
  for (int e = tid; e < l_pad * l_pad; e += kBlkThreads) {
    const int i = e / l_pad, j = e % l_pad;
    double t = 0.0;
    if (i < l1 && j < l1) t = T11[i * kBlk + j];
    if (i >= l1 && i < l && j >= l1 && j < l) t = T22[(i - l1) * kBlk + (j - l1)];
    if (!(i < l1 && j >= l1 && j < l)) T[e] = t;  // (T12 is written below)
  }
  blk_gemm(l1, l2, l1, 1.0, T11, kBlk, false, L21, kBlk, true, 0.0, nullptr, 0, M1, kBlk, As, Bs);
  blk_gemm(l1, l2, l2, -1.0, M1, kBlk, false, T22, kBlk, false, 0.0, nullptr, 0, T + l1, l_pad, As, Bs);
}

// ---- Rayleigh-Ritz eigensolve ---------------------------------------------
// Diagonalises the symmetrised B, sorts, records the rotations; meta[0] =
// rounds, meta[1..l] = permutation (sorted position -> original index).
template <bool IN_LDS, int NT>
__global__ __launch_bounds__(NT) void k_small_eig(const double* __restrict__ B, int l, int l_pad, int k,
                                                        double* __restrict__ theta, double* __restrict__ eigvals,
                                                        double2* __restrict__ rot, int* __restrict__ meta,
                                                        double* __restrict__ scratch, DevStatus* st) {
  __shared__ JacobiShared sh;
  __shared__ double Ml[IN_LDS ? kLdsMaxL * (kLdsMaxL + 1) : 1];
  __shared__ double th[kMaxL];
  __shared__ int perm[kMaxL];
  using MT = typename std::conditional<IN_LDS, lds_double*, double*>::type;
  MT M = IN_LDS ? (MT)(void*)Ml : (MT)(void*)scratch;
  const int tid = threadIdx.x;
  const int ldm = IN_LDS ? l_pad + 1 : l_pad;  // odd in LDS: the Jacobi's (min, max) accesses spread over banks
  const int le = l + (l & 1);

  for (int e = tid; e < l_pad * l_pad; e += NT) {
    const int i = e / l_pad, j = e % l_pad;
    M[i * ldm + j] = (i < l && j < l) ? 0.5 * (B[i * l_pad + j] + B[j * l_pad + i]) : 0.0;
  }
  __syncthreads();
  int rounds = 0;
  const int sweeps = jacobi<NT>(M, ldm, (double*)nullptr, 0, rot, le, sh, &rounds);
  __syncthreads();
  for (int i = tid; i < l; i += NT) th[i] = M[i * ldm + i];
  __syncthreads();
  for (int i = tid; i < l; i += NT) perm[desc_rank(th, l, i)] = i;  // a permutation, NaN included
  __syncthreads();
  for (int r = tid; r < l; r += NT) {
    const int src = perm[r];
    theta[r] = th[src];
    if (r < k) eigvals[r] = th[src];
    meta[1 + r] = src;
  }
  if (tid == 0) {
    meta[0] = rounds;
    st->jacobi_sweeps = sweeps < 0 ? -sweeps : sweeps;
    if (sweeps < 0) atomicAdd(&st->jacobi_unconv, 1);
  }
}

// ---- Rayleigh-Ritz eigensolve for l_pad > 128: tridiagonal QL ---------------
// The l x l matrix does not fit in LDS there, and a Jacobi round touches all
// of it, so a Jacobi from global memory is bound by one CU's L2 latency.
// Here the matrix is reduced once instead (Householder, Golub & Van Loan
// 8.3.1): for column j, x = A[j+1.., j], beta = -sign(x_0) ||x||,
// v = (x - beta e_1) / (x_0 - beta) (v_0 = 1), tau = (beta - x_0) / beta,
// H_j = I - tau v v^T; the trailing block becomes H_j A22 H_j = A22 - v w^T
// - w v^T with p = tau A22 v and w = p - (tau / 2)(p^T v) v.  That leaves
// the tridiagonal T (diagonal d, off-diagonal e) with A = Q T Q^T,
// Q = H_0 H_1 ... H_{l-3}.  T is diagonalised by implicit QL with Wilkinson
// shifts (Golub & Van Loan 8.3.3, the QL form): each step chases a bulge up
// the unreduced block l0..m with plane rotations of (i, i+1), i = m-1 .. l0.
// A block splits where |e_m| <= 2^-53 (|d_m| + |d_m+1|); an eigenvalue that
// needs more than kQLMaxSteps steps is left as it is and counted as
// unconverged.  The rotations are recorded, and the eigenvectors are made
// afterwards row by row: row i of V = e_i^T Q G_1 G_2 ... (k_ql_vectors).
//
// k_tri_reduce (one workgroup) keeps A symmetric in global
// scratch; thread (c, h) owns column c of the trailing block and the rows
// h, h + 4, .. of it, so its loads are coalesced across the columns of a
// wave and issued kTriBatch at a time; the column to be reduced next is
// published to LDS by its owners during the update (four barriers per
// column).  The QL steps run on one thread (the chain is sequential) with
// d, e in LDS.
constexpr int kQLMaxSteps = 30;
constexpr int kTriThreads = 1024;
constexpr int kTriBatch = 8;

// Record of the QL rotations (the rot buffer): int[4] header (steps,
// rotations), int2 (lo, hi) per step, then (c, s) per rotation in the order
// applied (per step i = hi-1 .. lo).
constexpr size_t kQLRecHead = 16;
__host__ __device__ inline size_t ql_rot_offset(int l) { return kQLRecHead + (size_t)kQLMaxSteps * l * 8; }
size_t ql_record_bytes(int l) { return ql_rot_offset(l) + (size_t)kQLMaxSteps * l * l * sizeof(double2); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_tri_reduce(const double* __restrict__ B, int l, int l_pad,
                                                   double* __restrict__ scratch) {
  constexpr int PC = NT / kMaxL;  // partial sums per column of the trailing block
  __shared__ double vb[kMaxL], pb[kMaxL], colx[kMaxL];
  __shared__ double part[PC][kMaxL];
  __shared__ double red[2][NT / 64];
  double* A = scratch;                            // row-major, ld l_pad, symmetric
  double* tau = scratch + (size_t)l_pad * l_pad;  // per reflector
  double* dd = tau + kMaxL;                       // diagonal and off-diagonal of T
  double* ee = dd + kMaxL;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ci = tid % kMaxL, ch = tid / kMaxL;

  for (int e = tid; e < l * l; e += NT) {
    const int i = e / l, j = e % l;
    A[(size_t)i * l_pad + j] = 0.5 * (B[i * l_pad + j] + B[j * l_pad + i]);
  }
  __syncthreads();
  for (int i = tid; i < l; i += NT) colx[i] = A[(size_t)i * l_pad];
  __syncthreads();

  // ---- Householder tridiagonalisation ----
  for (int j = 0; j + 2 < l; ++j) {
    const int m = l - j - 1;  // x = colx[j+1 .. l-1]
    double part_s = 0.0;      // sigma = ||x[1..]||^2, by every wave alike
    for (int i = j + 2 + lane; i < l; i += 64) part_s += colx[i] * colx[i];
    const double sigma = wave_sum(part_s);
    const double x0 = colx[j + 1];
    double beta = x0, t = 0.0, scal = 0.0;
    if (sigma != 0.0) {  // uniform
      const double mu = sqrt(x0 * x0 + sigma);
      beta = x0 <= 0.0 ? mu : -mu;
      t = (beta - x0) / beta;
      scal = 1.0 / (x0 - beta);
    }
    for (int i = tid; i < m; i += NT) {
      const double vi = i == 0 ? 1.0 : colx[j + 1 + i] * scal;
      vb[i] = vi;
      if (i > 0) A[(size_t)(j + 1 + i) * l_pad + j] = vi;  // kept for the eigenvectors
    }
    if (tid == 0) {
      dd[j] = colx[j];
      ee[j] = beta;
      tau[j] = t;
    }
    __syncthreads();
    if (t != 0.0) {  // uniform
      double* col = A + (size_t)(j + 1) * l_pad + (j + 1 + ci);  // column ci of the block, row 0
      double acc = 0.0;
      if (ci < m)
        for (int c0 = ch; c0 < m; c0 += PC * kTriBatch) {
          double x[kTriBatch];
#pragma unroll
          for (int u = 0; u < kTriBatch; ++u) {
            const int c = c0 + PC * u;
            x[u] = c < m ? col[(size_t)c * l_pad] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kTriBatch; ++u) {
            const int c = c0 + PC * u;
            acc += c < m ? x[u] * vb[c] : 0.0;
          }
        }
      part[ch][ci] = acc;
      __syncthreads();
      double qv = 0.0;
      if (ch == 0 && ci < m) {
        double sp = 0.0;
#pragma unroll
        for (int hh = 0; hh < PC; ++hh) sp += part[hh][ci];
        const double pi = t * sp;
        pb[ci] = pi;
        qv = pi * vb[ci];
      }
      qv = wave_sum(qv);
      if (lane == 0) red[j & 1][wave] = qv;
      __syncthreads();
      double sq = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) sq += red[j & 1][w];
      const double K = 0.5 * t * sq;
      if (ci < m) {
        const double vi = vb[ci], wi = pb[ci] - K * vi;
        for (int c0 = ch; c0 < m; c0 += PC * kTriBatch) {
          double x[kTriBatch];
#pragma unroll
          for (int u = 0; u < kTriBatch; ++u) {
            const int c = c0 + PC * u;
            x[u] = c < m ? col[(size_t)c * l_pad] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kTriBatch; ++u) {
            const int c = c0 + PC * u;
            if (c < m) {
              const double vc = vb[c], wc = pb[c] - K * vc;
              const double y = x[u] - (vc * wi + wc * vi);
              col[(size_t)c * l_pad] = y;
              if (ci == 0) colx[j + 1 + c] = y;  // the next column to reduce
            }
          }
        }
      }
      __syncthreads();
    } else {
      for (int i = tid; i < m; i += NT) colx[j + 1 + i] = A[(size_t)(j + 1 + i) * l_pad + (j + 1)];
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (l >= 2) {
      dd[l - 2] = colx[l - 2];
      ee[l - 2] = colx[l - 1];
      dd[l - 1] = A[(size_t)(l - 1) * l_pad + l - 1];
    } else {
      dd[0] = colx[0];
    }
    ee[l - 1] = 0.0;
  }
}

// Implicit QL on (d, e) by one thread, the rotations recorded; then the
// eigenvalues in descending order.
__global__ __launch_bounds__(256) void k_tri_ql(int l, int l_pad, int k, double* __restrict__ theta,
                                               double* __restrict__ eigvals, int* __restrict__ meta,
                                               const double* __restrict__ scratch, unsigned char* __restrict__ rec,
                                               DevStatus* st) {
  __shared__ double dd[kMaxL], ee[kMaxL];
  __shared__ int perm[kMaxL];
  const int tid = threadIdx.x;
  const double* tdiag = scratch + (size_t)l_pad * l_pad + kMaxL;
  for (int i = tid; i < l; i += 256) {
    dd[i] = tdiag[i];
    ee[i] = tdiag[kMaxL + i];
  }
  __syncthreads();
  if (tid == 0) {
    int* head = reinterpret_cast<int*>(rec);
    int2* steps = reinterpret_cast<int2*>(rec + kQLRecHead);
    double2* rot = reinterpret_cast<double2*>(rec + ql_rot_offset(l));
    int nstep = 0, nrot = 0, most = 0, unconv = 0;
    bool finite = true;
    for (int i = 0; i < l; ++i) finite = finite && isfinite(dd[i]) && isfinite(ee[i]);
    int l0 = finite ? 0 : l, cnt = 0;  // NaN or Inf: the values stay as the reduction left them
    while (l0 < l) {
      int m = l0;
      for (; m + 1 < l; ++m)
        if (fabs(ee[m]) <= 0x1p-53 * (fabs(dd[m]) + fabs(dd[m + 1]))) break;
      if (m == l0) {
        ++l0;
        cnt = 0;
        continue;
      }
      if (cnt == kQLMaxSteps) {
        unconv = 1;
        ++l0;
        cnt = 0;
        continue;
      }
      most = ++cnt > most ? cnt : most;
      double g = (dd[l0 + 1] - dd[l0]) / (2.0 * ee[l0]);
      double r = sqrt(g * g + 1.0);
      g = dd[m] - dd[l0] + ee[l0] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      double ei = ee[m - 1], di = dd[m - 1], di1 = dd[m];  // this rotation's inputs
      const int first = nrot;
      int i = m - 1;
      bool split = false;
      for (; i >= l0; --i) {
        // the next rotation's inputs, loaded unconditionally (index clamped,
        // the value replaced by 0 at the end of the block) so that the load
        // overlaps this rotation instead of being waited for at its start
        const bool more = i > l0;
        const int inx = more ? i - 1 : i;
        const double en_l = ee[inx], dn_l = dd[inx];
        const double f = s * ei, bb = c * ei;
        const double t2 = f * f + g * g;
        if (t2 == 0.0) {  // the block splits at i + 1: finish with the rotations so far
          ee[i + 1] = 0.0;
          dd[i + 1] -= p;
          ee[m] = 0.0;
          split = true;
          break;
        }
        // 1 / sqrt(t2): the hardware estimate and two Newton steps (normal range)
        const double rq = (t2 > 1e-300 && t2 < 1e300) ? rsqrt_newton(t2) : 1.0 / sqrt(t2);
        ee[i + 1] = t2 * rq;
        s = f * rq;
        c = g * rq;
        g = di1 - p;
        r = (di - g) * s + 2.0 * c * bb;
        p = s * r;
        dd[i + 1] = g + p;
        g = c * r - bb;
        rot[nrot++] = make_double2(c, s);
        di1 = di;
        di = more ? dn_l : 0.0;
        ei = more ? en_l : 0.0;
      }
      if (!split) {
        dd[l0] -= p;
        ee[l0] = g;
        ee[m] = 0.0;
      }
      if (nrot > first) steps[nstep++] = make_int2(split ? i + 1 : l0, m);
    }
    head[0] = nstep;
    head[1] = nrot;
    st->jacobi_sweeps = most;
    if (unconv) atomicAdd(&st->jacobi_unconv, 1);
  }
  __syncthreads();
  for (int i = tid; i < l; i += 256) perm[desc_rank(dd, l, i)] = i;
  __syncthreads();
  for (int r = tid; r < l; r += 256) {
    theta[r] = dd[perm[r]];
    if (r < k) eigvals[r] = dd[perm[r]];
    meta[1 + r] = perm[r];
  }
}

// Rows of V, 64 per workgroup (one wave, one row per lane, the row in LDS):
// x = e_i^T, then x <- x H_j for j = 0 .. l-3 (x - tau (x . v) v^T), then the
// recorded rotations in order; V[i][r] = x[perm[r]], Tc as in k_rot_apply.
__global__ __launch_bounds__(64) void k_ql_vectors(int l, int l_pad, int k, const double* __restrict__ scratch,
                                                   const unsigned char* __restrict__ rec,
                                                   const int* __restrict__ meta, const double* __restrict__ theta,
                                                   double* __restrict__ Vout, double* __restrict__ Tc) {
  __shared__ double x[kMaxL * 64];  // x[p * 64 + lane]
  __shared__ double vs[kMaxL];
  __shared__ double2 cs[kMaxL];
  const int lane = threadIdx.x;
  const int row = blockIdx.x * 64 + lane;
  const double* A = scratch;
  const double* tau = scratch + (size_t)l_pad * l_pad;
  for (int p = 0; p < l; ++p) x[p * 64 + lane] = (p == row) ? 1.0 : 0.0;
  for (int j = 0; j + 2 < l; ++j) {
    const double t = tau[j];
    if (t == 0.0) continue;  // uniform
    const int m = l - j - 1;
    for (int i = lane; i < m; i += 64) vs[i] = i == 0 ? 1.0 : A[(size_t)(j + 1 + i) * l_pad + j];
    wave_sync();
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
    const double* xr = x + (j + 1) * 64 + lane;
    int i = 0;
    for (; i + 3 < m; i += 4) {
      d0 += xr[i * 64] * vs[i];
      d1 += xr[(i + 1) * 64] * vs[i + 1];
      d2 += xr[(i + 2) * 64] * vs[i + 2];
      d3 += xr[(i + 3) * 64] * vs[i + 3];
    }
    for (; i < m; ++i) d0 += xr[i * 64] * vs[i];
    const double f = t * ((d0 + d1) + (d2 + d3));
    double* xw = x + (j + 1) * 64 + lane;
    for (int q = 0; q < m; ++q) xw[q * 64] -= f * vs[q];
    wave_sync();
  }
  const int nstep = reinterpret_cast<const int*>(rec)[0];
  const int2* steps = reinterpret_cast<const int2*>(rec + kQLRecHead);
  const double2* rot = reinterpret_cast<const double2*>(rec + ql_rot_offset(l));
  size_t pos = 0;
  for (int q = 0; q < nstep; ++q) {
    const int lo = steps[q].x, hi = steps[q].y, n = hi - lo;
    for (int i = lane; i < n; i += 64) cs[i] = rot[pos + i];
    wave_sync();
    double carry = x[hi * 64 + lane];
    double xi = x[(hi - 1) * 64 + lane];
    double2 r = cs[0];
    for (int t = 0; t < n; ++t) {
      const int i = hi - 1 - t;
      const double xn = t + 1 < n ? x[(i - 1) * 64 + lane] : 0.0;
      const double2 rn = cs[t + 1 < n ? t + 1 : t];
      x[(i + 1) * 64 + lane] = r.y * xi + r.x * carry;
      carry = r.x * xi - r.y * carry;
      xi = xn;
      r = rn;
    }
    x[lo * 64 + lane] = carry;
    pos += n;
    wave_sync();
  }
  if (row < l)
    for (int r = 0; r < l; ++r) {
      const double v = x[meta[1 + r] * 64 + lane];
      Vout[row * l_pad + r] = v;
      if (r < k) Tc[row * k + r] = v * sqrt(fmax(theta[r], 0.0));
    }
}

// Row i of V = e_i^T J_1 J_2 ... J_N from the recorded rotations (one wave
// per row), then Vout[i][r] = V[i][perm[r]] and Tc[i][r] = Vout[i][r] *
// sqrt(max(theta_r, 0)) for r < k.
constexpr int kRotChunk = 16;  // rounds staged in LDS at a time

__global__ __launch_bounds__(64) void k_rot_apply(const double2* __restrict__ rot, const int* __restrict__ meta,
                                                  const double* __restrict__ theta, int l, int l_pad, int k,
                                                  double* __restrict__ Vout, double* __restrict__ Tc) {
  __shared__ double v[kMaxL];
  __shared__ double2 cs[kRotChunk * kMaxPairs];
  const int i = blockIdx.x;  // row of V
  const int tid = threadIdx.x;
  const int le = l + (l & 1);
  const int np = le / 2;
  for (int j = tid; j < le; j += 64) v[j] = (j == i) ? 1.0 : 0.0;
  const int rounds = meta[0];
  int r = 0;  // round within the sweep: (r0 + rr) mod (le - 1)
  for (int r0 = 0; r0 < rounds; r0 += kRotChunk) {
    const int nrc = (rounds - r0 < kRotChunk) ? rounds - r0 : kRotChunk;
    __syncthreads();
    for (int e = tid; e < nrc * np; e += 64) cs[e] = rot[(int64_t)r0 * np + e];
    __syncthreads();
    for (int rr = 0; rr < nrc; ++rr, r = (r + 1 == le - 1) ? 0 : r + 1) {
      for (int t = tid; t < np; t += 64) {
        const double2 c = cs[rr * np + t];
        if (c.y != 0.0) {
          int p, q;
          round_robin_pair(le, r, t, p, q);
          const double vp = v[p], vq = v[q];
          v[p] = c.x * vp - c.y * vq;
          v[q] = c.y * vp + c.x * vq;
        }
      }
      __syncthreads();
    }
  }
  for (int r = tid; r < l; r += 64) {
    const double x = v[meta[1 + r]];
    Vout[i * l_pad + r] = x;
    if (r < k) Tc[i * k + r] = x * sqrt(fmax(theta[r], 0.0));
  }
}

}  // namespace

size_t small_eig_rot_bytes(int l) {
  const int le = l + (l & 1);
  const size_t jac = (size_t)kMaxSweeps * (le - 1) * (le / 2) * sizeof(double2);
  return l > kLdsMaxL ? ql_record_bytes(l) : jac;
}

hipError_t launch_orth_factor(const double* W, int l, int l_pad, double* T, double* scratch, DevStatus* st,
                              int near_identity, hipStream_t s) {
  if (l > kMaxL || l_pad > kMaxL || l < 1) return hipErrorInvalidValue;
  // l_pad <= 64: a quarter of the threads (the register factor still holds
  // 16 rows per thread), so each column step synchronises 4 waves, not 16
  if (l_pad <= kSmallLMax) {
    hipLaunchKernelGGL((k_orth_factor<kOrthRegThreadsSmall>), dim3(1), dim3(kOrthRegThreadsSmall), 0, s, W, l, l_pad,
                       l_pad, T, l_pad, (const double*)nullptr, 0, st, near_identity, 0, (const int*)nullptr);
    return hipGetLastError();
  }
  if (l_pad <= kLdsMaxL) {
    hipLaunchKernelGGL((k_orth_factor<kOrthRegThreads>), dim3(1), dim3(kOrthRegThreads), 0, s, W, l, l_pad, l_pad, T,
                       l_pad, (const double*)nullptr, 0, st, near_identity, 0, (const int*)nullptr);
    return hipGetLastError();
  }
  // two diagonal blocks (see k_blk_schur); scratch: T11, S / M1, T22, L21, flag
  double* T11 = scratch;
  double* S = scratch + kBlk * kBlk;
  double* T22 = scratch + 2 * kBlk * kBlk;
  double* L21 = scratch + 3 * kBlk * kBlk;
  int* flag = reinterpret_cast<int*>(scratch + 4 * kBlk * kBlk);
  const int l1 = (l + 1) / 2, l2 = l - l1;
  const int* skip = nullptr;
  if (near_identity) {
    hipLaunchKernelGGL(k_orth_near_identity, dim3(1), dim3(kBlkThreads), 0, s, W, l, l_pad, T, st, flag);
    skip = flag;
  }
  hipLaunchKernelGGL((k_orth_factor<kOrthRegThreads>), dim3(1), dim3(kOrthRegThreads), 0, s, W, l1,
                     (l1 + 15) / 16 * 16, l_pad, T11, kBlk, (const double*)nullptr, 0, st, 0, 0, skip);
  hipLaunchKernelGGL(k_blk_schur, dim3(1), dim3(kBlkThreads), 0, s, W, l, l_pad, T11, L21, S, skip);
  hipLaunchKernelGGL((k_orth_factor<kOrthRegThreads>), dim3(1), dim3(kOrthRegThreads), 0, s, (const double*)S, l2,
                     (l2 + 15) / 16 * 16, kBlk, T22, kBlk, W + (size_t)l1 * l_pad + l1, l_pad, st, 0, 1, skip);
  hipLaunchKernelGGL(k_blk_assemble, dim3(1), dim3(kBlkThreads), 0, s, l, l_pad, (const double*)T11,
                     (const double*)L21, (const double*)T22, S, T, skip);
  return hipGetLastError();
}

size_t orth_factor_scratch_bytes(int l_pad) {
  return l_pad <= kLdsMaxL ? 0 : (size_t)4 * kBlk * kBlk * sizeof(double) + 256;
}

hipError_t launch_small_eig(const double* B, int l, int l_pad, int k, double* theta, double* V, double* Tc,
                            double* eigvals_out, double* scratch, void* rot, int* meta, DevStatus* st,
                            hipStream_t s) {
  if (l > kMaxL || l_pad > kMaxL || k < 1 || k > l) return hipErrorInvalidValue;
  if (l_pad > kLdsMaxL) {
    hipLaunchKernelGGL((k_tri_reduce<kTriThreads>), dim3(1), dim3(kTriThreads), 0, s, B, l, l_pad, scratch);
    hipLaunchKernelGGL(k_tri_ql, dim3(1), dim3(256), 0, s, l, l_pad, k, theta, eigvals_out, meta,
                       (const double*)scratch, (unsigned char*)rot, st);
    hipLaunchKernelGGL(k_ql_vectors, dim3((unsigned)((l + 63) / 64)), dim3(64), 0, s, l, l_pad, k,
                       (const double*)scratch, (const unsigned char*)rot, (const int*)meta, (const double*)theta, V,
                       Tc);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_small_eig<true, kEigThreads>), dim3(1), dim3(kEigThreads), 0, s, B, l, l_pad, k, theta,
                     eigvals_out, (double2*)rot, meta, scratch, st);
  hipLaunchKernelGGL(k_rot_apply, dim3((unsigned)l), dim3(64), 0, s, (const double2*)rot, meta, theta, l, l_pad, k,
                     V, Tc);
  return hipGetLastError();
}

}  // namespace mds
