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
//                back substitution per column of R^{-1}); larger l use the
//                blocked versions on a global-memory copy.
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
// touches only LDS.  For l_pad <= 128 the working matrix lives in LDS;
// larger l use a global scratch buffer.
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

template <bool IN_LDS, int NT>
__global__ __launch_bounds__(NT) void k_orth_factor(const double* __restrict__ W, int l, int l_pad,
                                                     double* __restrict__ T, double* __restrict__ scratch,
                                                     DevStatus* st, int near_identity) {
  __shared__ JacobiShared sh;
  __shared__ double Ml[IN_LDS ? kLdsMaxL * (kLdsMaxL + 1) : 1];  // ld l_pad + 1 (R, then the Jacobi)
  __shared__ double wdiag[kMaxL];
  __shared__ double P[IN_LDS ? 1 : kMaxL * kNB];
  __shared__ __attribute__((aligned(16))) double colbuf[IN_LDS ? 2 * kLdsMaxL : 1];
  __shared__ double rdinv[IN_LDS ? kMaxL : 1];
  __shared__ int defl[IN_LDS ? 1 : kMaxL];
  __shared__ int ndefl;
  using MT = typename std::conditional<IN_LDS, lds_double*, double*>::type;
  MT M = IN_LDS ? (MT)(void*)Ml : (MT)(void*)scratch;
  const int tid = threadIdx.x;
  const int ldm = IN_LDS ? l_pad + 1 : l_pad;  // odd in LDS: column reads of R spread over banks

  if (!IN_LDS)
    for (int i = tid / 64; i < l_pad; i += NT / 64)
      for (int j = tid % 64; j < l_pad; j += 64) M[i * ldm + j] = (i < l && j < l) ? W[i * l_pad + j] : 0.0;
  for (int i = tid; i < l; i += NT) wdiag[i] = W[i * l_pad + i];
  if (tid == 0) ndefl = 0;
  __syncthreads();

  if (near_identity) {
    // Second CholeskyQR step: W = Q1^T Q1 = I + E.  If max|E| < 1e-9, then
    // chol(I + E) = I + U + O(|E|^2) with U = triu(E), diag(E)/2 on the
    // diagonal, and R^{-1} = I - U + O(|E|^2): no factorization needed.
    double emax = 0.0;
    for (int i = tid / 64; i < l; i += NT / 64)
      for (int j = tid % 64; j < l; j += 64) emax = fmax(emax, fabs(W[i * l_pad + j] - (i == j ? 1.0 : 0.0)));
    emax = block_max<NT>(emax, sh.red);
    if (emax < 1e-9) {
      for (int i = tid / 64; i < l_pad; i += NT / 64)
        for (int j = tid % 64; j < l_pad; j += 64) {
          double t = 0.0;
          if (i < l && j < l) {
            const double e = W[i * l_pad + j] - (i == j ? 1.0 : 0.0);
            t = (i == j) ? 1.0 - 0.5 * e : (j > i ? -e : 0.0);
          }
          T[i * l_pad + j] = t;
        }
      if (tid == 0) st->rank_deficient = 0;
      return;
    }
  }

  if constexpr (IN_LDS) {
    chol_reg<NT>(W, l_pad, M, ldm, l, wdiag, colbuf, rdinv, &ndefl);
    trinv_reg<NT>(M, ldm, l, rdinv, T, l_pad);  // zero rows and columns of the dropped
  } else {
    chol_blocked<NT>(M, ldm, l, wdiag, defl, &ndefl);
    trinv_blocked<NT>(M, ldm, l, P);
    for (int i = tid / 64; i < l_pad; i += NT / 64)
      for (int j = tid % 64; j < l_pad; j += 64)
        T[i * l_pad + j] = (i < l && j < l && j >= i && !defl[j]) ? M[i * ldm + j] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    st->rank_deficient = ndefl;
    if (ndefl) atomicAdd(&st->orth_fallbacks, 1);
  }
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
  return (size_t)kMaxSweeps * (le - 1) * (le / 2) * sizeof(double2);
}

hipError_t launch_orth_factor(const double* W, int l, int l_pad, double* T, double* scratch, DevStatus* st,
                              int near_identity, hipStream_t s) {
  if (l > kMaxL || l_pad > kMaxL || l < 1) return hipErrorInvalidValue;
  // l_pad <= 64: a quarter of the threads (the register factor still holds
  // 16 rows per thread), so each column step synchronises 4 waves, not 16
  if (l_pad <= kSmallLMax)
    hipLaunchKernelGGL((k_orth_factor<true, kOrthRegThreadsSmall>), dim3(1), dim3(kOrthRegThreadsSmall), 0, s, W, l,
                       l_pad, T, scratch, st, near_identity);
  else if (l_pad <= kLdsMaxL)
    hipLaunchKernelGGL((k_orth_factor<true, kOrthRegThreads>), dim3(1), dim3(kOrthRegThreads), 0, s, W, l, l_pad, T,
                       scratch, st, near_identity);
  else
    hipLaunchKernelGGL((k_orth_factor<false, kOrthThreads>), dim3(1), dim3(kOrthThreads), 0, s, W, l, l_pad, T,
                       scratch, st, near_identity);
  return hipGetLastError();
}

hipError_t launch_small_eig(const double* B, int l, int l_pad, int k, double* theta, double* V, double* Tc,
                            double* eigvals_out, double* scratch, void* rot, int* meta, DevStatus* st,
                            hipStream_t s) {
  if (l > kMaxL || l_pad > kMaxL || k < 1 || k > l) return hipErrorInvalidValue;
  if (l_pad <= kLdsMaxL)
    hipLaunchKernelGGL((k_small_eig<true, kEigThreads>), dim3(1), dim3(kEigThreads), 0, s, B, l, l_pad, k, theta,
                       eigvals_out, (double2*)rot, meta, scratch, st);
  else
    hipLaunchKernelGGL((k_small_eig<false, kEigThreads>), dim3(1), dim3(kEigThreads), 0, s, B, l, l_pad, k, theta,
                       eigvals_out, (double2*)rot, meta, scratch, st);
  hipLaunchKernelGGL(k_rot_apply, dim3((unsigned)l), dim3(64), 0, s, (const double2*)rot, meta, theta, l, l_pad, k,
                     V, Tc);
  return hipGetLastError();
}

}  // namespace mds
