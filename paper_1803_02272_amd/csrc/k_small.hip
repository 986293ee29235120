// Small dense kernels (one workgroup of 1024 threads, fp64):
//
//   orth_factor  From W = Y^T Y build T with Y T orthonormal.  First choice is
//                Cholesky W = R^T R and T = R^{-1} (one CholeskyQR step;
//                applied twice this is CholeskyQR2, Fukaya et al. 2014).  When
//                a pivot collapses (rank-deficient or too ill-conditioned Y)
//                it falls back to the eigendecomposition W = V S V^T and
//                T = V S^{-1/2}, dropping directions with s <= 1e-13 s_max, so
//                those columns of Q become exactly zero.
//   small_eig    Rayleigh-Ritz on B = Q^T G Q (symmetrised): eigenpairs in
//                algebraic descending order (Sec. 6.2, step 2 on the projected
//                matrix), eigenvalues keep their sign (G need not be PSD,
//                Sec. 6.3), and Tc = V_k diag(sqrt(max(theta, 0))) for the
//                coordinates X = Q Tc (Sec. 6.2, step 3).
//
// The symmetric eigensolver is cyclic Jacobi with the round-robin parallel
// ordering: every round rotates l/2 disjoint pairs at once, each thread
// updating whole 2x2 blocks J_p^T M_pq J_q, so a round needs two barriers.
// A rotation is skipped when |m_pq| <= 1e-17 ||M||_F; a sweep with no
// rotation ends the iteration (cap 40 sweeps).  For l <= 128 the working
// matrix lives in LDS; larger l use a global scratch buffer.
#include "mds_internal.h"

namespace mds {
namespace {

constexpr int kThreads = 1024;
constexpr int kMaxPairs = kMaxL / 2;
constexpr int kMaxSweeps = 40;

struct JacobiShared {
  int p[kMaxPairs], q[kMaxPairs];
  double c[kMaxPairs], s[kMaxPairs], t[kMaxPairs];
  int active[kMaxPairs];
  int nrot;
  double red[kThreads / 64];
};

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

// Cyclic Jacobi on the symmetric le x le matrix M (ld ldm), accumulating the
// rotations into V (ld ldv, identity on entry).  le is even; a padding
// row/column of zeros is never rotated.  Returns the number of sweeps, or
// -1 if the sweep cap was reached.
__device__ int jacobi(double* M, int ldm, double* V, int ldv, int le, JacobiShared& sh) {
  const int tid = threadIdx.x;
  const int np = le / 2;
  double fro = 0.0;
  for (int e = tid; e < le * le; e += kThreads) {
    const double v = M[(e / le) * ldm + e % le];
    fro += v * v;
  }
  fro = sqrt(block_sum(fro, sh.red));
  const double thr = 1e-17 * fro;
  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) sh.nrot = 0;
    __syncthreads();
    for (int r = 0; r < le - 1; ++r) {
      if (tid < np) {
        int p, q;
        if (tid == 0) {
          p = le - 1;
          q = r;
        } else {
          p = (r + tid) % (le - 1);
          q = (r - tid + (le - 1)) % (le - 1);
        }
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        const double app = M[p * ldm + p], aqq = M[q * ldm + q], apq = M[p * ldm + q];
        double c = 1.0, s = 0.0, t = 0.0;
        int act = 0;
        if (fabs(apq) > thr) {
          const double tau = (aqq - app) / (2.0 * apq);
          if (fabs(tau) > 1e150) {
            t = 0.5 / tau;
          } else {
            t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          }
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          act = 1;
          atomicAdd(&sh.nrot, 1);
        }
        sh.p[tid] = p;
        sh.q[tid] = q;
        sh.c[tid] = c;
        sh.s[tid] = s;
        sh.t[tid] = t;
        sh.active[tid] = act;
      }
      __syncthreads();
      // M <- J^T M J, one 2x2 block (pair a rows, pair b columns) at a time
      for (int e = tid; e < np * np; e += kThreads) {
        const int a = e / np, b = e % np;
        if (!sh.active[a] && !sh.active[b]) continue;
        const int pa = sh.p[a], qa = sh.q[a], pb = sh.p[b], qb = sh.q[b];
        const double ca = sh.c[a], sa = sh.s[a], cb = sh.c[b], sb = sh.s[b];
        const double m00 = M[pa * ldm + pb], m01 = M[pa * ldm + qb];
        const double m10 = M[qa * ldm + pb], m11 = M[qa * ldm + qb];
        if (a == b) {
          const double t = sh.t[a];
          M[pa * ldm + pa] = m00 - t * m01;
          M[qa * ldm + qa] = m11 + t * m01;
          M[pa * ldm + qa] = 0.0;
          M[qa * ldm + pa] = 0.0;
        } else {
          // rows: r_p = c x_p - s x_q, r_q = s x_p + c x_q
          const double r00 = ca * m00 - sa * m10, r01 = ca * m01 - sa * m11;
          const double r10 = sa * m00 + ca * m10, r11 = sa * m01 + ca * m11;
          // columns: y_p = c r_p - s r_q, y_q = s r_p + c r_q
          M[pa * ldm + pb] = cb * r00 - sb * r01;
          M[pa * ldm + qb] = sb * r00 + cb * r01;
          M[qa * ldm + pb] = cb * r10 - sb * r11;
          M[qa * ldm + qb] = sb * r10 + cb * r11;
        }
      }
      // V <- V J
      for (int e = tid; e < le * np; e += kThreads) {
        const int i = e / np, b = e % np;
        if (!sh.active[b]) continue;
        const int pb = sh.p[b], qb = sh.q[b];
        const double cb = sh.c[b], sb = sh.s[b];
        const double vp = V[i * ldv + pb], vq = V[i * ldv + qb];
        V[i * ldv + pb] = cb * vp - sb * vq;
        V[i * ldv + qb] = sb * vp + cb * vq;
      }
      __syncthreads();
    }
    if (sh.nrot == 0) return sweep + 1;
    __syncthreads();
  }
  return -1;
}

// ---- orthonormalisation factor ----------------------------------------------
template <bool IN_LDS>
__global__ __launch_bounds__(kThreads) void k_orth_factor(const double* __restrict__ W, int l, int l_pad,
                                                          double* __restrict__ T, double* __restrict__ scratch,
                                                          DevStatus* st) {
  __shared__ JacobiShared sh;
  __shared__ double Ml[IN_LDS ? kLdsMaxL * kLdsMaxL : 1];
  __shared__ double wdiag[kMaxL];
  __shared__ double part[kThreads];
  __shared__ int failed;
  const int tid = threadIdx.x;
  const int ldm = l_pad;
  double* M = IN_LDS ? Ml : scratch;
  double* V = scratch + (IN_LDS ? 0 : (int64_t)l_pad * l_pad);
  const int le = l + (l & 1);

  for (int e = tid; e < l_pad * l_pad; e += kThreads) {
    const int i = e / l_pad, j = e % l_pad;
    M[e] = (i < l && j < l) ? W[e] : 0.0;
  }
  if (tid < l) wdiag[tid] = W[tid * l_pad + tid];
  if (tid == 0) failed = 0;
  __syncthreads();

  // Cholesky, upper: W = R^T R, R overwrites the upper triangle of M
  for (int kk = 0; kk < l; ++kk) {
    const double piv = M[kk * ldm + kk];
    if (!(piv > 1e-12 * wdiag[kk]) || !(piv > 0.0)) {
      if (tid == 0) failed = 1;
      break;  // uniform: every thread read the same pivot
    }
    const double rkk = sqrt(piv);
    __syncthreads();
    for (int j = kk + 1 + tid; j < l; j += kThreads) M[kk * ldm + j] /= rkk;
    if (tid == 0) M[kk * ldm + kk] = rkk;
    __syncthreads();
    const int rem = l - kk - 1;
    for (int e = tid; e < rem * rem; e += kThreads) {
      const int i = kk + 1 + e / rem, j = kk + 1 + e % rem;
      if (j >= i) M[i * ldm + j] -= M[kk * ldm + i] * M[kk * ldm + j];
    }
    __syncthreads();
  }
  __syncthreads();

  if (!failed) {
    // In-place inverse of the upper triangular R (column by column):
    // T[j][j] = 1/R[j][j];  T[0:j, j] = -T[j][j] * T[0:j, 0:j] R[0:j, j]
    constexpr int kSub = 8;  // threads cooperating on one output row
    constexpr int kRowsPerPass = kThreads / kSub;
    for (int j = 0; j < l; ++j) {
      const int sub = tid % kSub;
      const double tjj = 1.0 / M[j * ldm + j];
      for (int ib = 0; ib < j; ib += kRowsPerPass) {
        const int i = ib + tid / kSub;
        double acc = 0.0;
        if (i < j) {
          for (int m = i + sub; m < j; m += kSub) acc += M[i * ldm + m] * M[m * ldm + j];
        }
        for (int off = kSub / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (i < j && sub == 0) part[i] = -tjj * acc;
      }
      __syncthreads();
      if (tid < j) M[tid * ldm + j] = part[tid];
      if (tid == 0) M[j * ldm + j] = tjj;
      __syncthreads();
    }
    for (int e = tid; e < l_pad * l_pad; e += kThreads) {
      const int i = e / l_pad, j = e % l_pad;
      T[e] = (i < l && j < l && j >= i) ? M[i * ldm + j] : 0.0;
    }
    if (tid == 0) st->rank_deficient = 0;
    return;
  }

  // Fallback: T = V diag(s^{-1/2}) over the retained eigen-directions of W.
  for (int e = tid; e < l_pad * l_pad; e += kThreads) {
    const int i = e / l_pad, j = e % l_pad;
    M[e] = (i < l && j < l) ? W[e] : 0.0;
    V[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi(M, ldm, V, l_pad, le, sh);
  __syncthreads();
  double smax = -1.0;
  for (int i = tid; i < l; i += kThreads) smax = fmax(smax, M[i * ldm + i]);
  smax = block_max(smax, sh.red);
  __shared__ double scale[kMaxL];
  __shared__ int dropped;
  if (tid == 0) dropped = 0;
  __syncthreads();
  if (tid < l) {
    const double sv = M[tid * ldm + tid];
    const bool keep = smax > 0.0 && sv > 1e-13 * smax;
    scale[tid] = keep ? 1.0 / sqrt(sv) : 0.0;
    if (!keep) atomicAdd(&dropped, 1);
  }
  __syncthreads();
  for (int e = tid; e < l_pad * l_pad; e += kThreads) {
    const int i = e / l_pad, j = e % l_pad;
    T[e] = (i < l && j < l) ? V[i * l_pad + j] * scale[j] : 0.0;
  }
  if (tid == 0) {
    atomicAdd(&st->orth_fallbacks, 1);
    st->rank_deficient = dropped;
  }
}

// ---- Rayleigh-Ritz eigensolve ---------------------------------------------
template <bool IN_LDS>
__global__ __launch_bounds__(kThreads) void k_small_eig(const double* __restrict__ B, int l, int l_pad, int k,
                                                        double* __restrict__ theta, double* __restrict__ Vout,
                                                        double* __restrict__ Tc, double* __restrict__ eigvals,
                                                        double* __restrict__ scratch, DevStatus* st) {
  __shared__ JacobiShared sh;
  __shared__ double Ml[IN_LDS ? kLdsMaxL * kLdsMaxL : 1];
  __shared__ double th[kMaxL];
  __shared__ int perm[kMaxL];
  const int tid = threadIdx.x;
  const int ldm = l_pad;
  double* M = IN_LDS ? Ml : scratch;
  double* V = scratch + (IN_LDS ? 0 : (int64_t)l_pad * l_pad);
  const int le = l + (l & 1);

  for (int e = tid; e < l_pad * l_pad; e += kThreads) {
    const int i = e / l_pad, j = e % l_pad;
    M[e] = (i < l && j < l) ? 0.5 * (B[i * l_pad + j] + B[j * l_pad + i]) : 0.0;
    V[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int sweeps = jacobi(M, ldm, V, l_pad, le, sh);
  __syncthreads();
  if (tid < l) {
    th[tid] = M[tid * ldm + tid];
    perm[tid] = tid;
  }
  __syncthreads();
  if (tid < l) {
    const double v = th[tid];
    int rank = 0;
    for (int j = 0; j < l; ++j) {
      const double w = th[j];
      rank += (w > v || (w == v && j < tid)) ? 1 : 0;
    }
    perm[rank] = tid;
  }
  __syncthreads();
  if (tid < l) theta[tid] = th[perm[tid]];
  if (tid < k) eigvals[tid] = th[perm[tid]];
  for (int e = tid; e < l * l; e += kThreads) {
    const int a = e / l, r = e % l;
    const double v = V[a * l_pad + perm[r]];
    Vout[a * l_pad + r] = v;
    if (r < k) Tc[a * k + r] = v * sqrt(fmax(th[perm[r]], 0.0));
  }
  if (tid == 0) {
    st->jacobi_sweeps = sweeps;
    if (sweeps < 0) atomicAdd(&st->jacobi_unconv, 1);
  }
}

}  // namespace

hipError_t launch_orth_factor(const double* W, int l, int l_pad, double* T, double* scratch, DevStatus* st,
                              hipStream_t s) {
  if (l > kMaxL || l_pad > kMaxL || l < 1) return hipErrorInvalidValue;
  if (l_pad <= kLdsMaxL)
    hipLaunchKernelGGL(k_orth_factor<true>, dim3(1), dim3(kThreads), 0, s, W, l, l_pad, T, scratch, st);
  else
    hipLaunchKernelGGL(k_orth_factor<false>, dim3(1), dim3(kThreads), 0, s, W, l, l_pad, T, scratch, st);
  return hipGetLastError();
}

hipError_t launch_small_eig(const double* B, int l, int l_pad, int k, double* theta, double* V, double* Tc,
                            double* eigvals_out, double* scratch, DevStatus* st, hipStream_t s) {
  if (l > kMaxL || l_pad > kMaxL || k < 1 || k > l) return hipErrorInvalidValue;
  if (l_pad <= kLdsMaxL)
    hipLaunchKernelGGL(k_small_eig<true>, dim3(1), dim3(kThreads), 0, s, B, l, l_pad, k, theta, V, Tc,
                       eigvals_out, scratch, st);
  else
    hipLaunchKernelGGL(k_small_eig<false>, dim3(1), dim3(kThreads), 0, s, B, l, l_pad, k, theta, V, Tc,
                       eigvals_out, scratch, st);
  return hipGetLastError();
}

}  // namespace mds
