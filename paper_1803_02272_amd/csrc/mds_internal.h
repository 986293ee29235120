// Internal declarations shared by the kernels and the host runtime of the
// MI355X (gfx950) random-projection classical MDS library.
//
// Data layout in HBM (all buffers live in one workspace):
//   D      caller's n x n distance matrix, row-major, ld = n (fp32 or fp64).
//   G      Gram matrix, n_pad x ldg row-major, n_pad = ldg = round_up(n, 256);
//          rows/cols >= n are zero so the G-pass kernels need no bounds checks.
//   "Tall" n x l operands (Omega, Y, Q) are stored transposed: l_pad x ldg
//          row-major ("column j of the tall matrix is a contiguous row"), with
//          zero padding in rows >= l and columns >= n.  Both MFMA operands of
//          the G-pass and of the Gram kernel are then contiguous in K.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mds {

typedef uint16_t bf16_t;  // raw bfloat16 bits

// Vector types for MFMA operands/accumulators.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4_t;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4_t;

enum GKind { GK_F64 = 0, GK_F32 = 1, GK_BF16 = 2 };

constexpr int kPadN = 256;     // padding granule of n (rows and ld of G)
constexpr int kMaxL = 256;     // largest oversampled rank l = k + p
constexpr int kLdsMaxL = 128;  // small kernels keep an l x l fp64 matrix in LDS up to this l

// Device-side status words (written by kernels, read back by the host).
struct DevStatus {
  int nonfinite;        // D produced a non-finite sum of squares
  int orth_fallbacks;   // orthonormalisations that left the Cholesky path
  int jacobi_sweeps;    // sweeps used by the last eigensolve
  int jacobi_unconv;    // eigensolves that hit the sweep cap
  int rank_deficient;   // last orthonormalisation dropped directions
  int pad_[3];
  double sum_sq;        // sum_ij d_ij^2
  double frob2;         // ||G||_F^2
  double trace;         // tr(G)
};

// ---- centring (Sec. 6.2, step 1) ------------------------------------------
constexpr int kStatsCols = 1024;  // columns per stats tile
constexpr int kStatsRows = 1024;  // rows per stats tile
hipError_t launch_center_stats(const void* D, int d_is_f64, int64_t n, double* rowpart, double* colpart,
                               double* r, double* c, double* rsum, double* mean_all, DevStatus* st,
                               hipStream_t s);
// Writes G (kind gk, ld = ldg, n_pad rows) and, if gref != nullptr, an fp32
// copy used by the refinement pass.  frob/trace partials go to fpart.
int64_t center_write_blocks(int64_t n_pad, int64_t ldg);
hipError_t launch_center_write(const void* D, int d_is_f64, int64_t n, int64_t n_pad, int64_t ldg,
                               const double* r, const double* c, const double* mean_all, int gk, void* G,
                               float* gref, double* fpart, DevStatus* st, hipStream_t s);

// ---- Gaussian test matrix ---------------------------------------------------
hipError_t launch_omega(uint64_t seed, int64_t n, int l, int l_pad, int64_t ldg, int xk, void* Xt,
                        hipStream_t s);

// ---- G-pass: Ypart[s] = G * X over K-split s (MFMA) ------------------------
struct GPassCfg {
  int rg;      // 16-row groups per wave
  int bm;      // rows per workgroup
  int split;   // K splits
  int64_t steps_total, steps_per_split;
};
GPassCfg gpass_config(int gk, int l_pad, int64_t n_pad, int64_t ldg, int split_hint);
hipError_t launch_gpass(int gk, const void* G, int64_t ldg, int64_t n_pad, const void* Xt, int l_pad,
                        const GPassCfg& cfg, void* Ypart, hipStream_t s);
// Y (fp64, l_pad x ldg) = sum_s Ypart[s] in split order.
hipError_t launch_splitk_reduce(int gk, const void* Ypart, int split, int64_t elems, double* Y,
                                hipStream_t s);

// ---- skinny fp64 kernels ----------------------------------------------------
int64_t gram_chunks(int64_t ldg);
// Wpart[p] = A_p B_p^T over column chunk p; then W = sum_p Wpart[p].
hipError_t launch_gram(const double* A, const double* B, int l_pad, int64_t ldg, double* Wpart,
                       double* W, hipStream_t s);
// Out = T^T In (In, Out: l_pad x ldg transposed tall matrices; T: l x lt, ld = ldt).
// Out rows >= lt are zeroed.  Optional cast copy of Out into Xc (kind xk).
hipError_t launch_apply(const double* In, int l, int64_t ldg, const double* T, int ldt, int lt,
                        int l_pad, double* Out, int xk, void* Xc, hipStream_t s);
// coords (n x k row-major) = Q^T-layout times Tc (l x k)
hipError_t launch_coords(const double* Qt, int l, int64_t n, int64_t ldg, const double* Tc, int k,
                         double* coords, double* sign_part, int64_t* idx_part, hipStream_t s);

// ---- small dense kernels (one workgroup) ------------------------------------
// T such that Y T has orthonormal columns, from W = Y^T Y (Cholesky, or an
// eigen-based inverse square root when Cholesky breaks down).
hipError_t launch_orth_factor(const double* W, int l, int l_pad, double* T, double* scratch,
                              DevStatus* st, hipStream_t s);
// Eigenpairs of the symmetrised B (algebraic descending); Tc = V_k diag(sqrt(max(theta,0))).
hipError_t launch_small_eig(const double* B, int l, int l_pad, int k, double* theta, double* V,
                            double* Tc, double* eigvals_out, double* scratch, DevStatus* st,
                            hipStream_t s);
hipError_t launch_finalize_stats(const double* fpart, int64_t nparts, DevStatus* st, hipStream_t s);

}  // namespace mds
