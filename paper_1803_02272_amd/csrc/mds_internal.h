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

// Kind of the G operand of a pass.  GK_FP8: OCP E4M3 codes with one fp32
// scale per 256 x 256 block, multiplied on bf16 MFMA (the X operand is bf16).
// GK_F32S: the fp32 pass (recentring D) computed on bf16 MFMA from exact
// three-term bf16 splits of both operands; X is stored split (see k_gpass).
// GK_S2: the same pass with G as its two-term split (about 16 significant
// bits) and X as bf16 (the first plane of the same split X layout): two
// products instead of six, each exact in fp32 (the 16-bit range passes).
// GK_S2X: G and X both as two-term splits (the first two planes of X) and
// three products, a0 b0 + a0 b1 + a1 b0 (the 16-bit projection).
enum GKind { GK_F64 = 0, GK_F32 = 1, GK_BF16 = 2, GK_FP8 = 3, GK_F32S = 4, GK_S2 = 5, GK_S2X = 6 };
inline bool gk_split(int gk) { return gk == GK_F32S || gk == GK_S2 || gk == GK_S2X; }
// terms of the G and X operands of a split pass kind
inline int gk_g_terms(int gk) { return gk == GK_F32S ? 3 : 2; }
inline int gk_x_terms(int gk) { return gk == GK_F32S ? 3 : (gk == GK_S2X ? 2 : 1); }
constexpr int kF8Block = 256;  // side of the blocks sharing one FP8 scale

constexpr int kPadN = 256;     // padding granule of n (rows and ld of G)
constexpr int kMaxL = 256;     // largest oversampled rank l = k + p
constexpr int kLdsMaxL = 128;  // small kernels keep an l x l fp64 matrix in LDS up to this l

// Device-side status words (written by kernels, read back by the host).
struct DevStatus {
  int nonfinite;        // D produced a non-finite sum of squares
  int orth_fallbacks;   // orthonormalisations that deflated directions
  int jacobi_sweeps;    // sweeps used by the last eigensolve
  int jacobi_unconv;    // eigensolves that hit the sweep cap
  int rank_deficient;   // last orthonormalisation dropped directions
  int pad_[3];
  double sum_sq;        // sum_ij d_ij^2
  double frob2;         // ||G||_F^2
  double trace;         // tr(G)
  unsigned long long asym_pairs;    // check_input: pairs i < j with d_ij != d_ji
  unsigned long long diag_nonzero;  // check_input: entries d_ii != 0
};

// ---- centring (Sec. 6.2, step 1) ------------------------------------------
constexpr int kStatsCols = 1024;  // columns per stats tile
constexpr int kStatsRows = 1024;  // rows per stats tile
// r, c, m (fp64), hc = fl32(c/2) (ldg floats, zero beyond n), and
// ||G||_F^2, tr(G) in the status words.  p4part: stats_parts(n) doubles.
// sym: read the tiles on and above the diagonal only (D symmetric), r = c.
int64_t stats_parts(int64_t n);
hipError_t launch_center_stats(const void* D, int d_is_f64, int64_t n, int64_t ldg, double* rowpart,
                               double* colpart, double* p4part, double* r, double* c, double* rsum, float* hc,
                               double* mean_all, DevStatus* st, int sym, hipStream_t s);
// FP8 storage of G: per 256 x 256 block, g = fl32(gamma) (gamma in fp64),
// s = fl32(max|g| / 448) (1 for an all-zero block), code = E4M3(fl32(g / s))
// rounded to nearest even and saturated at 448.  scales: nsb x nsb fp32,
// nsb = n_pad / 256.
hipError_t launch_center_write_fp8(const void* D, int d_is_f64, int64_t n, int64_t n_pad, int64_t ldg,
                                   const double* r, const double* c, const double* mean_all, uint8_t* G8,
                                   float* scales, hipStream_t s);
// Writes G (kind gk, ld = ldg, n_pad rows) and, if gref != nullptr, an fp32 copy.
int64_t center_write_blocks(int64_t n_pad, int64_t ldg);
hipError_t launch_center_write(const void* D, int d_is_f64, int64_t n, int64_t n_pad, int64_t ldg,
                               const double* r, const double* c, const double* mean_all, int gk, void* G,
                               float* gref, hipStream_t s);

// Finite-metric contract of D (symmetric, zero diagonal), whole matrix:
// adds the counts of asymmetric pairs and nonzero diagonal entries to st.
hipError_t launch_check_input(const void* D, int d_is_f64, int64_t n, DevStatus* st, hipStream_t s);

// ---- Gaussian test matrix ---------------------------------------------------
// Raw Philox4x64-10 blocks (counter words 0..3 and key words 0..1 per item).
hipError_t launch_philox(const uint64_t* in, uint64_t* out, int64_t count, hipStream_t s);
hipError_t launch_omega(uint64_t seed, int64_t n, int l, int l_pad, int64_t ldg, int xk, void* Xt,
                        hipStream_t s);

// ---- G-pass: Ypart[s] = G * X over K-split s (MFMA) ------------------------
struct GPassCfg {
  int rg;      // 16-row groups per wave
  int bm;      // rows per workgroup
  int split;   // K splits
  int sym;     // symmetric mode: upper triangle only, Ypart holds 2 (W o G) X
  int64_t steps_total, steps_per_split;
  int64_t sym_nbx;             // row blocks per XCD (symmetric mode and the LDS-ring split kernel)
  int64_t sym_cols_per_split;  // K columns per split (symmetric mode)
  int dma;                     // pass through an LDS ring: k_split (fp32 D, n % 4 == 0, aligned D) or k_gstream (bf16 G)
};
// sym (recentring passes only): the projection's symmetric mode, see k_gpass.
// d8: D holds fp64 (recentring passes keep more raw values in registers).
// gk == GK_BF16 with from_d: the fused centring write and first range pass
// on bf16 MFMA; gk == GK_F32S with a G argument: the fused centring write and
// an fp32 first range pass (three-term split).
// dma_ok (split kinds from D): n % 4 == 0 and D 16-byte aligned, so the pass
// may stream D through LDS (needs the same alignment at launch); (GK_BF16
// over the stored G): stream G through LDS (k_gstream).
GPassCfg gpass_config(int gk, int l_pad, int64_t n_pad, int64_t ldg, int split_hint, bool from_d, bool sym,
                      bool d8, bool dma_ok = false);
// With D != nullptr the A operand is recentred on the fly from D (ld = n)
// and G is unused.  fp64 passes: gamma_ij = -1/2 (((d_ij^2 - c_j) - r_i) + m)
// in fp64 (the stored-G value).  fp32 passes: gamma_ij =
// fma(-1/2, fl32(d_ij^2), hc_j + hr_i) in fp32 with hc_j = fl32(c_j / 2) and
// hr_i = fl32((r_i - m) / 2), a few fp32 ulps of the terms from the rounded
// exact value.
struct GPassDSrc {
  // (with gk == GK_BF16, GK_F32S or GK_S2 and D set, a non-null G argument of the pass
  // is the bf16 G that it writes: the fused centring write)
  const float* g8_scales = nullptr;  // GK_FP8: scale of block (I, J) at [I * g8_nsb + J]
  int64_t g8_nsb = 0;
  const void* D = nullptr;
  int64_t n = 0;
  const double* r = nullptr;
  const double* c = nullptr;
  const float* hc = nullptr;
  const double* m = nullptr;
  int vec = 0;
  int d_is_f64 = 0;
};
// The same pass (split, K ranges, summation order) with the register-prefetch
// kernel instead of the LDS-ring split kernel, for a D that is not 16-byte
// aligned.
GPassCfg gpass_config_nodma(const GPassCfg& c, int l_pad, int64_t n_pad, bool d8);
int64_t gpass_blocks(const GPassCfg& cfg, int64_t n_pad);
// The pipelined split pass (fp32 D, n % 4 == 0, 16-byte aligned D, l_pad <=
// 128; cfg.dma configurations): full pass, symmetric projection, or with Gw
// the fused centring write.  split_pass_rows(): rows per workgroup.
int split_pass_rows();
// The range pass over a stored bf16 G through an LDS ring (k_gstream):
// 256-row blocks, l_pad <= 128, a configuration from gpass_config with dma set.
int gstream_rows();
hipError_t launch_gstream(const void* G, int64_t ldg, const void* Xt, int l_pad, const GPassCfg& cfg, int64_t n,
                          int64_t blocks, void* Yp, hipStream_t s);
// Persisted autotune choices (tune_cache.hip, MDS_TUNE_CACHE): splits are
// range, projection, fused write, end passes.
struct TuneKey {
  int form, flags, d_dtype, l_pad, q;
  int64_t n;
};
bool tune_cache_lookup(const TuneKey& k, int (&splits)[4]);
bool tune_cache_store(const TuneKey& k, const int (&splits)[4]);
// Pairwise distances (k_dist.hip): D row-major n x n in fp32 or fp64.
constexpr int kMaxHammingLength = 2048;
constexpr int64_t kMaxDistanceN = 4000000;
hipError_t launch_hamming(const uint8_t* codes, int64_t n, int L, bool f64, void* D, hipStream_t s);
hipError_t launch_euclid(const double* X, int64_t n, int dim, bool f64, void* D, hipStream_t s);
// Connected components of the threshold graph (k_cc.hip); n_components may be null.
hipError_t launch_components(const void* D, bool f64, int64_t n, double theta, bool full, int32_t* labels,
                             int64_t* n_components, hipStream_t s);
// Tile (I, J), I <= J, of linear index t in the row-ordered upper triangle of
// nt x nt tiles: row I starts at S(I) = I nt - I (I - 1) / 2; the largest I
// with S(I) <= t from the root of the quadratic, corrected by whole steps.
__device__ inline void upper_tile(int64_t t, int64_t nt, int64_t& I, int64_t& J) {
  auto row_start = [&](int64_t r) { return r * nt - r * (r - 1) / 2; };
  const double b2 = 2.0 * (double)nt + 1.0;
  int64_t r = (int64_t)((b2 - __builtin_sqrt(b2 * b2 - 8.0 * (double)t)) * 0.5);
  if (r < 0) r = 0;
  if (r > nt - 1) r = nt - 1;
  while (r > 0 && row_start(r) > t) --r;
  while (r + 1 < nt && row_start(r + 1) <= t) ++r;
  I = r;
  J = r + (t - row_start(r));
}
// Zero the padding of the bf16 G (rows >= n, columns >= n) left by the fused write.
hipError_t launch_split_zero_pad(void* G, int64_t n, int64_t n_pad, int64_t ldg, hipStream_t s);
// gterms / xterms: terms of the G and X operands, (3, 3), (2, 1) or (2, 2)
hipError_t launch_split_pass(int gterms, int xterms, const void* Xt, int64_t ldg, int l_pad, const GPassCfg& cfg,
                             int64_t blocks, void* Yp, const GPassDSrc& src, void* Gw, hipStream_t s);
hipError_t launch_gpass(int gk, const void* G, int64_t ldg, int64_t n_pad, const void* Xt, int l_pad,
                        const GPassCfg& cfg, void* Ypart, const GPassDSrc& src, hipStream_t s);
// Y (fp64, l_pad x ldg) = sum_s Ypart[s] in split order (symmetric mode:
// over the splits that hold a partial for the row).
hipError_t launch_splitk_reduce(int gk, const GPassCfg& cfg, const void* Ypart, int64_t ldg, int64_t elems,
                                double* Y, hipStream_t s);

// ---- skinny fp64 kernels ----------------------------------------------------
int64_t gram_chunks(int64_t ldg);
// Wpart[p] = A_p B_p^T over column chunk p; then W = sum_p Wpart[p].
hipError_t launch_gram(const double* A, const double* B, int l_pad, int64_t ldg, double* Wpart,
                       double* W, hipStream_t s);
// Out = T^T In (In, Out: l_pad x ldg transposed tall matrices; T: l x lt, ld = ldt).
// Out rows >= lt are zeroed.  Optional cast copy of Out into Xc (kind xk).
hipError_t launch_apply(const double* In, int l, int64_t ldg, const double* T, int ldt, int lt,
                        int l_pad, double* Out, int xk, void* Xc, hipStream_t s);
int64_t coords_anchor_chunks(int64_t n);
// coords (n x k row-major) = Q Tc (Tc: l x k), columns sign-normalised.
// Ct is a transposed scratch of k_pad16 x ldg doubles.
hipError_t launch_coords(const double* Qt, int l, int64_t n, int64_t ldg, const double* Tc, int k,
                         double* Ct, double* coords, double* sign_part, int64_t* idx_part, hipStream_t s);

// ---- small dense kernels (one workgroup) ------------------------------------
// T such that Y T has orthonormal columns, from W = Y^T Y (deflating
// Cholesky, T = R^{-1}; for l_pad > 128 as two diagonal blocks).
// near_identity: W is the Gram matrix of an almost orthonormal basis (second
// CholeskyQR step); a first-order factor is used when W is within 1e-9 of I.
// scratch: orth_factor_scratch_bytes(l_pad) bytes of device memory.
hipError_t launch_orth_factor(const double* W, int l, int l_pad, double* T, double* scratch,
                              DevStatus* st, int near_identity, hipStream_t s);
size_t orth_factor_scratch_bytes(int l_pad);
// Eigenpairs of the symmetrised B (algebraic descending); Tc = V_k diag(sqrt(max(theta,0))).
size_t small_eig_rot_bytes(int l);
hipError_t launch_small_eig(const double* B, int l, int l_pad, int k, double* theta, double* V,
                            double* Tc, double* eigvals_out, double* scratch, void* rot, int* meta,
                            DevStatus* st, hipStream_t s);

}  // namespace mds
