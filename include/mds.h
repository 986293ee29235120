/*
 * mds.h -- C ABI of the MI355X (gfx950) random-projection classical MDS library.
 *
 * Method (Blanchard et al., "A geometric view of Biodiversity: scaling to
 * metagenomics", Inria RR-9144):
 *   - Sec. 6.2, step 1: Gram matrix by double centring of the squared
 *     distances, gamma_ij = -1/2 (d_ij^2 - c_j - r_i + m) with r_i, c_j the
 *     row/column means of d^2 and m their grand mean.
 *   - Sec. 3.2-3.3: approximate rank-k eigendecomposition of G by random
 *     projection (the randomized range finder of Halko, Martinsson and Tropp,
 *     2011): Gaussian test matrix Omega (n x l, l = k + oversample), q power
 *     iterations (each = two applications of G, orthonormalised after each
 *     application), then Rayleigh-Ritz on B = Q^T G Q.
 *   - Sec. 6.2, steps 2-3: eigenpairs in descending algebraic order and
 *     coordinates X = U diag(sqrt(max(lambda, 0))), first k columns.
 *
 * Conventions shared by every entry point:
 *   - Pointers named "dev" or documented as device memory must be device
 *     allocations valid on the current HIP device; the library never frees
 *     caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it; calls return once work is enqueued.
 *   - Errors are reported by status code only; no exception crosses the ABI.
 *     mds_last_error() gives a thread-local text for the last failure.
 *   - Argument errors are detected on the host before any device call.
 *   - A plan is not thread-safe: calls on one plan must be serialised, and
 *     two runs of one plan on different streams must not overlap.
 */
#ifndef MDS_H_
#define MDS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mds_status {
  MDS_OK = 0,
  MDS_PENDING = 1,
  MDS_ERR_INVALID_ARG = -1, /* bad size, pointer or option */
  MDS_ERR_NO_DEVICE = -2,   /* no HIP device visible */
  MDS_ERR_OOM = -3,         /* device allocation failed */
  MDS_ERR_BUDGET = -4,      /* job can never fit the server's memory budget */
  MDS_ERR_NONFINITE = -5,   /* D holds NaN or Inf (detected by the centring sums) */
  MDS_ERR_NUMERICAL = -6,   /* eigensolver did not converge */
  MDS_ERR_HIP = -7,         /* a HIP runtime call or kernel launch failed */
  MDS_ERR_CANCELLED = -8,   /* job cancelled before it ran */
  MDS_ERR_STATE = -9,       /* call not valid in the plan's current state */
  MDS_ERR_NOT_METRIC = -10  /* MDS_FLAG_CHECK_INPUT: D is not symmetric with a zero diagonal */
} mds_status;

/* Arithmetic form of the G-passes (dtype of the G operand).
 *   FP64: G entries in fp64, fp64 MFMA.
 *   FP32: G entries rounded to fp32, fp32 MFMA.
 *   BF16: G stored in bf16 (rounded from fp64 through fp32).  Of the 2q+1
 *         range passes, the first and the last are 16-bit passes over D and
 *         the q*2-1 between them run on the stored bf16 G against bf16 X
 *         (bf16 MFMA, fp32 accumulation); the projection pass
 *         ("refinement") is a 16-bit pass too.  A 16-bit pass takes the fp32
 *         value a of each G entry as the two-term bf16 expansion a0 + a1
 *         (a0 = bf16(a), a1 = bf16(a - a0), nearest even: about 16
 *         significant bits) and X as b = bf16(x), and accumulates a1 b + a0 b
 *         on bf16 MFMA in fp32 (each product exact).  The first range pass
 *         also writes the stored G
 *         (fused centring write, fp32 D).  Running the two end passes at 16
 *         bits keeps the bf16 rounding of G out of the sketch of Omega and
 *         out of the final basis: the Ritz values then stay within 1e-3
 *         (relative, per eigenvalue) of the fp64 method also where the k-th
 *         eigenvalue lies in a near-degenerate bulk, where a sketch made
 *         entirely of bf16 passes moves them by about 1e-3
 *         (MDS_FLAG_LOWP_ALL_RANGE restores that faster schedule).  The
 *         bf16 rounding of X enters the Ritz values only through inner
 *         products over n rows, which average it: about 1e-4 relative at
 *         most in the parity cases (MDS_FLAG_FP32_PROJECTION makes the
 *         projection an fp32 pass).
 *         An fp32 pass (the FP32 form with MDS_FLAG_SPLIT_FP32, the
 *         projection with MDS_FLAG_FP32_PROJECTION) multiplies fp32 G
 *         entries with fp32 X to fp32 accuracy: each fp32 operand is split
 *         exactly into three bf16 terms (a = a0 + a1 + a2, each rounded to
 *         nearest even) and the six products a_p b_q with p + q <= 2 run on
 *         bf16 MFMA with fp32 accumulation (the dropped terms are below
 *         2^-22 |a b|).
 *   FP8:  G stored as OCP FP8 E4M3 codes with one fp32 scale per 256 x 256
 *         block: g = fl32(gamma), s = fl32(max|g| / 448) over the block (1
 *         for an all-zero block), code = E4M3(fl32(g / s)), nearest even,
 *         saturating.  The range passes between the first and the last
 *         multiply bf16(fl32(s * code)) with bf16 X on bf16 MFMA, fp32
 *         accumulation; the first and last range passes and the projection
 *         are 16-bit passes as in the bf16 form.
 * G is stored only in the bf16 and fp8 forms (and only when q >= 1: with q = 0
 * the one range pass is a 16-bit pass from D).  Every other pass recomputes each
 * entry from D: fp64 passes with the centring equation in fp64 (the values a
 * stored fp64 G would hold), fp32 passes as fma(-1/2, fl32(d^2),
 * fl32(c_j/2) + fl32((r_i - m)/2)) in fp32, within a few fp32 ulps of the
 * terms of the rounded exact value (the fused first pass of the bf16 form
 * uses fl32(gamma) of the fp64 gamma itself).
 * In every form the centring sums, CholeskyQR2, the Gram products of the
 * tall matrices and the small eigensolve run in fp64. */
typedef enum mds_form { MDS_FORM_FP64 = 0, MDS_FORM_FP32 = 1, MDS_FORM_BF16 = 2, MDS_FORM_FP8 = 3 } mds_form;

/* Element type of the caller's distance matrix D. */
typedef enum mds_dtype { MDS_DTYPE_F32 = 0, MDS_DTYPE_F64 = 1 } mds_dtype;

/* Option flags.
 *   MDS_FLAG_FULL_PROJECTION: stream all of G in the projection pass.  By
 *   default the projection uses the symmetry of G (D symmetric is the
 *   contract): B = Q^T G Q is assembled as S + S^T from the upper triangle
 *   of G only, S = Q^T (W o G) Q with W = 1 above, 1/2 on and 0 below the
 *   diagonal, which halves that pass's reads and MFMA work.  Both give the
 *   same B up to rounding for a symmetric D; for a D that breaks the
 *   contract, the default reads only its upper triangle (j >= i) there. */
#define MDS_FLAG_FULL_PROJECTION 1
/*   MDS_FLAG_FP32_MFMA_PROJECTION: BF16 and FP8 forms, run the projection as
 *   an fp32 pass on fp32 MFMA (same fp32 operands as MDS_FLAG_FP32_PROJECTION;
 *   the results differ by fp32 rounding only, the split is about 2.5x
 *   faster).  No effect in the other forms. */
#define MDS_FLAG_FP32_MFMA_PROJECTION 2
/*   MDS_FLAG_SPLIT_FP32: FP32 form, run every G-pass (range passes and
 *   projection) as the three-term bf16 split on bf16 MFMA described under
 *   MDS_FORM_BF16: the same fp32 operands and fp32 accumulation as the plain
 *   FP32 form, to fp32 accuracy, in less time.  No effect in the other
 *   forms (the BF16 and FP8 forms' projection already uses it). */
#define MDS_FLAG_SPLIT_FP32 4
/*   MDS_FLAG_FULL_STATS: read all of D in the centring statistics.  By
 *   default that pass uses the symmetry of D (the contract) and reads only
 *   its 1024 x 1024 tiles on and above the diagonal, half of D: the row
 *   means r_i = (1/n) sum_j d_ij^2 are assembled from the row sums of the
 *   tiles right of the diagonal and the column sums of the tiles above it,
 *   and c = r.  With the flag, r and c are the row and column means of all
 *   of D as written in the double-centring formula; both agree up to
 *   rounding for a symmetric D. */
#define MDS_FLAG_FULL_STATS 8
/*   MDS_FLAG_CHECK_INPUT: before the centring, test the finite-metric
 *   contract on the whole of D (one extra read of D): d_ij == d_ji exactly
 *   for every pair and d_ii == 0.  Violations are counted on the device and
 *   reported by mds_get_info (asym_pairs, diag_nonzero) with status
 *   MDS_ERR_NOT_METRIC; the run itself still completes (its result is that
 *   of the upper triangle of D, see MDS_FLAG_FULL_STATS and
 *   MDS_FLAG_FULL_PROJECTION).  A NaN entry counts as asymmetric. */
#define MDS_FLAG_CHECK_INPUT 16
/*   MDS_FLAG_LOWP_ALL_RANGE: BF16 and FP8 forms, run all 2q+1 range passes
 *   on the stored low-precision G (no 16-bit first and last range pass):
 *   faster by two passes over D less, with Ritz values that may move by ~1e-3
 *   relative when the k-th eigenvalue lies in a near-degenerate bulk (bf16;
 *   ~1e-1 for fp8).  No effect in the other forms. */
#define MDS_FLAG_LOWP_ALL_RANGE 32
/*   MDS_FLAG_FP32_PROJECTION: BF16 and FP8 forms, run the projection as an
 *   fp32 pass (three-term bf16 split of both operands, six products) instead
 *   of the 16-bit pass (two-term G, bf16 X, two products).  No effect in the
 *   other forms. */
#define MDS_FLAG_FP32_PROJECTION 64

typedef struct mds_opts {
  int32_t form;        /* mds_form (default MDS_FORM_FP32) */
  int32_t d_dtype;     /* mds_dtype (default MDS_DTYPE_F32) */
  int32_t gpass_split; /* K-splits of the range passes, 0 = automatic */
  int32_t flags;       /* MDS_FLAG_* bits, 0 = defaults; other bits are rejected */
  int32_t proj_split;  /* K-splits of the projection pass, 0 = as gpass_split */
  int32_t write_split; /* K-splits of the fused centring write + first range pass, 0 = as gpass_split */
  int32_t f32_split;   /* K-splits of the fp32 end range passes of the BF16/FP8 forms that are not
                          fused with the write, 0 = as gpass_split */
} mds_opts;

typedef struct mds_plan_s* mds_plan_t;

/* Largest oversampled rank l = k + oversample supported. */
#define MDS_MAX_L 256

/* Create a plan for n points, k output axes, `oversample` extra sketch
 * columns, q power iterations and the seed of the test matrix.  Valid:
 * 2 <= n <= 1000000, k >= 1, oversample >= 0, q >= 0,
 * k + oversample <= min(n, MDS_MAX_L).
 * Makes no device call.  *out receives an opaque handle owned by the caller
 * (free with mds_destroy).  mds_plan uses default options. */
mds_status mds_plan(mds_plan_t* out, int64_t n, int32_t k, int32_t oversample, int32_t q, uint64_t seed);
mds_status mds_plan_ex(mds_plan_t* out, int64_t n, int32_t k, int32_t oversample, int32_t q, uint64_t seed,
                       const mds_opts* opts);

/* Device workspace needed by mds_run, in bytes (host-only computation). */
mds_status mds_workspace_size(mds_plan_t plan, size_t* bytes);

/* Hand the plan a caller-owned device buffer of at least mds_workspace_size
 * bytes (e.g. allocated by PyTorch).  It must stay valid while any run of the
 * plan is in flight.  Without it, the first run allocates the workspace with
 * hipMalloc and mds_destroy frees it. */
mds_status mds_set_workspace(mds_plan_t plan, void* dev_ptr, size_t bytes);

/* Run the whole method on `stream`:
 *   D       device, n x n row-major (ld = n), dtype from the plan options;
 *           a finite metric: symmetric with zero diagonal is the contract,
 *           the centring uses both row and column means as written.
 *   coords  device, n x k row-major fp64: X = Q V_k diag(sqrt(max(theta,0))),
 *           each column's entry of largest magnitude made positive.
 *   eigvals device, k fp64: the k largest Ritz values, algebraic descending.
 * Returns MDS_OK once enqueued.  Numerical outcome (non-finite input, solver
 * convergence) is available from mds_get_info after the stream completes. */
mds_status mds_run(mds_plan_t plan, const void* D, double* coords, double* eigvals, void* stream);

/* Stages for partial runs (tests and diagnostics). */
typedef enum mds_stage {
  MDS_STAGE_CENTER = 1, /* stop after the centring pass (G, r, c, m ready) */
  MDS_STAGE_OMEGA = 2,  /* ... after drawing Omega into the pass operand */
  MDS_STAGE_RANGE = 3,  /* ... after `range_passes` orthonormalised G-applications */
  MDS_STAGE_ALL = 100
} mds_stage;

/* Like mds_run, stopping after `stop_after`.  For MDS_STAGE_RANGE,
 * range_passes is in [1, 2q+1]; coords/eigvals may be NULL unless
 * stop_after == MDS_STAGE_ALL. */
mds_status mds_run_stages(mds_plan_t plan, const void* D, double* coords, double* eigvals, void* stream,
                          int32_t stop_after, int32_t range_passes);

/* Internal buffers exposed read-only for inspection after a (partial) run. */
typedef enum mds_buffer_id {
  MDS_BUF_G = 0,       /* stored Gram matrix, n_pad x ldg: bf16 (BF16 form) or E4M3 codes (FP8 form) */
  MDS_BUF_GREF = 1,    /* reserved (no fp32 copy of G is stored) */
  MDS_BUF_ROWMEAN = 2, /* r, n fp64 */
  MDS_BUF_COLMEAN = 3, /* c, n fp64 */
  MDS_BUF_MEAN = 4,    /* m, 1 fp64 */
  MDS_BUF_X = 5,       /* current G-pass operand, transposed l_pad x ldg; in the split
                          passes (the BF16/FP8 forms' projection, MDS_FLAG_SPLIT_FP32),
                          l_pad rows of 3 ldg bf16: per 32 columns the 32 x0, 32 x1 and
                          32 x2 terms */
  MDS_BUF_Q = 6,       /* orthonormal basis, transposed l_pad x ldg fp64 */
  MDS_BUF_Y = 7,       /* last G-pass product, transposed l_pad x ldg fp64 (after the
                          symmetric projection: 2 (W o G) Q, see MDS_FLAG_FULL_PROJECTION) */
  MDS_BUF_B = 8,       /* projected matrix Q^T G Q, l_pad x l_pad fp64 */
  MDS_BUF_THETA = 9,   /* all l Ritz values, descending, fp64 */
  MDS_BUF_V = 10,      /* Ritz vectors in the Q basis, l x l (ld l_pad) fp64 */
  MDS_BUF_W = 11,      /* last small Gram product (Y^T Y or Q1^T Q1), l_pad x l_pad fp64 */
  MDS_BUF_T = 12,      /* last orthonormalising factor, l_pad x l_pad fp64 */
  MDS_BUF_Q1 = 13,     /* first CholeskyQR iterate, transposed l_pad x ldg fp64 */
  MDS_BUF_GSCALE = 14  /* FP8 form: block scales, (n_pad/256) x (n_pad/256) fp32 */
} mds_buffer_id;

typedef struct mds_buffer {
  void* ptr;      /* device pointer into the workspace */
  int32_t dtype;  /* 0 fp64, 1 fp32, 2 bf16, 3 fp8 e4m3 codes */
  int32_t pad_;
  int64_t rows, cols, ld; /* logical shape and leading dimension (elements) */
} mds_buffer;

mds_status mds_get_buffer(mds_plan_t plan, int32_t which, mds_buffer* out);

typedef struct mds_info {
  int32_t status;            /* numerical outcome of the last run */
  int32_t nonfinite;         /* 1 if D contained NaN/Inf */
  int32_t orth_fallbacks;    /* orthonormalisations that deflated (dropped) directions */
  int32_t jacobi_sweeps;     /* sweeps of the last small eigensolve */
  int32_t jacobi_unconverged;
  int32_t rank_deficient;    /* directions dropped by the last orthonormalisation */
  int32_t k, l, l_pad, q, form, gpass_split;
  int64_t n, ldg;
  double sum_sq;             /* sum_ij d_ij^2 */
  double frob2;              /* ||G||_F^2 (fp64, closed form in the centring sums) */
  double trace;              /* tr(G) */
  int64_t asym_pairs;        /* MDS_FLAG_CHECK_INPUT: pairs i < j with d_ij != d_ji */
  int64_t diag_nonzero;      /* MDS_FLAG_CHECK_INPUT: entries d_ii != 0 */
  int32_t tuned_from_cache;  /* 1: the splits came from the MDS_TUNE_CACHE file */
} mds_info;

/* Synchronise `stream`, then report the plan's last-run diagnostics. */
mds_status mds_get_info(mds_plan_t plan, mds_info* out, void* stream);

/* Per-phase timing with HIP events recorded on the run's stream.  Phases: */
enum {
  MDS_PH_STATS = 0,    /* centring statistics (read D) */
  MDS_PH_WRITE = 1,    /* centring write (read D, write G); bf16 form on fp32 D: fused with range pass 1 */
  MDS_PH_OMEGA = 2,    /* test matrix */
  MDS_PH_GPASS = 3,    /* one range-pass kernel over the form's G (per launch); the fp32 end
                          passes of the BF16/FP8 forms are MDS_PH_WRITE or MDS_PH_GPASS_F32 */
  MDS_PH_REDUCE = 4,   /* split-K reduction of a G-pass */
  MDS_PH_ORTH = 5,     /* one CholeskyQR2 */
  MDS_PH_GPASS_REF = 6,/* the projection G-pass kernel */
  MDS_PH_SMALL = 7,    /* B = Q^T (G Q) and the small eigensolve */
  MDS_PH_COORDS = 8,   /* coordinates and signs */
  MDS_PH_GPASS_F32 = 9,/* an fp32 range pass of the BF16/FP8 forms that is not fused with the write
                          (the last one; the first as well on fp64 D or in the FP8 form) */
  MDS_PH_CHECK = 10,   /* MDS_FLAG_CHECK_INPUT: the symmetry and diagonal test */
  MDS_NUM_PHASES = 11
};
typedef struct mds_phase_time {
  int32_t count;   /* launches timed since the last read */
  float total_ms;
  float min_ms;
  float max_ms;
} mds_phase_time;
/* Enable (1) or disable (0) event timing for subsequent runs of the plan. */
mds_status mds_set_timing(mds_plan_t plan, int32_t enable);
/* Synchronise `stream`, then fill out[MDS_NUM_PHASES] with the phases timed
 * since the previous call, and reset the accumulators. */
mds_status mds_get_timings(mds_plan_t plan, mds_phase_time* out, void* stream);

/* Autotuner of a plan: times every split-K candidate (the K extent of a
 * workgroup's tile) of the range pass, the projection pass, the fp32 end
 * range passes of the BF16/FP8 forms and, in the bf16 form on fp32 D, the
 * fused centring write, on this plan's shape and the
 * given D; stores the fastest in the plan's options (copies made by the
 * server inherit them) and reports them.  Must be called before a workspace
 * is attached; allocates and frees a temporary one; synchronises `stream`. */
typedef struct mds_tune_result {
  int32_t range_split, proj_split, write_split, f32_split;
  float range_ms, proj_ms, write_ms, f32_ms; /* best per-launch times (pass + split-K reduction) */
  int32_t candidates;                        /* configurations timed */
} mds_tune_result;
mds_status mds_autotune(mds_plan_t plan, const void* D, void* stream, mds_tune_result* out);
/* Persisted choices: when the environment variable MDS_TUNE_CACHE names a
 * file, mds_autotune records the splits it chose there (one text line per
 * key: device architecture and CU count, form, flags, D dtype, n, l_pad, q),
 * and mds_plan / mds_plan_ex start a plan whose splits are all automatic
 * from the recorded choice of its key (mds_info.tuned_from_cache = 1).  The
 * file is rewritten whole through a rename; an unreadable or missing file is
 * ignored. */

void mds_destroy(mds_plan_t plan);

/* The generator behind Omega, exposed for validation against published
 * known-answer vectors: Philox4x64-10 (Salmon, Moraes, Dror and Shaw,
 * "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11; the test matrix of
 * the random projection, Sec. 3.2, draws entry (i, j) from the block at
 * counter (i, j / 4, 0, 0) with key (seed, 0)).  in: device, count x 6
 * uint64 (counter words 0..3, key words 0..1); out: device, count x 4 uint64
 * (the block).  Enqueued on `stream`; caller-owned buffers. */
mds_status mds_philox4x64_10(const uint64_t* in, uint64_t* out, int64_t count, void* stream);

/* Pairwise distances on the device: the dissimilarity matrix between reads
 * that the method takes as input (Sec. 2.2; in Table 1 its computation is
 * the dominant cost of the pipeline), written as the D that mds_run reads:
 * row-major n x n, ld = n, element type d_dtype (MDS_DTYPE_F32 or _F64).
 * Caller-owned device buffers, enqueued on `stream` (no allocation, no
 * synchronisation).  Argument errors (NULL pointer, sizes out of range, bad
 * dtype) return MDS_ERR_INVALID_ARG before any device call; no device:
 * MDS_ERR_NO_DEVICE.  Exact in the sense that each entry is the stated
 * formula with its stated roundings: the same bits as a CPU evaluation.
 *
 * mds_hamming_distances: codes is n x length bytes (row-major, ld = length),
 * one base per byte as 0..3 (A, C, G, T); d_ij = (number of positions p at
 * which codes differ) / length, the fp64 quotient rounded to nearest even
 * in d_dtype.  A byte outside 0..3 matches nothing, itself included (an
 * unknown base is a mismatch).  The Hamming distance stands in for the
 * alignment-based dissimilarity of Sec. 2.2 (reads that differ by
 * substitutions only).  1 <= n <= 4e6, 1 <= length <= 2048.
 *
 * mds_euclidean_distances: X is n x dim fp64 points (row-major, ld = dim);
 * d_ij = sqrt(sum_k (x_ik - x_jk)^2) with the square and each partial sum
 * rounded to fp64 (no fused multiply-add), k increasing, then the square
 * root rounded to d_dtype.  D is exactly symmetric with a zero diagonal.
 * 1 <= n <= 4e6, 1 <= dim <= 2^20. */
mds_status mds_hamming_distances(const uint8_t* codes, int64_t n, int32_t length, int32_t d_dtype, void* D,
                                 void* stream);
mds_status mds_euclidean_distances(const double* X, int64_t n, int32_t dim, int32_t d_dtype, void* D, void* stream);

/* Connected components of the threshold graph on D (Sec. 7, Conclusions and
 * perspectives: the n items are the vertices and (i, j), i != j, is an edge
 * iff d_ij <= threshold; the components are candidate clusters of reads).
 * D: device n x n, row-major, ld = n, element type d_dtype; each entry is
 * compared as an fp64 value (exact for fp32 D); a NaN entry is no edge.  By
 * default only the upper triangle j > i is read (D symmetric by contract,
 * half the reads); with MDS_CC_FULL_MATRIX every off-diagonal entry is read
 * and (i, j) is an edge iff d_ij <= threshold or d_ji <= threshold.
 * labels: device int32[n], written with labels[i] = the smallest index of
 * the component of i (canonical: the same labels whatever the evaluation
 * order).  n_components: device int64, the number of components, or NULL.
 * Caller-owned buffers; enqueued on `stream`, no allocation and no
 * synchronisation; labels and n_components are valid once the stream
 * reaches that point.  Argument errors (NULL D or labels, n outside
 * 1..4e6, bad dtype or flags, NaN threshold) return MDS_ERR_INVALID_ARG
 * before any device call; no device: MDS_ERR_NO_DEVICE. */
#define MDS_CC_FULL_MATRIX 1
mds_status mds_threshold_components(const void* D, int32_t d_dtype, int64_t n, double threshold, int32_t flags,
                                    int32_t* labels, int64_t* n_components, void* stream);

/* ---- Batched small instances ------------------------------------------------
 * Many independent MDS instances of uneven n in one persistent launch: one
 * workgroup runs a whole instance (centring, Omega, range passes with
 * CholeskyQR2, projection, eigensolve, coordinates), so a launch fills the
 * GPU with instances rather than with tiles of one instance.  Limits per
 * instance: 2 <= n <= 16384 and k + oversample rounded up to 16 <= 64.  All
 * instances of a call share one form.  The values of every dtype follow
 * mds_run (same G entries, same Omega, same sign convention); sums run in
 * another order, so results agree with mds_run to rounding, not bit for bit. */
typedef struct mds_batch_job {
  const void* D;   /* device, n x n row-major, dtype d_dtype */
  double* coords;  /* device, n x k row-major fp64 */
  double* eigvals; /* device, k fp64 */
  int64_t n;
  int32_t k, oversample, q, d_dtype;
  uint64_t seed;
} mds_batch_job;
/* Device workspace for the batch (host-only computation). */
mds_status mds_batch_workspace_size(const mds_batch_job* jobs, int32_t count, int32_t form, size_t* bytes);
/* Enqueue the batch on `stream` (256-byte aligned workspace of at least the
 * size above, caller-owned, valid until the stream work completes).  tile:
 * K depth of the G-pass register tile (1, 2 or 4), 0 = the autotuned choice
 * for the batch's size class (4 if none was tuned). */
mds_status mds_run_batch(const mds_batch_job* jobs, int32_t count, int32_t form, void* workspace, size_t bytes,
                         int32_t tile, void* stream);
/* Autotuner of the batched kernel.  Times every tile shape of the batched
 * kernel's G-pass (the K depth of the register tile: 1, 2 or 4 MFMA chunks
 * of operands loaded ahead) on `batch` instances of size n (a synthetic
 * full-rank distance matrix), records the fastest in a process-wide table
 * that mds_run_batch consults for that size class of n, form and l, and
 * also times the plan path on one instance.  Allocates and frees its own
 * device memory; synchronises `stream`. */
typedef struct mds_batch_tune {
  int32_t tile;                /* chosen K depth */
  int32_t pad_;
  float batch_ms_per_job[3];   /* per instance, tile 1, 2, 4 */
  float batch_ms_best;         /* per instance, chosen tile */
  float plan_ms;               /* one instance through mds_run */
} mds_batch_tune;
mds_status mds_autotune_batch(int32_t form, int64_t n, int32_t k, int32_t oversample, int32_t q, int32_t batch,
                              void* stream, mds_batch_tune* out);
/* Synchronise `stream` and write the numerical status of each instance of
 * the last batch run in `workspace` (MDS_OK, MDS_ERR_NONFINITE or
 * MDS_ERR_NUMERICAL) to host statuses[count]. */
mds_status mds_batch_status(const void* workspace, int32_t count, int32_t* statuses, void* stream);

/* mds_run_batch without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The batch workspace is a static device
 * array of MDS_BATCH_STATIC_BYTES (128 MiB) that the library holds on every
 * device it runs on until the process ends; no hipMalloc,
 * hipFree or allocating library routine is called.  The same kernels as
 * mds_run_batch, so each instance's result equals mds_run_batch's.
 *   jobs, count, form, tile: as for mds_run_batch.
 *   statuses: optional device array of count int32 (NULL: none), written
 *             with each instance's final status (MDS_OK, MDS_ERR_NONFINITE,
 *             MDS_ERR_NUMERICAL) by the batched kernel itself.
 * Errors (host-side, before any device work): MDS_ERR_INVALID_ARG for bad
 * jobs or a batch whose workspace (mds_batch_workspace_size) exceeds the
 * capacity, MDS_ERR_NO_DEVICE.  All calls on one device share its array and
 * each call overwrites what the last one left: calls that overlap on one
 * device (different streams, or threads) race and must be serialised by the
 * caller. */
#define MDS_BATCH_STATIC_BYTES ((size_t)128 << 20)
mds_status mds_run_batch_static(const mds_batch_job* jobs, int32_t count, int32_t form, int32_t tile,
                                int32_t* statuses, void* stream);

/* ---- Serving: continuous batching of MDS jobs (spec serving loop) ----
 * A server owns a device arena of hbm_budget_bytes, allocated once by
 * mds_server_create (nothing is allocated on the device while serving), and
 * max_slots HIP streams.  Submitted jobs wait in a FIFO queue; a worker thread
 * inside the server admits the queue head as soon as a slot is free and the
 * arena has room for the job's workspace, enqueues the whole run on that
 * slot's stream, and retires finished jobs, whose slot and memory then admit
 * the next ones.  Admitted jobs run concurrently on the device.  Each job runs
 * on the server's own copy of the plan, so its result is bit-identical to
 * mds_run of the same plan alone (small jobs: see mds_server_set_batching),
 * and the caller may reuse or destroy `plan` right after mds_submit.  Server calls are thread-safe; no call may be in
 * flight on a server that is being destroyed. */
typedef struct mds_server_s* mds_server_t;
typedef uint64_t mds_ticket;

typedef struct mds_job_times {
  double queue_ms;   /* submit -> admitted (host clock) */
  double run_ms;     /* admitted -> completion observed by the server */
  double latency_ms; /* submit -> completion observed */
} mds_job_times;

typedef struct mds_server_info {
  int32_t queued, running, slots, pad_;
  uint64_t completed;
  uint64_t batches; /* batched launches of small jobs */
  size_t budget_bytes, used_bytes, peak_bytes; /* arena size, bytes held by admitted jobs, peak */
} mds_server_info;

/* Create a server on the current HIP device.  1 <= max_slots <= 256.
 * Errors: MDS_ERR_INVALID_ARG, MDS_ERR_NO_DEVICE, MDS_ERR_OOM (arena), MDS_ERR_HIP. */
mds_status mds_server_create(mds_server_t* out, size_t hbm_budget_bytes, int32_t max_slots);
/* Queue one job.  D, coords, eigvals as for mds_run (device memory of the
 * server's device); they must stay valid until the job is terminal.
 * MDS_ERR_BUDGET if the plan's workspace can never fit the arena. */
mds_status mds_submit(mds_server_t server, mds_plan_t plan, const void* D, double* coords, double* eigvals,
                      mds_ticket* out);
/* Non-blocking.  *job_status = MDS_PENDING while queued or running, else the
 * terminal status: MDS_OK, MDS_ERR_NONFINITE, MDS_ERR_NUMERICAL, MDS_ERR_HIP
 * or MDS_ERR_CANCELLED.  Returning a terminal status releases the ticket (a
 * later call reports MDS_ERR_INVALID_ARG).  times may be NULL. */
mds_status mds_poll(mds_server_t server, mds_ticket ticket, mds_status* job_status, mds_job_times* times);
/* Like mds_poll, but blocks until the job is terminal. */
mds_status mds_wait(mds_server_t server, mds_ticket ticket, mds_status* job_status, mds_job_times* times);
/* Cancel a job that has not been admitted yet (its status becomes
 * MDS_ERR_CANCELLED); MDS_ERR_STATE once it has started: a running job
 * completes. */
mds_status mds_cancel(mds_server_t server, mds_ticket ticket);
mds_status mds_server_stats(mds_server_t server, mds_server_info* out);
/* Batching of small jobs: when the queue head has n <= small_n_max and
 * k + oversample rounded up to 16 <= 64, and at least one more such job of
 * the same form waits right behind it, the longest run of them (at most
 * max_batch, 1..256) is admitted together and runs as one mds_run_batch
 * launch on one slot (results then agree with mds_run to rounding, not bit
 * for bit); a lone small job runs through the plan path.  small_n_max = 0 turns batching
 * off.  Default: small_n_max = 2048, max_batch = 32. */
mds_status mds_server_set_batching(mds_server_t server, int64_t small_n_max, int32_t max_batch);
/* Pick small_n_max with the autotuner: for n = 128, 256, ... (while the
 * batched kernel supports it), run mds_autotune_batch at the server's
 * max_batch and keep batching a size class while a full batch costs less
 * than a quarter of the plan path's time per instance.  Also leaves the
 * chosen tile shapes in the process-wide table.  Call while the server is
 * idle (it times kernels on the null stream). */
mds_status mds_server_autotune(mds_server_t server, int32_t form, int32_t k, int32_t oversample, int32_t q,
                               int64_t* small_n_max);
/* Cancel queued jobs, wait for admitted ones, free the arena and streams. */
void mds_server_destroy(mds_server_t server);

const char* mds_status_string(mds_status s);
const char* mds_last_error(void);
/* Library version as "major.minor.patch". */
const char* mds_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MDS_H_ */
