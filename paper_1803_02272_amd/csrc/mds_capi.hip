// Host runtime behind the C ABI: plan validation, workspace layout and the
// stream-ordered sequence of kernels that make up one run of
// random-projection classical MDS (see include/mds.h).
//
// Sequence of one run (everything enqueued on the caller's stream):
//   centring stats -> centring write (G in the pass dtype) -> Omega ->
//   (2q+1) x [G-pass -> split-K reduce -> CholeskyQR2] ->
//   projection G-pass -> B = Q^T (G Q) -> eigensolve -> coordinates.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/mds.h"
#include "mds_internal.h"
#include "plan.h"

using namespace mds;

namespace {
thread_local std::string g_last_error;
inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
// bytes per element of G or X of a pass kind (GK_F32S: three bf16 terms of X)
int gk_size(int gk) {
  return gk == GK_F64 ? 8 : (gk == GK_F32 ? 4 : (gk == GK_BF16 ? 2 : (gk_split(gk) ? 6 : 1)));
}
// Element kind of the X operand of a pass with G of kind gk (FP8 G meets bf16 X).
// (the two-term split passes read the first one or two planes of the split layout)
int x_kind(int gk) { return gk == GK_FP8 ? GK_BF16 : ((gk == GK_S2 || gk == GK_S2X) ? GK_F32S : gk); }
bool stores_g(int form) { return form == MDS_FORM_BF16 || form == MDS_FORM_FP8; }
}  // namespace

namespace mds {

mds_status fail(mds_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

}  // namespace mds

namespace {

void add(mds_plan_s* P, Region& reg, size_t bytes) {
  reg.off = P->total;
  reg.bytes = bytes;
  P->total += (size_t)round_up((int64_t)bytes, 256);
}

// Kind of range pass `it` (0-based, of 2q + 1): the BF16/FP8 forms run the
// first and the last from D with G as a two-term bf16 split (about 16
// significant bits) unless MDS_FLAG_LOWP_ALL_RANGE; the sketch of Omega
// splits Omega into two terms as well, the last pass rounds X to bf16 (a
// pass that is both takes the first kind).
int pass_kind(const mds_plan_s* P, int it) {
  if (!P->refine) return P->gk;
  return it == 0 ? GK_S2X : (it == 2 * P->q ? GK_S2 : P->gk);
}

void layout(mds_plan_s* P) {
  const int64_t n = P->n, n_pad = P->n_pad, ldg = P->ldg, lp = P->l_pad;
  const size_t e = (size_t)gk_size(P->gk);
  P->total = 0;
  // G is stored only in the bf16/fp8 forms (their middle range passes stream
  // the 2- or 1-byte G); every other pass recentres D on the fly.
  add(P, P->G, P->needs_g ? (size_t)n_pad * ldg * e : 0);
  const int64_t nsb = n_pad / kF8Block;
  add(P, P->gscale, P->form == MDS_FORM_FP8 ? (size_t)nsb * nsb * 4 : 0);
  const int64_t ncb = (n + kStatsCols - 1) / kStatsCols, nrb = (n + kStatsRows - 1) / kStatsRows;
  add(P, P->rowpart, (size_t)ncb * n * 8);
  add(P, P->colpart, (size_t)nrb * n * 8);
  add(P, P->r, (size_t)n * 8);
  add(P, P->c, (size_t)n * 8);
  add(P, P->rsum, (size_t)n * 8);
  add(P, P->mean, 8);
  add(P, P->p4part, (size_t)stats_parts(n) * 8);
  add(P, P->hc, (size_t)ldg * 4);
  size_t xe = (size_t)(gk_size(x_kind(P->gk)) > gk_size(P->ref_gk) ? gk_size(x_kind(P->gk))
                                                                   : gk_size(P->ref_gk));
  if (P->refine && (size_t)gk_size(GK_S2) > xe) xe = (size_t)gk_size(GK_S2);
  add(P, P->X, (size_t)lp * ldg * xe);
  const size_t acc_main = P->gk == GK_F64 ? 8 : 4, acc_ref = P->ref_gk == GK_F64 ? 8 : 4;
  const size_t yp_main = (size_t)P->cfg.split * lp * ldg * acc_main;
  const int ref_split = P->ref_cfg.split > P->ref_cfg_alt.split ? P->ref_cfg.split : P->ref_cfg_alt.split;
  const size_t yp_ref = (size_t)ref_split * lp * ldg * acc_ref;
  const size_t yp_w = P->fused ? (size_t)P->wcfg.split * lp * ldg * 4 : 0;
  const size_t yp_f = P->refine ? (size_t)P->fcfg.split * lp * ldg * 4 : 0;
  size_t yp = yp_main > yp_ref ? yp_main : yp_ref;
  yp = yp > yp_w ? yp : yp_w;
  yp = yp > yp_f ? yp : yp_f;
  add(P, P->Ypart, yp > P->ypart_min ? yp : P->ypart_min);
  add(P, P->Y, (size_t)lp * ldg * 8);
  add(P, P->Q1, (size_t)lp * ldg * 8);
  add(P, P->Q, (size_t)lp * ldg * 8);
  add(P, P->Wpart, (size_t)gram_chunks(ldg) * lp * lp * 8);
  add(P, P->W, (size_t)lp * lp * 8);
  add(P, P->T, (size_t)lp * lp * 8);
  add(P, P->B, (size_t)lp * lp * 8);
  add(P, P->V, (size_t)lp * lp * 8);
  add(P, P->theta, (size_t)lp * 8);
  add(P, P->Tc, (size_t)lp * P->k * 8);
  // the eigensolve's working copies (l_pad > 128: A and Q) and the blocked factor's blocks
  const size_t small = (size_t)2 * lp * lp * 8;
  add(P, P->small, small > orth_factor_scratch_bytes(lp) ? small : orth_factor_scratch_bytes(lp));
  add(P, P->rot, small_eig_rot_bytes(P->l));
  add(P, P->meta, (size_t)(P->l + 1) * sizeof(int));
  const int64_t nch = coords_anchor_chunks(n);
  add(P, P->sval, (size_t)(nch * P->k + P->k) * 8);
  add(P, P->sidx, (size_t)nch * P->k * 8);
  add(P, P->status, sizeof(DevStatus));
}

// Pass configurations from the plan's options (split-K per pass kind), then
// the workspace layout.
void configure(mds_plan_s* P) {
  const mds_opts& o = P->opts;
  const bool d8 = o.d_dtype == MDS_DTYPE_F64;
  // default split-K of the range passes at mid-size n (fewer than 256 row
  // blocks): about three workgroups per CU.  The pass library's own default
  // aims at eight, which there only adds partials (a bf16 solve at n = 30,000
  // takes 4.35 ms instead of 4.49); with more row blocks (n = 1e5) its larger
  // split is the faster one (at l_pad = 224, three splits against one).
  int64_t range_split = o.gpass_split;
  if (range_split == 0) {
    const GPassCfg c0 = gpass_config(P->gk, P->l_pad, P->n_pad, P->ldg, 0, !stores_g(P->form), false, d8);
    const int64_t rows = P->n_pad / c0.bm;
    if (rows < 256) range_split = (768 + rows - 1) / rows;
  }
  P->cfg = gpass_config(P->gk, P->l_pad, P->n_pad, P->ldg, (int)range_split, !stores_g(P->form), false, d8,
                        P->gk == GK_BF16 || (P->gk == GK_F32S && P->n % 4 == 0));
  const int ps = o.proj_split ? o.proj_split : o.gpass_split;
  const bool psym = (o.flags & MDS_FLAG_FULL_PROJECTION) == 0;
  P->ref_cfg = gpass_config(P->ref_gk, P->l_pad, P->n_pad, P->ldg, ps, true, psym, d8, P->n % 4 == 0);
  P->ref_cfg_alt = gpass_config(P->ref_gk, P->l_pad, P->n_pad, P->ldg, ps, true, psym, d8, false);
  // fp32 end range passes of the bf16/fp8 forms (full passes recentring D)
  P->refine = stores_g(o.form) && (o.flags & MDS_FLAG_LOWP_ALL_RANGE) == 0;
  P->needs_g = stores_g(o.form) && !(P->refine && P->q == 0);
  if (P->refine)
    P->fcfg = gpass_config(GK_S2, P->l_pad, P->n_pad, P->ldg, o.f32_split ? o.f32_split : o.gpass_split, true,
                           false, d8, P->n % 4 == 0);
  // bf16 form on fp32 D: the centring write is fused with the first range
  // pass (an fp32 split pass when refining, else a bf16 pass)
  P->fused = o.form == MDS_FORM_BF16 && !d8 && P->needs_g;
  if (P->fused)
    P->wcfg = gpass_config(P->refine ? GK_S2X : GK_BF16, P->l_pad, P->n_pad, P->ldg,
                           o.write_split ? o.write_split : o.gpass_split, true, false, false, P->n % 4 == 0);
  layout(P);
}

// Bracket a phase with events on the stream when timing is enabled.
struct PhaseTimer {
  mds_plan_s* P;
  hipStream_t s;
  int phase;
  bool on;
  PhaseTimer(mds_plan_s* P_, hipStream_t s_, int ph) : P(P_), s(s_), phase(ph), on(P_->timing) {
    if (!on) return;
    const size_t need = 2 * (P->rec_phase.size() + 1);
    while (P->events.size() < need) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        return;
      }
      P->events.push_back(e);
    }
    (void)hipEventRecord(P->events[2 * P->rec_phase.size()], s);
  }
  ~PhaseTimer() {
    if (!on) return;
    (void)hipEventRecord(P->events[2 * P->rec_phase.size() + 1], s);
    P->rec_phase.push_back(phase);
  }
};

__global__ void k_status_init(DevStatus* st) {
  DevStatus z = {};
  *st = z;
}

}  // namespace

mds_status mds::hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return MDS_OK;
  return fail(MDS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {

#define MDS_TRY(expr, what)                          \
  do {                                               \
    mds_status _s = hip_check((expr), (what));       \
    if (_s != MDS_OK) return _s;                     \
  } while (0)

mds_status device_present() {
  int count = 0;
  const hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) return fail(MDS_ERR_NO_DEVICE, "no HIP device available");
  return MDS_OK;
}

mds_status ensure_workspace(mds_plan_s* P) {
  if (P->ws) return MDS_OK;
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, P->total);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(MDS_ERR_OOM, "hipMalloc(%zu bytes) failed", P->total);
  }
  P->ws = p;
  P->ws_bytes = P->total;
  P->ws_owned = true;
  return MDS_OK;
}

// Orthonormalise the tall matrix Y (fp64, transposed) into Q by CholeskyQR2
// (with the eigen fallback inside orth_factor); also cast Q into the operand
// of the next G-pass with kind xk.
mds_status orthonormalize(mds_plan_s* P, hipStream_t s, int xk) {
  double* Y = P->at<double>(P->Y);
  double* Q1 = P->at<double>(P->Q1);
  double* Q = P->at<double>(P->Q);
  double* W = P->at<double>(P->W);
  double* T = P->at<double>(P->T);
  double* Wp = P->at<double>(P->Wpart);
  double* sm = P->at<double>(P->small);
  DevStatus* st = P->at<DevStatus>(P->status);
  PhaseTimer tm(P, s, MDS_PH_ORTH);
  MDS_TRY(launch_gram(Y, Y, P->l_pad, P->ldg, Wp, W, s), "gram(Y)");
  MDS_TRY(launch_orth_factor(W, P->l, P->l_pad, T, sm, st, 0, s), "orth_factor 1");
  MDS_TRY(launch_apply(Y, P->l, P->ldg, T, P->l_pad, P->l, P->l_pad, Q1, -1, nullptr, s), "apply 1");
  MDS_TRY(launch_gram(Q1, Q1, P->l_pad, P->ldg, Wp, W, s), "gram(Q1)");
  MDS_TRY(launch_orth_factor(W, P->l, P->l_pad, T, sm, st, 1, s), "orth_factor 2");
  MDS_TRY(launch_apply(Q1, P->l, P->ldg, T, P->l_pad, P->l, P->l_pad, Q, xk, P->at<void>(P->X), s), "apply 2");
  return MDS_OK;
}

// One G-pass Y = G X of kind gk with configuration cfg, then its split-K
// reduction.  from_d: the pass recentres D (else it reads the stored G);
// Gw: the fused centring write's target (the bf16 G).
GPassDSrc make_src(mds_plan_s* P, int gk, bool from_d, const void* D);

mds_status gpass(mds_plan_s* P, hipStream_t s, int gk, const GPassCfg& cfg0, bool from_d, const void* D, void* Gw,
                 int phase) {
  const GPassDSrc src = make_src(P, gk, from_d, D);
  // the LDS-ring split kernel needs a 16-byte aligned D: else the same split
  // with the register-prefetch kernel
  const GPassCfg cfg =
      (!src.D || src.vec) ? cfg0 : gpass_config_nodma(cfg0, P->l_pad, P->n_pad, P->d_dtype == MDS_DTYPE_F64);
  {
    PhaseTimer tm(P, s, phase);
    MDS_TRY(launch_gpass(gk, Gw ? Gw : (from_d ? nullptr : P->at<void>(P->G)), P->ldg, P->n_pad,
                         P->at<void>(P->X), P->l_pad, cfg, P->at<void>(P->Ypart), src, s),
            Gw ? "centring write + range pass 1" : "gpass");
  }
  PhaseTimer tm(P, s, MDS_PH_REDUCE);
  MDS_TRY(launch_splitk_reduce(gk, cfg, P->at<void>(P->Ypart), P->ldg, (int64_t)P->l_pad * P->ldg,
                               P->at<double>(P->Y), s),
          "splitk_reduce");
  return MDS_OK;
}

// Range pass `it` of the plan (kind, configuration, source and phase).
mds_status range_pass(mds_plan_s* P, hipStream_t s, int it, bool fused, const void* D) {
  const int gk = pass_kind(P, it);
  if (it == 0 && fused) {
    mds_status e = gpass(P, s, gk, P->wcfg, true, D, P->at<void>(P->G), MDS_PH_WRITE);
    if (e == MDS_OK && P->wcfg.dma)  // the LDS-ring kernel leaves the padding of G to this
      e = hip_check(launch_split_zero_pad(P->at<void>(P->G), P->n, P->n_pad, P->ldg, s), "zero padding of G");
    return e;
  }
  if (gk == GK_S2 || gk == GK_S2X) return gpass(P, s, gk, P->fcfg, true, D, nullptr, MDS_PH_GPASS_F32);
  return gpass(P, s, gk, P->cfg, !stores_g(P->form), D, nullptr, MDS_PH_GPASS);
}

// Source of a G-pass: block scales of a stored fp8 G, or D and the centring
// terms when the pass recentres D.
GPassDSrc make_src(mds_plan_s* P, int gk, bool from_d, const void* D) {
  GPassDSrc src;
  src.n = P->n;
  if (gk == GK_FP8) {
    src.g8_scales = P->at<float>(P->gscale);
    src.g8_nsb = P->n_pad / kF8Block;
  }
  if (from_d) {
    src.D = D;
    src.n = P->n;
    src.r = P->at<double>(P->r);
    src.c = P->at<double>(P->c);
    src.m = P->at<double>(P->mean);
    src.hc = P->at<float>(P->hc);
    src.vec = ((uintptr_t)D % 16) == 0;
    src.d_is_f64 = P->d_dtype == MDS_DTYPE_F64;
  }
  return src;
}

}  // namespace

mds_status mds::run_plan(mds_plan_s* P, const void* D, double* coords, double* eigvals, hipStream_t s,
                         int stop_after, int range_passes) {
  mds_status st0 = device_present();
  if (st0 != MDS_OK) return st0;
  st0 = ensure_workspace(P);
  if (st0 != MDS_OK) return st0;
  DevStatus* st = P->at<DevStatus>(P->status);
  P->last_stage = 0;
  P->last_xk = -1;
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(1), 0, s, st);
  MDS_TRY(hipGetLastError(), "status init");

  if (P->opts.flags & MDS_FLAG_CHECK_INPUT) {
    PhaseTimer tm(P, s, MDS_PH_CHECK);
    MDS_TRY(launch_check_input(D, P->d_dtype == MDS_DTYPE_F64, P->n, st, s), "input check");
  }
  {
  PhaseTimer tm(P, s, MDS_PH_STATS);
  MDS_TRY(launch_center_stats(D, P->d_dtype == MDS_DTYPE_F64, P->n, P->ldg, P->at<double>(P->rowpart),
                              P->at<double>(P->colpart), P->at<double>(P->p4part), P->at<double>(P->r),
                              P->at<double>(P->c), P->at<double>(P->rsum), P->at<float>(P->hc),
                              P->at<double>(P->mean), st, (P->opts.flags & MDS_FLAG_FULL_STATS) == 0 ? 1 : 0, s),
          "centring stats");
  }
  // fused: the bf16 G is written by the first range pass (needs Omega first)
  const bool fused = P->fused && stop_after >= MDS_STAGE_RANGE;
  if (P->form == MDS_FORM_FP8 && P->needs_g) {
    PhaseTimer tm(P, s, MDS_PH_WRITE);
    MDS_TRY(launch_center_write_fp8(D, P->d_dtype == MDS_DTYPE_F64, P->n, P->n_pad, P->ldg, P->at<double>(P->r),
                                    P->at<double>(P->c), P->at<double>(P->mean), P->at<uint8_t>(P->G),
                                    P->at<float>(P->gscale), s),
            "centring write fp8");
  } else if (P->form == MDS_FORM_BF16 && P->needs_g && !fused) {
    PhaseTimer tm(P, s, MDS_PH_WRITE);
    MDS_TRY(launch_center_write(D, P->d_dtype == MDS_DTYPE_F64, P->n, P->n_pad, P->ldg, P->at<double>(P->r),
                                P->at<double>(P->c), P->at<double>(P->mean), P->gk, P->at<void>(P->G), nullptr, s),
            "centring write");
  }
  P->last_stage = MDS_STAGE_CENTER;
  if (stop_after == MDS_STAGE_CENTER) return MDS_OK;

  {
    PhaseTimer tm(P, s, MDS_PH_OMEGA);
    const int xk0 = x_kind(pass_kind(P, 0));
    MDS_TRY(launch_omega(P->seed, P->n, P->l, P->l_pad, P->ldg, xk0, P->at<void>(P->X), s), "omega");
    P->last_xk = xk0;
  }
  P->last_stage = MDS_STAGE_OMEGA;
  if (stop_after == MDS_STAGE_OMEGA) return MDS_OK;

  const int total_range = 2 * P->q + 1;
  const int passes = stop_after == MDS_STAGE_RANGE ? range_passes : total_range;
  for (int it = 0; it < passes; ++it) {
    mds_status e = range_pass(P, s, it, fused, D);
    if (e != MDS_OK) return e;
    const int next_xk = x_kind((it == total_range - 1) ? P->ref_gk : pass_kind(P, it + 1));
    e = orthonormalize(P, s, next_xk);
    if (e != MDS_OK) return e;
    P->last_xk = next_xk;
  }
  P->last_stage = MDS_STAGE_RANGE;
  if (stop_after == MDS_STAGE_RANGE) return MDS_OK;

  // projection: Y = G_ref Q, B = Q^T Y (symmetric mode: Y = 2 (W o G_ref) Q,
  // whose symmetrised B is the same Q^T G_ref Q, see k_gpass)
  mds_status e = gpass(P, s, P->ref_gk, P->ref_cfg, true, D, nullptr, MDS_PH_GPASS_REF);
  if (e != MDS_OK) return e;
  {
    PhaseTimer tm(P, s, MDS_PH_SMALL);
    MDS_TRY(launch_gram(P->at<double>(P->Q), P->at<double>(P->Y), P->l_pad, P->ldg, P->at<double>(P->Wpart),
                        P->at<double>(P->B), s),
            "gram(Q, GQ)");
    MDS_TRY(launch_small_eig(P->at<double>(P->B), P->l, P->l_pad, P->k, P->at<double>(P->theta),
                             P->at<double>(P->V), P->at<double>(P->Tc), eigvals, P->at<double>(P->small),
                             P->at<void>(P->rot), P->at<int>(P->meta), st, s),
            "small_eig");
  }
  PhaseTimer tm(P, s, MDS_PH_COORDS);
  MDS_TRY(launch_coords(P->at<double>(P->Q), P->l, P->n, P->ldg, P->at<double>(P->Tc), P->k,
                        P->at<double>(P->Q1), coords,
                        P->at<double>(P->sval), P->at<int64_t>(P->sidx), s),
          "coords");
  P->last_stage = MDS_STAGE_ALL;
  return MDS_OK;
}

extern "C" {

const char* mds_version(void) { return "0.1.0"; }

const char* mds_last_error(void) { return g_last_error.c_str(); }

const char* mds_status_string(mds_status s) {
  switch (s) {
    case MDS_OK: return "ok";
    case MDS_PENDING: return "pending";
    case MDS_ERR_INVALID_ARG: return "invalid argument";
    case MDS_ERR_NO_DEVICE: return "no device";
    case MDS_ERR_OOM: return "out of device memory";
    case MDS_ERR_BUDGET: return "exceeds memory budget";
    case MDS_ERR_NONFINITE: return "non-finite input";
    case MDS_ERR_NUMERICAL: return "numerical failure";
    case MDS_ERR_HIP: return "HIP error";
    case MDS_ERR_CANCELLED: return "cancelled";
    case MDS_ERR_STATE: return "invalid state";
    case MDS_ERR_NOT_METRIC: return "D is not symmetric with a zero diagonal";
  }
  return "unknown status";
}

mds_status mds_plan_ex(mds_plan_t* out, int64_t n, int32_t k, int32_t oversample, int32_t q, uint64_t seed,
                       const mds_opts* opts) {
  if (!out) return fail(MDS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  mds_opts o = {MDS_FORM_FP32, MDS_DTYPE_F32, 0, 0, 0, 0, 0};
  if (opts) o = *opts;
  if (n < 2) return fail(MDS_ERR_INVALID_ARG, "n = %lld < 2", (long long)n);
  if (n > 1000000) return fail(MDS_ERR_INVALID_ARG, "n = %lld > 1000000", (long long)n);
  if (k < 1) return fail(MDS_ERR_INVALID_ARG, "k = %d < 1", k);
  if (oversample < 0) return fail(MDS_ERR_INVALID_ARG, "oversample = %d < 0", oversample);
  if (q < 0) return fail(MDS_ERR_INVALID_ARG, "q = %d < 0", q);
  const int64_t l = (int64_t)k + oversample;
  if (l > n) return fail(MDS_ERR_INVALID_ARG, "k + oversample = %lld > n = %lld", (long long)l, (long long)n);
  if (l > MDS_MAX_L) return fail(MDS_ERR_INVALID_ARG, "k + oversample = %lld > %d", (long long)l, MDS_MAX_L);
  if (o.form < MDS_FORM_FP64 || o.form > MDS_FORM_FP8)
    return fail(MDS_ERR_INVALID_ARG, "unknown form %d", o.form);
  if (o.d_dtype != MDS_DTYPE_F32 && o.d_dtype != MDS_DTYPE_F64)
    return fail(MDS_ERR_INVALID_ARG, "unknown D dtype %d", o.d_dtype);
  if (o.gpass_split < 0 || o.proj_split < 0 || o.write_split < 0 || o.f32_split < 0)
    return fail(MDS_ERR_INVALID_ARG, "negative split (%d, %d, %d, %d)", o.gpass_split, o.proj_split, o.write_split,
                o.f32_split);
  if (o.flags & ~(MDS_FLAG_FULL_PROJECTION | MDS_FLAG_FP32_MFMA_PROJECTION | MDS_FLAG_SPLIT_FP32 |
                  MDS_FLAG_FULL_STATS | MDS_FLAG_CHECK_INPUT | MDS_FLAG_LOWP_ALL_RANGE | MDS_FLAG_FP32_PROJECTION))
    return fail(MDS_ERR_INVALID_ARG, "unknown flags 0x%x", o.flags);
  if ((o.flags & MDS_FLAG_CHECK_INPUT) && (n + 63) / 64 > 65535)
    return fail(MDS_ERR_INVALID_ARG, "MDS_FLAG_CHECK_INPUT supports n <= %d", 65535 * 64);
  mds_plan_s* P = new (std::nothrow) mds_plan_s();
  if (!P) return fail(MDS_ERR_OOM, "host allocation failed");
  P->opts = o;
  P->n = n;
  P->n_pad = round_up(n, kPadN);
  P->ldg = P->n_pad;
  P->k = k;
  P->p = oversample;
  P->q = q;
  P->l = (int)l;
  P->l_pad = (int)round_up(l, 16);
  P->seed = seed;
  P->form = o.form;
  P->d_dtype = o.d_dtype;
  P->gk = o.form == MDS_FORM_FP64 ? GK_F64
          : (o.form == MDS_FORM_FP32 ? GK_F32 : (o.form == MDS_FORM_BF16 ? GK_BF16 : GK_FP8));
  // projection ("refinement") of the stored-G forms: a 16-bit pass (two-term
  // bf16 splits of G and X) by default, else fp32 as the three-term split or
  // on fp32 MFMA
  P->ref_gk = !stores_g(o.form)                             ? P->gk
              : (o.flags & MDS_FLAG_FP32_MFMA_PROJECTION) ? GK_F32
              : (o.flags & MDS_FLAG_FP32_PROJECTION)      ? GK_F32S
                                                          : GK_S2X;
  // FP32 form with every pass as the three-term bf16 split
  if (o.form == MDS_FORM_FP32 && (o.flags & MDS_FLAG_SPLIT_FP32)) P->gk = P->ref_gk = GK_F32S;
  P->flags = o.flags;
  // splits all automatic: a recorded autotune choice for this key, if any
  if (!P->opts.gpass_split && !P->opts.proj_split && !P->opts.write_split && !P->opts.f32_split) {
    int s[4];
    if (tune_cache_lookup(TuneKey{o.form, o.flags, o.d_dtype, P->l_pad, P->q, P->n}, s)) {
      P->opts.gpass_split = s[0];
      P->opts.proj_split = s[1];
      P->opts.write_split = s[2];
      P->opts.f32_split = s[3];
      P->tuned_from_cache = 1;
    }
  }
  configure(P);
  *out = P;
  return MDS_OK;
}

mds_status mds_plan(mds_plan_t* out, int64_t n, int32_t k, int32_t oversample, int32_t q, uint64_t seed) {
  return mds_plan_ex(out, n, k, oversample, q, seed, nullptr);
}

mds_status mds_workspace_size(mds_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  *bytes = plan->total;
  return MDS_OK;
}

mds_status mds_set_workspace(mds_plan_t plan, void* dev_ptr, size_t bytes) {
  if (!plan || !dev_ptr) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  if (bytes < plan->total)
    return fail(MDS_ERR_INVALID_ARG, "workspace of %zu bytes < required %zu", bytes, plan->total);
  if (((uintptr_t)dev_ptr) % 256 != 0) return fail(MDS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (plan->ws_owned) {
    (void)hipFree(plan->ws);
    plan->ws_owned = false;
  }
  plan->ws = dev_ptr;
  plan->ws_bytes = bytes;
  return MDS_OK;
}

mds_status mds_run_stages(mds_plan_t plan, const void* D, double* coords, double* eigvals, void* stream,
                          int32_t stop_after, int32_t range_passes) {
  if (!plan || !D) return fail(MDS_ERR_INVALID_ARG, "NULL plan or D");
  if (stop_after != MDS_STAGE_CENTER && stop_after != MDS_STAGE_OMEGA && stop_after != MDS_STAGE_RANGE &&
      stop_after != MDS_STAGE_ALL)
    return fail(MDS_ERR_INVALID_ARG, "unknown stage %d", stop_after);
  if (stop_after == MDS_STAGE_RANGE && (range_passes < 1 || range_passes > 2 * plan->q + 1))
    return fail(MDS_ERR_INVALID_ARG, "range_passes %d outside [1, %d]", range_passes, 2 * plan->q + 1);
  if (stop_after == MDS_STAGE_ALL && (!coords || !eigvals))
    return fail(MDS_ERR_INVALID_ARG, "NULL coords or eigvals");
  return run_plan(plan, D, coords, eigvals, (hipStream_t)stream, stop_after, range_passes);
}

mds_status mds_run(mds_plan_t plan, const void* D, double* coords, double* eigvals, void* stream) {
  return mds_run_stages(plan, D, coords, eigvals, stream, MDS_STAGE_ALL, 0);
}

mds_status mds_get_buffer(mds_plan_t plan, int32_t which, mds_buffer* out) {
  if (!plan || !out) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  if (!plan->ws) return fail(MDS_ERR_STATE, "plan has no workspace yet");
  mds_buffer b = {};
  const int64_t lp = plan->l_pad;
  // X dtype (FP8: bf16; split passes: bf16 planes)
  const int xdt = plan->gk == GK_F64 ? 0 : (plan->gk == GK_F32 ? 1 : 2);
  switch (which) {
    case MDS_BUF_G:
      if (!plan->needs_g) return fail(MDS_ERR_STATE, "G is not stored in this form");
      b = {plan->at<void>(plan->G), plan->form == MDS_FORM_FP8 ? 3 : xdt, 0, plan->n_pad, plan->ldg, plan->ldg};
      break;
    case MDS_BUF_GSCALE:
      if (plan->form != MDS_FORM_FP8) return fail(MDS_ERR_STATE, "no block scales in this form");
      b = {plan->at<void>(plan->gscale), 1, 0, plan->n_pad / kF8Block, plan->n_pad / kF8Block,
           plan->n_pad / kF8Block};
      break;
    case MDS_BUF_GREF: return fail(MDS_ERR_STATE, "no fp32 copy of G is stored");
    case MDS_BUF_ROWMEAN: b = {plan->at<void>(plan->r), 0, 0, plan->n, 1, 1}; break;
    case MDS_BUF_COLMEAN: b = {plan->at<void>(plan->c), 0, 0, plan->n, 1, 1}; break;
    case MDS_BUF_MEAN: b = {plan->at<void>(plan->mean), 0, 0, 1, 1, 1}; break;
    case MDS_BUF_X: {
      // dtype of the operand that the last pass or cast wrote
      const int xk = plan->last_xk >= 0 ? plan->last_xk : x_kind(plan->gk);
      const int dt = xk == GK_F64 ? 0 : (xk == GK_F32 ? 1 : 2);
      const int64_t cols = xk == GK_F32S ? 3 * plan->ldg : plan->ldg;
      b = {plan->at<void>(plan->X), dt, 0, lp, cols, cols};
      break;
    }
    case MDS_BUF_Q: b = {plan->at<void>(plan->Q), 0, 0, lp, plan->ldg, plan->ldg}; break;
    case MDS_BUF_Y: b = {plan->at<void>(plan->Y), 0, 0, lp, plan->ldg, plan->ldg}; break;  // see mds.h
    case MDS_BUF_B: b = {plan->at<void>(plan->B), 0, 0, lp, lp, lp}; break;
    case MDS_BUF_THETA: b = {plan->at<void>(plan->theta), 0, 0, plan->l, 1, 1}; break;
    case MDS_BUF_V: b = {plan->at<void>(plan->V), 0, 0, plan->l, plan->l, lp}; break;
    case MDS_BUF_W: b = {plan->at<void>(plan->W), 0, 0, lp, lp, lp}; break;
    case MDS_BUF_T: b = {plan->at<void>(plan->T), 0, 0, lp, lp, lp}; break;
    case MDS_BUF_Q1: b = {plan->at<void>(plan->Q1), 0, 0, lp, plan->ldg, plan->ldg}; break;
    default: return fail(MDS_ERR_INVALID_ARG, "unknown buffer %d", which);
  }
  *out = b;
  return MDS_OK;
}

mds_status mds_get_info(mds_plan_t plan, mds_info* out, void* stream) {
  if (!plan || !out) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  mds_info info = {};
  info.k = plan->k;
  info.l = plan->l;
  info.l_pad = plan->l_pad;
  info.q = plan->q;
  info.form = plan->form;
  info.gpass_split = plan->cfg.split;
  info.tuned_from_cache = plan->tuned_from_cache;
  info.n = plan->n;
  info.ldg = plan->ldg;
  info.status = MDS_OK;
  if (plan->ws && plan->last_stage > 0) {
    MDS_TRY(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
    DevStatus d = {};
    MDS_TRY(hipMemcpy(&d, plan->at<void>(plan->status), sizeof(d), hipMemcpyDeviceToHost), "hipMemcpy status");
    info.nonfinite = d.nonfinite;
    info.orth_fallbacks = d.orth_fallbacks;
    info.jacobi_sweeps = d.jacobi_sweeps;
    info.jacobi_unconverged = d.jacobi_unconv;
    info.rank_deficient = d.rank_deficient;
    info.sum_sq = d.sum_sq;
    info.frob2 = d.frob2;
    info.trace = d.trace;
    info.asym_pairs = (int64_t)d.asym_pairs;
    info.diag_nonzero = (int64_t)d.diag_nonzero;
    if (d.nonfinite)
      info.status = MDS_ERR_NONFINITE;
    else if ((plan->opts.flags & MDS_FLAG_CHECK_INPUT) && (d.asym_pairs || d.diag_nonzero))
      info.status = MDS_ERR_NOT_METRIC;
    else if (d.jacobi_unconv)
      info.status = MDS_ERR_NUMERICAL;
  }
  *out = info;
  return MDS_OK;
}

mds_status mds_set_timing(mds_plan_t plan, int32_t enable) {
  if (!plan) return fail(MDS_ERR_INVALID_ARG, "NULL plan");
  plan->timing = enable != 0;
  return MDS_OK;
}

mds_status mds_get_timings(mds_plan_t plan, mds_phase_time* out, void* stream) {
  if (!plan || !out) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  for (int i = 0; i < MDS_NUM_PHASES; ++i) out[i] = mds_phase_time{0, 0.f, 0.f, 0.f};
  if (plan->rec_phase.empty()) return MDS_OK;
  MDS_TRY(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
  for (size_t i = 0; i < plan->rec_phase.size(); ++i) {
    float ms = 0.f;
    MDS_TRY(hipEventElapsedTime(&ms, plan->events[2 * i], plan->events[2 * i + 1]), "hipEventElapsedTime");
    mds_phase_time& t = out[plan->rec_phase[i]];
    t.min_ms = t.count ? (ms < t.min_ms ? ms : t.min_ms) : ms;
    t.max_ms = t.count ? (ms > t.max_ms ? ms : t.max_ms) : ms;
    t.total_ms += ms;
    t.count += 1;
  }
  plan->rec_phase.clear();
  return MDS_OK;
}

mds_status mds_autotune(mds_plan_t P, const void* D, void* stream, mds_tune_result* out) {
  if (!P || !D || !out) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  if (P->ws) return fail(MDS_ERR_STATE, "autotune before a workspace is attached or allocated");
  mds_status st = device_present();
  if (st != MDS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  static const int kCands[] = {0, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48};
  const bool d8 = P->d_dtype == MDS_DTYPE_F64;
  const bool sym = (P->opts.flags & MDS_FLAG_FULL_PROJECTION) == 0;
  // pass kinds: 0 range passes over the form's G, 1 projection, 2 fused
  // centring write + first range pass, 3 fp32 end range passes (refine)
  enum { kRange = 0, kProj = 1, kWrite = 2, kF32 = 3, kKinds = 4 };
  const bool has_kind[kKinds] = {!P->refine || P->q >= 1, true, P->fused, P->refine};
  auto gk_of = [&](int kind) {
    if (kind == kRange) return P->gk;
    if (kind == kProj) return P->ref_gk;
    if (kind == kWrite) return P->refine ? (int)GK_S2X : (int)GK_BF16;
    return (int)GK_S2;
  };
  auto cfg_of = [&](int kind, int split) {
    if (kind == kRange)
      return gpass_config(P->gk, P->l_pad, P->n_pad, P->ldg, split, !stores_g(P->form), false, d8,
                          P->gk == GK_BF16 || (P->gk == GK_F32S && P->n % 4 == 0 && (uintptr_t)D % 16 == 0));
    if (kind == kProj)
      return gpass_config(P->ref_gk, P->l_pad, P->n_pad, P->ldg, split, true, sym, d8,
                          P->n % 4 == 0 && (uintptr_t)D % 16 == 0);
    const bool dma_ok = P->n % 4 == 0 && (uintptr_t)D % 16 == 0;
    if (kind == kWrite)
      return gpass_config(gk_of(kWrite), P->l_pad, P->n_pad, P->ldg, split, true, false, false, dma_ok);
    return gpass_config(GK_S2, P->l_pad, P->n_pad, P->ldg, split, true, false, d8, dma_ok);
  };
  // workspace sized for the largest candidate's partials
  size_t ymax = 0;
  for (int kind = 0; kind < kKinds; ++kind) {
    if (!has_kind[kind]) continue;
    for (int c : kCands) {
      const GPassCfg g = cfg_of(kind, c);
      const size_t b = (size_t)g.split * P->l_pad * P->ldg * (gk_of(kind) == GK_F64 ? 8 : 4);
      ymax = b > ymax ? b : ymax;
    }
  }
  P->ypart_min = ymax;
  layout(P);
  st = ensure_workspace(P);
  if (st != MDS_OK) {
    P->ypart_min = 0;
    layout(P);
    return st;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto finish = [&](mds_status r) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(P->ws);
    P->ws = nullptr;
    P->ws_owned = false;
    P->ws_bytes = 0;
    P->ypart_min = 0;
    configure(P);
    return r;
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return finish(fail(MDS_ERR_HIP, "event creation failed"));
  // centring, stored G and Omega in the workspace
  st = run_plan(P, D, nullptr, nullptr, s, MDS_STAGE_OMEGA, 0);
  if (st != MDS_OK) return finish(st);
  int best[kKinds] = {0, 0, 0, 0};
  float best_ms[kKinds] = {0.f, 0.f, 0.f, 0.f};
  int timed = 0;
  for (int kind = 0; kind < kKinds; ++kind) {
    if (!has_kind[kind]) continue;
    const int gk = gk_of(kind);
    const bool from_d = kind != kRange || !stores_g(P->form);
    const GPassDSrc src = make_src(P, gk, from_d, D);
    void* G = (kind == kWrite || !from_d) ? P->at<void>(P->G) : nullptr;
    // the pass operand X holds the split-K test data of any kind: Omega in
    // the dtype of the first pass (its contents do not change the timing of
    // the other kinds, which read the same number of bytes from it)
    float kbest = 1e30f;
    int last_split = -1;
    for (int c : kCands) {
      const GPassCfg g = cfg_of(kind, c);
      if (g.split == last_split && c != 0) continue;  // same configuration as a candidate already timed
      last_split = g.split;
      float ms_best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {  // first launch warms up
        float ms = 0.f;
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess)
          e = launch_gpass(gk, G, P->ldg, P->n_pad, P->at<void>(P->X), P->l_pad, g, P->at<void>(P->Ypart), src, s);
        // the split-K reduction grows with the split: it is part of the cost
        if (e == hipSuccess)
          e = launch_splitk_reduce(gk == GK_F64 ? GK_F64 : GK_F32, g, P->at<void>(P->Ypart), P->ldg,
                                   (int64_t)P->l_pad * P->ldg, P->at<double>(P->Y), s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) return finish(hip_check(e, "autotune gpass"));
        if (rep > 0 && ms < ms_best) ms_best = ms;
      }
      ++timed;
      if (ms_best < kbest) {
        kbest = ms_best;
        best[kind] = g.split;
      }
    }
    best_ms[kind] = kbest;
  }
  P->opts.gpass_split = best[kRange];
  P->opts.proj_split = best[kProj];
  P->opts.write_split = P->fused ? best[kWrite] : 0;
  P->opts.f32_split = P->refine ? best[kF32] : 0;
  out->range_split = best[kRange];
  out->proj_split = best[kProj];
  out->write_split = P->opts.write_split;
  out->f32_split = P->opts.f32_split;
  out->range_ms = best_ms[kRange];
  out->proj_ms = best_ms[kProj];
  out->write_ms = P->fused ? best_ms[kWrite] : 0.f;
  out->f32_ms = P->refine ? best_ms[kF32] : 0.f;
  out->candidates = timed;
  const int rec[4] = {P->opts.gpass_split, P->opts.proj_split, P->opts.write_split, P->opts.f32_split};
  tune_cache_store(TuneKey{P->opts.form, P->opts.flags, P->opts.d_dtype, P->l_pad, P->q, P->n}, rec);
  return finish(MDS_OK);
}

mds_status mds_philox4x64_10(const uint64_t* in, uint64_t* out, int64_t count, void* stream) {
  if (count < 0 || (count > 0 && (!in || !out))) return fail(MDS_ERR_INVALID_ARG, "NULL pointer or count < 0");
  if (count == 0) return MDS_OK;
  if (count > ((int64_t)1 << 36)) return fail(MDS_ERR_INVALID_ARG, "count = %lld too large", (long long)count);
  const mds_status st = device_present();
  if (st != MDS_OK) return st;
  return hip_check(launch_philox(in, out, count, (hipStream_t)stream), "philox");
}

mds_status mds_hamming_distances(const uint8_t* codes, int64_t n, int32_t length, int32_t d_dtype, void* D,
                                 void* stream) {
  if (!codes || !D) return fail(MDS_ERR_INVALID_ARG, "NULL codes or D");
  if (n < 1 || n > kMaxDistanceN) return fail(MDS_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (length < 1 || length > kMaxHammingLength)
    return fail(MDS_ERR_INVALID_ARG, "length = %d out of range 1..%d", length, kMaxHammingLength);
  if (d_dtype != MDS_DTYPE_F32 && d_dtype != MDS_DTYPE_F64) return fail(MDS_ERR_INVALID_ARG, "bad d_dtype");
  const mds_status st = device_present();
  if (st != MDS_OK) return st;
  return hip_check(launch_hamming(codes, n, length, d_dtype == MDS_DTYPE_F64, D, (hipStream_t)stream),
                   "hamming distances");
}

mds_status mds_euclidean_distances(const double* X, int64_t n, int32_t dim, int32_t d_dtype, void* D, void* stream) {
  if (!X || !D) return fail(MDS_ERR_INVALID_ARG, "NULL X or D");
  if (n < 1 || n > kMaxDistanceN) return fail(MDS_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (dim < 1 || dim > (1 << 20)) return fail(MDS_ERR_INVALID_ARG, "dim = %d out of range", dim);
  if (d_dtype != MDS_DTYPE_F32 && d_dtype != MDS_DTYPE_F64) return fail(MDS_ERR_INVALID_ARG, "bad d_dtype");
  const mds_status st = device_present();
  if (st != MDS_OK) return st;
  return hip_check(launch_euclid(X, n, dim, d_dtype == MDS_DTYPE_F64, D, (hipStream_t)stream), "euclidean distances");
}

mds_status mds_threshold_components(const void* D, int32_t d_dtype, int64_t n, double threshold, int32_t flags,
                                    int32_t* labels, int64_t* n_components, void* stream) {
  if (!D || !labels) return fail(MDS_ERR_INVALID_ARG, "NULL D or labels");
  if (n < 1 || n > kMaxDistanceN) return fail(MDS_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (d_dtype != MDS_DTYPE_F32 && d_dtype != MDS_DTYPE_F64) return fail(MDS_ERR_INVALID_ARG, "bad d_dtype");
  if (flags & ~MDS_CC_FULL_MATRIX) return fail(MDS_ERR_INVALID_ARG, "unknown flags 0x%x", (unsigned)flags);
  if (threshold != threshold) return fail(MDS_ERR_INVALID_ARG, "NaN threshold");
  const mds_status st = device_present();
  if (st != MDS_OK) return st;
  return hip_check(launch_components(D, d_dtype == MDS_DTYPE_F64, n, threshold, (flags & MDS_CC_FULL_MATRIX) != 0,
                                     labels, n_components, (hipStream_t)stream),
                   "threshold components");
}

void mds_destroy(mds_plan_t plan) {
  if (!plan) return;
  for (hipEvent_t e : plan->events) (void)hipEventDestroy(e);
  if (plan->ws_owned && plan->ws) (void)hipFree(plan->ws);
  delete plan;
}

}  // extern "C"
