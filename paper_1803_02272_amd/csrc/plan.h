// Host-side plan object shared by the C ABI (mds_capi.hip) and the serving
// runtime (mds_server.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/mds.h"
#include "mds_internal.h"

namespace mds {

struct Region {
  size_t off = 0, bytes = 0;
};

}  // namespace mds

struct mds_plan_s {
  int64_t n = 0, n_pad = 0, ldg = 0;
  int k = 0, p = 0, q = 0, l = 0, l_pad = 0;
  uint64_t seed = 0;
  mds_opts opts{};      // options the plan was created with
  int tuned_from_cache = 0;  // splits taken from the MDS_TUNE_CACHE file
  int form = MDS_FORM_FP32;
  int d_dtype = MDS_DTYPE_F32;
  int gk = mds::GK_F32;      // dtype of G and of the range passes
  int ref_gk = mds::GK_F32;  // dtype of the projection pass
  int flags = 0;
  // ref_cfg_alt: the projection's configuration for a D that is not 16-byte
  // aligned (equal to ref_cfg unless ref_cfg streams D through LDS)
  mds::GPassCfg cfg{}, ref_cfg{}, ref_cfg_alt{};
  // refine: BF16/FP8 forms whose first and last range passes run in fp32
  // (three-term split) around the passes over the stored low-precision G
  bool refine = false;
  bool needs_g = false;  // G is stored (BF16/FP8 forms with at least one pass over it)
  mds::GPassCfg fcfg{};  // the fp32 end range passes that are not fused with the write
  bool fused = false;   // bf16 centring write fused with the first range pass (fp32 D)
  mds::GPassCfg wcfg{};  // its configuration (an fp32 split pass when refine, else a bf16 pass)
  int last_xk = -1;      // kind of the operand currently in X (inspection)
  size_t ypart_min = 0;   // lower bound on the split-K partials region (autotuning)
  // workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  mds::Region G, gscale, rowpart, colpart, p4part, r, c, hc, rsum, mean, X, Ypart, Y, Q1, Q, Wpart, W, T, B, V, theta, Tc,
      small, rot, meta, sval, sidx, status;
  size_t total = 0;
  int last_stage = 0;
  // event timing
  bool timing = false;
  std::vector<hipEvent_t> events;  // pool
  std::vector<int> rec_phase;      // phase of recorded pair i (events 2i, 2i+1)

  template <typename T>
  T* at(const mds::Region& reg) const {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + reg.off);
  }
};

namespace mds {

// Record a thread-local error text (mds_last_error) and return s.
mds_status fail(mds_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
mds_status hip_check(hipError_t e, const char* what);
// Enqueue one (partial) run of the plan on stream s; the plan's workspace
// is allocated on first use if none was set.
mds_status run_plan(mds_plan_s* P, const void* D, double* coords, double* eigvals, hipStream_t s, int stop_after,
                    int range_passes);
// Limits of the batched small-instance kernel (l_pad and n).
int batch_max_l();
int64_t batch_max_n();

}  // namespace mds
