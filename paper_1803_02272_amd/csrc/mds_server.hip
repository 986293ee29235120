// Serving runtime: continuous batching of MDS jobs on one GPU.
//
// A server owns one device arena of `hbm_budget_bytes` (allocated once, at
// creation: nothing is allocated on the device while serving) and
// `max_slots` HIP streams at the default priority.  Submitted jobs wait in a
// FIFO queue; a worker thread admits the queue head as soon as a slot is free
// and the arena has room for the job's workspace (first fit), enqueues the
// whole run on the slot's stream, and retires jobs whose completion event has
// fired, releasing their slot and memory for the next admissions.  Admitted
// jobs therefore overlap on the device: a small job runs beside a large one
// instead of behind it.  Each job runs on its own copy of the caller's plan,
// so its result is bit-identical to mds_run of the same plan alone.
//
// Small jobs are batched: when the queue head is small (n <= small_n_max and
// l_pad <= 64) and at least one more small job of the same form waits right
// behind it, the longest such run (up to max_batch) is admitted together and
// runs as one persistent launch of the batched kernel (mds_run_batch), one
// workgroup per job.  A lone small job takes the plan path, whose latency is
// lower.  Batched results agree with mds_run to rounding, not bit for bit.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mds.h"
#include "mds_internal.h"
#include "plan.h"

using namespace mds;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
 public:
  explicit Arena(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += bytes;
      if (used_ > peak_) peak_ = used_;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  static constexpr size_t kAlign = 256;
  size_t used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

enum JobState { kQueued, kRunning, kDone };

struct Job {
  mds_ticket id = 0;
  mds_plan_s* plan = nullptr;
  const void* D = nullptr;
  double* coords = nullptr;
  double* eigvals = nullptr;
  JobState state = kQueued;
  mds_status result = MDS_PENDING;
  size_t ws_off = 0, ws_bytes = 0;
  int slot = -1;
  Clock::time_point t_submit, t_start, t_done;
};

constexpr int kMaxGroup = 256;  // largest batch of small jobs

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  DevStatus* host_status = nullptr;  // pinned, kMaxGroup entries
  std::vector<Job*> group;           // jobs running on this slot (empty: free)
  bool batched = false;
  size_t ws_off = 0, ws_bytes = 0;
};

// The batched kernel runs the default schedule of each form (fp32 end passes
// in bf16, full-matrix centring and projection), so plans with option flags
// always take the plan path.
bool batchable(const Job* j, int64_t small_n_max) {
  const mds_plan_s* P = j->plan;
  return P->form <= MDS_FORM_BF16 && P->opts.flags == 0 && P->n <= small_n_max && P->l_pad <= batch_max_l() &&
         P->n <= batch_max_n();
}

mds_batch_job batch_entry(const Job* j) {
  mds_batch_job b{};
  b.D = j->D;
  b.coords = j->coords;
  b.eigvals = j->eigvals;
  b.n = j->plan->n;
  b.k = j->plan->k;
  b.oversample = j->plan->p;
  b.q = j->plan->q;
  b.d_dtype = j->plan->d_dtype;
  b.seed = j->plan->seed;
  return b;
}

}  // namespace

struct mds_server_s {
  int device = 0;
  size_t budget = 0;
  void* arena_ptr = nullptr;
  Arena* arena = nullptr;
  std::vector<Slot> slots;
  int64_t small_n_max = 2048;  // batching threshold (0: never batch)
  int max_batch = 32;
  uint64_t batches = 0;        // batched launches so far
  std::deque<Job*> queue;
  std::vector<Job*> running;
  std::unordered_map<mds_ticket, Job*> jobs;
  mds_ticket next_ticket = 1;
  uint64_t completed = 0;
  std::mutex mu;
  std::condition_variable work_cv;  // wakes the worker
  std::condition_variable done_cv;  // wakes mds_wait
  std::thread worker;
  bool stop = false;
};

namespace {

void free_job(Job* j) {
  if (j->plan) mds_destroy(j->plan);
  delete j;
}

// Enqueue the slot's group (one job through the plan path, or a batch of
// small jobs through the batched kernel); called by the worker without the lock.
mds_status launch(mds_server_s* S, Slot& sl) {
  char* ws = static_cast<char*>(S->arena_ptr) + sl.ws_off;
  mds_status st = MDS_OK;
  if (sl.batched) {
    std::vector<mds_batch_job> bj;
    for (Job* j : sl.group) bj.push_back(batch_entry(j));
    st = mds_run_batch(bj.data(), (int32_t)bj.size(), sl.group[0]->plan->form, ws, sl.ws_bytes, 0, sl.stream);
    if (st == MDS_OK)
      st = hip_check(hipMemcpyAsync(sl.host_status, ws, bj.size() * sizeof(DevStatus), hipMemcpyDeviceToHost,
                                    sl.stream),
                     "status copy");
  } else {
    Job* j = sl.group[0];
    st = mds_set_workspace(j->plan, ws, sl.ws_bytes);
    if (st == MDS_OK) st = run_plan(j->plan, j->D, j->coords, j->eigvals, sl.stream, MDS_STAGE_ALL, 0);
    if (st == MDS_OK)
      st = hip_check(hipMemcpyAsync(sl.host_status, j->plan->at<void>(j->plan->status), sizeof(DevStatus),
                                    hipMemcpyDeviceToHost, sl.stream),
                     "status copy");
  }
  // the event is recorded whatever happened so that retirement waits for
  // every kernel this group managed to enqueue
  const mds_status ev = hip_check(hipEventRecord(sl.done, sl.stream), "hipEventRecord");
  return st != MDS_OK ? st : ev;
}

// Workspace bytes of the first `count` jobs of grp as one batch.
size_t batch_bytes(const std::vector<Job*>& grp, size_t count) {
  std::vector<mds_batch_job> bj;
  for (size_t i = 0; i < count; ++i) bj.push_back(batch_entry(grp[i]));
  size_t bytes = 0;
  if (mds_batch_workspace_size(bj.data(), (int32_t)count, grp[0]->plan->form, &bytes) != MDS_OK) return 0;
  return bytes;
}

void worker_main(mds_server_s* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progressed = false;
    // retire finished jobs
    for (size_t si = 0; si < S->slots.size(); ++si) {
      Slot& sl = S->slots[si];
      if (sl.group.empty()) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      const Clock::time_point now = Clock::now();
      for (size_t g = 0; g < sl.group.size(); ++g) {
        Job* j = sl.group[g];
        if (j->result == MDS_PENDING) {
          if (q != hipSuccess) {
            j->result = fail(MDS_ERR_HIP, "job %llu: %s", (unsigned long long)j->id, hipGetErrorString(q));
          } else {
            const DevStatus& d = sl.host_status[sl.batched ? g : 0];
            j->result = d.nonfinite ? MDS_ERR_NONFINITE : (d.jacobi_unconv ? MDS_ERR_NUMERICAL : MDS_OK);
          }
        }
        j->t_done = now;
        j->state = kDone;
        ++S->completed;
        for (size_t r = 0; r < S->running.size(); ++r)
          if (S->running[r] == j) {
            S->running[r] = S->running.back();
            S->running.pop_back();
            break;
          }
      }
      S->arena->release(sl.ws_off, sl.ws_bytes);
      sl.group.clear();
      progressed = true;
    }
    if (progressed) S->done_cv.notify_all();
    if (S->stop && S->queue.empty() && S->running.empty()) break;
    // admit from the queue head while a slot and arena room are free
    while (!S->queue.empty() && !S->stop) {
      int slot = -1;
      for (size_t si = 0; si < S->slots.size(); ++si)
        if (S->slots[si].group.empty()) {
          slot = (int)si;
          break;
        }
      if (slot < 0) break;
      Job* head = S->queue.front();
      std::vector<Job*> grp;
      size_t bytes = 0, off = 0;
      bool batched = false;
      if (S->small_n_max > 0 && batchable(head, S->small_n_max)) {
        for (Job* j : S->queue) {
          if ((int)grp.size() >= S->max_batch || !batchable(j, S->small_n_max) || j->plan->form != head->plan->form)
            break;
          grp.push_back(j);
        }
        // shrink the batch until it fits the free arena
        size_t count = grp.size();
        for (; count > 0; --count) {
          bytes = batch_bytes(grp, count);
          if (bytes && S->arena->alloc(bytes, &off)) break;
        }
        if (count > 1) {
          grp.resize(count);
          batched = true;
        } else {
          // a lone small job, or no batch that fits: the plan path (lower
          // latency; its workspace fits the budget, checked at submit)
          if (count == 1) S->arena->release(off, bytes);
          grp.assign(1, head);
          bytes = head->ws_bytes;
          if (!S->arena->alloc(bytes, &off)) break;
        }
      } else {
        bytes = head->ws_bytes;
        if (!S->arena->alloc(bytes, &off)) break;
        grp.push_back(head);
      }
      for (size_t g = 0; g < grp.size(); ++g) S->queue.pop_front();
      Slot& sl = S->slots[slot];
      sl.group = grp;
      sl.batched = batched;
      sl.ws_off = off;
      sl.ws_bytes = bytes;
      const Clock::time_point now = Clock::now();
      for (Job* j : grp) {
        j->slot = slot;
        j->state = kRunning;
        j->t_start = now;
        S->running.push_back(j);
      }
      if (batched) ++S->batches;
      lk.unlock();
      const mds_status st = launch(S, sl);
      lk.lock();
      if (st != MDS_OK)
        for (Job* j : grp) j->result = st;
      progressed = true;
    }
    if (!progressed) {
      if (S->running.empty())
        S->work_cv.wait_for(lk, std::chrono::milliseconds(20));
      else
        S->work_cv.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

mds_status take_result(mds_server_s* S, std::unordered_map<mds_ticket, Job*>::iterator it, mds_status* job_status,
                       mds_job_times* times) {
  Job* j = it->second;
  if (job_status) *job_status = j->result;
  if (times) {
    const bool ran = j->slot >= 0;
    times->queue_ms = ran ? ms_between(j->t_submit, j->t_start) : ms_between(j->t_submit, j->t_done);
    times->run_ms = ran ? ms_between(j->t_start, j->t_done) : 0.0;
    times->latency_ms = ms_between(j->t_submit, j->t_done);
  }
  S->jobs.erase(it);
  free_job(j);
  return MDS_OK;
}

}  // namespace

extern "C" {

mds_status mds_server_create(mds_server_t* out, size_t hbm_budget_bytes, int32_t max_slots) {
  if (!out) return fail(MDS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes < 256) return fail(MDS_ERR_INVALID_ARG, "budget of %zu bytes", hbm_budget_bytes);
  if (max_slots < 1 || max_slots > 256) return fail(MDS_ERR_INVALID_ARG, "max_slots = %d outside [1, 256]", max_slots);
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(MDS_ERR_NO_DEVICE, "no HIP device available");
  }
  mds_server_s* S = new (std::nothrow) mds_server_s();
  if (!S) return fail(MDS_ERR_OOM, "host allocation failed");
  auto cleanup = [&](mds_status st) {
    for (Slot& sl : S->slots) {
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.host_status) (void)hipHostFree(sl.host_status);
    }
    if (S->arena_ptr) (void)hipFree(S->arena_ptr);
    delete S;
    return st;
  };
  if (hipGetDevice(&S->device) != hipSuccess) return cleanup(fail(MDS_ERR_HIP, "hipGetDevice failed"));
  S->budget = hbm_budget_bytes;
  if (hipMalloc(&S->arena_ptr, hbm_budget_bytes) != hipSuccess || !S->arena_ptr) {
    (void)hipGetLastError();
    S->arena_ptr = nullptr;
    return cleanup(fail(MDS_ERR_OOM, "hipMalloc of the %zu-byte arena failed", hbm_budget_bytes));
  }
  S->slots.resize((size_t)max_slots);
  for (Slot& sl : S->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&sl.host_status, kMaxGroup * sizeof(DevStatus), hipHostMallocDefault) != hipSuccess)
      return cleanup(fail(MDS_ERR_HIP, "stream/event/pinned-buffer creation failed"));
  }
  S->arena = new Arena(hbm_budget_bytes);
  S->worker = std::thread(worker_main, S);
  *out = S;
  return MDS_OK;
}

mds_status mds_submit(mds_server_t S, mds_plan_t plan, const void* D, double* coords, double* eigvals,
                      mds_ticket* out) {
  if (!S || !plan || !D || !coords || !eigvals || !out) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  *out = 0;
  if (plan->total > S->budget)
    return fail(MDS_ERR_BUDGET, "job needs %zu bytes of workspace, the budget is %zu", plan->total, S->budget);
  mds_plan_t copy = nullptr;
  mds_status st = mds_plan_ex(&copy, plan->n, plan->k, plan->p, plan->q, plan->seed, &plan->opts);
  if (st != MDS_OK) return st;
  Job* j = new (std::nothrow) Job();
  if (!j) {
    mds_destroy(copy);
    return fail(MDS_ERR_OOM, "host allocation failed");
  }
  j->plan = copy;
  j->D = D;
  j->coords = coords;
  j->eigvals = eigvals;
  j->ws_bytes = copy->total;
  j->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(S->mu);
    j->id = S->next_ticket++;
    S->jobs[j->id] = j;
    S->queue.push_back(j);
  }
  S->work_cv.notify_one();
  *out = j->id;
  return MDS_OK;
}

mds_status mds_poll(mds_server_t S, mds_ticket ticket, mds_status* job_status, mds_job_times* times) {
  if (!S || !job_status) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return fail(MDS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second->state != kDone) {
    *job_status = MDS_PENDING;
    return MDS_OK;
  }
  return take_result(S, it, job_status, times);
}

mds_status mds_wait(mds_server_t S, mds_ticket ticket, mds_status* job_status, mds_job_times* times) {
  if (!S || !job_status) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return fail(MDS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  // the predicate looks the ticket up again: another thread may have taken the result
  S->done_cv.wait(lk, [&] {
    auto f = S->jobs.find(ticket);
    return f == S->jobs.end() || f->second->state == kDone;
  });
  it = S->jobs.find(ticket);
  if (it == S->jobs.end())
    return fail(MDS_ERR_STATE, "ticket %llu was released by another call", (unsigned long long)ticket);
  return take_result(S, it, job_status, times);
}

mds_status mds_cancel(mds_server_t S, mds_ticket ticket) {
  if (!S) return fail(MDS_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return fail(MDS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  Job* j = it->second;
  if (j->state != kQueued) return fail(MDS_ERR_STATE, "job %llu has already started", (unsigned long long)ticket);
  for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
    if (*q == j) {
      S->queue.erase(q);
      break;
    }
  j->state = kDone;
  j->result = MDS_ERR_CANCELLED;
  j->t_done = Clock::now();
  S->done_cv.notify_all();
  S->work_cv.notify_one();
  return MDS_OK;
}

mds_status mds_server_stats(mds_server_t S, mds_server_info* out) {
  if (!S || !out) return fail(MDS_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  out->queued = (int32_t)S->queue.size();
  out->running = (int32_t)S->running.size();
  out->slots = (int32_t)S->slots.size();
  out->pad_ = 0;
  out->completed = S->completed;
  out->batches = S->batches;
  out->budget_bytes = S->budget;
  out->used_bytes = S->arena->used();
  out->peak_bytes = S->arena->peak();
  return MDS_OK;
}

mds_status mds_server_set_batching(mds_server_t S, int64_t small_n_max, int32_t max_batch) {
  if (!S) return fail(MDS_ERR_INVALID_ARG, "NULL server");
  if (small_n_max < 0 || max_batch < 1 || max_batch > kMaxGroup)
    return fail(MDS_ERR_INVALID_ARG, "small_n_max = %lld, max_batch = %d (need >= 0 and 1..%d)",
                (long long)small_n_max, max_batch, kMaxGroup);
  std::lock_guard<std::mutex> g(S->mu);
  S->small_n_max = small_n_max;
  S->max_batch = max_batch;
  return MDS_OK;
}

mds_status mds_server_autotune(mds_server_t S, int32_t form, int32_t k, int32_t oversample, int32_t q,
                               int64_t* small_n_max) {
  if (!S) return fail(MDS_ERR_INVALID_ARG, "NULL server");
  int max_batch;
  {
    std::lock_guard<std::mutex> g(S->mu);
    max_batch = S->max_batch;
  }
  // batch a size class only if a full batch costs under a quarter of the
  // plan path's time per instance (the plan path also overlaps across slots)
  int64_t chosen = 0;
  for (int64_t n = 128; n <= 8192; n *= 2) {
    if ((int64_t)k + oversample > n) continue;
    mds_batch_tune t{};
    const mds_status st = mds_autotune_batch(form, n, k, oversample, q, max_batch, nullptr, &t);
    if (st == MDS_ERR_INVALID_ARG) break;  // past the batched kernel's limits
    if (st != MDS_OK) return st;
    if (!(4.0f * t.batch_ms_best < t.plan_ms)) break;
    chosen = n;
  }
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->small_n_max = chosen;
  }
  if (small_n_max) *small_n_max = chosen;
  return MDS_OK;
}

void mds_server_destroy(mds_server_t S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    for (Job* j : S->queue) {
      j->state = kDone;
      j->result = MDS_ERR_CANCELLED;
    }
    S->queue.clear();
    S->stop = true;
  }
  S->work_cv.notify_one();
  if (S->worker.joinable()) S->worker.join();  // returns once every admitted job has completed
  for (auto& kv : S->jobs) free_job(kv.second);
  for (Slot& sl : S->slots) {
    (void)hipStreamDestroy(sl.stream);
    (void)hipEventDestroy(sl.done);
    (void)hipHostFree(sl.host_status);
  }
  (void)hipFree(S->arena_ptr);
  delete S->arena;
  delete S;
}

}  // extern "C"
