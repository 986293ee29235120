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

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  DevStatus* host_status = nullptr;  // pinned
  Job* job = nullptr;
};

}  // namespace

struct mds_server_s {
  int device = 0;
  size_t budget = 0;
  void* arena_ptr = nullptr;
  Arena* arena = nullptr;
  std::vector<Slot> slots;
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

// Enqueue the whole run of j on its slot; called by the worker without the lock.
mds_status launch(mds_server_s* S, Job* j) {
  Slot& sl = S->slots[j->slot];
  mds_status st = mds_set_workspace(j->plan, static_cast<char*>(S->arena_ptr) + j->ws_off, j->ws_bytes);
  if (st == MDS_OK) st = run_plan(j->plan, j->D, j->coords, j->eigvals, sl.stream, MDS_STAGE_ALL, 0);
  if (st == MDS_OK)
    st = hip_check(hipMemcpyAsync(sl.host_status, j->plan->at<void>(j->plan->status), sizeof(DevStatus),
                                  hipMemcpyDeviceToHost, sl.stream),
                   "status copy");
  // the event is recorded whatever happened so that retirement waits for
  // every kernel this run managed to enqueue
  const mds_status ev = hip_check(hipEventRecord(sl.done, sl.stream), "hipEventRecord");
  return st != MDS_OK ? st : ev;
}

void worker_main(mds_server_s* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progressed = false;
    // retire finished jobs
    for (size_t i = 0; i < S->running.size();) {
      Job* j = S->running[i];
      Slot& sl = S->slots[j->slot];
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (j->result == MDS_PENDING) {
        if (q != hipSuccess) {
          j->result = fail(MDS_ERR_HIP, "job %llu: %s", (unsigned long long)j->id, hipGetErrorString(q));
        } else {
          const DevStatus& d = *sl.host_status;
          j->result = d.nonfinite ? MDS_ERR_NONFINITE : (d.jacobi_unconv ? MDS_ERR_NUMERICAL : MDS_OK);
        }
      }
      j->t_done = Clock::now();
      j->state = kDone;
      S->arena->release(j->ws_off, j->ws_bytes);
      sl.job = nullptr;
      S->running[i] = S->running.back();
      S->running.pop_back();
      ++S->completed;
      progressed = true;
    }
    if (progressed) S->done_cv.notify_all();
    if (S->stop && S->queue.empty() && S->running.empty()) break;
    // admit from the queue head while a slot and arena room are free
    while (!S->queue.empty() && !S->stop) {
      int slot = -1;
      for (size_t s = 0; s < S->slots.size(); ++s)
        if (!S->slots[s].job) {
          slot = (int)s;
          break;
        }
      if (slot < 0) break;
      Job* j = S->queue.front();
      size_t off = 0;
      if (!S->arena->alloc(j->ws_bytes, &off)) break;
      S->queue.pop_front();
      j->ws_off = off;
      j->slot = slot;
      j->state = kRunning;
      j->t_start = Clock::now();
      S->slots[slot].job = j;
      S->running.push_back(j);
      lk.unlock();
      const mds_status st = launch(S, j);
      lk.lock();
      if (st != MDS_OK) j->result = st;
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
        hipHostMalloc((void**)&sl.host_status, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess)
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
  out->budget_bytes = S->budget;
  out->used_bytes = S->arena->used();
  out->peak_bytes = S->arena->peak();
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
