// Serving scheduler: continuous batching of integration jobs on one GPU.
//
// The real-time correlator of Sec. 5 keeps the GPU fed with large batches and
// overlaps host staging with device work.  Here independent integration jobs
// (each its own N_I, N_C, T) arrive at any time.  One scheduler thread admits
// them in arrival order as soon as their HBM footprint fits in the caller's
// arena (first-fit free list; a job that does not fit does not block smaller
// ones behind it for longer than kMaxHeadWait), and runs each admitted job on
// one of a pool of HIP streams, so the jobs' kernels overlap on the device.
// Per job: fill (or caller samples) -> int8 X-engine (a corr_plan carved from
// the arena) -> copy of the integration to the job's result buffer -> host
// callback that stamps the completion time.  The arena region is recycled once the
// scheduler thread sees the completion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "corr.h"
#include "plan_internal.h"

namespace {

constexpr size_t kAlign = 256;
constexpr double kMaxHeadWait = 0.020;   // s a blocked head job lets smaller jobs pass
constexpr int kLookahead = 16;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum JobState { kQueued = 0, kRunning = 1, kDone = 2 };

struct Job {
  uint64_t id = 0;
  corr_job_desc d{};
  double t_arrival = 0, t_admit = 0;
  std::atomic<double> t_done{0.0};
  size_t off = 0, bytes = 0, samples_bytes = 0;
  corr_plan* plan = nullptr;
  int stream = -1;
  int64_t n_out = 0;
  std::atomic<int> state{kQueued};
  corr_status status = CORR_OK;
  bool released = false;       // arena region returned
  struct corr_sched* owner = nullptr;
};

// First-fit allocator over [0, size) with coalescing.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t peak() const { return peak_; }

 private:
  size_t size_;
  size_t used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

corr_config job_config(const corr_job_desc& d) {
  corr_config c;
  std::memset(&c, 0, sizeof(c));
  c.n_inputs = d.n_inputs;
  c.n_channels = d.n_channels;
  c.fft_size = 0;
  c.sample_type = CORR_CI8;
  c.engine = CORR_X_I8;
  c.max_abs = d.max_abs;
  return c;
}

}  // namespace

struct corr_sched {
  uint8_t* arena_base = nullptr;
  Arena arena{0};
  std::vector<hipStream_t> streams;
  std::vector<int> stream_jobs;            // running jobs per stream
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job*> pending;
  std::vector<Job*> running;
  std::unordered_map<uint64_t, Job*> jobs;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  int64_t n_submitted = 0, n_admitted = 0, n_completed = 0, n_failed = 0;

  explicit corr_sched(size_t bytes) : arena(bytes) {}
};

namespace {

void on_done(void* arg) {
  // Runs on a HIP runtime thread once the job's copy has landed.  It makes no
  // HIP call and takes no lock (the scheduler thread may hold the lock while
  // it waits on a stream); the scheduler's bounded wait catches a missed
  // notification.
  Job* j = static_cast<Job*>(arg);
  j->t_done.store(now_s());
  j->state.store(kDone);
  j->owner->cv.notify_all();
}

// Admit one job (lock held): carve its region, create its plan, queue its work.
void launch_job(corr_sched* s, Job* j) {
  const corr_config cfg = job_config(j->d);
  uint8_t* base = s->arena_base + j->off;
  int best = 0;
  for (int k = 1; k < (int)s->streams.size(); ++k)
    if (s->stream_jobs[k] < s->stream_jobs[best]) best = k;
  j->stream = best;
  s->stream_jobs[best]++;
  hipStream_t st = s->streams[best];
  j->t_admit = now_s();
  j->state.store(kRunning);
  s->running.push_back(j);
  s->n_admitted++;

  const void* samples = j->d.d_samples;
  if (j->d.fill) {
    samples = base;
    j->d.fill(j->d.fill_user, j->id, base, j->d.n_channels, j->d.n_inputs, j->d.n_samples, st);
  }
  corr_status rc = corr_create(&cfg, base + j->samples_bytes, j->bytes - j->samples_bytes, st, &j->plan);
  const int64_t stride = j->d.fill ? 0 : j->d.row_stride;
  if (rc == CORR_OK) rc = corr_correlate(j->plan, samples, j->d.n_samples, stride);
  if (rc == CORR_OK) rc = corr_internal_dump_async(j->plan, j->d.dst, j->d.dst_is_device, &j->n_out);
  if (rc == CORR_OK && hipLaunchHostFunc(st, on_done, j) != hipSuccess) rc = CORR_E_HIP;
  if (rc != CORR_OK) {
    // Nothing will signal this job: wait for whatever was queued, then fail it.
    hipStreamSynchronize(st);
    j->status = rc;
    j->t_done.store(now_s());
    j->state.store(kDone);
  }
}

void worker_loop(corr_sched* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // Retire completed jobs: free their plan and arena region.
    for (size_t k = 0; k < s->running.size();) {
      Job* j = s->running[k];
      if (j->state.load() == kDone) {
        if (j->plan) corr_destroy(j->plan);
        j->plan = nullptr;
        s->arena.release(j->off, j->bytes);
        j->released = true;
        s->stream_jobs[j->stream]--;
        if (j->status == CORR_OK) s->n_completed++;
        else s->n_failed++;
        s->running[k] = s->running.back();
        s->running.pop_back();
      } else {
        ++k;
      }
    }
    // Admit in arrival order; smaller jobs may pass a head that does not fit
    // while the head has waited less than kMaxHeadWait.
    bool admitted = true;
    while (admitted && !s->pending.empty()) {
      admitted = false;
      const double t = now_s();
      const int look = (t - s->pending.front()->t_arrival < kMaxHeadWait) ? kLookahead : 1;
      for (int k = 0; k < look && k < (int)s->pending.size(); ++k) {
        Job* j = s->pending[k];
        size_t off;
        if (s->arena.alloc(j->bytes, &off)) {
          j->off = off;
          s->pending.erase(s->pending.begin() + k);
          launch_job(s, j);
          admitted = true;
          break;
        }
      }
    }
    if (s->stop && s->pending.empty() && s->running.empty()) break;
    s->cv.wait_for(lk, std::chrono::microseconds(200));
  }
}

}  // namespace

extern "C" {

double corr_sched_now(void) { return now_s(); }

corr_status corr_sched_create(void* d_arena, size_t arena_bytes, int32_t n_streams, corr_sched** out) {
  try {
    if (!out || n_streams < 1 || n_streams > 16) return CORR_E_INVAL;
    if (!d_arena || arena_bytes < kAlign || (reinterpret_cast<uintptr_t>(d_arena) % kAlign) != 0)
      return CORR_E_WORKSPACE;
    corr_sched* s = new (std::nothrow) corr_sched(arena_bytes / kAlign * kAlign);
    if (!s) return CORR_E_INVAL;
    s->arena_base = static_cast<uint8_t*>(d_arena);
    for (int k = 0; k < n_streams; ++k) {
      hipStream_t st;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        for (hipStream_t x : s->streams) hipStreamDestroy(x);
        delete s;
        return CORR_E_HIP;
      }
      s->streams.push_back(st);
      s->stream_jobs.push_back(0);
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

corr_status corr_sched_submit(corr_sched* s, const corr_job_desc* d, double t_arrival, uint64_t* job_id) {
  try {
    if (!s || !d || !job_id) return CORR_E_INVAL;
    if (!d->dst || d->n_samples < 1 || (!d->fill && !d->d_samples)) return CORR_E_INVAL;
    if (d->row_stride < 0 || (d->row_stride > 0 && d->row_stride < d->n_samples)) return CORR_E_INVAL;
    const corr_config cfg = job_config(*d);
    size_t ws = 0;
    const corr_status v = corr_workspace_bytes(&cfg, &ws);
    if (v != CORR_OK) return v;
    if (2.0 * d->max_abs * d->max_abs * (double)d->n_samples > 2147483647.0) return CORR_E_OVERFLOW;
    Job* j = new (std::nothrow) Job();
    if (!j) return CORR_E_INVAL;
    j->d = *d;
    j->t_arrival = t_arrival;
    j->owner = s;
    j->samples_bytes = d->fill ? align_up((size_t)d->n_channels * d->n_inputs * d->n_samples * 2) : 0;
    j->bytes = j->samples_bytes + align_up(ws);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (j->bytes > s->arena.size()) {
        delete j;
        return CORR_E_WORKSPACE;
      }
      j->id = s->next_id++;
      s->jobs[j->id] = j;
      s->pending.push_back(j);
      s->n_submitted++;
    }
    s->cv.notify_all();
    *job_id = j->id;
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

corr_status corr_sched_poll(corr_sched* s, uint64_t job_id, int64_t* n_samples_out, double* t_admit,
                            double* t_done) {
  if (!s) return CORR_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return CORR_E_INVAL;
  Job* j = it->second;
  if (j->state.load() != kDone || !j->released) return CORR_E_BUSY;
  const corr_status st = j->status;
  if (n_samples_out) *n_samples_out = j->n_out;
  if (t_admit) *t_admit = j->t_admit;
  if (t_done) *t_done = j->t_done.load();
  s->jobs.erase(it);
  delete j;
  return st;
}

corr_status corr_sched_stats(corr_sched* s, int64_t stats[8]) {
  if (!s || !stats) return CORR_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  stats[0] = s->n_submitted;
  stats[1] = s->n_admitted;
  stats[2] = s->n_completed;
  stats[3] = s->n_failed;
  stats[4] = (int64_t)s->pending.size();
  stats[5] = (int64_t)s->running.size();
  stats[6] = (int64_t)s->arena.peak();
  stats[7] = (int64_t)s->arena.size();
  return CORR_OK;
}

corr_status corr_sched_destroy(corr_sched* s) {
  if (!s) return CORR_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (hipStream_t st : s->streams) {
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  for (auto& kv : s->jobs) delete kv.second;
  delete s;
  return CORR_OK;
}

}  // extern "C"
