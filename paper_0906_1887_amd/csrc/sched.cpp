// Serving scheduler: continuous batching of integration jobs on one GPU.
//
// The real-time correlator of Sec. 5 keeps the GPU fed by batching many
// unpack-FFT-CMAC cycles per GPU call and overlaps host staging with device
// work.  Here independent integration jobs (each its own N_I, N_C, T) arrive
// at any time.  One scheduler thread admits them in arrival order as soon as
// their HBM footprint fits in the caller's arena (first-fit free list; a job
// that does not fit lets smaller ones behind it pass for at most kMaxHeadWait)
// and a queue slot is free.
//
// Device queue (the batched path).  An admitted job is published in a slot
// of a job queue in the arena's head: its pass (sample and result pointers,
// shape) and the claim limit of its work items, one per (channel, 128-row
// baseline tile).  A persistent serving grid (xeng_serve_kernel, as many
// workgroups as the GPU holds at once but kCopyReserve) runs while published
// work remains.  Its workgroups claim items round robin over the listed jobs,
// so jobs that arrive while others run are taken up by the grid already on
// the device and a small job is not queued behind a large one.  A job whose
// items are all claimed leaves the list.  Once the queue
// has been idle for kIdleUs the grid closes as a whole; the scheduler
// launches a new full-size grid (alternating between two streams, so it can
// start while the closing one finishes its last tiles) when work is published
// after the last launch and no open grid is running.  The workgroup that
// finishes a job's last item writes the job's completion word in pinned host
// memory.  Results go straight to a device
// destination; a host destination gets the integration through a copy from
// the arena (the latency end point is then the landed copy).  There is no
// per-job plan and no per-job kernel launch.
//
// Rows that are not 16-byte aligned (caller buffers with an odd stride) take
// the per-job path instead: a corr_plan carved from the arena, the plan's
// X-engine launch and a copy, on one of the scheduler's streams.
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

#include "common.h"
#include "corr.h"
#include "launch.h"
#include "plan_internal.h"

namespace {

constexpr size_t kAlign = 256;
constexpr double kMaxHeadWait = 0.020;   // s a blocked head job lets smaller jobs pass
constexpr int kLookahead = 16;
constexpr int kSlots = 64;               // jobs on the device queue at once
constexpr int kStage = 512;              // pinned staging entries for queue updates
constexpr size_t kStageBytes = 512;
constexpr double kIdleUs = 100.0;        // queue idle this long: the serving grid closes
constexpr int kMaxPolls = 1 << 18;       // bound on one serving workgroup's empty polls
constexpr int kCopyStreams = 4;          // streams a large host copy is split over
constexpr size_t kCopyPart = 32u << 20;  // at least this many bytes per part
constexpr int kCopyReserve = 16;         // workgroup slots a serving grid leaves free (the runtime's
                                         // copy kernels for host destinations run there)

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum JobState { kQueued = 0, kRunning = 1, kCopying = 2, kDone = 3 };

struct Job {
  uint64_t id = 0;
  corr_job_desc d{};
  double t_arrival = 0, t_admit = 0, t_device = 0;
  std::atomic<double> t_done{0.0};
  size_t off = 0, bytes = 0;           // arena region: samples (fill), then result (host destination)
  size_t samples_bytes = 0, result_bytes = 0;
  int64_t fill_stride = 0;             // samples between rows of a filled job
  bool queued_path = true;             // device queue, else per-job plan
  int slot = -1;
  uint64_t items = 0;
  uint64_t limit = 0;                  // claim limit of the job's items
  bool claimed_all = false;            // the device has claimed every item
  uint32_t flag_value = 0;
  corr_plan* plan = nullptr;
  int stream = -1;
  int64_t n_out = 0;
  std::atomic<int> state{kQueued};
  corr_status status = CORR_OK;
  bool released = false;               // arena region returned
  struct corr_sched* owner = nullptr;
};

// First-fit allocator over [base, size) with coalescing.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  void reset(size_t base, size_t size) {
    free_.clear();
    free_[base] = size - base;
    size_ = size - base;
  }
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
    if (bytes == 0) return;
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

// Device-queue layout in the arena's head (byte offsets).
struct QueueLayout {
  size_t slots = 0, limit = 0, claim = 0, done = 0, active = 0, rr = 0, last_claim = 0, closing = 0, total = 0;
};
QueueLayout queue_layout() {
  QueueLayout q;
  size_t off = 0;
  q.slots = off;
  off = align_up(off + kSlots * sizeof(corr::ServeJob));
  q.limit = off;
  off = align_up(off + kSlots * corr::kServeLine * 4);
  q.claim = off;
  off = align_up(off + kSlots * corr::kServeLine * 4);
  q.done = off;
  off = align_up(off + kSlots * corr::kServeLine * 4);
  q.active = off;
  off = align_up(off + (kSlots + 1) * 4);
  q.rr = off;
  off = align_up(off + 128);
  q.last_claim = off;
  off = align_up(off + 128);
  q.closing = off;
  off = align_up(off + 128);
  q.total = off;
  return q;
}

}  // namespace

struct corr_sched {
  uint8_t* arena_base = nullptr;
  Arena arena{0};
  std::vector<hipStream_t> streams;        // per-job path
  std::vector<int> stream_jobs;            // running per-job-path jobs per stream
  hipStream_t s_ctl = nullptr;             // fills and queue updates
  hipStream_t s_grid[2] = {nullptr, nullptr};  // serving grids, alternately
  hipStream_t s_copy = nullptr;            // results to host destinations (and the completion callback)
  hipStream_t s_copy_x[kCopyStreams - 1] = {};  // further parts of large host copies
  hipEvent_t ev_copy_x[kCopyStreams - 1] = {};
  hipEvent_t ev_pub = nullptr;             // after the latest queue update
  hipEvent_t ev_grid[2] = {nullptr, nullptr};
  bool grid_alive[2] = {false, false};     // launched, completion not yet seen
  uint32_t grid_gen[2] = {0, 0};           // generation of the grid on each stream
  uint32_t next_gen = 0;
  bool work_since_launch = false;          // a job was published after the latest grid launch
  int grid_cap = 0;                        // workgroups the GPU holds at once
  QueueLayout ql;
  corr::ServeQueue q{};
  uint32_t* flags = nullptr;               // pinned host: completion words, one line per slot,
                                           // then the closed-grid generation
  uint32_t* d_flags = nullptr;             // their device view
  uint8_t* stage = nullptr;                // pinned host staging ring for queue updates
  hipEvent_t stage_ev[kStage] = {};
  bool stage_used[kStage] = {};
  int stage_next = 0;
  uint64_t slot_limit[kSlots] = {};        // claim limit of each slot's latest job
  Job* slot_job[kSlots] = {};
  std::vector<int> free_slots;
  bool active_dirty = false;
  uint32_t next_flag = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job*> pending;
  std::vector<Job*> running;
  std::unordered_map<uint64_t, Job*> jobs;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  int64_t n_submitted = 0, n_admitted = 0, n_completed = 0, n_failed = 0;
  std::atomic<int64_t> callbacks{0};       // host callbacks queued and not yet finished

  explicit corr_sched(size_t bytes) : arena(bytes) {}
};

namespace {

void on_done(void* arg) {
  // Runs on a HIP runtime thread once the job's copy has landed.  It makes no
  // HIP call and takes no lock (the scheduler thread may hold the lock while
  // it waits on a stream); the scheduler's bounded wait catches a missed
  // notification.  Once kDone is published the job may be retired and freed
  // at any moment, so the owner is read first and the job is not touched
  // after the store; the owner outlives the callback because
  // corr_sched_destroy waits for the count of callbacks in flight to drop to
  // zero, which is this function's last access to it.
  Job* j = static_cast<Job*>(arg);
  corr_sched* o = j->owner;
  j->t_done.store(now_s());
  j->state.store(kDone);
  o->cv.notify_all();
  o->callbacks.fetch_sub(1);
}

// Copy `bytes` through a pinned staging entry (whose previous copy has
// completed) to the arena at arena_off, on the control stream (lock held).
hipError_t stage_copy(corr_sched* s, size_t arena_off, const void* src, size_t bytes) {
  const int k = s->stage_next;
  s->stage_next = (k + 1) % kStage;
  if (s->stage_used[k]) hipEventSynchronize(s->stage_ev[k]);
  s->stage_used[k] = true;
  uint8_t* e = s->stage + (size_t)k * kStageBytes;
  std::memcpy(e, src, bytes);
  hipError_t r = hipMemcpyAsync(s->arena_base + arena_off, e, bytes, hipMemcpyHostToDevice, s->s_ctl);
  if (r == hipSuccess) r = hipEventRecord(s->stage_ev[k], s->s_ctl);
  return r;
}

// Publish the list of slots holding jobs with unclaimed items (lock held).
hipError_t publish_active(corr_sched* s) {
  int32_t list[kSlots + 1];
  int n = 0;
  for (int k = 0; k < kSlots; ++k) {
    const Job* j = s->slot_job[k];
    if (j && j->state.load() == kRunning && !j->claimed_all) list[1 + n++] = k;
  }
  list[0] = n;
  s->active_dirty = false;
  hipError_t r = stage_copy(s, s->ql.active, list, sizeof(int32_t) * (n + 1));
  if (r == hipSuccess) r = hipEventRecord(s->ev_pub, s->s_ctl);
  return r;
}

// Admit one job on the device queue (lock held).
corr_status launch_queued(corr_sched* s, Job* j) {
  const corr_job_desc& d = j->d;
  j->slot = s->free_slots.back();
  s->free_slots.pop_back();
  s->slot_job[j->slot] = j;
  j->t_admit = now_s();
  j->state.store(kRunning);
  s->running.push_back(j);
  s->n_admitted++;

  const void* samples = d.d_samples;
  int64_t stride = d.row_stride ? d.row_stride : d.n_samples;
  if (d.fill) {
    samples = s->arena_base + j->off;
    stride = j->fill_stride;
    d.fill(d.fill_user, j->id, const_cast<void*>(samples), d.n_channels, d.n_inputs, d.n_samples, stride,
           s->s_ctl);
  }
  corr::ServeJob sj;
  std::memset(&sj, 0, sizeof(sj));
  const int64_t nb = (d.n_inputs + 127) / 128;
  corr::XArgs& a = sj.x;
  a.x = samples;
  a.row_stride_b = stride * 2;
  a.ch_stride_b = (int64_t)d.n_inputs * a.row_stride_b;
  a.k_bytes = d.n_samples * 2;
  a.k_split_bytes = a.k_bytes;
  a.out = d.dst_is_device ? d.dst : static_cast<void*>(s->arena_base + j->off + j->samples_bytes);
  a.n_products = (int64_t)d.n_inputs * (d.n_inputs + 1) / 2;
  a.n_in = d.n_inputs;
  a.n_ch = d.n_channels;
  a.n_tiles = (int32_t)(nb * (nb + 1) / 2);
  a.n_split = 1;
  a.n_items = (int32_t)j->items;
  a.accumulate = 0;
  j->flag_value = ++s->next_flag;
  if (j->flag_value == 0) j->flag_value = ++s->next_flag;
  sj.flag = s->d_flags + (size_t)j->slot * corr::kServeLine;
  sj.flag_value = j->flag_value;
  sj.base = s->slot_limit[j->slot];
  s->slot_limit[j->slot] += j->items;
  const uint64_t lim = s->slot_limit[j->slot];
  j->limit = lim;
  // The job, then its claim limit (a grid claims an item only below the
  // limit, so it sees the job -- and the fill before it -- first), then the
  // list of active slots.
  hipError_t r = stage_copy(s, s->ql.slots + (size_t)j->slot * sizeof(corr::ServeJob), &sj, sizeof(sj));
  if (r == hipSuccess) r = stage_copy(s, s->ql.limit + (size_t)j->slot * corr::kServeLine * 4, &lim, sizeof(lim));
  if (r == hipSuccess) r = publish_active(s);
  s->work_since_launch = true;
  return r == hipSuccess ? CORR_OK : CORR_E_HIP;
}

// Admit one job on the per-job path (lock held): carve its region, create its
// plan, queue its work.
void launch_plan_job(corr_sched* s, Job* j) {
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
  int64_t stride = j->d.row_stride;
  if (j->d.fill) {
    samples = base;
    stride = j->fill_stride;
    j->d.fill(j->d.fill_user, j->id, base, j->d.n_channels, j->d.n_inputs, j->d.n_samples, stride, st);
  }
  corr_status rc = corr_create(&cfg, base + j->samples_bytes, j->bytes - j->samples_bytes, st, &j->plan);
  if (rc == CORR_OK) rc = corr_correlate(j->plan, samples, j->d.n_samples, stride);
  if (rc == CORR_OK) rc = corr_internal_dump_async(j->plan, j->d.dst, j->d.dst_is_device, &j->n_out);
  if (rc == CORR_OK) {
    s->callbacks.fetch_add(1);
    if (hipLaunchHostFunc(st, on_done, j) != hipSuccess) {
      s->callbacks.fetch_sub(1);
      rc = CORR_E_HIP;
    }
  }
  if (rc != CORR_OK) {
    // Nothing will signal this job: wait for whatever was queued, then fail it.
    hipStreamSynchronize(st);
    j->status = rc;
    j->t_done.store(now_s());
    j->state.store(kDone);
  }
}

// Launch a full-size serving grid when a job was published after the latest
// launch and no open grid is running (lock held).  An open grid takes new work
// itself; a closing one takes none, so the work waits for the new grid, which
// may start on the other stream while the closing grid finishes its tiles.
void launch_grids(corr_sched* s) {
  for (int g = 0; g < 2; ++g)
    if (s->grid_alive[g] && hipEventQuery(s->ev_grid[g]) != hipErrorNotReady) s->grid_alive[g] = false;
  if (!s->work_since_launch || s->grid_cap <= 0) return;
  const uint32_t closed = __atomic_load_n(s->flags + (size_t)kSlots * corr::kServeLine, __ATOMIC_ACQUIRE);
  int free_g = -1;
  for (int g = 0; g < 2; ++g) {
    if (s->grid_alive[g] && s->grid_gen[g] > closed) return;   // an open grid is running
    if (!s->grid_alive[g] && free_g < 0) free_g = g;
  }
  if (free_g < 0) return;                                        // both streams hold closing grids
  corr::ServeQueue q = s->q;
  q.gen = s->next_gen + 1;
  if (hipStreamWaitEvent(s->s_grid[free_g], s->ev_pub, 0) != hipSuccess) return;
  if (corr::launch_xeng_serve(q, s->grid_cap, s->s_grid[free_g]) != hipSuccess) return;
  if (hipEventRecord(s->ev_grid[free_g], s->s_grid[free_g]) != hipSuccess) return;
  s->next_gen = q.gen;
  s->grid_gen[free_g] = q.gen;
  s->grid_alive[free_g] = true;
  s->work_since_launch = false;
}

void retire_job(corr_sched* s, Job* j) {
  if (j->plan) corr_destroy(j->plan);
  j->plan = nullptr;
  s->arena.release(j->off, j->bytes);
  j->released = true;
  if (!j->queued_path) s->stream_jobs[j->stream]--;
  if (j->status == CORR_OK) s->n_completed++;
  else s->n_failed++;
}

// Jobs whose completion word has been written: free the queue slot, then
// finish (device destination) or copy the result to the host destination.
void collect_queue(corr_sched* s) {
  for (Job* j : s->running) {
    if (!j->queued_path || j->state.load() != kRunning) continue;
    if (!j->claimed_all) {
      const uint64_t c = __atomic_load_n(reinterpret_cast<const uint64_t*>(s->flags) +
                                             (size_t)j->slot * (corr::kServeLine / 2) + 1,
                                         __ATOMIC_ACQUIRE);
      if (c == j->limit) {
        // every item is claimed: list the job no more, so the grid's
        // workgroups do not scan past it
        j->claimed_all = true;
        s->active_dirty = true;
      }
    }
    const uint32_t f = __atomic_load_n(s->flags + (size_t)j->slot * corr::kServeLine, __ATOMIC_ACQUIRE);
    if (f != j->flag_value) continue;
    j->t_device = now_s();
    j->n_out = j->d.n_samples;
    s->slot_job[j->slot] = nullptr;
    s->free_slots.push_back(j->slot);
    s->active_dirty = true;
    if (j->d.dst_is_device) {
      j->t_done.store(j->t_device);
      j->state.store(kDone);
      continue;
    }
    j->state.store(kCopying);
    // A large result goes to the host in up to kCopyStreams parts on as many
    // streams (copy engines run in parallel); the callback follows them all.
    const uint8_t* src = s->arena_base + j->off + j->samples_bytes;
    uint8_t* dst = static_cast<uint8_t*>(j->d.dst);
    const int parts = (int)std::min<size_t>(kCopyStreams, std::max<size_t>(1, j->result_bytes / kCopyPart));
    const size_t piece = (j->result_bytes / parts + 255) / 256 * 256;
    hipError_t e = hipSuccess;
    for (int k = 1; k < parts && e == hipSuccess; ++k) {
      const size_t o = k * piece;
      if (o >= j->result_bytes) break;
      e = hipMemcpyAsync(dst + o, src + o, std::min(piece, j->result_bytes - o), hipMemcpyDeviceToHost,
                         s->s_copy_x[k - 1]);
      if (e == hipSuccess) e = hipEventRecord(s->ev_copy_x[k - 1], s->s_copy_x[k - 1]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s->s_copy, s->ev_copy_x[k - 1], 0);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(dst, src, std::min(piece, j->result_bytes), hipMemcpyDeviceToHost, s->s_copy);
    if (e == hipSuccess) {
      s->callbacks.fetch_add(1);
      e = hipLaunchHostFunc(s->s_copy, on_done, j);
      if (e != hipSuccess) s->callbacks.fetch_sub(1);
    }
    if (e != hipSuccess) {
      hipStreamSynchronize(s->s_copy);
      for (hipStream_t x : s->s_copy_x) hipStreamSynchronize(x);
      j->status = CORR_E_HIP;
      j->t_done.store(now_s());
      j->state.store(kDone);
    }
  }
}

void worker_loop(corr_sched* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    collect_queue(s);
    // Retire completed jobs: free their plan and arena region.
    for (size_t k = 0; k < s->running.size();) {
      Job* j = s->running[k];
      if (j->state.load() == kDone) {
        retire_job(s, j);
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
        if (j->queued_path && s->free_slots.empty()) continue;
        size_t off;
        if (!s->arena.alloc(j->bytes, &off)) continue;
        j->off = off;
        s->pending.erase(s->pending.begin() + k);
        if (j->queued_path) {
          const corr_status rc = launch_queued(s, j);
          if (rc != CORR_OK) {
            hipStreamSynchronize(s->s_ctl);
            j->status = rc;
            s->slot_job[j->slot] = nullptr;
            s->free_slots.push_back(j->slot);
            j->t_done.store(now_s());
            j->state.store(kDone);
          }
        } else {
          launch_plan_job(s, j);
        }
        admitted = true;
        break;
      }
    }
    if (s->active_dirty) publish_active(s);
    launch_grids(s);
    if (s->stop && s->pending.empty() && s->running.empty()) break;
    bool busy = s->work_since_launch || s->grid_alive[0] || s->grid_alive[1];
    for (const Job* j : s->running) busy = busy || (j->queued_path && j->state.load() == kRunning);
    s->cv.wait_for(lk, std::chrono::microseconds(busy ? 20 : 200));
  }
}

}  // namespace

extern "C" {

double corr_sched_now(void) { return now_s(); }

corr_status corr_sched_create(void* d_arena, size_t arena_bytes, int32_t n_streams, corr_sched** out) {
  try {
    if (!out || n_streams < 1 || n_streams > 16) return CORR_E_INVAL;
    if (!d_arena || (reinterpret_cast<uintptr_t>(d_arena) % kAlign) != 0) return CORR_E_WORKSPACE;
    const QueueLayout ql = queue_layout();
    const size_t size = arena_bytes / kAlign * kAlign;
    if (size < ql.total + kAlign) return CORR_E_WORKSPACE;
    corr_sched* s = new (std::nothrow) corr_sched(size);
    if (!s) return CORR_E_INVAL;
    s->arena_base = static_cast<uint8_t*>(d_arena);
    s->arena.reset(ql.total, size);
    s->ql = ql;
    bool ok = true;
    for (int k = 0; k < n_streams && ok; ++k) {
      hipStream_t st;
      ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
      if (ok) {
        s->streams.push_back(st);
        s->stream_jobs.push_back(0);
      }
    }
    for (hipStream_t* st : {&s->s_ctl, &s->s_grid[0], &s->s_grid[1], &s->s_copy})
      ok = ok && hipStreamCreateWithFlags(st, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k < kCopyStreams - 1; ++k) {
      ok = ok && hipStreamCreateWithFlags(&s->s_copy_x[k], hipStreamNonBlocking) == hipSuccess;
      ok = ok && hipEventCreateWithFlags(&s->ev_copy_x[k], hipEventDisableTiming) == hipSuccess;
    }
    for (hipEvent_t* e : {&s->ev_pub, &s->ev_grid[0], &s->ev_grid[1]})
      ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < kStage && ok; ++k)
      ok = hipEventCreateWithFlags(&s->stage_ev[k], hipEventDisableTiming) == hipSuccess;
    // Pinned host memory (allocated, not registered): completion words the
    // serving grids write, and the staging ring for queue updates.
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&s->flags), (kSlots + 1) * corr::kServeLine * 4,
                             hipHostMallocMapped) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&s->stage), kStage * kStageBytes, hipHostMallocDefault) ==
                   hipSuccess;
    void* d_flags = nullptr;
    ok = ok && hipHostGetDevicePointer(&d_flags, s->flags, 0) == hipSuccess;
    // The queue's words start at zero.
    ok = ok && corr::launch_fill_zero(s->arena_base, (int64_t)ql.total, s->s_ctl) == hipSuccess;
    ok = ok && hipStreamSynchronize(s->s_ctl) == hipSuccess;
    if (!ok) {
      corr_sched_destroy(s);
      return CORR_E_HIP;
    }
    std::memset(s->flags, 0, (kSlots + 1) * corr::kServeLine * 4);
    s->d_flags = static_cast<uint32_t*>(d_flags);
    int dev = 0, cus = 0, clock_khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
      cus = 0;   // no serving grid: every job takes the per-job path
    s->grid_cap = std::max(0, corr::serve_blocks_per_cu() * cus - kCopyReserve);
    s->q.slots = reinterpret_cast<const corr::ServeJob*>(s->arena_base + ql.slots);
    s->q.limit = reinterpret_cast<const uint64_t*>(s->arena_base + ql.limit);
    s->q.claim = reinterpret_cast<uint64_t*>(s->arena_base + ql.claim);
    s->q.done = reinterpret_cast<uint32_t*>(s->arena_base + ql.done);
    s->q.active = reinterpret_cast<const int32_t*>(s->arena_base + ql.active);
    s->q.n_slots = kSlots;
    s->q.last_claim = reinterpret_cast<uint64_t*>(s->arena_base + ql.last_claim);
    s->q.closing = reinterpret_cast<uint32_t*>(s->arena_base + ql.closing);
    s->q.host_closing = s->d_flags + (size_t)kSlots * corr::kServeLine;
    s->q.host_claimed = reinterpret_cast<uint64_t*>(s->d_flags);
    s->q.rr = reinterpret_cast<uint32_t*>(s->arena_base + ql.rr);
    s->q.idle_ticks = (uint32_t)std::max(1.0, (double)clock_khz * 1e3 * kIdleUs * 1e-6);
    s->q.max_polls = kMaxPolls;
    for (int k = kSlots - 1; k >= 0; --k) s->free_slots.push_back(k);
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
    const int64_t nb = (d->n_inputs + 127) / 128;
    j->items = (uint64_t)d->n_channels * (uint64_t)(nb * (nb + 1) / 2);
    // Filled rows are padded to a multiple of 8 samples (16 bytes).
    j->fill_stride = (d->n_samples + 7) / 8 * 8;
    const int64_t stride = d->row_stride ? d->row_stride : d->n_samples;
    const bool aligned =
        d->fill || ((reinterpret_cast<uintptr_t>(d->d_samples) % 16) == 0 && (stride * 2) % 16 == 0);
    j->queued_path = aligned && j->items < (1ull << 31) && s->grid_cap > 0;
    j->samples_bytes = d->fill ? align_up((size_t)d->n_channels * d->n_inputs * j->fill_stride * 2) : 0;
    j->result_bytes = (size_t)d->n_channels * (size_t)((int64_t)d->n_inputs * (d->n_inputs + 1) / 2) * 8;
    j->bytes = j->queued_path ? j->samples_bytes + (d->dst_is_device ? 0 : align_up(j->result_bytes))
                              : j->samples_bytes + align_up(ws);
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
                            double* t_device, double* t_done) {
  if (!s) return CORR_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return CORR_E_INVAL;
  Job* j = it->second;
  if (j->state.load() != kDone || !j->released) return CORR_E_BUSY;
  const corr_status st = j->status;
  if (n_samples_out) *n_samples_out = j->n_out;
  if (t_admit) *t_admit = j->t_admit;
  if (t_device) *t_device = j->t_device > 0 ? j->t_device : j->t_done.load();
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
  std::vector<hipStream_t> all = s->streams;
  for (hipStream_t st : {s->s_ctl, s->s_grid[0], s->s_grid[1], s->s_copy})
    if (st) all.push_back(st);
  for (hipStream_t st : s->s_copy_x)
    if (st) all.push_back(st);
  for (hipStream_t st : all) hipStreamSynchronize(st);
  // A callback may still be returning after its stream has passed it.
  while (s->callbacks.load() != 0) std::this_thread::yield();
  for (hipStream_t st : all) hipStreamDestroy(st);
  for (hipEvent_t e : {s->ev_pub, s->ev_grid[0], s->ev_grid[1]})
    if (e) hipEventDestroy(e);
  for (hipEvent_t e : s->ev_copy_x)
    if (e) hipEventDestroy(e);
  for (int k = 0; k < kStage; ++k)
    if (s->stage_ev[k]) hipEventDestroy(s->stage_ev[k]);
  if (s->flags) hipHostFree(s->flags);
  if (s->stage) hipHostFree(s->stage);
  for (auto& kv : s->jobs) delete kv.second;
  delete s;
  return CORR_OK;
}

}  // extern "C"
