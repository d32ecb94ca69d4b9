// Serving form: continuous (iteration-level) batching of independent jobs over
// a caller-owned device arena.
//
// A job is the per-job pass sequence of the filter: down(0) .. down(L-2), then
// up(L-2) .. up(0) (a single-level job is one copy).  Each step enqueues the
// next pass of every admitted job; passes of one kernel class share a launch
// (the batched launches of the batched form, with levels mixed), so jobs that
// arrive while others are in flight join at the next step and their passes
// overlap on the device with everybody else's.  Admission is by device-memory
// footprint: a job's workspace is a first-fit block of the arena, held from
// admission until its last pass has completed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "fllf_internal.h"

namespace {

using fllf::align_up;
using fllf::kAlign;

// First-fit allocator over [lo, hi) with coalescing of freed blocks.
class Arena {
 public:
  void init(size_t lo, size_t hi) {
    free_.clear();
    if (hi > lo) free_[lo] = hi - lo;
    capacity_ = hi > lo ? hi - lo : 0;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
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
  size_t capacity() const { return capacity_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;  // offset -> bytes
  size_t capacity_ = 0, used_ = 0, peak_ = 0;
};

struct Job {
  fllf_job job;
  uint64_t tag;
  hipEvent_t ready;
  size_t ws_off = 0, ws_bytes = 0;
  fllf::JobPlan plan;
  int pass = 0, npasses = 1;  // passes enqueued so far / in total
};

// pass p of a job with L levels: down(p) for p < L - 1, else up(2L - 3 - p)
fllf::PassItem pass_item(const Job &j) {
  const int L = j.plan.levels;
  if (L == 1) return fllf::PassItem{&j.plan, 0, true};
  if (j.pass < L - 1) return fllf::PassItem{&j.plan, j.pass, true};
  return fllf::PassItem{&j.plan, 2 * L - 3 - j.pass, false};
}

struct Step {
  hipEvent_t ev;
  int slot;
  std::vector<Job *> finishing;
};

constexpr int kSlots = 4;  // launch tables in flight

}  // namespace

struct fllf_server {
  fllf_ctx *ctx = nullptr;
  char *base = nullptr;
  size_t bytes = 0;
  int max_active = 0;
  size_t slot_bytes = 0;
  Arena arena;
  void *stage = nullptr;  // pinned host copies of the kSlots tables
  bool slot_busy[kSlots] = {};
  int next_slot = 0;
  std::deque<Job *> queue;
  std::vector<Job *> active;
  std::deque<Step> inflight;
  std::deque<uint64_t> done;
  std::vector<hipEvent_t> events;
  int64_t steps = 0, launches = 0, completed = 0, passes = 0;
  int max_step_jobs = 0;
  int finishing = 0;
};

namespace {

hipEvent_t get_event(fllf_server *s, hipError_t *err) {
  if (!s->events.empty()) {
    hipEvent_t e = s->events.back();
    s->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  *err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
  return e;
}

// Retires completed steps in order: their finishing jobs become done and give
// their workspace back.  wait_slot >= 0: first block until the step that uses
// that table slot has completed.
fllf_status reclaim(fllf_server *s, int wait_slot) {
  while (!s->inflight.empty()) {
    Step &st = s->inflight.front();
    hipError_t e = hipSuccess;
    if (wait_slot >= 0 && s->slot_busy[wait_slot]) {
      e = hipEventSynchronize(st.ev);
    } else {
      e = hipEventQuery(st.ev);
      if (e == hipErrorNotReady) break;
    }
    if (e != hipSuccess)
      return fllf::ctx_fail(s->ctx, FLLF_EDEVICE, "server: step failed on the device: %s", hipGetErrorString(e));
    for (Job *j : st.finishing) {
      if (j->ws_bytes) s->arena.release(j->ws_off, j->ws_bytes);
      s->done.push_back(j->tag);
      --s->finishing;
      delete j;
    }
    s->slot_busy[st.slot] = false;
    s->events.push_back(st.ev);
    s->inflight.pop_front();
  }
  return FLLF_OK;
}

}  // namespace

extern "C" {

fllf_status fourier_llf_server_create(fllf_ctx *ctx, void *arena, size_t arena_bytes, int max_active,
                                      fllf_server **out) {
  if (!out) return fllf::ctx_fail(ctx, FLLF_EINVAL, "server_create: out is NULL");
  *out = nullptr;
  if (!ctx) return fllf::ctx_fail(nullptr, FLLF_EINVAL, "server_create: ctx is NULL");
  if (!arena || ((uintptr_t)arena) % kAlign != 0)
    return fllf::ctx_fail(ctx, FLLF_EINVAL, "server_create: arena must be non-NULL and %zu-byte aligned", kAlign);
  if (max_active < 1 || max_active > 4096)
    return fllf::ctx_fail(ctx, FLLF_EINVAL, "server_create: max_active=%d outside [1, 4096]", max_active);
  const size_t slot = fllf::step_table_bound(max_active);
  if (arena_bytes <= kSlots * slot)
    return fllf::ctx_fail(ctx, FLLF_ENOMEM, "server_create: arena of %zu bytes holds only the launch tables (%zu)",
                          arena_bytes, kSlots * slot);
  hipError_t e = hipSetDevice(fllf::ctx_device(ctx));
  void *stage = nullptr;
  if (e == hipSuccess) e = hipHostMalloc(&stage, kSlots * slot, hipHostMallocDefault);
  if (e != hipSuccess) return fllf::ctx_fail(ctx, FLLF_EDEVICE, "server_create: %s", hipGetErrorString(e));
  fllf_server *s = new fllf_server();
  s->ctx = ctx;
  s->base = (char *)arena;
  s->bytes = arena_bytes;
  s->max_active = max_active;
  s->slot_bytes = slot;
  s->stage = stage;
  s->arena.init(kSlots * slot, arena_bytes - arena_bytes % kAlign);
  *out = s;
  return FLLF_OK;
}

fllf_status fourier_llf_server_submit(fllf_server *s, const fllf_job *job, uint64_t tag, void *ready_event) {
  if (!s) return fllf::ctx_fail(nullptr, FLLF_EINVAL, "server_submit: server is NULL");
  fllf_ctx *ctx = s->ctx;
  const fllf_storage storage = fllf::ctx_storage(ctx);
  fllf_status st = fllf::validate_jobs(ctx, job, 1, storage);
  if (st != FLLF_OK) return st;
  if (job->flags) return fllf::ctx_fail(ctx, FLLF_EUNSUPPORTED, "server_submit: Fourier LLF jobs only");
  auto hits = [&](const void *p, size_t bytes) { return fllf::spans_overlap(p, bytes, s->base, s->bytes); };
  if (hits(job->out, fllf::out_span(*job)) || hits(job->in, fllf::in_span(*job)) ||
      hits(job->m_map, fllf::map_span(*job)) || hits(job->sigma_map, fllf::map_span(*job)))
    return fllf::ctx_fail(ctx, FLLF_EINVAL, "server_submit: the job's images overlap the arena");
  Job *j = new Job();
  j->job = *job;
  j->tag = tag;
  j->ready = (hipEvent_t)ready_event;
  fllf::plan_job(*job, storage, 0, &j->plan);
  j->ws_bytes = j->plan.bytes;
  j->npasses = job->levels == 1 ? 1 : 2 * (job->levels - 1);
  if (align_up(j->ws_bytes) > s->arena.capacity()) {
    const size_t need = j->ws_bytes;
    delete j;
    return fllf::ctx_fail(ctx, FLLF_ENOMEM, "server_submit: workspace of %zu bytes exceeds the arena (%zu)",
                          need, s->arena.capacity());
  }
  s->queue.push_back(j);
  return FLLF_OK;
}

fllf_status fourier_llf_server_step(fllf_server *s, void *hip_stream, int *pending) {
  if (!s) return fllf::ctx_fail(nullptr, FLLF_EINVAL, "server_step: server is NULL");
  fllf_ctx *ctx = s->ctx;
  const fllf_storage storage = fllf::ctx_storage(ctx);
  hipStream_t stream = (hipStream_t)hip_stream;
  hipError_t e = hipSetDevice(fllf::ctx_device(ctx));
  if (e != hipSuccess) return fllf::ctx_fail(ctx, FLLF_EDEVICE, "server_step: %s", hipGetErrorString(e));
  fllf_status st = reclaim(s, -1);
  if (st != FLLF_OK) return st;
  // admission: arrival order, first fit, no overtaking
  while (!s->queue.empty() && (int)s->active.size() < s->max_active) {
    Job *j = s->queue.front();
    size_t off = 0;
    if (j->ws_bytes && !s->arena.alloc(j->ws_bytes, &off)) break;
    j->ws_off = off;
    fllf::plan_job(j->job, storage, off, &j->plan);
    if (j->ready) {
      e = hipStreamWaitEvent(stream, j->ready, 0);
      if (e != hipSuccess) {
        if (j->ws_bytes) s->arena.release(off, j->ws_bytes);
        return fllf::ctx_fail(ctx, FLLF_EDEVICE, "server_step: wait for input: %s", hipGetErrorString(e));
      }
    }
    s->queue.pop_front();
    s->active.push_back(j);
  }
  if (!s->active.empty()) {
    const int slot = s->next_slot;
    if (s->slot_busy[slot]) {
      st = reclaim(s, slot);
      if (st != FLLF_OK) return st;
    }
    std::vector<fllf::PassItem> items;
    items.reserve(s->active.size());
    for (Job *j : s->active) items.push_back(pass_item(*j));
    fllf::BatchSchedule sched;
    fllf::build_step(items.data(), (int)items.size(), storage, s->base, fllf::ctx_tuning(ctx), &sched);
    if (sched.table_bytes > s->slot_bytes)
      return fllf::ctx_fail(ctx, FLLF_EINVAL, "server_step: launch table of %zu bytes exceeds its slot (%zu)",
                            sched.table_bytes, s->slot_bytes);
    char *table = s->base + slot * s->slot_bytes;
    char *stage = (char *)s->stage + slot * s->slot_bytes;
    if (sched.table_bytes) {
      std::memcpy(stage, sched.blob.data(), sched.table_bytes);
      e = hipMemcpyAsync(table, stage, sched.table_bytes, hipMemcpyHostToDevice, stream);
      if (e != hipSuccess) return fllf::ctx_fail(ctx, FLLF_EDEVICE, "server_step: table upload: %s", hipGetErrorString(e));
    }
    e = fllf::launch_batch(sched, storage, table, stream, fllf::ctx_hook(ctx), fllf::ctx_tuning(ctx));
    if (e != hipSuccess) return fllf::ctx_fail(ctx, FLLF_EDEVICE, "server_step: launch: %s", hipGetErrorString(e));
    Step rec;
    rec.slot = slot;
    rec.ev = get_event(s, &e);
    if (e == hipSuccess) e = hipEventRecord(rec.ev, stream);
    if (e != hipSuccess) return fllf::ctx_fail(ctx, FLLF_EDEVICE, "server_step: event: %s", hipGetErrorString(e));
    std::vector<Job *> still;
    still.reserve(s->active.size());
    for (Job *j : s->active) {
      if (++j->pass == j->npasses) {
        rec.finishing.push_back(j);
        ++s->finishing;
      } else {
        still.push_back(j);
      }
    }
    s->active.swap(still);
    s->slot_busy[slot] = true;
    s->inflight.push_back(rec);
    s->next_slot = (slot + 1) % kSlots;
    ++s->steps;
    s->launches += (int64_t)sched.launches.size();
    s->passes += (int64_t)items.size();
    s->max_step_jobs = std::max(s->max_step_jobs, (int)items.size());
  }
  if (pending) *pending = (int)(s->queue.size() + s->active.size()) + s->finishing + (int)s->done.size();
  return FLLF_OK;
}

fllf_status fourier_llf_server_poll(fllf_server *s, uint64_t *tags, int max, int *n) {
  if (!s || !n || (max > 0 && !tags)) return fllf::ctx_fail(s ? s->ctx : nullptr, FLLF_EINVAL, "server_poll: bad arguments");
  *n = 0;
  fllf_status st = reclaim(s, -1);
  if (st != FLLF_OK) return st;
  while (*n < max && !s->done.empty()) {
    tags[(*n)++] = s->done.front();
    s->done.pop_front();
    ++s->completed;
  }
  return FLLF_OK;
}

fllf_status fourier_llf_server_stats(const fllf_server *s, fllf_server_stats *out) {
  if (!s || !out) return fllf::ctx_fail(nullptr, FLLF_EINVAL, "server_stats: bad arguments");
  out->queued = (int32_t)s->queue.size();
  out->active = (int32_t)s->active.size();
  out->finishing = s->finishing;
  out->max_active = s->max_active;
  out->steps = s->steps;
  out->launches = s->launches;
  out->completed = s->completed;
  out->passes = s->passes;
  out->max_step_jobs = s->max_step_jobs;
  out->reserved = 0;
  out->arena_bytes = s->arena.capacity();
  out->arena_used = s->arena.used();
  out->arena_peak = s->arena.peak();
  return FLLF_OK;
}

void fourier_llf_server_destroy(fllf_server *s) {
  if (!s) return;
  for (Step &st : s->inflight) {
    (void)hipEventSynchronize(st.ev);
    for (Job *j : st.finishing) delete j;
    (void)hipEventDestroy(st.ev);
  }
  for (Job *j : s->queue) delete j;
  for (Job *j : s->active) delete j;
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  if (s->stage) (void)hipHostFree(s->stage);
  delete s;
}

}  // extern "C"
