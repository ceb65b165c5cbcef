// Request server: continuous batching of matches (Algorithm 1 per request)
// over the public batch call.  A worker thread keeps up to max_inflight
// batches on the device, one HIP stream each, so a new batch is formed and
// launched while earlier ones still run; requests are admitted first in,
// first out while the device workspace of the batches in flight stays within
// the budget.  Results come back through pinned host memory; each request's
// latency is measured from submission to the moment the worker sees its batch
// complete.  The worker sleeps until a request arrives or a batch finishes
// (a host function enqueued after each batch's result copy wakes it).  The
// device memory the server's streams hold stays within the budget: a slot's
// workspace pool grows to exactly what its batches need, and a batch is
// launched only while the pools of all slots fit the budget (idle slots
// release theirs first); one request larger than the budget runs alone.

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include <hip/hip_runtime.h>

#include "tm.h"
#include "tm_internal.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  uint64_t ticket;
  tm_plan plan;
  const void* x;
  int64_t footprint;
  int64_t t_submit;
};

struct Done {
  tm_result result;
  tm_status status;
  int64_t t_submit;
  int64_t t_done;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  tm_result* dev_out = nullptr;
  tm_result* host_out = nullptr;
  bool busy = false;
  std::vector<Req> reqs;
  int64_t footprint = 0;
};

}  // namespace

struct tm_server_s {
  tm_server_desc desc{};
  int device = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req> pending;
  std::unordered_map<uint64_t, Done> done;
  std::unordered_set<uint64_t> outstanding;      // submitted, result not yet taken
  uint64_t next_ticket = 1;
  int64_t inflight_bytes = 0;
  bool stop = false;
  bool kick = false;               // a request arrived or a batch finished
  bool poll_mode = false;          // a wake-up host function could not be enqueued
  tm_server_stats stats{};
  std::thread worker;
};

namespace {

// FIFO admission: requests join the current batch while it holds fewer than
// max_batch and the bytes in flight stay within the budget; a batch is never
// empty (one request larger than the budget goes alone).  Returns how many of
// the first `count` footprints form the next batch.
int32_t admit_prefix(int32_t count, const int64_t* fp, int64_t inflight, int64_t budget, int32_t max_batch) {
  int32_t n = 0;
  int64_t used = inflight;
  while (n < count && n < max_batch) {
    if (used + fp[n] > budget && !(n == 0 && inflight == 0)) break;
    used += fp[n];
    ++n;
  }
  return n;
}

void finish_slot(tm_server_s* s, Slot& sl, tm_status st) {
  const int64_t t = now_ns();
  std::lock_guard<std::mutex> lock(s->mu);
  for (size_t i = 0; i < sl.reqs.size(); ++i) {
    Done d{};
    d.status = st;
    if (st == TM_OK) d.result = sl.host_out[i];
    d.t_submit = sl.reqs[i].t_submit;
    d.t_done = t;
    s->done[sl.reqs[i].ticket] = d;
  }
  s->stats.completed += (int64_t)sl.reqs.size();
  if (st != TM_OK) s->stats.failed += (int64_t)sl.reqs.size();
  s->inflight_bytes -= sl.footprint;
  sl.busy = false;
  sl.reqs.clear();
  sl.footprint = 0;
  s->cv_done.notify_all();
}

void wake(tm_server_s* s) {
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->kick = true;
  }
  s->cv_work.notify_one();
}

void batch_done_cb(void* user) { wake(static_cast<tm_server_s*>(user)); }

// Device bytes the slots' pools hold, and the admission test on them: a
// batch of `fp` bytes may run in slot `mine` while every slot's pool, that
// slot's grown to the batch, fits the budget (or the batch is alone and
// larger than the budget).  Idle slots give their pools back first.
int64_t held_bytes(tm_server_s* s) {
  int64_t h = 0;
  for (Slot& sl : s->slots) h += (int64_t)tmi::stream_pool_device_bytes(s->device, sl.stream);
  return h;
}

bool make_room(tm_server_s* s, Slot& mine, int64_t fp) {
  const int64_t budget = std::max(s->desc.budget_bytes, fp);
  auto fits = [&] {
    int64_t h = 0;
    for (Slot& sl : s->slots) {
      const int64_t b = (int64_t)tmi::stream_pool_device_bytes(s->device, sl.stream);
      h += &sl == &mine ? std::max(b, fp) : b;
    }
    return h <= budget;
  };
  if (fits()) return true;
  for (Slot& sl : s->slots) {
    if (sl.busy && &sl != &mine) continue;
    (void)tmi::stream_pool_release(s->device, sl.stream, true);
    if (fits()) return true;
  }
  return false;
}

void worker_loop(tm_server_s* s) {
  (void)hipSetDevice(s->device);
  std::vector<tm_plan> plans;
  std::vector<const void*> xs;
  std::vector<int64_t> fps;
  for (;;) {
    // 1. batches that completed
    bool any_busy = false;
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.event);
      if (q == hipSuccess) finish_slot(s, sl, TM_OK);
      else if (q != hipErrorNotReady) finish_slot(s, sl, TM_ERR_DEVICE);
      else any_busy = true;
    }
    // 2. new batches into free slots
    for (Slot& sl : s->slots) {
      if (sl.busy) continue;
      {
        std::unique_lock<std::mutex> lock(s->mu);
        if (s->pending.empty()) break;
        fps.clear();
        const size_t look = std::min<size_t>(s->pending.size(), (size_t)s->desc.max_batch);
        for (size_t i = 0; i < look; ++i) fps.push_back(s->pending[i].footprint);
        const int32_t n = admit_prefix((int32_t)fps.size(), fps.data(), s->inflight_bytes, s->desc.budget_bytes,
                                       s->desc.max_batch);
        if (n == 0) break;   // budget full until a batch completes
        int64_t fp = 0;
        for (int32_t i = 0; i < n; ++i) fp += fps[(size_t)i];
        lock.unlock();       // pools are released outside the request lock
        const bool room = make_room(s, sl, fp);
        lock.lock();
        if (!room) break;    // the pools in flight hold the budget until a batch completes
        const int64_t held = held_bytes(s);
        s->stats.peak_held_bytes = std::max(s->stats.peak_held_bytes, held);
        sl.reqs.assign(s->pending.begin(), s->pending.begin() + n);
        s->pending.erase(s->pending.begin(), s->pending.begin() + n);
        for (const Req& r : sl.reqs) sl.footprint += r.footprint;
        s->inflight_bytes += sl.footprint;
        s->stats.peak_inflight_bytes = std::max(s->stats.peak_inflight_bytes, s->inflight_bytes);
        s->stats.batches += 1;
        sl.busy = true;
      }
      plans.clear();
      xs.clear();
      for (const Req& r : sl.reqs) {
        plans.push_back(r.plan);
        xs.push_back(r.x);
      }
      tm_status st = tm_match_batch((int32_t)plans.size(), plans.data(), xs.data(), sl.dev_out, sl.stream);
      if (st == TM_OK &&
          hipMemcpyAsync(sl.host_out, sl.dev_out, sizeof(tm_result) * plans.size(), hipMemcpyDeviceToHost,
                         sl.stream) != hipSuccess)
        st = TM_ERR_DEVICE;
      if (st == TM_OK && hipEventRecord(sl.event, sl.stream) != hipSuccess) st = TM_ERR_DEVICE;
      if (st == TM_OK && !s->poll_mode && hipLaunchHostFunc(sl.stream, batch_done_cb, s) != hipSuccess) {
        (void)hipGetLastError();
        s->poll_mode = true;   // no wake-up from the device: poll the events instead
      }
      if (st != TM_OK) finish_slot(s, sl, st);
      else any_busy = true;
    }
    // 3. sleep until a request arrives or a batch finishes
    std::unique_lock<std::mutex> lock(s->mu);
    if (s->stop && s->pending.empty() && !any_busy) return;
    if (any_busy && s->poll_mode)
      s->cv_work.wait_for(lock, std::chrono::microseconds(50), [&] { return s->kick; });
    else
      s->cv_work.wait(lock, [&] { return s->kick; });
    s->kick = false;
  }
}

}  // namespace

extern "C" {

tm_status tm_admit_batches(int32_t count, const int64_t* footprint, int64_t budget_bytes, int32_t max_batch,
                           int32_t* batch_of) {
  // host arithmetic only
  if (count < 0 || (count > 0 && (!footprint || !batch_of)) || max_batch < 1 || budget_bytes < 0)
    return TM_ERR_INVALID;
  int32_t i = 0, b = 0;
  while (i < count) {
    const int32_t n = admit_prefix(count - i, footprint + i, 0, budget_bytes, max_batch);
    for (int32_t j = 0; j < n; ++j) batch_of[i + j] = b;
    i += n;
    ++b;
  }
  return TM_OK;
}

tm_status tm_server_create(const tm_server_desc* desc, tm_server* out) {
  if (!out) return TM_ERR_INVALID;
  *out = nullptr;
  tm_server_desc d{};
  if (desc) d = *desc;
  if (d.budget_bytes < 0 || d.max_batch < 0 || d.max_inflight < 0) return TM_ERR_INVALID;
  if (d.budget_bytes == 0) d.budget_bytes = int64_t(1) << 30;
  if (d.max_batch == 0) d.max_batch = 1024;
  if (d.max_inflight == 0) d.max_inflight = 2;
  if (d.max_inflight > 8) return TM_ERR_INVALID;
  tm_server_s* s = new tm_server_s();
  s->desc = d;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return TM_ERR_DEVICE;
  }
  s->slots.resize((size_t)d.max_inflight);
  bool ok = true;
  for (Slot& sl : s->slots) {
    ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
    if (ok) tmi::stream_pool_set_exact(s->device, sl.stream);
    ok = ok && hipEventCreateWithFlags(&sl.event, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc(&sl.dev_out, sizeof(tm_result) * (size_t)d.max_batch) == hipSuccess;
    ok = ok && hipHostMalloc(&sl.host_out, sizeof(tm_result) * (size_t)d.max_batch, hipHostMallocDefault) ==
                   hipSuccess;
    if (!ok) break;
  }
  if (!ok) {
    for (Slot& sl : s->slots) {
      if (sl.event) (void)hipEventDestroy(sl.event);
      if (sl.stream) (void)tmi::stream_pool_release(s->device, sl.stream, false);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.dev_out) (void)hipFree(sl.dev_out);
      if (sl.host_out) (void)hipHostFree(sl.host_out);
    }
    delete s;
    return TM_ERR_DEVICE;
  }
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return TM_OK;
}

tm_status tm_server_submit(tm_server s, tm_plan plan, const void* x, uint64_t* ticket) {
  if (!s || !plan || !x || !ticket) return TM_ERR_INVALID;
  tm_plan_info info;
  const tm_status st = tm_plan_get_info(plan, &info);
  if (st != TM_OK) return st;
  if (!info.fft_in_lds && !info.fft_global && !info.corr_gemm) return TM_ERR_UNSUPPORTED;
  Req r;
  r.plan = plan;
  r.x = x;
  // workspace, result slot, and the request's entry in the batch's instance
  // table and launch list
  r.footprint = info.workspace_bytes + (int64_t)sizeof(tm_result) + (int64_t)sizeof(tmi::Inst) + 16;
  r.t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) return TM_ERR_INVALID;
    r.ticket = s->next_ticket++;
    s->outstanding.insert(r.ticket);
    s->pending.push_back(r);
    s->stats.submitted += 1;
    s->kick = true;
  }
  s->cv_work.notify_one();
  *ticket = r.ticket;
  return TM_OK;
}

static tm_status take_done(tm_server s, uint64_t ticket, tm_result* out, int64_t* latency_ns) {
  auto it = s->done.find(ticket);
  const Done d = it->second;
  s->done.erase(it);
  s->outstanding.erase(ticket);
  if (out) *out = d.result;
  if (latency_ns) *latency_ns = d.t_done - d.t_submit;
  return d.status;
}

tm_status tm_server_poll(tm_server s, uint64_t ticket, tm_result* out, int64_t* latency_ns, int* done) {
  if (!s || !done) return TM_ERR_INVALID;
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->outstanding.find(ticket) == s->outstanding.end()) return TM_ERR_INVALID;
  if (s->done.find(ticket) == s->done.end()) {
    *done = 0;
    return TM_OK;
  }
  *done = 1;
  return take_done(s, ticket, out, latency_ns);
}

tm_status tm_server_wait(tm_server s, uint64_t ticket, tm_result* out, int64_t* latency_ns) {
  if (!s || ticket == 0) return TM_ERR_INVALID;
  std::unique_lock<std::mutex> lock(s->mu);
  if (s->outstanding.find(ticket) == s->outstanding.end()) return TM_ERR_INVALID;
  s->cv_done.wait(lock, [&] { return s->done.find(ticket) != s->done.end(); });
  return take_done(s, ticket, out, latency_ns);
}

tm_status tm_server_get_stats(tm_server s, tm_server_stats* out) {
  if (!s || !out) return TM_ERR_INVALID;
  std::lock_guard<std::mutex> lock(s->mu);
  *out = s->stats;
  return TM_OK;
}

tm_status tm_server_destroy(tm_server s) {
  if (!s) return TM_OK;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
    s->kick = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  tm_status st = TM_OK;
  for (Slot& sl : s->slots) {
    // the stream drains (wake-up host functions included), then its pool goes
    if (tmi::stream_pool_release(s->device, sl.stream, false) != hipSuccess) st = TM_ERR_DEVICE;
    if (hipStreamSynchronize(sl.stream) != hipSuccess) st = TM_ERR_DEVICE;
    (void)hipEventDestroy(sl.event);
    (void)hipStreamDestroy(sl.stream);
    (void)hipFree(sl.dev_out);
    (void)hipHostFree(sl.host_out);
  }
  delete s;
  return st;
}

}  // extern "C"
