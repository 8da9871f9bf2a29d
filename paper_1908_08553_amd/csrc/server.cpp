// Served request loop: continuous admission of lattice contractions.
//
// Requests of different sizes arrive at any time.  A scheduler thread admits
// them in arrival order as soon as a slot (a HIP stream of its own) and a
// contiguous region of the caller's arena large enough for the request's
// whole workspace (boundary buffers, staged sites, bookkeeping) are free; the
// request's sites are copied in, every step of its contraction is enqueued on
// its slot's stream, and its boundary tensors stay on the device until the
// scalar comes out.  Work of different requests overlaps on the device: the
// hardware queues interleave their kernels step by step, so a small request
// admitted next to a large one finishes without waiting for it.  Completion
// is detected with events; the result record is copied back and the slot and
// arena region are released for the next request.  Admission is strictly
// first-come-first-served (a large request at the head of the queue is not
// overtaken), which keeps the largest requests from starving.
#include "server.hpp"
#include "server_arena.hpp"

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "exec.hpp"
#include "plan.hpp"

namespace tn {
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

enum ReqState { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Request {
  uint64_t ticket = 0;
  Plan plan;
  int32_t prec = 0;
  std::vector<std::vector<double>> sites;   // host copies taken at submit
  std::vector<const double*> site_ptrs;
  size_t footprint = 0;
  size_t arena_off = 0;
  size_t state_off = 0;
  size_t result_off = 0;                    // result record in the slot's pinned image
  int32_t slot = -1;
  hipEvent_t done = nullptr;
  int64_t t_submit = 0, t_admit = 0, t_done = 0;
  tn_result result{};
  tn_status status = TN_OK;
  int32_t state = QUEUED;
};

}  // namespace

struct ServerImpl {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int32_t max_slots = 1, queue_depth = 1;
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<int32_t> slot_busy;
  // pinned upload image per slot: a slot runs one request at a time and is
  // released only after that request's stream work has finished
  std::vector<std::unique_ptr<HostKeep>> keeps;
  Arena alloc{0};
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
  std::mutex mu;
  std::condition_variable cv;
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1;
  int64_t n_submitted = 0, n_completed = 0, peak_used = 0, peak_active = 0;
  std::string fatal;
};

namespace {

void complete(ServerImpl* s, Request* r) {
  const hipStream_t st = s->streams[r->slot];
  tn_result* staged = reinterpret_cast<tn_result*>(s->keeps[r->slot]->data() + r->result_off);
  hipError_t e = hipMemcpyAsync(staged, s->arena + r->state_off, sizeof(tn_result),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    std::memset(&r->result, 0, sizeof(r->result));
    r->status = TN_EDEVICE;
  } else {
    r->result = *staged;
    r->status = r->result.status;
  }
  r->t_done = now_ns();
}

void scheduler(ServerImpl* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // admission: first come, first served, by footprint and free slot
    std::vector<Request*> admitted;
    while (!s->queue.empty()) {
      Request* r = s->queue.front();
      int32_t slot = -1;
      for (int32_t k = 0; k < s->max_slots; ++k)
        if (!s->slot_busy[k]) { slot = k; break; }
      size_t off = 0;
      if (slot < 0 || !s->alloc.alloc(r->footprint, &off)) break;
      s->queue.pop_front();
      s->slot_busy[slot] = 1;
      r->slot = slot;
      r->arena_off = off;
      r->state = RUNNING;
      r->t_admit = now_ns();
      s->active.push_back(r);
      admitted.push_back(r);
      s->peak_used = std::max<int64_t>(s->peak_used, static_cast<int64_t>(s->alloc.used()));
      s->peak_active = std::max<int64_t>(s->peak_active, static_cast<int64_t>(s->active.size()));
    }
    std::vector<Request*> running = s->active;
    lk.unlock();

    for (Request* r : admitted) {
      std::string err;
      const hipStream_t st = s->streams[r->slot];
      LaunchTimer timer(st, false);
      tn_status rc = enqueue(r->plan, r->site_ptrs.data(), false, r->prec, s->arena + r->arena_off,
                             r->footprint, st, *s->keeps[r->slot], timer, err);
      const Layout L = make_layout(r->plan, r->prec);
      r->state_off = r->arena_off + L.state;
      r->result_off = head_bytes(r->plan, L);
      if (rc == TN_OK && hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess)
        rc = TN_EDEVICE;
      if (rc == TN_OK && hipEventRecord(r->done, st) != hipSuccess) rc = TN_EDEVICE;
      if (rc != TN_OK) {
        r->status = rc;
        if (r->done) { (void)hipEventDestroy(r->done); r->done = nullptr; }
        (void)hipStreamSynchronize(st);   // let any work already issued drain
      }
    }

    std::vector<Request*> finished;
    for (Request* r : running) {
      if (r->status != TN_OK && !r->done) { r->t_done = now_ns(); finished.push_back(r); continue; }
      if (!r->done) continue;
      const hipError_t q = hipEventQuery(r->done);
      if (q == hipErrorNotReady) continue;
      complete(s, r);
      (void)hipEventDestroy(r->done);
      r->done = nullptr;
      finished.push_back(r);
    }

    lk.lock();
    for (Request* r : finished) {
      s->alloc.release(r->arena_off, r->footprint);
      s->slot_busy[r->slot] = 0;
      r->state = DONE;
      r->sites.clear();
      for (size_t k = 0; k < s->active.size(); ++k)
        if (s->active[k] == r) { s->active.erase(s->active.begin() + k); break; }
      s->n_completed += 1;
    }
    if (!finished.empty()) s->cv.notify_all();
    if (s->stop && s->queue.empty() && s->active.empty()) break;
    if (s->active.empty() && s->queue.empty()) {
      // idle: sleep until a submit (or destroy) arrives
      s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    } else if (admitted.empty() && finished.empty()) {
      // work in flight: poll completions again shortly, without the lock
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

}  // namespace

tn_status server_create(void* arena, size_t arena_bytes, int32_t max_slots, int32_t queue_depth,
                        ServerImpl** out, std::string& err) {
  if (!arena || !out) { err = "null argument"; return TN_EINVAL; }
  if (reinterpret_cast<uintptr_t>(arena) % kAlign != 0) { err = "arena must be 256-byte aligned"; return TN_EINVAL; }
  if (max_slots < 1 || max_slots > 64) { err = "max_slots must be 1..64"; return TN_EINVAL; }
  if (queue_depth < 1) { err = "queue_depth must be >= 1"; return TN_EINVAL; }
  auto* s = new ServerImpl;
  s->arena = static_cast<char*>(arena);
  s->arena_bytes = arena_bytes / kAlign * kAlign;
  s->alloc = Arena(s->arena_bytes);
  s->max_slots = max_slots;
  s->queue_depth = queue_depth;
  if (hipGetDevice(&s->device) != hipSuccess) { err = "hipGetDevice failed"; delete s; return TN_EDEVICE; }
  s->streams.resize(max_slots, nullptr);
  s->slot_busy.assign(max_slots, 0);
  for (int32_t k = 0; k < max_slots; ++k) s->keeps.push_back(std::make_unique<HostKeep>());
  for (int32_t k = 0; k < max_slots; ++k) {
    if (hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking) != hipSuccess) {
      for (int32_t j = 0; j < k; ++j) (void)hipStreamDestroy(s->streams[j]);
      err = "hipStreamCreateWithFlags failed";
      delete s;
      return TN_EDEVICE;
    }
  }
  s->th = std::thread(scheduler, s);
  *out = s;
  return TN_OK;
}

tn_status server_submit(ServerImpl* s, const tn_grid& grid, int32_t order, int32_t prec,
                        const double* const* host_sites, uint64_t* ticket, std::string& err) {
  if (!host_sites || !ticket) { err = "null argument"; return TN_EINVAL; }
  if (prec < TN_PREC_F64 || prec > TN_PREC_BF16X3) { err = "unknown precision"; return TN_EINVAL; }
  auto r = std::make_unique<Request>();
  tn_status rc = build_plan(grid, order, 0, 0, r->plan, err);
  if (rc != TN_OK) return rc;
  r->prec = prec;
  r->footprint = align_up(make_layout(r->plan, prec).total);
  if (r->footprint > s->arena_bytes) {
    err = "request footprint " + std::to_string(r->footprint) + " exceeds the arena";
    return TN_ENOMEM;
  }
  const int32_t nsites = r->plan.rows * r->plan.cols;
  std::vector<int64_t> entries(nsites, 1);
  for (const Step& st : r->plan.steps) entries[st.r * r->plan.cols + st.c] = st.site_entries;
  r->sites.resize(nsites);
  r->site_ptrs.resize(nsites);
  for (int32_t k = 0; k < nsites; ++k) {
    if (!host_sites[k]) { err = "null site pointer"; return TN_EINVAL; }
    r->sites[k].assign(host_sites[k], host_sites[k] + entries[k]);
    r->site_ptrs[k] = r->sites[k].data();
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (static_cast<int32_t>(s->queue.size()) >= s->queue_depth) {
    err = "submit queue full";
    return TN_EBUSY;
  }
  r->ticket = s->next_ticket++;
  r->t_submit = now_ns();
  *ticket = r->ticket;
  s->queue.push_back(r.get());
  s->all.emplace(r->ticket, std::move(r));
  s->n_submitted += 1;
  s->cv.notify_all();
  return TN_OK;
}

tn_status server_poll(ServerImpl* s, uint64_t ticket, tn_result* out, int64_t* times_ns,
                      std::string& err) {
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) { err = "unknown or retired ticket"; return TN_ENOTFOUND; }
  Request* r = it->second.get();
  if (r->state != DONE) return TN_PENDING;
  if (out) *out = r->result;
  if (times_ns) {
    times_ns[0] = r->t_submit;
    times_ns[1] = r->t_admit;
    times_ns[2] = r->t_done;
  }
  const tn_status st = r->status;
  s->all.erase(it);
  if (st != TN_OK) err = st == TN_ENONFINITE ? "non-finite value in the request" : "request failed";
  return st;
}

void server_info(ServerImpl* s, tn_server_info* o) {
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(o, 0, sizeof(*o));
  o->submitted = s->n_submitted;
  o->completed = s->n_completed;
  o->queued = static_cast<int64_t>(s->queue.size());
  o->active = static_cast<int64_t>(s->active.size());
  o->arena_bytes = static_cast<int64_t>(s->arena_bytes);
  o->arena_in_use = static_cast<int64_t>(s->alloc.used());
  o->peak_arena_in_use = s->peak_used;
  o->peak_active = s->peak_active;
}

void server_destroy(ServerImpl* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  delete s;
}

}  // namespace tn
