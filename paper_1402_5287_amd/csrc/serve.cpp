// Request scheduler for sessions of planned matvecs (continuous batching).
//
// The motivating use (Section 1) is a Lanczos iteration: many matvecs with
// one fixed Hankel matrix per session.  The server keeps the plans (the
// resident spectra of h) and a caller-provided device memory pool.  Each
// request is one planned matvec; it is admitted onto a free stream slot as
// soon as the pool can hold its workspace, so requests of different
// sessions overlap on the device and new work enters while earlier work is
// still running.  Requests of one session run in submission order.
// Admission is oldest-first with a reservation: while the oldest waiting
// request cannot get memory, younger requests are admitted only if they
// leave enough free memory for it (no starvation of large matrices).  It is
// also size-aware: a request whose workspace exceeds large_bytes is large,
// and at most max_large of those run at once; a large request that finds
// the cap reached is passed over (smaller ones behind it may start), so
// small requests keep finding slots and do not queue behind the device
// time of many large products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <set>
#include <vector>

#include "common.h"
#include "hmv.h"
#include "plan.h"

using namespace hmv;

namespace {

// first-fit allocator over [0, size) with kAlign granularity
struct PoolAlloc {
  int64_t size = 0;
  std::map<int64_t, int64_t> free_;   // offset -> length
  int64_t used = 0, peak = 0;

  void init(int64_t sz) {
    size = sz / kAlign * kAlign;
    free_.clear();
    if (size > 0) free_[0] = size;
    used = peak = 0;
  }
  int64_t largest() const {
    int64_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  int64_t alloc(int64_t bytes) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used += bytes;
        peak = std::max(peak, used);
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = align_up(bytes);
    used -= bytes;
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
};

struct Request {
  int64_t id = 0;
  int mid = 0;
  int64_t session = 0;
  const uint64_t* x = nullptr;
  uint64_t* y = nullptr;
  int64_t ws_off = -1, ws_bytes = 0;
  hipEvent_t ready = nullptr;   // recorded on the submitter's stream at submit
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  bool large = false;
  Request req;
};

}  // namespace

struct hmv_server {
  char* pool = nullptr;
  PoolAlloc alloc;
  std::vector<Slot> slots;
  std::vector<const hmv_plan*> plans;
  std::deque<Request> waiting;
  std::vector<hipEvent_t> spare_events;   // recycled ordering events
  std::set<int64_t> busy_sessions;
  int64_t next_id = 1;
  int64_t completed = 0, admitted = 0;
  int max_inflight = 0;
  int64_t large_bytes = 0;        // workspace above which a request is large
  int max_large = 1;              // large requests in flight at most
  int large_inflight = 0, max_large_seen = 0;
};

namespace {

int admit(hmv_server* S) {
  int64_t reserve = 0;             // memory promised to the oldest blocked request
  bool blocked = false;
  for (auto it = S->waiting.begin(); it != S->waiting.end();) {
    Request& r = *it;
    if (S->busy_sessions.count(r.session)) {
      ++it;
      continue;
    }
    int slot = -1;
    for (int k = 0; k < (int)S->slots.size(); ++k)
      if (!S->slots[k].busy) {
        slot = k;
        break;
      }
    if (slot < 0) break;
    const int64_t need = align_up(r.ws_bytes);
    const bool large = need > S->large_bytes;
    if (large && S->large_inflight >= S->max_large) {
      ++it;
      continue;
    }
    if (blocked && S->alloc.largest() - need < reserve) {
      ++it;
      continue;
    }
    const int64_t off = S->alloc.alloc(need);
    if (off < 0) {
      if (!blocked) {
        blocked = true;
        reserve = need;
      }
      ++it;
      continue;
    }
    r.ws_off = off;
    Slot& sl = S->slots[slot];
    const hmv_plan* p = S->plans[r.mid];
    // the request starts after the submitter's work that preceded submit
    int rc = hipStreamWaitEvent(sl.stream, r.ready, 0) == hipSuccess ? HMV_OK : HMV_EDEVICE;
    if (rc == HMV_OK) rc = hmv_plan_matvec(p, r.x, r.y, S->pool + off, r.ws_bytes, sl.stream);
    if (rc == HMV_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) rc = HMV_EDEVICE;
    if (rc != HMV_OK) {
      S->alloc.release(off, need);
      return rc;
    }
    sl.busy = true;
    sl.large = large;
    if (large) {
      ++S->large_inflight;
      S->max_large_seen = std::max(S->max_large_seen, S->large_inflight);
    }
    sl.req = r;
    S->busy_sessions.insert(r.session);
    ++S->admitted;
    it = S->waiting.erase(it);
    int inflight = 0;
    for (auto& s2 : S->slots) inflight += s2.busy ? 1 : 0;
    S->max_inflight = std::max(S->max_inflight, inflight);
  }
  return HMV_OK;
}

}  // namespace

extern "C" {

int hmv_server_create(hmv_server** out, void* pool, int64_t pool_bytes, int32_t max_slots) {
  if (!out || !pool || pool_bytes <= 0 || max_slots < 1 || max_slots > 64) return HMV_EINVAL;
  *out = nullptr;
  hmv_server* S = new (std::nothrow) hmv_server();
  if (!S) return HMV_ENOMEM;
  S->pool = static_cast<char*>(pool);
  S->alloc.init(pool_bytes);
  S->slots.resize(max_slots);
  S->large_bytes = S->alloc.size / 8;
  S->max_large = std::max(1, max_slots / 4);
  for (auto& sl : S->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      hmv_server_destroy(S);
      return HMV_EDEVICE;
    }
  }
  *out = S;
  return HMV_OK;
}

int hmv_server_add_plan(hmv_server* S, const hmv_plan* plan, int32_t* matrix_id) {
  if (!S || !plan || !matrix_id) return HMV_EINVAL;
  if (kStatusBytes + plan->mv_scratch > S->alloc.size) return HMV_ENOMEM;
  S->plans.push_back(plan);
  *matrix_id = (int32_t)S->plans.size() - 1;
  return HMV_OK;
}

int hmv_server_submit(hmv_server* S, int32_t matrix_id, int64_t session, const uint64_t* x,
                      uint64_t* y, void* stream, int64_t* request_id) {
  if (!S || !x || !y || matrix_id < 0 || matrix_id >= (int32_t)S->plans.size()) return HMV_EINVAL;
  clear_stale_error();
  hipEvent_t ev = nullptr;
  if (!S->spare_events.empty()) {
    ev = S->spare_events.back();
    S->spare_events.pop_back();
  } else {
    const hipError_t ec = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (ec != hipSuccess) return status_from_hip(ec, "server event");
  }
  const hipError_t er = hipEventRecord(ev, static_cast<hipStream_t>(stream));
  if (er != hipSuccess) {
    S->spare_events.push_back(ev);
    return status_from_hip(er, "server submit event");
  }
  Request r;
  r.ready = ev;
  r.id = S->next_id++;
  r.mid = matrix_id;
  r.session = session;
  r.x = x;
  r.y = y;
  r.ws_bytes = kStatusBytes + S->plans[matrix_id]->mv_scratch;
  S->waiting.push_back(r);
  if (request_id) *request_id = r.id;
  return admit(S);
}

int hmv_server_poll(hmv_server* S, int64_t* done_ids, int32_t* done_status, int32_t cap,
                    int32_t* n_done) {
  if (!S || !n_done || (cap > 0 && !done_ids)) return HMV_EINVAL;
  *n_done = 0;
  clear_stale_error();
  for (auto& sl : S->slots) {
    if (!sl.busy || *n_done >= cap) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return status_from_hip(q, "server poll");
    int32_t flags = 0;
    const int rc = hmv_read_status(S->pool + sl.req.ws_off, sl.stream, &flags, nullptr);
    done_ids[*n_done] = sl.req.id;
    if (done_status) done_status[*n_done] = rc == HMV_OK ? flags : rc;
    ++*n_done;
    S->alloc.release(sl.req.ws_off, align_up(sl.req.ws_bytes));
    S->spare_events.push_back(sl.req.ready);   // its wait has been consumed
    S->busy_sessions.erase(sl.req.session);
    if (sl.large) --S->large_inflight;
    sl.busy = false;
    sl.large = false;
    ++S->completed;
  }
  (void)hipGetLastError();
  return admit(S);
}

int hmv_server_stats(const hmv_server* S, hmv_server_stats_t* st) {
  if (!S || !st) return HMV_EINVAL;
  std::memset(st, 0, sizeof(*st));
  for (auto& sl : S->slots) st->in_flight += sl.busy ? 1 : 0;
  st->waiting = (int64_t)S->waiting.size();
  st->admitted = S->admitted;
  st->completed = S->completed;
  st->max_in_flight = S->max_inflight;
  st->pool_used = S->alloc.used;
  st->pool_peak = S->alloc.peak;
  st->pool_bytes = S->alloc.size;
  st->large_in_flight = S->large_inflight;
  st->max_large_in_flight = S->max_large_seen;
  st->large_bytes = S->large_bytes;
  st->max_large = S->max_large;
  return HMV_OK;
}

int hmv_server_set_policy(hmv_server* S, int64_t large_bytes, int32_t max_large) {
  if (!S || large_bytes < 0 || max_large < 1 || max_large > (int32_t)S->slots.size())
    return HMV_EINVAL;
  S->large_bytes = large_bytes;
  S->max_large = max_large;
  return HMV_OK;
}

int hmv_server_destroy(hmv_server* S) {
  if (!S) return HMV_EINVAL;
  for (auto& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.busy && sl.req.ready) (void)hipEventDestroy(sl.req.ready);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (auto& r : S->waiting)
    if (r.ready) (void)hipEventDestroy(r.ready);
  for (hipEvent_t ev : S->spare_events) (void)hipEventDestroy(ev);
  delete S;
  return HMV_OK;
}

}  // extern "C"
