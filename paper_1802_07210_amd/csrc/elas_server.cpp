// Serving loop of elas_mi355x: continuous batching of stereo pairs that
// arrive from many cameras.
//
// Callers submit pairs (device images and outputs of any supported size) and
// get a ticket back at once. One worker thread owns the device side: it
// keeps up to max_inflight batches on the device, each on its own stream,
// and whenever a stream is free and requests are waiting it takes the
// longest-waiting requests, as many as max_batch and the memory budget
// admit, and launches them as one elas_process_batch call. Requests that
// arrive while others run are therefore admitted as soon as a stream and
// memory free up, and their work overlaps the batches already on the device.
// The memory budget bounds the device memory the server's pairs keep
// resident: the buffer sets (elas_frame_bytes each) that the handles hold per
// (stream, size) between batches. New sets are admitted against it, and the
// sets of idle streams are released when the oldest request needs room. Latency is measured on the host
// from submission to the worker seeing the batch's completion event.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "elas.h"
#include "elas_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

enum class State { Pending, Done, Failed };

struct Request {
  int64_t ticket;
  elas_pair pair;
  int64_t bytes;
  hipEvent_t ready;  // recorded on the producer's stream at submission, or null
};

struct Result {
  State state = State::Pending;
  Clock::time_point submitted, finished;
  int code = ELAS_OK;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<int64_t> tickets;
  int64_t bytes = 0;
  // one pinned, device-mapped failure report word per pair of the batch: the
  // device mesh of a failing pair sets its word (cleared before each launch)
  int32_t* report_host = nullptr;
  int32_t* report_dev = nullptr;
  std::vector<int32_t*> report_ptrs;
};

}  // namespace

struct elas_server {
  elas_handle* h = nullptr;
  elas_server_config cfg{};
  std::mutex m;
  std::condition_variable work;  // submissions and shutdown
  std::condition_variable done;  // completions
  std::deque<Request> queue;
  std::vector<Slot> slots;
  std::unordered_map<int64_t, Result> results;
  std::map<std::tuple<elas_handle*, int32_t, int32_t>, int64_t> footprint;
  // buffer sets the library keeps for this server's pairs, per (slot, pair
  // parameter handle, w, h), and their device bytes
  std::map<std::tuple<int, elas_handle*, int32_t, int32_t>, int> sets;
  int64_t resident = 0;
  int64_t next_ticket = 1;
  int64_t in_flight = 0;
  std::vector<hipEvent_t> free_events;  // ready events not in use
  elas_server_stats stats{};
  bool stop = false;
  std::string err;
  std::thread worker;
};

namespace {

thread_local std::string g_server_error;

int server_fail(elas_server* s, int code, const std::string& msg) {
  if (s) {
    std::lock_guard<std::mutex> lk(s->m);
    s->err = msg;
  } else {
    g_server_error = msg;
  }
  return code;
}

void finish(elas_server* S, Slot& sl, State st, int code, Clock::time_point now) {
  for (size_t i = 0; i < sl.tickets.size(); ++i) {
    auto it = S->results.find(sl.tickets[i]);
    if (it == S->results.end()) continue;
    // a pair whose device mesh failed was matched without plane priors
    const int32_t rep =
        st == State::Done ? __atomic_load_n(&sl.report_host[i], __ATOMIC_ACQUIRE) : 0;
    if (rep != 0) {
      S->err = "the device mesh of ticket " + std::to_string(sl.tickets[i]) +
               " failed (status " + std::to_string(rep) + ")";
      it->second.state = State::Failed;
      it->second.code = ELAS_ERR_INTERNAL;
    } else {
      it->second.state = st;
      it->second.code = code;
    }
    it->second.finished = now;
  }
  S->stats.completed += (int64_t)sl.tickets.size();
  S->in_flight -= sl.bytes;
  sl.tickets.clear();
  sl.bytes = 0;
  sl.busy = false;
}

// Releases the buffer sets of every idle slot (their streams have finished);
// returns whether anything was released.
bool release_idle(elas_server* S) {
  bool any = false;
  for (size_t j = 0; j < S->slots.size(); ++j) {
    if (S->slots[j].busy) continue;
    std::map<elas_handle*, int64_t> held;  // per handle: bytes of its sets on this slot
    for (auto it = S->sets.begin(); it != S->sets.end();) {
      if (std::get<0>(it->first) != (int)j) {
        ++it;
        continue;
      }
      elas_handle* ph = std::get<1>(it->first);
      const auto kind = std::make_tuple(ph, std::get<2>(it->first), std::get<3>(it->first));
      held[ph] += S->footprint[kind] * it->second;
      it = S->sets.erase(it);
    }
    for (auto& kv : held) {
      (void)elas::release_stream_buffers(kv.first, S->slots[j].stream);
      S->resident -= kv.second;
      any = true;
    }
  }
  return any;
}

void worker_loop(elas_server* S) {
  std::unique_lock<std::mutex> lk(S->m);
  for (;;) {
    // completions
    bool any_done = false, any_busy = false;
    for (Slot& sl : S->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipSuccess) {
        finish(S, sl, State::Done, ELAS_OK, Clock::now());
        any_done = true;
      } else if (q != hipErrorNotReady) {
        S->err = std::string("batch failed on the device: ") + hipGetErrorString(q);
        finish(S, sl, State::Failed, ELAS_ERR_HIP, Clock::now());
        any_done = true;
      } else {
        any_busy = true;
      }
    }
    if (any_done) S->done.notify_all();
    // launches: oldest requests first, while a stream is free and the buffer
    // sets they need fit the budget. A batch with k pairs of one kind (pair
    // parameters and size) on a slot needs k buffer sets of that kind there;
    // sets the slot already holds are reused, new ones count against the
    // budget. When the oldest request does not fit, the sets of idle slots
    // are released once and it is tried again; otherwise it waits.
    for (size_t si = 0; si < S->slots.size(); ++si) {
      Slot& sl = S->slots[si];
      if (sl.busy || S->queue.empty()) continue;
      const int maxb = S->cfg.plain ? 1 : S->cfg.max_batch;
      std::vector<elas_pair> pairs;
      std::vector<int64_t> tickets;
      std::vector<hipEvent_t> ready;
      std::map<std::tuple<elas_handle*, int32_t, int32_t>, int> kinds;
      int64_t bytes = 0, grow = 0;
      bool released = false;
      while (!S->queue.empty() && (int)pairs.size() < maxb) {
        const Request& q = S->queue.front();
        elas_handle* ph = q.pair.params ? q.pair.params : S->h;
        const auto kind = std::make_tuple(ph, q.pair.w, q.pair.h);
        const int need = kinds.count(kind) ? kinds[kind] + 1 : 1;
        const auto skey = std::make_tuple((int)si, ph, q.pair.w, q.pair.h);
        const auto sit = S->sets.find(skey);
        const int have = sit == S->sets.end() ? 0 : sit->second;
        const int64_t extra = need > have ? q.bytes : 0;
        if (S->resident + grow + extra > S->cfg.memory_budget) {
          if (!pairs.empty() || released) break;
          released = true;
          if (release_idle(S)) continue;
          break;
        }
        kinds[kind] = need;
        grow += extra;
        pairs.push_back(q.pair);
        tickets.push_back(q.ticket);
        ready.push_back(q.ready);
        bytes += q.bytes;
        S->queue.pop_front();
      }
      if (pairs.empty()) break;  // the oldest request waits for memory
      for (auto& kv : kinds) {
        int& n = S->sets[std::make_tuple((int)si, std::get<0>(kv.first), std::get<1>(kv.first),
                                         std::get<2>(kv.first))];
        n = std::max(n, kv.second);
      }
      S->resident += grow;
      S->stats.peak_resident_bytes = std::max(S->stats.peak_resident_bytes, S->resident);
      for (size_t i = 0; i < pairs.size(); ++i)
        __atomic_store_n(&sl.report_host[i], 0, __ATOMIC_RELAXED);
      sl.busy = true;
      sl.tickets = tickets;
      sl.bytes = bytes;
      S->in_flight += bytes;
      S->stats.peak_bytes_in_flight = std::max(S->stats.peak_bytes_in_flight, S->in_flight);
      S->stats.batches += 1;
      S->stats.batched_pairs += (int64_t)pairs.size();
      lk.unlock();
      // the batch waits for the streams that produced its inputs
      hipError_t we = hipSuccess;
      for (hipEvent_t ev : ready)
        if (ev && we == hipSuccess) we = hipStreamWaitEvent(sl.stream, ev, 0);
      int rc = we == hipSuccess ? ELAS_OK : ELAS_ERR_HIP;
      if (rc != ELAS_OK) {
      } else if (S->cfg.plain) {
        const elas_pair& q = pairs[0];
        rc = elas::process_one(q.params ? q.params : S->h, q.left, q.right, q.w, q.h, q.stride,
                               sl.stream, q.disp_left, q.disp_right, sl.report_ptrs[0]);
      } else {
        rc = elas::process_batch(S->h, (int32_t)pairs.size(), pairs.data(), sl.stream,
                                 sl.report_ptrs.data());
      }
      const hipError_t re = rc == ELAS_OK ? hipEventRecord(sl.done, sl.stream) : hipSuccess;
      lk.lock();
      // the waits are enqueued: the events can be recorded again
      for (hipEvent_t ev : ready)
        if (ev) S->free_events.push_back(ev);
      if (we != hipSuccess) {
        S->err = std::string("hipStreamWaitEvent: ") + hipGetErrorString(we);
        finish(S, sl, State::Failed, ELAS_ERR_HIP, Clock::now());
        S->done.notify_all();
        continue;
      }
      if (rc != ELAS_OK || re != hipSuccess) {
        elas_handle* eh = S->cfg.plain && pairs[0].params ? pairs[0].params : S->h;
        S->err = rc != ELAS_OK ? std::string(elas_last_error(eh))
                               : std::string("hipEventRecord: ") + hipGetErrorString(re);
        finish(S, sl, State::Failed, rc != ELAS_OK ? rc : ELAS_ERR_HIP, Clock::now());
        S->done.notify_all();
      } else {
        any_busy = true;
      }
    }
    if (S->stop && S->queue.empty() && !any_busy) break;
    if (!any_busy && S->queue.empty())
      S->work.wait(lk);
    else
      S->work.wait_for(lk, std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

void elas_server_config_default(elas_server_config* c) {
  if (!c) return;
  c->max_batch = 32;
  c->max_inflight = 3;
  c->memory_budget = (int64_t)32 << 30;
  c->plain = 0;
}

int elas_server_create(elas_handle* h, const elas_server_config* cfg, elas_server** out) {
  if (!h || !cfg || !out) return server_fail(nullptr, ELAS_ERR_ARG, "null argument");
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->max_batch > 1024 || cfg->max_inflight < 1 ||
      cfg->max_inflight > 16 || cfg->memory_budget <= 0 || (cfg->plain != 0 && cfg->plain != 1))
    return server_fail(nullptr, ELAS_ERR_ARG,
                       "max_batch 1..1024, max_inflight 1..16, memory_budget > 0, plain 0/1");
  elas_server* S = new elas_server();
  S->h = h;
  S->cfg = *cfg;
  S->slots.resize(cfg->plain ? 1 : cfg->max_inflight);
  const int nrep = cfg->plain ? 1 : cfg->max_batch;
  for (Slot& sl : S->slots) {
    hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    void* rh = nullptr;
    if (e == hipSuccess)
      e = hipHostMalloc(&rh, sizeof(int32_t) * nrep, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
      sl.report_host = static_cast<int32_t*>(rh);
      void* rd = nullptr;
      e = hipHostGetDevicePointer(&rd, rh, 0);
      sl.report_dev = static_cast<int32_t*>(rd);
    }
    if (e != hipSuccess) {
      for (Slot& x : S->slots) {
        if (x.done) (void)hipEventDestroy(x.done);
        if (x.stream) (void)hipStreamDestroy(x.stream);
        if (x.report_host) (void)hipHostFree(x.report_host);
      }
      delete S;
      return server_fail(nullptr, ELAS_ERR_HIP, std::string("stream setup: ") + hipGetErrorString(e));
    }
    for (int i = 0; i < nrep; ++i) {
      sl.report_host[i] = 0;
      sl.report_ptrs.push_back(sl.report_dev + i);
    }
  }
  S->worker = std::thread(worker_loop, S);
  *out = S;
  return ELAS_OK;
}

}  // extern "C"

namespace {

// ordered: the pair waits on the device for the work enqueued on `producer`
// (the null stream when producer is null) at submission
int submit_pair(elas_server* s, const elas_pair* pair, bool ordered, hipStream_t producer,
                int64_t* ticket) {
  if (!s || !pair || !ticket) return server_fail(s, ELAS_ERR_ARG, "null argument");
  if (!pair->left || !pair->right || !pair->disp_left || !pair->disp_right || pair->w < 9 ||
      pair->h < 9 || pair->w > 8192 || pair->h > 8192 || pair->stride < pair->w)
    return server_fail(s, ELAS_ERR_ARG, "bad pair");
  elas_handle* ph = pair->params ? pair->params : s->h;
  int64_t bytes = 0;
  {
    std::lock_guard<std::mutex> lk(s->m);
    auto key = std::make_tuple(ph, pair->w, pair->h);
    auto it = s->footprint.find(key);
    if (it != s->footprint.end()) bytes = it->second;
  }
  if (bytes == 0) {
    const int rc = elas_frame_bytes(ph, pair->w, pair->h, &bytes);
    if (rc != ELAS_OK) return server_fail(s, rc, "footprint of the pair");
  }
  std::lock_guard<std::mutex> lk(s->m);
  s->footprint[std::make_tuple(ph, pair->w, pair->h)] = bytes;
  if (bytes > s->cfg.memory_budget) {
    s->err = "pair needs more device memory than the whole budget";
    return ELAS_ERR_ARG;
  }
  if (s->stop) {
    s->err = "server is shutting down";
    return ELAS_ERR_ARG;
  }
  hipEvent_t ready = nullptr;
  if (ordered) {  // order the pair after the work already on the producer's stream
    if (!s->free_events.empty()) {
      ready = s->free_events.back();
      s->free_events.pop_back();
    } else {
      const hipError_t e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
      if (e != hipSuccess) {
        s->err = std::string("hipEventCreate: ") + hipGetErrorString(e);
        return ELAS_ERR_HIP;
      }
    }
    const hipError_t e = hipEventRecord(ready, producer);
    if (e != hipSuccess) {
      s->free_events.push_back(ready);
      s->err = std::string("hipEventRecord on the producer stream: ") + hipGetErrorString(e);
      return ELAS_ERR_HIP;
    }
  }
  const int64_t t = s->next_ticket++;
  Result r;
  r.submitted = Clock::now();
  s->results.emplace(t, r);
  s->queue.push_back(Request{t, *pair, bytes, ready});
  s->stats.submitted += 1;
  *ticket = t;
  s->work.notify_one();
  return ELAS_OK;
}

}  // namespace

extern "C" {

int elas_server_submit(elas_server* s, const elas_pair* pair, int64_t* ticket) {
  return submit_pair(s, pair, false, nullptr, ticket);
}

int elas_server_submit_on(elas_server* s, const elas_pair* pair, hipStream_t producer,
                          int64_t* ticket) {
  return submit_pair(s, pair, true, producer, ticket);
}

static int take_result(elas_server* s, std::unordered_map<int64_t, Result>::iterator it,
                       double* latency_ms) {
  const Result r = it->second;
  s->results.erase(it);
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(r.finished - r.submitted).count();
  return r.state == State::Done ? ELAS_OK : r.code;
}

int elas_server_poll(elas_server* s, int64_t ticket, int32_t* done, double* latency_ms) {
  if (!s || !done) return server_fail(s, ELAS_ERR_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) {
    s->err = "unknown ticket";
    return ELAS_ERR_ARG;
  }
  *done = it->second.state != State::Pending;
  if (!*done) return ELAS_OK;
  return take_result(s, it, latency_ms);
}

int elas_server_wait(elas_server* s, int64_t ticket, double* latency_ms) {
  if (!s) return server_fail(nullptr, ELAS_ERR_ARG, "null server");
  std::unique_lock<std::mutex> lk(s->m);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) {
    s->err = "unknown ticket";
    return ELAS_ERR_ARG;
  }
  // submissions may rehash the table while this thread waits: look up again
  s->done.wait(lk, [&] {
    auto i = s->results.find(ticket);
    return i == s->results.end() || i->second.state != State::Pending;
  });
  it = s->results.find(ticket);
  if (it == s->results.end()) {
    s->err = "unknown ticket";
    return ELAS_ERR_ARG;
  }
  return take_result(s, it, latency_ms);
}

int elas_server_get_stats(elas_server* s, elas_server_stats* out) {
  if (!s || !out) return server_fail(s, ELAS_ERR_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->m);
  *out = s->stats;
  out->queued = (int64_t)s->queue.size();
  out->bytes_in_flight = s->in_flight;
  out->resident_bytes = s->resident;
  return ELAS_OK;
}

const char* elas_server_last_error(const elas_server* s) {
  return s ? s->err.c_str() : g_server_error.c_str();
}

int elas_server_destroy(elas_server* s) {
  if (!s) return ELAS_OK;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stop = true;
  }
  s->work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.report_host) (void)hipHostFree(sl.report_host);
  }
  for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
  delete s;
  return ELAS_OK;
}

}  // extern "C"
