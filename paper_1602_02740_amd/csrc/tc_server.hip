// tc_server.hip -- the serving loop of libtoom.so: continuous batching of
// product requests on one device.
//
// A scheduler thread owns a few HIP streams.  Requests wait in a FIFO queue;
// whenever a stream is free and the HBM budget allows, the oldest request is
// launched together with the queued requests of the same size (one merged
// launch through tc_mul_batch, section 2: the products are independent).
// Only products below kMergeLimbs are merged, and a batch takes a power of
// two of them: every merged shape is a compiled plan with scratch of its own,
// so this keeps the shapes (at most log2(max_batch) + 1 per size) and their
// device memory bounded, while a product of kMergeLimbs or more fills the
// device alone.
// Admission counts the plan scratch of the work in flight against the budget;
// the scratch itself stays device-resident in the plan cache between
// requests.  Batches on different streams overlap on the device, and requests
// that arrive meanwhile are admitted as streams and budget free up.  Each
// batch reports its items' exactness status into its stream's own pinned
// array, so an error is charged to exactly the request that had it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

#include "toom.h"

namespace {

using Clock = std::chrono::steady_clock;

// Operand width (limbs) from which a request runs as a batch of its own.
constexpr size_t kMergeLimbs = (size_t)1 << 16;

struct Request {
  uint64_t ticket;
  tc_mul_desc d;
  size_t bytes;
  double t_submit;
};

struct Batch {
  std::vector<Request> reqs;
  int stream;
  hipEvent_t ev = nullptr;
  double t_start;
  size_t bytes;
};

}  // namespace

struct tc_server {
  int dev = 0;
  size_t budget = 0, max_inflight = 0, max_queued = 0;
  int max_batch = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> pending;
  std::vector<Batch> inflight;
  std::unordered_set<uint64_t> live;                 // queued or in flight
  std::unordered_map<uint64_t, tc_result> finished;  // done, not yet polled
  std::map<std::pair<size_t, size_t>, size_t> footprint;  // scratch per size
  std::vector<hipStream_t> streams;
  std::vector<int32_t*> stat;  // per stream: pinned per-item status of its batch
  std::vector<bool> busy;
  std::vector<hipEvent_t> free_events;
  uint64_t next_ticket = 1;
  bool stop = false;
  // statistics
  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0;
  size_t inflight_reqs = 0, inflight_bytes = 0;
  double first_submit = -1.0, last_finish = 0.0, work = 0.0;
  std::vector<double> lat;
  std::thread thr;

  double now() const {
    return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
  }
  void run();
  void reap(std::unique_lock<std::mutex>& lk);
  bool admit(std::unique_lock<std::mutex>& lk);
};

// Completed batches: results (each request's status from its batch's
// status array), statistics, budget back.
void tc_server::reap(std::unique_lock<std::mutex>&) {
  std::vector<Batch> done;
  for (size_t i = 0; i < inflight.size();) {
    if (hipEventQuery(inflight[i].ev) == hipSuccess) {
      done.push_back(std::move(inflight[i]));
      inflight.erase(inflight.begin() + (long)i);
    } else {
      ++i;
    }
  }
  (void)hipGetLastError();
  if (done.empty()) return;
  const double t = now();
  for (auto& b : done) {
    for (size_t i = 0; i < b.reqs.size(); i++) {
      const Request& r = b.reqs[i];
      tc_result res;
      res.status = stat[(size_t)b.stream][i];
      res.submit_us = r.t_submit;
      res.start_us = b.t_start;
      res.finish_us = t;
      finished[r.ticket] = res;
      live.erase(r.ticket);
      completed++;
      lat.push_back(t - r.t_submit);
      work += (double)r.d.nu * (double)r.d.nv;
    }
    last_finish = t;
    inflight_reqs -= b.reqs.size();
    inflight_bytes -= b.bytes;
    busy[(size_t)b.stream] = false;
    free_events.push_back(b.ev);
  }
}

// Launches queued work while a stream, request slots and budget are free.
// Returns true if anything was launched.
bool tc_server::admit(std::unique_lock<std::mutex>& lk) {
  bool any = false;
  while (!pending.empty() && inflight_reqs < max_inflight) {
    int st = -1;
    for (size_t i = 0; i < busy.size(); i++)
      if (!busy[i]) {
        st = (int)i;
        break;
      }
    if (st < 0) break;
    // the oldest request and the queued requests of its size
    const size_t nu = pending.front().d.nu, nv = pending.front().d.nv;
    const size_t room = std::max(nu, nv) >= kMergeLimbs
                            ? 1
                            : std::min(max_inflight - inflight_reqs, (size_t)max_batch);
    std::vector<size_t> take;
    size_t bytes = 0;
    for (size_t i = 0; i < pending.size() && take.size() < room; i++) {
      const Request& r = pending[i];
      if (r.d.nu != nu || r.d.nv != nv) continue;
      if (!inflight.empty() || !take.empty())
        if (inflight_bytes + bytes + r.bytes > budget) break;
      take.push_back(i);
      bytes += r.bytes;
    }
    if (take.empty()) break;  // wait for memory to free up
    size_t keep = 1;  // the oldest power of two of them
    while (keep * 2 <= take.size()) keep *= 2;
    take.resize(keep);
    bytes = 0;
    for (const size_t i : take) bytes += pending[i].bytes;
    Batch b;
    b.stream = st;
    b.bytes = bytes;
    std::vector<tc_mul_desc> ds;
    for (size_t k = take.size(); k-- > 0;) {
      b.reqs.push_back(pending[take[k]]);
      pending.erase(pending.begin() + (long)take[k]);
    }
    std::reverse(b.reqs.begin(), b.reqs.end());
    for (auto& r : b.reqs) ds.push_back(r.d);
    if (free_events.empty()) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr;
      free_events.push_back(e);
    }
    b.ev = free_events.back();
    free_events.pop_back();
    b.t_start = now();
    busy[(size_t)st] = true;
    // launch without the lock: a first-seen batch shape compiles its plan
    // here, and submit/poll must not wait for that
    int rc = b.ev ? TC_OK : TC_ERR_HIP;
    lk.unlock();
    if (rc == TC_OK) rc = tc_mul_batch(ds.data(), ds.size(), stat[(size_t)st], streams[(size_t)st]);
    if (rc == TC_OK && hipEventRecord(b.ev, streams[(size_t)st]) != hipSuccess) rc = TC_ERR_HIP;
    lk.lock();
    if (rc != TC_OK) {
      // nothing usable was enqueued for these requests: fail them now
      const double t = now();
      for (auto& r : b.reqs) {
        tc_result res{rc, r.t_submit, b.t_start, t};
        finished[r.ticket] = res;
        live.erase(r.ticket);
        completed++;
      }
      if (b.ev) free_events.push_back(b.ev);
      busy[(size_t)st] = false;
      continue;
    }
    inflight_reqs += b.reqs.size();
    inflight_bytes += b.bytes;
    batches++;
    inflight.push_back(std::move(b));
    any = true;
  }
  return any;
}

void tc_server::run() {
  (void)hipSetDevice(dev);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    reap(lk);
    const bool launched = admit(lk);
    if (stop && pending.empty() && inflight.empty()) break;
    if (!launched) {
      // in-flight work is polled every few microseconds; an idle server
      // sleeps until a submit wakes it
      if (inflight.empty())
        cv.wait_for(lk, std::chrono::milliseconds(50));
      else
        cv.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

extern "C" {

int tc_server_create(const tc_server_cfg* cfg, tc_server** out) {
  if (!out) return TC_ERR_INVALID;
  *out = nullptr;
  tc_server_cfg c{};
  if (cfg) c = *cfg;
  int rc = tc_init();
  if (rc != TC_OK) return rc;
  auto* s = new (std::nothrow) tc_server;
  if (!s) return TC_ERR_NOMEM;
  if (hipGetDevice(&s->dev) != hipSuccess) {
    delete s;
    return TC_ERR_HIP;
  }
  if (c.hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      return TC_ERR_HIP;
    }
    c.hbm_budget = fr / 4;
  }
  s->budget = c.hbm_budget;
  s->max_inflight = c.max_inflight ? c.max_inflight : 256;
  s->max_queued = c.max_queued ? c.max_queued : 4096;
  s->max_batch = c.max_batch > 0 ? c.max_batch : 64;
  const int ns = c.streams > 0 ? c.streams : 4;
  for (int i = 0; i < ns; i++) {
    hipStream_t st;
    int32_t* h = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&h), (size_t)s->max_batch * sizeof(int32_t),
                      hipHostMallocDefault) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      for (auto x : s->stat) (void)hipHostFree(x);
      delete s;
      return TC_ERR_HIP;
    }
    s->streams.push_back(st);
    s->stat.push_back(h);
    s->busy.push_back(false);
  }
  s->t0 = Clock::now();
  s->thr = std::thread([s] { s->run(); });
  *out = s;
  return TC_OK;
}

int tc_submit(tc_server* s, tc_limb* w, const tc_limb* u, size_t nu, const tc_limb* v, size_t nv,
              uint64_t* ticket) {
  if (!s || !w || !u || !v || nu == 0 || nv == 0 || !ticket) return TC_ERR_INVALID;
  if (nu > ((size_t)1 << 31) || nv > ((size_t)1 << 31)) return TC_ERR_UNSUPPORTED;
  const uintptr_t W = (uintptr_t)w, U = (uintptr_t)u, V = (uintptr_t)v;
  const uintptr_t WE = W + (nu + nv) * 4;
  if ((U < WE && W < U + nu * 4) || (V < WE && W < V + nv * 4)) return TC_ERR_INVALID;
  size_t bytes = 0;
  bool known;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->footprint.find({nu, nv});
    known = it != s->footprint.end();
    if (known) bytes = it->second;
  }
  // a dry run of the default plan, once per size (0: the product is a single
  // leaf without scratch; an unsupported size fails at launch with its status)
  if (!known) bytes = tc_workspace_bytes(nu, nv);
  std::lock_guard<std::mutex> lk(s->mu);
  s->footprint[{nu, nv}] = bytes;
  if (bytes > s->budget) {
    s->rejected++;
    return TC_ERR_NOMEM;
  }
  if (s->pending.size() >= s->max_queued) {
    s->rejected++;
    return TC_ERR_AGAIN;
  }
  Request r;
  r.ticket = s->next_ticket++;
  r.d.w = w;
  r.d.u = u;
  r.d.nu = nu;
  r.d.v = v;
  r.d.nv = nv;
  r.bytes = bytes;
  r.t_submit = s->now();
  if (s->first_submit < 0) s->first_submit = r.t_submit;
  s->pending.push_back(r);
  s->live.insert(r.ticket);
  s->submitted++;
  *ticket = r.ticket;
  s->cv.notify_one();
  return TC_OK;
}

int tc_poll(tc_server* s, uint64_t ticket, tc_result* r) {
  if (!s || !r) return TC_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->finished.find(ticket);
  if (it != s->finished.end()) {
    *r = it->second;
    s->finished.erase(it);
    return TC_OK;
  }
  return s->live.count(ticket) ? TC_ERR_NOT_READY : TC_ERR_INVALID;
}

int tc_server_stats(tc_server* s, tc_stats* out) {
  if (!s || !out) return TC_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  tc_stats st{};
  st.submitted = s->submitted;
  st.completed = s->completed;
  st.rejected = s->rejected;
  st.batches = s->batches;
  st.queued = s->pending.size();
  st.inflight = s->inflight_reqs;
  st.inflight_bytes = s->inflight_bytes;
  if (!s->lat.empty()) {
    std::vector<double> l = s->lat;
    auto pct = [&](double q) {
      const size_t k = std::min(l.size() - 1, (size_t)(q * (double)(l.size() - 1) + 0.5));
      std::nth_element(l.begin(), l.begin() + (long)k, l.end());
      return l[k];
    };
    st.p50_us = pct(0.50);
    st.p99_us = pct(0.99);
  }
  if (s->completed > 0 && s->last_finish > s->first_submit) {
    st.window_s = (s->last_finish - s->first_submit) * 1e-6;
    st.limb_mults_per_s = s->work / st.window_s;
  }
  *out = st;
  return TC_OK;
}

int tc_server_reset_stats(tc_server* s) {
  if (!s) return TC_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  s->submitted = s->completed = s->rejected = s->batches = 0;
  s->first_submit = -1.0;
  s->last_finish = 0.0;
  s->work = 0.0;
  s->lat.clear();
  return TC_OK;
}

int tc_server_destroy(tc_server* s) {
  if (!s) return TC_ERR_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_one();
  }
  if (s->thr.joinable()) s->thr.join();
  for (auto e : s->free_events)
    if (e) (void)hipEventDestroy(e);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  for (auto h : s->stat) (void)hipHostFree(h);
  delete s;
  return TC_OK;
}

}  // extern "C"
