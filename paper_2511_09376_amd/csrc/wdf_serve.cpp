// Serving loop: continuous batching of explain requests over a resident
// background summary.
//
// Requests (1..max_rows rows of caller-owned host data) wait in a FIFO queue.
// The server owns a fixed set of batch slots, each with pinned host staging
// and device buffers for batch_rows rows of X and phi, a stream and events;
// the number of slots is what the memory budget pays for (at most four).  A
// worker thread takes a free slot and the oldest queued requests that fit in
// it, has its copy threads pack their rows into the slot's staging, then
// copies the batch in, runs wdf_explain and copies phi back, all
// asynchronously on the slot's stream, so the batches of different slots
// overlap on the device.  A completion thread takes launched slots in launch
// order, waits for each one's last event, has its own copy threads unpack
// each request's rows into its caller's buffer, records the requests'
// latencies (submit to result on host) and frees the slot; packing the next
// batch and unpacking the last one thus run at the same time.  Every row is
// explained independently of the others in its batch, so a request's result
// is bit-identical alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "wdf.h"
#include "wdf_impl.h"

using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0;
  const float *x = nullptr;  // caller's [F][ldx] host rows, valid until the ticket is waited on
  int64_t ldx = 0;
  float *phi_out = nullptr;
  Clock::time_point t_submit;
  bool done = false;
  int status = WDF_OK;
};

// Host threads that split a copy job into parts: run(parts, fn) calls
// fn(0) .. fn(parts - 1) on the helpers and the calling thread and returns
// when all have finished.
class CopyPool {
 public:
  explicit CopyPool(int threads) {
    for (int i = 1; i < threads; ++i) helpers_.emplace_back([this] { loop(); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> lock(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto &t : helpers_) t.join();
  }
  void run(int parts, const std::function<void(int)> &fn) {
    {
      std::lock_guard<std::mutex> lock(mu_);
      fn_ = &fn;
      parts_ = parts;
      next_ = 0;
      done_ = 0;
      ++gen_;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> lock(mu_);
    cv_done_.wait(lock, [&] { return done_ == parts_; });
    fn_ = nullptr;
  }

 private:
  void work() {
    for (;;) {
      int p;
      const std::function<void(int)> *fn;
      {
        std::lock_guard<std::mutex> lock(mu_);
        if (!fn_ || next_ >= parts_) return;
        p = next_++;
        fn = fn_;
      }
      (*fn)(p);
      std::lock_guard<std::mutex> lock(mu_);
      if (++done_ == parts_) cv_done_.notify_all();
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lock(mu_);
        cv_.wait(lock, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
      }
      work();
    }
  }
  std::vector<std::thread> helpers_;
  std::mutex mu_;
  std::condition_variable cv_, cv_done_;
  const std::function<void(int)> *fn_ = nullptr;
  int parts_ = 0, next_ = 0, done_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

struct Slot {
  float *hx = nullptr, *hphi = nullptr;  // pinned [F][batch_rows]
  float *dx = nullptr, *dphi = nullptr;  // device [F][batch_rows]
  hipStream_t stream = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // start, copied in, explained, copied out
  std::vector<std::shared_ptr<Request>> reqs;
  int64_t rows = 0;
  bool busy = false;
  uint64_t seq = 0;  // launch order
};

}  // namespace

struct wdf_server {
  const wdf_bg *bg = nullptr;
  int device = 0;
  int F = 0;
  int64_t max_rows = 0, batch_rows = 0;
  int queue_cap = 0;
  bool one_per_launch = false;
  std::vector<Slot> slots;
  std::unique_ptr<CopyPool> pack_pool, unpack_pool;
  int copy_parts = 1;

  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_launched;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> pending;
  std::deque<Slot *> launched;  // slots on the device, in launch order
  uint64_t next_ticket = 1, next_seq = 1;
  bool stop = false, paused = false, worker_done = false;
  std::thread worker, completer;

  // statistics; latencies of the most recent kLatencyWindow requests (a
  // ring once full), so that a long-running server's memory stays bounded
  static constexpr size_t kLatencyWindow = size_t(1) << 20;
  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, rows = 0;
  std::vector<double> latency_ms;
  uint64_t latency_next = 0;  // ring position once the window is full
  double busy_ms = 0.0, copy_in_ms = 0.0, explain_ms = 0.0, copy_out_ms = 0.0;
  double pack_ms = 0.0, unpack_ms = 0.0;
  bool any_submit = false;
  Clock::time_point first_submit, last_done;
  int worker_error = WDF_OK;

  void run();
  void complete();
  void launch(Slot &s);
  void drain(Slot &s);
  // request offsets inside a slot's batch
  static std::vector<int64_t> offsets(const Slot &s) {
    std::vector<int64_t> off(s.reqs.size());
    int64_t o = 0;
    for (size_t i = 0; i < s.reqs.size(); ++i) off[i] = o, o += s.reqs[i]->n;
    return off;
  }
};

void wdf_server::launch(Slot &s) {
  // pack: the copy threads split the features; request r's feature f goes to
  // column offset off[r] of staging row f
  const std::vector<int64_t> off = offsets(s);
  const auto t0 = Clock::now();
  const size_t ld = (size_t)batch_rows;
  pack_pool->run(copy_parts, [&](int p) {
    const int f0 = (int)((int64_t)F * p / copy_parts), f1 = (int)((int64_t)F * (p + 1) / copy_parts);
    for (size_t i = 0; i < s.reqs.size(); ++i) {
      const Request &r = *s.reqs[i];
      for (int f = f0; f < f1; ++f)
        std::memcpy(s.hx + (size_t)f * ld + (size_t)off[i], r.x + (size_t)f * (size_t)r.ldx, (size_t)r.n * sizeof(float));
    }
  });
  const double pm = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  s.rows = off.empty() ? 0 : off.back() + s.reqs.back()->n;
  const size_t pitch = ld * sizeof(float);
  hipError_t e = hipEventRecord(s.ev[0], s.stream);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(s.dx, pitch, s.hx, pitch, (size_t)s.rows * sizeof(float), (size_t)F, hipMemcpyHostToDevice,
                         s.stream);
  if (e == hipSuccess) e = hipEventRecord(s.ev[1], s.stream);
  int rc = e == hipSuccess ? WDF_OK : wdf::hip_error(e, "server: copy in");
  if (rc == WDF_OK) rc = wdf_explain(bg, s.dx, s.rows, batch_rows, s.dphi, batch_rows, s.stream);
  if (rc == WDF_OK) {
    e = hipEventRecord(s.ev[2], s.stream);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(s.hphi, pitch, s.dphi, pitch, (size_t)s.rows * sizeof(float), (size_t)F,
                           hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.ev[3], s.stream);
    if (e != hipSuccess) rc = wdf::hip_error(e, "server: copy out");
  }
  std::lock_guard<std::mutex> lock(mu);
  pack_ms += pm;
  if (rc != WDF_OK) {
    worker_error = rc;
    for (auto &r : s.reqs) {
      r->status = rc;
      r->done = true;
    }
    s.reqs.clear();
    s.busy = false;
    cv_done.notify_all();
    return;
  }
  s.seq = next_seq++;
  launched.push_back(&s);
  cv_launched.notify_one();
}

void wdf_server::drain(Slot &s) {
  float t[3] = {0.f, 0.f, 0.f};
  for (int k = 0; k < 3; ++k) (void)hipEventElapsedTime(&t[k], s.ev[k], s.ev[k + 1]);
  const std::vector<int64_t> off = offsets(s);
  const auto t0 = Clock::now();
  const size_t ld = (size_t)batch_rows;
  unpack_pool->run(copy_parts, [&](int p) {
    const int f0 = (int)((int64_t)F * p / copy_parts), f1 = (int)((int64_t)F * (p + 1) / copy_parts);
    for (size_t i = 0; i < s.reqs.size(); ++i) {
      const Request &r = *s.reqs[i];
      for (int f = f0; f < f1; ++f)
        std::memcpy(r.phi_out + (size_t)f * (size_t)r.n, s.hphi + (size_t)f * ld + (size_t)off[i],
                    (size_t)r.n * sizeof(float));
    }
  });
  const auto now = Clock::now();
  std::lock_guard<std::mutex> lock(mu);
  unpack_ms += std::chrono::duration<double, std::milli>(now - t0).count();
  copy_in_ms += t[0];
  explain_ms += t[1];
  copy_out_ms += t[2];
  busy_ms += (double)t[0] + (double)t[1] + (double)t[2];
  for (auto &r : s.reqs) {
    r->done = true;
    const double ms = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
    if (latency_ms.size() < kLatencyWindow)
      latency_ms.push_back(ms);
    else
      latency_ms[(size_t)(latency_next++ % kLatencyWindow)] = ms;
    ++completed;
  }
  last_done = now;
  ++batches;
  rows += (uint64_t)s.rows;
  s.reqs.clear();
  s.busy = false;
  cv_done.notify_all();
}

void wdf_server::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lock(mu);
  for (;;) {
    // a free slot and queued requests (FIFO; a batch takes the oldest
    // requests that fit in batch_rows rows), unless paused
    Slot *free_slot = nullptr;
    for (auto &s : slots)
      if (!s.busy) {
        free_slot = &s;
        break;
      }
    if (stop && queue.empty()) break;
    if (paused && !stop) {
      cv_work.wait(lock);
      continue;
    }
    if (queue.empty()) {
      cv_work.wait(lock);
      continue;
    }
    if (!free_slot) {
      cv_done.wait(lock);  // the completion thread frees slots
      continue;
    }
    Slot &s = *free_slot;
    int64_t rows_in = 0;
    while (!queue.empty() && rows_in + queue.front()->n <= batch_rows) {
      rows_in += queue.front()->n;
      s.reqs.push_back(queue.front());
      queue.pop_front();
      if (one_per_launch) break;
    }
    s.busy = true;
    lock.unlock();
    launch(s);  // packs without the lock, takes it to hand the slot over
    lock.lock();
  }
  worker_done = true;
  cv_launched.notify_all();
}

void wdf_server::complete() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lock(mu);
  for (;;) {
    cv_launched.wait(lock, [&] { return !launched.empty() || worker_done; });
    if (launched.empty()) break;  // the worker has stopped and every batch is drained
    Slot *s = launched.front();
    launched.pop_front();
    lock.unlock();
    (void)hipEventSynchronize(s->ev[3]);
    drain(*s);  // unpacks without the lock, takes it to record and free the slot
    lock.lock();
  }
}

extern "C" int wdf_server_create(const wdf_bg *bg, const wdf_server_config *cfg, wdf_server **out) {
  if (!bg || !cfg || !out) return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_create: NULL argument");
  *out = nullptr;
  if (bg->iv) return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_create: serving explains Shapley/Banzhaf values");
  const int64_t max_rows = cfg->max_rows;
  const int64_t batch_rows = cfg->batch_rows > 0 ? cfg->batch_rows : std::max<int64_t>(max_rows, 65536);
  if (max_rows < 1 || cfg->queue_cap < 1 || batch_rows < max_rows || batch_rows > (1 << 24) || cfg->copy_threads < 0 ||
      cfg->copy_threads > 64)
    return wdf::set_error(WDF_E_INVALID_ARG,
                          "wdf_server_create: need max_rows >= 1, max_rows <= batch_rows <= 2^24, queue_cap >= 1, "
                          "0 <= copy_threads <= 64");
  const bool one = (cfg->flags & WDF_SERVE_ONE_PER_LAUNCH) != 0;
  const int F = bg->model->n_features;
  // a plain one-request-per-launch server stages one request at a time
  const int64_t slot_rows = one ? max_rows : batch_rows;
  const size_t per_slot = (size_t)4 * (size_t)F * (size_t)slot_rows * sizeof(float);  // pinned + device, in + out
  const size_t n_slots = one ? 1 : std::min<size_t>(4, cfg->mem_budget / per_slot);
  if (n_slots < 1 || cfg->mem_budget < per_slot)
    return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_create: budget %zu bytes is below one batch slot (%zu bytes)",
                          cfg->mem_budget, per_slot);
  hipError_t e = hipSetDevice(bg->device);
  if (e != hipSuccess) return wdf::hip_error(e, "hipSetDevice");
  std::unique_ptr<wdf_server> S(new (std::nothrow) wdf_server());
  if (!S) return wdf::set_error(WDF_E_OOM, "wdf_server_create: out of host memory");
  S->bg = bg;
  S->device = bg->device;
  S->F = F;
  S->max_rows = max_rows;
  S->batch_rows = slot_rows;
  S->queue_cap = cfg->queue_cap;
  S->one_per_launch = one;
  S->paused = (cfg->flags & WDF_SERVE_START_PAUSED) != 0;
  const int threads = cfg->copy_threads > 0 ? cfg->copy_threads : 4;
  S->copy_parts = std::min(threads, F);
  S->pack_pool.reset(new CopyPool(S->copy_parts));
  S->unpack_pool.reset(new CopyPool(S->copy_parts));
  S->slots.resize(n_slots);
  const size_t bytes = (size_t)F * (size_t)slot_rows * sizeof(float);
  for (auto &s : S->slots) {
    if ((e = hipHostMalloc((void **)&s.hx, bytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&s.hphi, bytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipMalloc((void **)&s.dx, bytes)) != hipSuccess || (e = hipMalloc((void **)&s.dphi, bytes)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess) {
      wdf_server_destroy(S.release());
      return wdf::set_error(WDF_E_OOM, "wdf_server_create: %s", hipGetErrorString(e));
    }
    for (auto &ev : s.ev)
      if ((e = hipEventCreate(&ev)) != hipSuccess) {
        wdf_server_destroy(S.release());
        return wdf::set_error(WDF_E_OOM, "wdf_server_create: %s", hipGetErrorString(e));
      }
  }
  wdf_server *raw = S.release();
  raw->worker = std::thread([raw] { raw->run(); });
  raw->completer = std::thread([raw] { raw->complete(); });
  *out = raw;
  return WDF_OK;
}

extern "C" int wdf_server_pause(wdf_server *srv, int paused) {
  if (!srv) return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_pause: NULL server");
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->paused = paused != 0;
  }
  srv->cv_work.notify_all();
  return WDF_OK;
}

extern "C" int wdf_server_submit(wdf_server *srv, const float *X_host, int64_t n, int64_t ldx, float *phi_host,
                                 uint64_t *ticket) {
  if (!srv || !X_host || !phi_host || !ticket) return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_submit: NULL argument");
  if (n < 1 || n > srv->max_rows || ldx < n)
    return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_submit: need 1 <= n <= max_rows (%lld) and ldx >= n",
                          (long long)srv->max_rows);
  auto r = std::make_shared<Request>();
  r->n = n;
  r->x = X_host;
  r->ldx = ldx;
  r->phi_out = phi_host;
  std::lock_guard<std::mutex> lock(srv->mu);
  if ((int)srv->queue.size() >= srv->queue_cap) {
    ++srv->rejected;
    return wdf::set_error(WDF_E_BUSY, "wdf_server_submit: queue full (%d requests)", srv->queue_cap);
  }
  r->ticket = srv->next_ticket++;
  r->t_submit = Clock::now();
  if (!srv->any_submit) srv->first_submit = r->t_submit, srv->any_submit = true;
  srv->pending[r->ticket] = r;
  srv->queue.push_back(r);
  ++srv->submitted;
  *ticket = r->ticket;
  srv->cv_work.notify_one();
  return WDF_OK;
}

extern "C" int wdf_server_wait(wdf_server *srv, uint64_t ticket, int timeout_ms) {
  if (!srv) return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_wait: NULL server");
  std::unique_lock<std::mutex> lock(srv->mu);
  auto it = srv->pending.find(ticket);
  if (it == srv->pending.end()) return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_wait: unknown ticket %llu",
                                                        (unsigned long long)ticket);
  std::shared_ptr<Request> r = it->second;
  auto ready = [&] { return r->done; };
  if (timeout_ms < 0) srv->cv_done.wait(lock, ready);
  else if (!srv->cv_done.wait_for(lock, std::chrono::milliseconds(timeout_ms), ready))
    return wdf::set_error(WDF_E_TIMEOUT, "wdf_server_wait: ticket %llu not done after %d ms",
                          (unsigned long long)ticket, timeout_ms);
  srv->pending.erase(ticket);
  if (r->status != WDF_OK) return wdf::set_error(r->status, "wdf_server_wait: the batch failed");
  return WDF_OK;
}

extern "C" int wdf_server_stats(wdf_server *srv, wdf_stats *out) {
  if (!srv || !out) return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_stats: NULL argument");
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->batches = srv->batches;
    out->rows = srv->rows;
    out->busy_ms = srv->busy_ms;
    out->copy_in_ms = srv->copy_in_ms;
    out->explain_ms = srv->explain_ms;
    out->copy_out_ms = srv->copy_out_ms;
    out->pack_ms = srv->pack_ms;
    out->unpack_ms = srv->unpack_ms;
    out->active_ms = (srv->any_submit && srv->completed)
                         ? std::chrono::duration<double, std::milli>(srv->last_done - srv->first_submit).count()
                         : 0.0;
    out->slots = (int)srv->slots.size();
    out->batch_rows = srv->batch_rows;
    lat = srv->latency_ms;
  }
  out->p50_ms = out->p99_ms = out->mean_ms = out->max_ms = 0.0;
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto q = [&](double p) {  // nearest-rank percentile
      size_t k = (size_t)std::ceil(p * (double)lat.size());
      k = std::min(std::max<size_t>(k, 1), lat.size());
      return lat[k - 1];
    };
    out->p50_ms = q(0.50);
    out->p99_ms = q(0.99);
    double s = 0.0;
    for (double v : lat) s += v;
    out->mean_ms = s / (double)lat.size();
    out->max_ms = lat.back();
  }
  return WDF_OK;
}

extern "C" void wdf_server_destroy(wdf_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->stop = true;
    srv->paused = false;  // queued requests are explained before the worker stops
  }
  srv->cv_work.notify_all();
  srv->cv_done.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  if (srv->completer.joinable()) srv->completer.join();
  (void)hipSetDevice(srv->device);
  for (auto &s : srv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    for (auto &ev : s.ev)
      if (ev) (void)hipEventDestroy(ev);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.dx) (void)hipFree(s.dx);
    if (s.dphi) (void)hipFree(s.dphi);
    if (s.hx) (void)hipHostFree(s.hx);
    if (s.hphi) (void)hipHostFree(s.hphi);
  }
  // requests still queued at destruction complete with an error
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    for (auto &r : srv->queue) {
      r->status = WDF_E_INVALID_ARG;
      r->done = true;
    }
    srv->cv_done.notify_all();
  }
  delete srv;
}
