// Serving loop: continuous batching of explain requests over a resident
// background summary.
//
// Requests (1..max_rows rows of caller-owned host data) wait in a FIFO queue.  A worker
// thread owns a fixed set of slots, each with pinned host staging, device
// buffers for X and phi, a stream and an event; the number of slots is what
// the memory budget pays for.  Whenever a slot is free the worker packs the
// oldest queued requests that fit in max_rows rows into it, copies the batch
// in, runs wdf_explain and copies phi back, all asynchronously on the slot's
// stream, so the batches of different slots overlap on the device.  A slot
// whose event has completed is drained: each request's rows are copied to its
// caller's buffer and its latency (submit to result on host) is recorded.
// Every row is explained independently of the others in its batch, so a
// request's result is bit-identical alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
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

struct Slot {
  float *hx = nullptr, *hphi = nullptr;  // pinned [F][max_rows]
  float *dx = nullptr, *dphi = nullptr;  // device [F][max_rows]
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, done = nullptr;
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
  int64_t max_rows = 0;
  int queue_cap = 0;
  bool one_per_launch = false;
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> pending;
  uint64_t next_ticket = 1, next_seq = 1;
  bool stop = false;
  std::thread worker;

  // statistics; latencies of the most recent kLatencyWindow requests (a
  // ring once full), so that a long-running server's memory stays bounded
  static constexpr size_t kLatencyWindow = size_t(1) << 20;
  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, rows = 0;
  std::vector<double> latency_ms;
  uint64_t latency_next = 0;  // ring position once the window is full
  double busy_ms = 0.0;
  int worker_error = WDF_OK;

  void run();
  void launch(Slot &s);
  void drain(Slot &s);
};

void wdf_server::launch(Slot &s) {
  // pack: request r's feature f goes to column offset `off` of row f
  int64_t off = 0;
  for (auto &r : s.reqs) {
    for (int f = 0; f < F; ++f)
      std::memcpy(s.hx + (size_t)f * (size_t)max_rows + (size_t)off, r->x + (size_t)f * (size_t)r->ldx,
                  (size_t)r->n * sizeof(float));
    off += r->n;
  }
  s.rows = off;
  const size_t pitch = (size_t)max_rows * sizeof(float);
  hipError_t e = hipEventRecord(s.start, s.stream);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(s.dx, pitch, s.hx, pitch, (size_t)off * sizeof(float), (size_t)F,
                                  hipMemcpyHostToDevice, s.stream);
  int rc = e == hipSuccess ? WDF_OK : wdf::hip_error(e, "server: copy in");
  if (rc == WDF_OK) rc = wdf_explain(bg, s.dx, off, max_rows, s.dphi, max_rows, s.stream);
  if (rc == WDF_OK) {
    e = hipMemcpy2DAsync(s.hphi, pitch, s.dphi, pitch, (size_t)off * sizeof(float), (size_t)F, hipMemcpyDeviceToHost,
                         s.stream);
    if (e != hipSuccess) rc = wdf::hip_error(e, "server: copy out");
  }
  if (rc == WDF_OK && (e = hipEventRecord(s.done, s.stream)) != hipSuccess) rc = wdf::hip_error(e, "server: event");
  if (rc != WDF_OK) {
    std::lock_guard<std::mutex> lock(mu);
    worker_error = rc;
    for (auto &r : s.reqs) {
      r->status = rc;
      r->done = true;
    }
    s.reqs.clear();
    cv_done.notify_all();
    return;
  }
  s.busy = true;
  s.seq = next_seq++;
}

void wdf_server::drain(Slot &s) {
  int64_t off = 0;
  for (auto &r : s.reqs) {
    for (int f = 0; f < F; ++f)
      std::memcpy(r->phi_out + (size_t)f * (size_t)r->n, s.hphi + (size_t)f * (size_t)max_rows + (size_t)off,
                  (size_t)r->n * sizeof(float));
    off += r->n;
  }
  const auto now = Clock::now();
  std::lock_guard<std::mutex> lock(mu);
  for (auto &r : s.reqs) {
    r->done = true;
    const double ms = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
    if (latency_ms.size() < kLatencyWindow)
      latency_ms.push_back(ms);
    else
      latency_ms[(size_t)(latency_next++ % kLatencyWindow)] = ms;
    ++completed;
  }
  ++batches;
  rows += (uint64_t)s.rows;
  s.reqs.clear();
  s.busy = false;
  cv_done.notify_all();
}

void wdf_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    // 1. fill free slots from the queue (FIFO; a batch takes the oldest
    //    requests that fit in max_rows rows)
    std::vector<Slot *> to_launch;
    {
      std::lock_guard<std::mutex> lock(mu);
      for (auto &s : slots) {
        if (s.busy || queue.empty()) continue;
        int64_t rows_in = 0;
        while (!queue.empty() && rows_in + queue.front()->n <= max_rows) {
          rows_in += queue.front()->n;
          s.reqs.push_back(queue.front());
          queue.pop_front();
          if (one_per_launch) break;
        }
        if (!s.reqs.empty()) to_launch.push_back(&s);
      }
    }
    for (Slot *s : to_launch) launch(*s);
    // 2. drain every finished slot
    for (auto &s : slots) {
      if (!s.busy || hipEventQuery(s.done) != hipSuccess) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, s.start, s.done) == hipSuccess) {
        std::lock_guard<std::mutex> lock(mu);
        busy_ms += ms;
      }
      drain(s);
    }
    // 3. wait for something to do
    Slot *oldest = nullptr;
    bool any_free = false;
    for (auto &s : slots) {
      if (!s.busy) any_free = true;
      else if (!oldest || s.seq < oldest->seq) oldest = &s;
    }
    std::unique_lock<std::mutex> lock(mu);
    if (!oldest) {
      cv_work.wait(lock, [&] { return stop || !queue.empty(); });
      if (stop && queue.empty()) break;
    } else if (!any_free) {
      lock.unlock();
      (void)hipEventSynchronize(oldest->done);
    } else if (queue.empty()) {
      // a batch is in flight and a slot is free: wake on a new request or
      // shortly after, to collect the batch
      cv_work.wait_for(lock, std::chrono::microseconds(100), [&] { return stop || !queue.empty(); });
    }
  }
}

extern "C" int wdf_server_create(const wdf_bg *bg, size_t mem_budget, int max_rows, int queue_cap, int flags,
                                 wdf_server **out) {
  if (!bg || !out) return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_create: NULL argument");
  *out = nullptr;
  if (bg->iv) return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_create: serving explains Shapley/Banzhaf values");
  if (max_rows < 1 || queue_cap < 1)
    return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_create: max_rows and queue_cap must be >= 1");
  const int F = bg->model->n_features;
  const size_t per_slot = (size_t)4 * (size_t)F * (size_t)max_rows * sizeof(float);  // pinned + device, in + out
  const size_t n_slots = std::min<size_t>(4, mem_budget / per_slot);
  if (n_slots < 1)
    return wdf::set_error(WDF_E_INVALID_ARG, "wdf_server_create: budget %zu bytes is below one batch slot (%zu bytes)",
                          mem_budget, per_slot);
  hipError_t e = hipSetDevice(bg->device);
  if (e != hipSuccess) return wdf::hip_error(e, "hipSetDevice");
  std::unique_ptr<wdf_server> S(new (std::nothrow) wdf_server());
  if (!S) return wdf::set_error(WDF_E_OOM, "wdf_server_create: out of host memory");
  S->bg = bg;
  S->device = bg->device;
  S->F = F;
  S->max_rows = max_rows;
  S->queue_cap = queue_cap;
  S->one_per_launch = (flags & WDF_SERVE_ONE_PER_LAUNCH) != 0;
  S->slots.resize(n_slots);
  const size_t bytes = (size_t)F * (size_t)max_rows * sizeof(float);
  for (auto &s : S->slots) {
    if ((e = hipHostMalloc((void **)&s.hx, bytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&s.hphi, bytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipMalloc((void **)&s.dx, bytes)) != hipSuccess || (e = hipMalloc((void **)&s.dphi, bytes)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreate(&s.start)) != hipSuccess || (e = hipEventCreate(&s.done)) != hipSuccess) {
      wdf_server_destroy(S.release());
      return wdf::set_error(WDF_E_OOM, "wdf_server_create: %s", hipGetErrorString(e));
    }
  }
  wdf_server *raw = S.release();
  raw->worker = std::thread([raw] { raw->run(); });
  *out = raw;
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
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  (void)hipSetDevice(srv->device);
  for (auto &s : srv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    if (s.start) (void)hipEventDestroy(s.start);
    if (s.done) (void)hipEventDestroy(s.done);
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
