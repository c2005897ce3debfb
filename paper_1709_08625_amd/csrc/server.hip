// Serving runtime: a request loop over many likelihood evaluations with a
// pool of worker threads, one HIP stream each, admission by a device-memory
// estimate, and resident data sets for repeated evaluations on the same
// locations (the optimiser's outer loop, Sec. 4 of the paper).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hcov.h"

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// stream-ordered device allocation for the contexts of one stream
void* async_alloc(size_t bytes, void* user) {
  void* p = nullptr;
  if (hipMallocAsync(&p, bytes, (hipStream_t)user) != hipSuccess) return nullptr;
  return p;
}
void async_free(void* p, void* user) { (void)hipFreeAsync(p, (hipStream_t)user); }

struct Request {
  uint64_t id;
  std::vector<double> locs, z;
  int64_t n;
  hcov_theta theta;
  double eps;
  int leaf;
  double eta;
  int dataset;
  size_t est;
  double t_submit;
};

struct Dataset {
  hcov_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  size_t bytes = 0;
  bool busy = false;
  bool released = false;
  int queued = 0;
};

}  // namespace

struct hcov_server {
  int device = 0;
  size_t budget = 0;
  hcov_opts opts{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> queue;
  std::unordered_map<uint64_t, hcov_result> done;
  std::unordered_map<uint64_t, int> live;   // queued or running tickets
  std::unordered_map<int, Dataset> datasets;
  size_t in_use = 0;
  int running = 0;
  bool stop = false;
  uint64_t next_ticket = 1;
  int next_dataset = 1;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;

  // index of the next request to admit, or -1 (caller holds mu).  Requests
  // are taken in arrival order; one whose data set is busy is passed over
  // (order within a data set is kept); the first request whose memory does
  // not fit blocks everything behind it, unless nothing is running.
  long pick() {
    for (size_t i = 0; i < queue.size(); ++i) {
      const Request& r = queue[i];
      if (r.dataset) {
        auto it = datasets.find(r.dataset);
        if (it != datasets.end() && it->second.busy) continue;
        return long(i);
      }
      if (in_use + r.est <= budget || running == 0) return long(i);
      return -1;
    }
    return -1;
  }

  void finish(uint64_t id, const hcov_result& res) {
    done[id] = res;
    live.erase(id);
  }

  void work(int slot) {
    (void)hipSetDevice(device);
    hipStream_t st = streams[slot];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      long i = -1;
      cv_work.wait(lk, [&] { return stop || (i = pick()) >= 0; });
      if (stop) return;
      Request r = std::move(queue[size_t(i)]);
      queue.erase(queue.begin() + i);
      running += 1;
      Dataset* ds = nullptr;
      if (r.dataset) {
        ds = &datasets[r.dataset];
        ds->busy = true;
      } else {
        in_use += r.est;
      }
      const double t_adm = now_ms();
      lk.unlock();

      hcov_result res{};
      res.loglik = res.logdet = res.quad = 0.0;
      if (ds) {
        int rc = hcov_set_theta(ds->ctx, r.theta);
        if (rc == HCOV_OK) rc = hcov_loglik(ds->ctx, r.z.data(), HCOV_HOST, &res.loglik, &res.logdet, &res.quad);
        res.status = rc;
      } else {
        hcov_opts o = opts;
        o.alloc = async_alloc;
        o.free = async_free;
        o.alloc_user = (void*)st;
        o.use_graphs = 0;   // a one-shot context would not replay a captured sweep
        o.autotune = 0;     // nor profit from timing its GEMM launches
        hcov_ctx* c = nullptr;
        int rc = hcov_build(r.locs.data(), r.n, r.theta, r.eps, r.leaf, r.eta, &o, (void*)st, &c);
        if (rc == HCOV_OK || rc == HCOV_ERANK) {
          rc = hcov_loglik(c, r.z.data(), HCOV_HOST, &res.loglik, &res.logdet, &res.quad);
        }
        if (c) hcov_destroy(c);
        (void)hipStreamSynchronize(st);
        res.status = rc;
      }
      const double t_end = now_ms();
      res.queue_ms = t_adm - r.t_submit;
      res.service_ms = t_end - t_adm;
      res.latency_ms = t_end - r.t_submit;

      lk.lock();
      running -= 1;
      if (ds) {
        ds->busy = false;
        ds->queued -= 1;
      } else {
        in_use -= r.est;
      }
      finish(r.id, res);
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

int hcov_server_create(int slots, size_t mem_budget_bytes, const hcov_opts* opts, hcov_server** out) {
  if (!out) return HCOV_EINVAL;
  *out = nullptr;
  if (slots < 1 || slots > 64) return HCOV_EINVAL;
  auto* s = new hcov_server();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return HCOV_EDEVICE;
  }
  hcov_opts_default(&s->opts);
  if (opts) s->opts = *opts;
  if (mem_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      return HCOV_EDEVICE;
    }
    mem_budget_bytes = size_t(0.9 * double(fr));
  }
  s->budget = mem_budget_bytes;
  s->streams.resize(size_t(slots), nullptr);
  for (int i = 0; i < slots; ++i) {
    if (hipStreamCreateWithFlags(&s->streams[size_t(i)], hipStreamNonBlocking) != hipSuccess) {
      for (auto st : s->streams)
        if (st) (void)hipStreamDestroy(st);
      delete s;
      return HCOV_EDEVICE;
    }
  }
  for (int i = 0; i < slots; ++i) s->workers.emplace_back([s, i] { s->work(i); });
  *out = s;
  return HCOV_OK;
}

int hcov_server_dataset(hcov_server* s, const double* locs, int64_t n, hcov_theta theta, double eps, int leaf,
                        double eta, int* id) {
  if (!s || !locs || !id) return HCOV_EINVAL;
  size_t est = 0;
  int rc = hcov_estimate_bytes(locs, n, eps, leaf, eta, &s->opts, &est);
  if (rc != HCOV_OK) return rc;
  Dataset d;
  d.n = n;
  d.bytes = est;
  if (hipStreamCreateWithFlags(&d.stream, hipStreamNonBlocking) != hipSuccess) return HCOV_EDEVICE;
  hcov_opts o = s->opts;
  o.alloc = async_alloc;
  o.free = async_free;
  o.alloc_user = (void*)d.stream;
  rc = hcov_build(locs, n, theta, eps, leaf, eta, &o, (void*)d.stream, &d.ctx);
  if (rc != HCOV_OK && rc != HCOV_ERANK) {
    if (d.ctx) hcov_destroy(d.ctx);
    (void)hipStreamSynchronize(d.stream);
    (void)hipStreamDestroy(d.stream);
    return rc;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  *id = s->next_dataset++;
  s->in_use += est;
  s->datasets[*id] = d;
  return HCOV_OK;
}

int hcov_server_release(hcov_server* s, int id) {
  if (!s) return HCOV_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->datasets.find(id);
  if (it == s->datasets.end() || it->second.released) return HCOV_EINVAL;
  it->second.released = true;
  s->cv_done.wait(lk, [&] { return it->second.queued == 0 && !it->second.busy; });
  Dataset d = it->second;
  s->datasets.erase(it);
  s->in_use -= d.bytes;
  lk.unlock();
  hcov_destroy(d.ctx);
  (void)hipStreamSynchronize(d.stream);
  (void)hipStreamDestroy(d.stream);
  s->cv_work.notify_all();
  return HCOV_OK;
}

int hcov_server_submit(hcov_server* s, const hcov_request* q, uint64_t* ticket) {
  if (!s || !q || !ticket || !q->z || q->n < 1) return HCOV_EINVAL;
  Request r;
  r.n = q->n;
  r.theta = q->theta;
  r.eps = q->eps;
  r.leaf = q->leaf;
  r.eta = q->eta;
  r.dataset = q->dataset;
  r.est = 0;
  if (!q->dataset) {
    if (!q->locs) return HCOV_EINVAL;
    int rc = hcov_estimate_bytes(q->locs, q->n, q->eps, q->leaf, q->eta, &s->opts, &r.est);
    if (rc != HCOV_OK) return rc;
    r.locs.assign(q->locs, q->locs + 2 * q->n);
  }
  r.z.assign(q->z, q->z + q->n);
  std::lock_guard<std::mutex> lk(s->mu);
  if (q->dataset) {
    auto it = s->datasets.find(q->dataset);
    if (it == s->datasets.end() || it->second.released || it->second.n != q->n) return HCOV_EINVAL;
    it->second.queued += 1;
  }
  r.id = s->next_ticket++;
  r.t_submit = now_ms();
  *ticket = r.id;
  s->live[r.id] = 1;
  s->queue.push_back(std::move(r));
  s->cv_work.notify_one();
  return HCOV_OK;
}

int hcov_server_poll(hcov_server* s, uint64_t ticket, hcov_result* out) {
  if (!s || !out) return HCOV_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->done.find(ticket);
  if (it != s->done.end()) {
    *out = it->second;
    s->done.erase(it);
    return HCOV_OK;
  }
  return s->live.count(ticket) ? HCOV_EAGAIN : HCOV_EINVAL;
}

int hcov_server_wait(hcov_server* s, uint64_t ticket, hcov_result* out) {
  if (!s || !out) return HCOV_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->done.count(ticket) && !s->live.count(ticket)) return HCOV_EINVAL;
  s->cv_done.wait(lk, [&] { return s->done.count(ticket) > 0; });
  *out = s->done[ticket];
  s->done.erase(ticket);
  return HCOV_OK;
}

void hcov_server_destroy(hcov_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->datasets) {
    hcov_destroy(kv.second.ctx);
    (void)hipStreamSynchronize(kv.second.stream);
    (void)hipStreamDestroy(kv.second.stream);
  }
  for (auto st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  delete s;
}

}  // extern "C"
