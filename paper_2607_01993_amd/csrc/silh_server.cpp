// Request-serving runtime (include/silh_server.h): resident datasets, a FIFO
// queue with admission against a device-memory budget, and worker threads
// that each own a HIP stream and a cache of device blocks.  A request is the
// C-ABI sequence silh_sample_init -> silh_pps_sample -> silh_scores (mean
// only) -> silh_destroy, so results equal those of a direct call.
#include "../../include/silh_server.h"

#include <hip/hip_runtime.h>

#include <cmath>

#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "silh_internal.hpp"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Device blocks cached per worker: a freed block is reused by a later request
// of the same worker (same stream, so no cross-stream hazard); a block is
// reused for a request of at most twice smaller size.
struct Pool {
  std::multimap<size_t, void*> free_blocks;
  std::unordered_map<void*, size_t> size_of;

  static size_t granule(size_t b) {
    const size_t g = b >= ((size_t)1 << 26) ? ((size_t)1 << 21) : ((size_t)1 << 16);
    return (b + g - 1) / g * g;
  }
  void* get(size_t bytes) {
    const size_t want = granule(bytes ? bytes : 1);
    auto it = free_blocks.lower_bound(want);
    if (it != free_blocks.end() && it->first <= 2 * want) {
      void* p = it->second;
      free_blocks.erase(it);
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      release();  // give the cache back and try once more
      if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    size_of[p] = want;
    return p;
  }
  void put(void* p) {
    auto it = size_of.find(p);
    if (it != size_of.end()) free_blocks.emplace(it->second, p);
  }
  void release() {
    for (auto& kv : free_blocks) {
      size_of.erase(kv.second);
      (void)hipFree(kv.second);
    }
    free_blocks.clear();
  }
  ~Pool() {
    release();
    for (auto& kv : size_of) (void)hipFree(kv.first);  // blocks never returned
  }
};

void* pool_alloc(size_t bytes, void* user) { return static_cast<Pool*>(user)->get(bytes); }
void pool_free(void* p, void* user) { static_cast<Pool*>(user)->put(p); }

struct Dataset {
  const float* X;
  int64_t n;
  int32_t d;
};

struct Job {
  silh_request req{};
  silh_result res{};
  uint64_t est = 0;
  bool done = false;
};

}  // namespace

struct silh_server {
  int device = 0;
  uint64_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<Dataset> datasets;
  std::unordered_map<int64_t, Job> jobs;
  std::deque<int64_t> queue;
  int64_t next_ticket = 1;
  uint64_t in_flight = 0;
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;
};

namespace {

// Device bytes one request needs at most, roughly: the cluster index and the
// Phase-1 arrays (about 24 bytes per element), the distances kept between the
// W pass and the draw, plus the packed sample, sized for S = 2 k t + 32 k rows
// (a few times the expected 1-1.5 k t).
uint64_t estimate_bytes(const Dataset& ds, const silh_request& r) {
  const int DM = silh::dm_for(ds.d);
  const uint64_t n = (uint64_t)ds.n;
  uint64_t S = 2ull * (uint64_t)r.k * (uint64_t)r.t + 32ull * (uint64_t)r.k;
  if (S > n + 32ull * (uint64_t)r.k) S = n + 32ull * (uint64_t)r.k;
  const bool mfma = (r.metric == SILH_EUCL || r.metric == SILH_COS) && r.prec != SILH_FP32_VALU;
  const int mprec = r.prec == SILH_BF16 ? 1 : (r.prec == SILH_FP8 ? 2 : 0);
  const uint64_t kp = mfma ? (uint64_t)silh::mfma_kp(mprec, DM) : 0;
  const uint64_t row = (uint64_t)DM * 4 + kp * 4 + 24;
  const uint64_t m = r.m > 0 ? (uint64_t)r.m : 0;  // row draws: ids, gathered rows, outputs
  // d > 128 Manhattan / Canberra: float64 partial sums per element and cluster
  const uint64_t split = (DM > 128 && (r.metric == SILH_MANH || r.metric == SILH_CANB)) ? n * (uint64_t)r.k * 8 : 0;
  // PPS with d <= 128: the W pass keeps its distances for the draw (allocated
  // at their capacity)
  const uint64_t kept = (r.sampler == SILH_PPS && DM <= 128)
                            ? 8 * (uint64_t)silh::dist_capacity((int64_t)n, std::log(5.0 * r.k / r.delta))
                            : 0;
  return 24 * n + S * row + m * ((uint64_t)ds.d * 4 + 32) + split + kept + ((uint64_t)1 << 20);
}

void run_job(Dataset ds, const silh_request& r, Pool& pool, hipStream_t st, silh_result& res) {
  silh_params p{};
  p.n = ds.n;
  p.d = ds.d;
  p.k = r.k;
  p.metric = (silh_metric)r.metric;
  p.prec = (silh_prec)r.prec;
  p.sampler = (silh_sampler)r.sampler;
  p.t = r.t;
  p.eps = 0.0;
  p.delta = r.delta;
  p.seed = r.seed;
  p.alloc = pool_alloc;
  p.free = pool_free;
  p.alloc_user = &pool;
  silh_ctx* ctx = nullptr;
  silh_status s = silh_sample_init(&p, ds.X, r.labels, (silh_stream)st, &ctx);
  int64_t S = 0;
  double mean = 0.0;
  int32_t* rows = nullptr;
  if (s == SILH_OK) s = silh_pps_sample(ctx, &S, nullptr);
  if (s == SILH_OK && r.m > 0) {
    rows = static_cast<int32_t*>(pool.get((size_t)r.m * sizeof(int32_t)));
    if (!rows) s = SILH_E_NOMEM;
    if (s == SILH_OK) s = silh_draw_rows(r.seed, ds.n, r.m, rows, (silh_stream)st);
    if (s == SILH_OK) s = silh_scores_rows(ctx, rows, r.m, nullptr, nullptr, nullptr, &mean);
  } else if (s == SILH_OK) {
    s = silh_scores(ctx, nullptr, nullptr, nullptr, &mean);
  }
  if (s != SILH_OK) std::snprintf(res.message, sizeof(res.message), "%s", silh_last_error());
  silh_destroy(ctx);  // synchronises the stream: the row buffer is free again
  if (rows) {
    (void)hipStreamSynchronize(st);
    pool.put(rows);
  }
  res.status = s;
  res.S = S;
  res.s_mean = mean;
}

void worker_main(silh_server* srv) {
  (void)hipSetDevice(srv->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  Pool pool;
  for (;;) {
    int64_t ticket = 0;
    silh_request req{};
    Dataset ds{};
    uint64_t est = 0;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      // first in, first out: the head waits until its estimate fits
      srv->cv_work.wait(lk, [&] {
        if (srv->stop) return true;
        if (srv->queue.empty()) return false;
        const Job& head = srv->jobs[srv->queue.front()];
        return srv->in_flight == 0 || srv->in_flight + head.est <= srv->budget;
      });
      if (srv->queue.empty()) return;  // stop requested and nothing left
      ticket = srv->queue.front();
      srv->queue.pop_front();
      Job& job = srv->jobs[ticket];
      req = job.req;
      ds = srv->datasets[req.dataset];
      est = job.est;
      srv->in_flight += est;
      srv->running += 1;
      job.res.start_ns = now_ns();
    }
    silh_result res{};
    if (st == nullptr) {
      res.status = SILH_E_HIP;
      std::snprintf(res.message, sizeof(res.message), "worker stream creation failed");
    } else {
      run_job(ds, req, pool, st, res);
    }
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      Job& job = srv->jobs[ticket];
      res.submit_ns = job.res.submit_ns;
      res.start_ns = job.res.start_ns;
      res.done_ns = now_ns();
      job.res = res;
      job.done = true;
      srv->in_flight -= est;
      srv->running -= 1;
    }
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

int64_t silh_server_now_ns(void) { return now_ns(); }

silh_status silh_server_create(const silh_server_cfg* cfg, silh_server** out) {
  if (!cfg || !out) return SILH_E_ARG;
  *out = nullptr;
  if (cfg->workers < 1 || cfg->workers > 64 || cfg->reserved0 != 0 || cfg->hbm_budget_bytes == 0)
    return SILH_E_ARG;
  silh_server* srv = new (std::nothrow) silh_server();
  if (!srv) return SILH_E_NOMEM;
  if (hipGetDevice(&srv->device) != hipSuccess) {
    delete srv;
    return SILH_E_HIP;
  }
  srv->budget = cfg->hbm_budget_bytes;
  for (int i = 0; i < cfg->workers; ++i) srv->workers.emplace_back(worker_main, srv);
  *out = srv;
  return SILH_OK;
}

silh_status silh_server_add_dataset(silh_server* srv, const float* X, int64_t n, int32_t d, int32_t* id) {
  if (!srv || !X || !id) return SILH_E_ARG;
  if (n < 2 || n > ((int64_t)1 << 30) || d < 1 || d > 256) return SILH_E_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->datasets.push_back({X, n, d});
  *id = (int32_t)srv->datasets.size() - 1;
  return SILH_OK;
}

silh_status silh_server_submit(silh_server* srv, const silh_request* req, int64_t* ticket) {
  if (!srv || !req || !ticket) return SILH_E_ARG;
  if (req->reserved0 != 0) return SILH_E_ARG;
  Dataset ds{};
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (req->dataset < 0 || req->dataset >= (int32_t)srv->datasets.size()) return SILH_E_ARG;
    ds = srv->datasets[req->dataset];
  }
  silh_params p{};
  p.n = ds.n;
  p.d = ds.d;
  p.k = req->k;
  p.metric = (silh_metric)req->metric;
  p.prec = (silh_prec)req->prec;
  p.sampler = (silh_sampler)req->sampler;
  p.t = req->t;
  p.delta = req->delta;
  p.seed = req->seed;
  int64_t t = 0;
  silh_status s = silh::validate_params(&p, ds.X, req->labels, &t);
  if (s != SILH_OK) return s;
  if (req->t < 1 || req->m < 0 || req->m > ((int64_t)1 << 30)) return SILH_E_ARG;
  const uint64_t est = estimate_bytes(ds, *req);
  if (est > srv->budget) return SILH_E_NOMEM;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    const int64_t tk = srv->next_ticket++;
    Job& job = srv->jobs[tk];
    job.req = *req;
    job.est = est;
    job.res.submit_ns = now_ns();
    srv->queue.push_back(tk);
    *ticket = tk;
  }
  srv->cv_work.notify_all();
  return SILH_OK;
}

silh_status silh_server_wait(silh_server* srv, int64_t ticket, silh_result* out) {
  if (!srv || !out) return SILH_E_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  if (srv->jobs.find(ticket) == srv->jobs.end()) return SILH_E_ARG;
  // another waiter may retire the same ticket first
  srv->cv_done.wait(lk, [&] {
    auto it = srv->jobs.find(ticket);
    return it == srv->jobs.end() || it->second.done;
  });
  auto it = srv->jobs.find(ticket);
  if (it == srv->jobs.end()) return SILH_E_ARG;
  *out = it->second.res;
  srv->jobs.erase(it);
  return SILH_OK;
}

silh_status silh_server_drain(silh_server* srv) {
  if (!srv) return SILH_E_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->queue.empty() && srv->running == 0; });
  return SILH_OK;
}

void silh_server_destroy(silh_server* srv) {
  if (!srv) return;
  (void)silh_server_drain(srv);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& th : srv->workers) th.join();
  delete srv;
}

silh_status silh_sweep(const silh_params* base, const float* X, const int32_t* labels, const int32_t* ks,
                       int32_t K, int64_t m, int32_t workers, uint64_t hbm_budget_bytes, silh_stream stream,
                       double* means_host, int32_t* best_host) {
  if (!base || !X || !labels || !ks || !means_host || K < 1) return SILH_E_ARG;
  if (base->n < 2 || base->n > ((int64_t)1 << 30)) return SILH_E_ARG;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SILH_E_HIP;
  silh_server_cfg cfg{workers, 0, hbm_budget_bytes};
  silh_server* srv = nullptr;
  silh_status s = silh_server_create(&cfg, &srv);
  if (s != SILH_OK) return s;
  int32_t did = 0;
  s = silh_server_add_dataset(srv, X, base->n, base->d, &did);
  std::vector<int64_t> tickets((size_t)K, 0);
  silh_status first_bad = SILH_OK;
  for (int32_t i = 0; i < K && s == SILH_OK; ++i) {
    silh_request r{};
    r.dataset = did;
    r.k = ks[i];
    r.labels = labels + (size_t)i * (size_t)base->n;
    r.metric = base->metric;
    r.prec = base->prec;
    r.sampler = base->sampler;
    r.t = base->t;
    r.delta = base->delta;
    r.seed = base->seed;
    r.m = m;
    const silh_status q = silh_server_submit(srv, &r, &tickets[i]);
    if (q != SILH_OK) {
      tickets[i] = 0;
      means_host[i] = __builtin_nan("");
      if (first_bad == SILH_OK) first_bad = q;
    }
  }
  for (int32_t i = 0; i < K && s == SILH_OK; ++i) {
    if (tickets[i] == 0) continue;
    silh_result res{};
    silh_server_wait(srv, tickets[i], &res);
    means_host[i] = res.status == SILH_OK ? res.s_mean : __builtin_nan("");
    if (res.status != SILH_OK && first_bad == SILH_OK) first_bad = (silh_status)res.status;
  }
  silh_server_destroy(srv);
  if (s != SILH_OK) return s;
  if (best_host) {
    int32_t best = -1;
    for (int32_t i = 0; i < K; ++i)
      if (means_host[i] == means_host[i] && (best < 0 || means_host[i] > means_host[best])) best = i;
    *best_host = best;
  }
  return first_bad;
}

}  // extern "C"
