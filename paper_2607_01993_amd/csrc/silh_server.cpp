// Request-serving runtime (include/silh_server.h): resident datasets,
// admission against a device-memory budget, worker threads that run each
// admitted request's cluster index and Phase 1 on their own streams, and a
// batcher that runs the Phase 2 of every request whose Phase 1 is done in
// shared launches over (request, row-block) work items (continuous batching:
// requests join the next launch as they become ready and leave when their
// last block has run).  A request is the C-ABI sequence silh_sample_init ->
// silh_pps_sample -> Phase 2 -> mean -> silh_destroy; its Phase-2 blocks are
// those of its own launch, so results equal those of a direct call.
#include "../../include/silh_server.h"

#include <hip/hip_runtime.h>

#include <algorithm>
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
// of the same worker (its allocations and frees all happen on the worker's
// thread, after the work that used the block has completed); a block is
// reused for a request of at most twice smaller size.  `cached` counts the
// bytes of free blocks, which the worker trims after each request.
struct Pool {
  std::multimap<size_t, void*> free_blocks;
  std::unordered_map<void*, size_t> size_of;
  size_t cached = 0;

  static size_t granule(size_t b) {
    const size_t g = b >= ((size_t)1 << 26) ? ((size_t)1 << 21) : ((size_t)1 << 16);
    return (b + g - 1) / g * g;
  }
  void* get(size_t bytes) {
    const size_t want = granule(bytes ? bytes : 1);
    auto it = free_blocks.lower_bound(want);
    if (it != free_blocks.end() && it->first <= 2 * want) {
      void* p = it->second;
      cached -= it->first;
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
    if (it != size_of.end()) {
      free_blocks.emplace(it->second, p);
      cached += it->second;
    }
  }
  // free cached blocks, largest first, until at most `keep` bytes stay cached
  void trim(size_t keep) {
    while (cached > keep && !free_blocks.empty()) {
      auto it = std::prev(free_blocks.end());
      cached -= it->first;
      size_of.erase(it->second);
      (void)hipFree(it->second);
      free_blocks.erase(it);
    }
  }
  void release() { trim(0); }
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
  int passed = 0;  // admissions that went past it while it waited at the head
};

// A request in Phase 2: handed by its worker to the batcher, back to the
// worker once its last block has run.
struct Active {
  int64_t ticket = 0;
  int worker = 0;
  silh_ctx* ctx = nullptr;
  int64_t S = 0;
  silh::P2Job job{};
  silh::P2Class cls{};
  int64_t issued = 0, finished = 0;  // blocks launched / completed
  bool failed = false;               // a launch with its blocks could not be issued
};

// one launch of the batcher: its staging and device buffers (a ring of
// kSlots), the requests it covers and how many blocks of each
constexpr int kSlots = 2;
constexpr int kMaxTickJobs = 256;
constexpr int kMaxTickItems = 1 << 16;
struct Tick {
  hipStream_t st = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  silh::P2Job* jobs_h = nullptr;  // pinned
  int2* items_h = nullptr;        // pinned
  silh::P2Job* jobs_d = nullptr;
  int2* items_d = nullptr;
  std::vector<std::pair<Active*, int64_t>> parts;
  double pairs = 0.0;
  int64_t blocks = 0;
  bool busy = false;
};

// The launches of one kernel class go to streams of their own (so the
// launches of a class with long blocks do not hold another class's), two in
// flight at a time, each slot on its own stream: the next launch of the class
// starts on the CUs that the tail of the previous one leaves idle.
struct Lane {
  Tick ticks[kSlots];
  int next = 0;              // slot of the next launch (the older one when both are busy)
  double ns_per_pair = 0.0;  // measured time per (element, sample) pair of the whole device, 0: none yet
};

void free_lane(Lane* L) {
  if (!L) return;
  for (Tick& t : L->ticks) {
    if (t.t0) (void)hipEventDestroy(t.t0);
    if (t.t1) (void)hipEventDestroy(t.t1);
    if (t.jobs_h) (void)hipHostFree(t.jobs_h);
    if (t.items_h) (void)hipHostFree(t.items_h);
    if (t.jobs_d) (void)hipFree(t.jobs_d);
    if (t.items_d) (void)hipFree(t.items_d);
    if (t.st) (void)hipStreamDestroy(t.st);
  }
  delete L;
}

Lane* new_lane() {
  Lane* L = new (std::nothrow) Lane();
  if (!L) return nullptr;
  bool ok = true;
  for (Tick& t : L->ticks) {
    ok = ok && hipStreamCreateWithFlags(&t.st, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreate(&t.t0) == hipSuccess && hipEventCreate(&t.t1) == hipSuccess &&
         hipHostMalloc((void**)&t.jobs_h, sizeof(silh::P2Job) * kMaxTickJobs, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void**)&t.items_h, sizeof(int2) * kMaxTickItems, hipHostMallocDefault) == hipSuccess &&
         hipMalloc((void**)&t.jobs_d, sizeof(silh::P2Job) * kMaxTickJobs) == hipSuccess &&
         hipMalloc((void**)&t.items_d, sizeof(int2) * kMaxTickItems) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    free_lane(L);
    return nullptr;
  }
  return L;
}

}  // namespace

struct silh_server {
  int device = 0;
  int mode = 0;  // 0: Phase 2 in shared launches; 1: each request's own launch
  uint64_t budget = 0;
  size_t pool_keep = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_batch;
  std::vector<Dataset> datasets;
  std::unordered_map<int64_t, Job> jobs;
  std::deque<int64_t> queue;
  std::vector<std::deque<Active*>> finish;  // per worker
  std::vector<Active*> ready;               // Phase 1 done, not yet taken by the batcher
  int64_t next_ticket = 1;
  uint64_t in_flight = 0;
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::thread batcher;
  // batcher state (its thread only, except `launches`)
  std::map<int, Lane*> lanes;         // per kernel class
  int fill_blocks = 512;              // work items that keep every CU busy
  int64_t launches = 0;
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
  const uint64_t kp = mfma ? (uint64_t)silh::mfma_row_bytes(mprec, DM) : 0;
  const uint64_t row = (uint64_t)DM * 4 + kp + 24;
  const uint64_t m = r.m > 0 ? (uint64_t)r.m : 0;  // row draws: ids, gathered rows, outputs
  // d > 128 Manhattan / Canberra: float64 partial sums per element and cluster
  const uint64_t split = (DM > 128 && (r.metric == SILH_MANH || r.metric == SILH_CANB)) ? n * (uint64_t)r.k * 8 : 0;
  // PPS: the W pass keeps its distances for the draw (allocated at their
  // capacity)
  const uint64_t kept = r.sampler == SILH_PPS
                            ? 8 * (uint64_t)silh::dist_capacity((int64_t)n, std::log(5.0 * r.k / r.delta))
                            : 0;
  // cosine: one float32 reciprocal norm per element
  const uint64_t rn = r.metric == SILH_COS ? 4 * n : 0;
  return 24 * n + S * row + m * ((uint64_t)ds.d * 4 + 32) + split + kept + rn + ((uint64_t)1 << 20);
}

silh_params request_params(const Dataset& ds, const silh_request& r, Pool* pool) {
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
  if (pool) {
    p.alloc = pool_alloc;
    p.free = pool_free;
    p.alloc_user = pool;
  }
  return p;
}

void complete(silh_server* srv, int64_t ticket, silh_result res) {
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    Job& job = srv->jobs[ticket];
    res.submit_ns = job.res.submit_ns;
    res.start_ns = job.res.start_ns;
    res.done_ns = now_ns();
    job.res = res;
    job.done = true;
    srv->in_flight -= job.est;
    srv->running -= 1;
  }
  srv->cv_done.notify_all();
  srv->cv_work.notify_all();
}

void fail_result(silh_result& res, silh_status s) {
  res.status = s;
  std::snprintf(res.message, sizeof(res.message), "%s", silh_last_error());
}

// Phase 1 of one admitted request on the worker's stream.  Its Phase 2 goes
// to the batcher when it has a multi-request kernel (mode 0), else it runs
// here (the request's own launch, or the row draws of Eq. 10).
void start_request(silh_server* srv, int w, int64_t ticket, const Dataset& ds, const silh_request& r, Pool& pool,
                   hipStream_t st) {
  silh_result res{};
  silh_params p = request_params(ds, r, &pool);
  silh_ctx* ctx = nullptr;
  silh_status s = silh_sample_init(&p, ds.X, r.labels, (silh_stream)st, &ctx);
  int64_t S = 0;
  if (s == SILH_OK) s = silh_pps_sample(ctx, &S, nullptr);
  if (s == SILH_OK && srv->mode == 0 && r.m == 0) {
    Active* a = new (std::nothrow) Active();
    if (a && silh::phase2_job(ctx, &a->job, &a->cls)) {
      // the packing kernels of Phase 1 complete before another stream reads
      // their output
      if (hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        delete a;
        res.status = SILH_E_HIP;
        std::snprintf(res.message, sizeof(res.message), "worker stream failed");
        silh_destroy(ctx);
        complete(srv, ticket, res);
        return;
      }
      a->ticket = ticket;
      a->worker = w;
      a->ctx = ctx;
      a->S = S;
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->ready.push_back(a);
      }
      srv->cv_batch.notify_one();
      return;
    }
    delete a;
  }
  double mean = 0.0;
  int32_t* rows = nullptr;
  if (s == SILH_OK && r.m > 0) {
    rows = static_cast<int32_t*>(pool.get((size_t)r.m * sizeof(int32_t)));
    if (!rows) s = SILH_E_NOMEM;
    if (s == SILH_OK) s = silh_draw_rows(r.seed, ds.n, r.m, rows, (silh_stream)st);
    if (s == SILH_OK) s = silh_scores_rows(ctx, rows, r.m, nullptr, nullptr, nullptr, &mean);
  } else if (s == SILH_OK) {
    s = silh_scores(ctx, nullptr, nullptr, nullptr, &mean);
  }
  if (s != SILH_OK) fail_result(res, s);
  silh_destroy(ctx);  // synchronises the stream: the row buffer is free again
  if (rows) {
    (void)hipStreamSynchronize(st);
    pool.put(rows);
  }
  res.status = s;
  res.S = S;
  res.s_mean = mean;
  complete(srv, ticket, res);
}

// a request whose Phase-2 blocks have all run: the mean, then its buffers go
// back to the worker's pool
void finish_request(silh_server* srv, Active* a) {
  silh_result res{};
  double mean = 0.0;
  silh_status s = SILH_E_HIP;
  if (a->failed) {
    std::snprintf(res.message, sizeof(res.message), "a shared Phase-2 launch failed");
  } else {
    s = silh::phase2_job_mean(a->ctx, &mean);
    if (s != SILH_OK) fail_result(res, s);
  }
  silh_destroy(a->ctx);
  res.status = s;
  res.S = a->S;
  res.s_mean = mean;
  const int64_t ticket = a->ticket;
  delete a;
  complete(srv, ticket, res);
}

// next request to admit: the first in arrival order whose estimate fits what
// the admitted ones leave of the budget; once the head has been passed over
// 8 times, nothing goes past it until it fits
bool pick_admission(silh_server* srv, int64_t* ticket) {
  for (size_t i = 0; i < srv->queue.size(); ++i) {
    Job& job = srv->jobs[srv->queue[i]];
    if (srv->in_flight == 0 || srv->in_flight + job.est <= srv->budget) {
      if (i > 0) {
        Job& head = srv->jobs[srv->queue.front()];
        head.passed += 1;
      }
      *ticket = srv->queue[i];
      srv->queue.erase(srv->queue.begin() + (std::ptrdiff_t)i);
      return true;
    }
    if (i == 0 && job.passed >= 8) return false;
  }
  return false;
}

void worker_main(silh_server* srv, int w) {
  (void)hipSetDevice(srv->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  Pool pool;
  for (;;) {
    Active* fin = nullptr;
    int64_t ticket = 0;
    silh_request req{};
    Dataset ds{};
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv_work.wait(lk, [&] {
        if (!srv->finish[w].empty()) return true;
        if (pick_admission(srv, &ticket)) return true;
        return srv->stop && srv->queue.empty();
      });
      if (!srv->finish[w].empty()) {
        fin = srv->finish[w].front();
        srv->finish[w].pop_front();
        if (ticket != 0) {  // admitted in the same wake-up: back to the head
          srv->queue.push_front(ticket);
          ticket = 0;
        }
      } else if (ticket != 0) {
        Job& job = srv->jobs[ticket];
        req = job.req;
        ds = srv->datasets[req.dataset];
        srv->in_flight += job.est;
        srv->running += 1;
        job.res.start_ns = now_ns();
      } else {
        break;  // stop requested, nothing queued; this worker has no request in Phase 2
      }
    }
    if (fin) {
      finish_request(srv, fin);
    } else if (st == nullptr) {
      silh_result res{};
      res.status = SILH_E_HIP;
      std::snprintf(res.message, sizeof(res.message), "worker stream creation failed");
      complete(srv, ticket, res);
    } else {
      start_request(srv, w, ticket, ds, req, pool, st);
    }
    pool.trim(srv->pool_keep);
  }
  if (st) (void)hipStreamDestroy(st);
}

// ---- the batcher -------------------------------------------------------------

int class_key(const silh::P2Class& c) {
  return ((c.mfma * 4 + c.metric) * 4 + (c.prec + 1)) * 2048 + c.DM * 4 + c.pb;
}

// a first guess of the device's time per (element, sample) pair for a class,
// in ns, from the measured rates of each path (replaced by the class's own
// measurement after its first launch that fills the device)
double guess_ns_per_pair(const silh::P2Class& c) {
  const double dd = std::max(1.0, c.DM / 32.0);
  if (c.mfma) return (c.prec == 0 ? 6.3e-4 : 1.8e-4) * dd;
  switch (c.metric) {
    case SILH_MANH: return 1.1e-3 * dd;
    case SILH_CANB: return 5.1e-3 * dd;
    default: return 1.5e-3 * dd;
  }
}

constexpr double kTickNs = 4.0e6;  // target duration of one shared launch

bool tick_done(const Tick& t) {
  if (!t.busy) return false;
  const hipError_t e = hipEventQuery(t.t1);
  if (e == hipErrorNotReady) return false;
  if (e != hipSuccess) (void)hipGetLastError();
  return true;
}

// blocks of launch t have run: requests whose last block was among them
// leave `act` and go back to their workers (which delete them)
void retire(silh_server* srv, Lane& L, Tick& t, std::vector<Active*>& act) {
  (void)hipEventSynchronize(t.t1);
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, t.t0, t.t1) == hipSuccess) {
    // only a launch that filled the device measures the device's rate
    if (t.pairs > 0 && t.blocks >= srv->fill_blocks) {
      const double v = ms * 1.0e6 / t.pairs;
      L.ns_per_pair = L.ns_per_pair > 0.0 ? 0.5 * L.ns_per_pair + 0.5 * v : v;
    }
  } else {
    (void)hipGetLastError();
  }
  std::vector<Active*> done;
  for (auto& part : t.parts) {
    part.first->finished += part.second;
    if (part.first->finished == part.first->cls.blocks) done.push_back(part.first);
  }
  t.parts.clear();
  t.busy = false;
  if (!done.empty()) {
    act.erase(std::remove_if(act.begin(), act.end(),
                             [&](const Active* a) { return std::find(done.begin(), done.end(), a) != done.end(); }),
              act.end());
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      for (Active* a : done) srv->finish[a->worker].push_back(a);
    }
    srv->cv_work.notify_all();
  }
}

// Fill launch t with blocks of the requests of class `key` in `act`: the
// request with the least remaining work first (shortest remaining first, so
// a small request is not held behind a large one), about kTickNs of work
// but at least fill_blocks items (fewer blocks would leave CUs idle); the
// oldest request of the class gets at least a quarter, so large requests
// keep moving.
void issue(silh_server* srv, Lane& L, Tick& t, int key, std::vector<Active*>& act) {
  auto rest = [](const Active* a) { return (double)(a->cls.blocks - a->issued) * a->cls.rows * (double)a->cls.S_pad; };
  std::vector<Active*> same;
  Active* oldest = nullptr;
  for (Active* a : act) {
    if (a->issued >= a->cls.blocks || class_key(a->cls) != key) continue;
    same.push_back(a);
    if (!oldest || a->ticket < oldest->ticket) oldest = a;
  }
  if (same.empty()) return;
  std::sort(same.begin(), same.end(), [&](const Active* x, const Active* y) { return rest(x) < rest(y); });
  const silh::P2Class cls = same.front()->cls;
  const double nspp = L.ns_per_pair > 0.0 ? L.ns_per_pair : guess_ns_per_pair(cls);
  double budget = kTickNs / nspp;  // pairs
  int64_t want = srv->fill_blocks;  // items
  int nj = 0, ni = 0;
  t.parts.clear();
  t.pairs = 0.0;
  auto take = [&](Active* a, double pairs, int64_t blocks) {
    if (nj >= kMaxTickJobs || ni >= kMaxTickItems) return;
    const double per = (double)a->cls.rows * (double)a->cls.S_pad;
    int64_t nb = std::max<int64_t>((int64_t)(pairs / per), blocks);
    nb = std::max<int64_t>(nb, 1);
    nb = std::min<int64_t>(nb, a->cls.blocks - a->issued);
    nb = std::min<int64_t>(nb, kMaxTickItems - ni);
    if (nb <= 0) return;
    t.jobs_h[nj] = a->job;
    for (int64_t b = 0; b < nb; ++b) t.items_h[ni + b] = int2{nj, (int)(a->issued + b)};
    a->issued += nb;
    ni += (int)nb;
    t.parts.emplace_back(a, nb);
    t.pairs += (double)nb * per;
    budget -= (double)nb * per;
    want -= nb;
    ++nj;
  };
  if (oldest != same.front()) take(oldest, 0.25 * budget, want / 4);
  for (Active* a : same) {
    if (budget <= 0.0 && want <= 0) break;
    bool seen = false;
    for (auto& part : t.parts) seen = seen || part.first == a;
    if (!seen) take(a, budget, want);
  }
  if (ni == 0) return;
  t.blocks = ni;
  const hipStream_t st = t.st;
  bool ok = hipMemcpyAsync(t.jobs_d, t.jobs_h, sizeof(silh::P2Job) * (size_t)nj, hipMemcpyHostToDevice, st) ==
                hipSuccess &&
            hipMemcpyAsync(t.items_d, t.items_h, sizeof(int2) * (size_t)ni, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipEventRecord(t.t0, st) == hipSuccess && silh::launch_phase2_class(st, cls, t.jobs_d, t.items_d, ni) &&
            hipGetLastError() == hipSuccess && hipEventRecord(t.t1, st) == hipSuccess;
  if (!ok) {
    // the requests complete with an error; their blocks still count as done
    (void)hipGetLastError();
    for (auto& part : t.parts) part.first->failed = true;
    (void)hipEventRecord(t.t1, st);
  }
  t.busy = true;
  L.next = (L.next + 1) % kSlots;
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->launches += 1;
}

void batcher_main(silh_server* srv) {
  (void)hipSetDevice(srv->device);
  std::vector<Active*> act;
  for (;;) {
    bool busy = false;
    for (auto& kv : srv->lanes)
      for (const Tick& t : kv.second->ticks) busy = busy || t.busy;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      bool pending = false;
      for (const Active* a : act) pending = pending || a->issued < a->cls.blocks;
      if (srv->ready.empty() && !pending) {
        if (!busy) {
          srv->cv_batch.wait(lk, [&] { return !srv->ready.empty() || srv->stop; });
          if (srv->ready.empty() && srv->stop) break;
        } else {
          // launches in flight, nothing to issue: poll them, and wake early
          // for a request that becomes ready
          srv->cv_batch.wait_for(lk, std::chrono::microseconds(100), [&] { return !srv->ready.empty(); });
        }
      }
      for (Active* a : srv->ready) act.push_back(a);
      srv->ready.clear();
    }
    // retire every completed launch (per lane in issue order)
    for (auto& kv : srv->lanes) {
      Lane& L = *kv.second;
      for (int i = 0; i < kSlots; ++i) {
        Tick& t = L.ticks[(L.next + i) % kSlots];  // the older launch first
        if (!t.busy) continue;
        if (!tick_done(t)) break;
        retire(srv, L, t, act);
      }
    }
    // issue where a class has blocks left and a free slot
    std::vector<int> keys;
    for (const Active* a : act)
      if (a->issued < a->cls.blocks && std::find(keys.begin(), keys.end(), class_key(a->cls)) == keys.end())
        keys.push_back(class_key(a->cls));
    bool issued = false, blocked = false;
    for (int key : keys) {
      Lane*& L = srv->lanes[key];
      if (!L) L = new_lane();
      if (!L) {  // no stream or buffers for this class: its requests fail
        for (Active* a : act)
          if (class_key(a->cls) == key && a->issued < a->cls.blocks) {
            a->failed = true;
            a->finished += a->cls.blocks - a->issued;
            a->issued = a->cls.blocks;
          }
        continue;
      }
      Tick& t = L->ticks[L->next];
      if (t.busy) {
        blocked = true;
        continue;
      }
      issue(srv, *L, t, key, act);
      issued = true;
    }
    // requests failed above whose blocks are all accounted go back now
    std::vector<Active*> done;
    for (Active* a : act)
      if (a->failed && a->finished == a->cls.blocks) done.push_back(a);
    if (!done.empty()) {
      act.erase(std::remove_if(act.begin(), act.end(),
                               [&](const Active* a) { return std::find(done.begin(), done.end(), a) != done.end(); }),
                act.end());
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (Active* a : done) srv->finish[a->worker].push_back(a);
      }
      srv->cv_work.notify_all();
    }
    if (!issued && blocked) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

}  // namespace

extern "C" {

int64_t silh_server_now_ns(void) { return now_ns(); }

silh_status silh_server_create(const silh_server_cfg* cfg, silh_server** out) {
  if (!cfg || !out) return SILH_E_ARG;
  *out = nullptr;
  if (cfg->workers < 1 || cfg->workers > 64 || cfg->mode < 0 || cfg->mode > 1 || cfg->hbm_budget_bytes == 0)
    return SILH_E_ARG;
  silh_server* srv = new (std::nothrow) silh_server();
  if (!srv) return SILH_E_NOMEM;
  if (hipGetDevice(&srv->device) != hipSuccess) {
    delete srv;
    return SILH_E_HIP;
  }
  srv->mode = cfg->mode;
  srv->budget = cfg->hbm_budget_bytes;
  // each worker keeps at most this many bytes of free blocks between requests
  srv->pool_keep = (size_t)(cfg->hbm_budget_bytes / (2 * (uint64_t)cfg->workers));
  srv->finish.resize((size_t)cfg->workers);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, srv->device) == hipSuccess && cus > 0)
    srv->fill_blocks = 2 * cus;
  srv->batcher = std::thread(batcher_main, srv);
  for (int i = 0; i < cfg->workers; ++i) srv->workers.emplace_back(worker_main, srv, i);
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
  srv->cv_batch.notify_all();
  for (auto& th : srv->workers) th.join();
  if (srv->batcher.joinable()) srv->batcher.join();
  for (auto& kv : srv->lanes) free_lane(kv.second);
  delete srv;
}

int64_t silh_server_launches(silh_server* srv) {
  if (!srv) return -1;
  std::lock_guard<std::mutex> lk(srv->mu);
  return srv->launches;
}

silh_status silh_sweep(const silh_params* base, const float* X, const int32_t* labels, const int32_t* ks,
                       int32_t K, int64_t m, int32_t workers, uint64_t hbm_budget_bytes, silh_stream stream,
                       double* means_host, int32_t* best_host) {
  if (!base || !X || !labels || !ks || !means_host || K < 1) return SILH_E_ARG;
  if (base->n < 2 || base->n > ((int64_t)1 << 30)) return SILH_E_ARG;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SILH_E_HIP;
  silh_server_cfg cfg{workers, 0, hbm_budget_bytes};  // Phase 2 in shared launches
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
