// C ABI of the silhouette library: argument checks, the per-clustering
// context, the call order, device-memory management through the caller's
// allocator, and the order of kernel launches on the caller's stream.
#include "../../include/silh.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <atomic>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "silh_internal.hpp"

using namespace silh;

namespace {

thread_local std::string g_err;

silh_status fail(silh_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(SILH_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define CHK(expr)                      \
  do {                                 \
    silh_status s_ = (expr);           \
    if (s_ != SILH_OK) return s_;      \
  } while (0)

enum Slot {
  K_SORT_HIST = 0,
  K_SORT_SCAN,
  K_SORT_SCATTER,
  K_F0_FLAG,
  K_SCAN,
  K_F0_PACK,
  K_W_PARTIAL,
  K_W_FINAL,
  K_DRAW,
  K_PACK,
  K_CENTER,
  K_PACK_MFMA,
  K_PHASE2,
  K_MEAN,
  K_NSLOTS
};
const char* const kSlotNames[K_NSLOTS] = {
    "sort_hist", "sort_scan", "sort_scatter", "f0_flag", "scan", "f0_pack",
    "w_partial", "w_final", "draw",      "pack",         "center",  "pack_mfma", "phase2", "mean"};

constexpr int64_t kMaxN = (int64_t)1 << 30;
constexpr int kMaxK = 4096;
constexpr int kMaxD = 256;
constexpr int kFp8MinD = 64;

}  // namespace

struct silh_ctx {
  silh_params prm{};
  int64_t t = 0;
  hipStream_t st = nullptr;
  const float* X = nullptr;
  const int32_t* labels = nullptr;
  int n = 0, d = 0, k = 0, DM = 0;
  bool mfma = false;  // Phase 2 on the matrix cores
  int mprec = 0;      // MFMA operand type: 0 float32, 1 bf16, 2 fp8
  int p2_rows = kP2Rows;
  int state = 0;  // 0 = indexed, 1 = sampled

  std::vector<void*> alloc_init, alloc_sample, alloc_rows, alloc_p2;

  // host copies
  std::vector<uint32_t> counts_h;
  std::vector<int32_t> csize_h, off_h;
  std::vector<double> q_h;
  std::vector<int32_t> f0_off32_h, s_off32_h, sp_off_h, cnt_h, items_h, citem_first_h, citem_count_h;
  std::vector<int64_t> f0_off_h, s_off_h;
  double mean_h = 0.0;

  // index
  int32_t* csize = nullptr;  // u32 counts reinterpreted (sizes < 2^31)
  int32_t* off = nullptr;
  int32_t* uh = nullptr;
  int32_t* perm = nullptr;
  int32_t* slab = nullptr;
  float* rn = nullptr;  // cosine: reciprocal row norms of X
  double* q = nullptr;

  // sample
  int64_t S = 0, S_pad = 0, F0 = 0;
  int32_t *flag = nullptr, *pos = nullptr, *scan_tmp = nullptr;
  int32_t *f0_off = nullptr, *f0_cl = nullptr, *items = nullptr, *citem_first = nullptr,
          *citem_count = nullptr, *imeta = nullptr;
  int64_t* ibase = nullptr;
  int64_t* dbase = nullptr;
  double* dkeep = nullptr;   // member-to-F0 distances kept by the W pass for the draw
  int* p1_status = nullptr;  // capacity bits of the device-built W work items
  int p1_status_h = 0;
  int64_t *f0_gid = nullptr, *gid_view = nullptr;
  double *f0X = nullptr, *W0 = nullptr, *partial = nullptr, *p_gid = nullptr;
  int32_t *s_off = nullptr, *sp_off = nullptr, *cnt = nullptr, *gid_pk = nullptr;
  float *w32 = nullptr, *aux32 = nullptr, *Y32 = nullptr, *mu = nullptr, *bnorm = nullptr;
  void* Ym = nullptr;
  double *bpart = nullptr, *mean_d = nullptr;

  // pinned staging for the small host <-> device transfers (from a
  // process-wide pool): host-to-device copies from it are asynchronous
  unsigned char* pin = nullptr;
  size_t pin_size = 0, pin_used = 0;

  // profiling
  bool prof_on = false;
  int prof_mode = 1;  // 1: every kernel, 2: the Phase-2 launches only
  struct Pending {
    int slot;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double tot_ms[K_NSLOTS] = {};
  int64_t launches[K_NSLOTS] = {};
};

namespace {

// Without an allocator callback, device memory comes from a cache of blocks
// the library keeps per (device, stream) until the process ends: a block
// freed by a context goes back to its stream's list, and a later allocation
// on the same stream takes the smallest cached block of at least the size
// asked for and at most twice it.  Work on one stream runs in order, so the
// next user of a block starts after the previous one's last kernel; no call
// synchronises the device once the cache is warm.  New blocks: hipMalloc.
struct CachedBlock {
  void* p;
  size_t bytes;
};
std::mutex g_dcache_mu;
std::map<std::pair<int, hipStream_t>, std::vector<CachedBlock>> g_dcache;
std::map<void*, std::pair<std::pair<int, hipStream_t>, size_t>> g_dlive;

void* raw_alloc(silh_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (c->prm.alloc) return c->prm.alloc(bytes, c->prm.alloc_user);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  const auto key = std::make_pair(dev, c->st);
  {
    std::lock_guard<std::mutex> lk(g_dcache_mu);
    auto& v = g_dcache[key];
    size_t best = v.size();
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i].bytes >= bytes && v[i].bytes / 2 <= bytes && (best == v.size() || v[i].bytes < v[best].bytes))
        best = i;
    if (best < v.size()) {
      const CachedBlock b = v[best];
      v[best] = v.back();
      v.pop_back();
      g_dlive[b.p] = {key, b.bytes};
      return b.p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_dcache_mu);
  g_dlive[p] = {key, bytes};
  return p;
}

void raw_free(silh_ctx* c, void* p) {
  if (!p) return;
  if (c->prm.alloc) {
    if (c->prm.free) c->prm.free(p, c->prm.alloc_user);
    return;
  }
  std::lock_guard<std::mutex> lk(g_dcache_mu);
  auto it = g_dlive.find(p);
  if (it == g_dlive.end()) return;  // not ours
  g_dcache[it->second.first].push_back({p, it->second.second});
  g_dlive.erase(it);
}

// Buffers of one stage are carved out of a single allocation (one allocator
// call per stage instead of one per buffer), each at a 256-byte boundary.
struct Carve {
  struct Req {
    void** out;
    size_t bytes;
  };
  std::vector<Req> reqs;
  template <class T>
  Carve& add(T** out, size_t count) {
    reqs.push_back({(void**)out, count * sizeof(T)});
    return *this;
  }
  // every request gets an address of its own, also an empty one
  static size_t span(size_t b) { return b == 0 ? 256 : (b + 255) / 256 * 256; }
  silh_status commit(silh_ctx* c, std::vector<void*>& list) {
    size_t tot = 0;
    for (const Req& r : reqs) tot += span(r.bytes);
    void* base = raw_alloc(c, tot);
    if (!base) return fail(SILH_E_NOMEM, "device allocation of %zu bytes failed", tot);
    list.push_back(base);
    size_t off = 0;
    for (const Req& r : reqs) {
      *r.out = (void*)((char*)base + off);
      off += span(r.bytes);
    }
    return SILH_OK;
  }
};

void free_list(silh_ctx* c, std::vector<void*>& list) {
  for (void* p : list) raw_free(c, p);
  list.clear();
}

// Timing events outlive the contexts that used them: a per-device pool
// shared by every context of the process (creating events per request costs
// more than the short kernels they time).
std::mutex g_event_mu;
std::map<int, std::vector<hipEvent_t>> g_event_pool;

hipEvent_t get_event(silh_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_event_mu);
    auto& v = g_event_pool[dev];
    if (!v.empty()) {
      hipEvent_t e = v.back();
      v.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void return_events(std::vector<hipEvent_t>& evs) {
  int dev = 0;
  if (evs.empty()) return;
  if (hipGetDevice(&dev) != hipSuccess) {
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  } else {
    std::lock_guard<std::mutex> lk(g_event_mu);
    auto& v = g_event_pool[dev];
    v.insert(v.end(), evs.begin(), evs.end());
  }
  evs.clear();
}

// Brackets a kernel launch with events when profiling is on, and checks the
// launch status afterwards.
struct Launch {
  silh_ctx* c;
  int slot;
  hipEvent_t a = nullptr;
  Launch(silh_ctx* ctx, int s) : c(ctx), slot(s) {
    if (c->prof_on && (c->prof_mode == 1 || s == K_PHASE2)) {
      a = get_event(c);
      if (a) (void)hipEventRecord(a, c->st);
    }
  }
  silh_status done() {
    hipError_t e = hipGetLastError();
    if (c->prof_on && a) {
      hipEvent_t b = get_event(c);
      if (b) {
        (void)hipEventRecord(b, c->st);
        c->pending.push_back({slot, a, b});
      } else {
        c->pool.push_back(a);
      }
      a = nullptr;
    }
    if (e != hipSuccess) return fail(SILH_E_HIP, "kernel %s: %s", kSlotNames[slot], hipGetErrorString(e));
    return SILH_OK;
  }
};

silh_status drain_prof(silh_ctx* c) {
  if (c->pending.empty()) return SILH_OK;
  HIPCHK(hipStreamSynchronize(c->st));
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->tot_ms[p.slot] += ms;
      c->launches[p.slot] += 1;
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
  return SILH_OK;
}

// ---- pinned staging ------------------------------------------------------------
// Blocks of page-locked host memory are shared by the process: a context takes
// one at its first transfer and returns it at silh_destroy.  Inside a block,
// transfers take consecutive slices; the slices are reused only after the
// context's stream has been synchronised (every copy from them is then done).
std::mutex g_pin_mu;
std::vector<std::pair<unsigned char*, size_t>> g_pin_free;
constexpr size_t kPinBlock = (size_t)1 << 18;

void pin_release(silh_ctx* c) {
  if (!c->pin) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.emplace_back(c->pin, c->pin_size);
  c->pin = nullptr;
  c->pin_size = c->pin_used = 0;
}

silh_status pin_acquire(silh_ctx* c, size_t min_bytes) {
  pin_release(c);
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    for (size_t i = 0; i < g_pin_free.size(); ++i) {
      if (g_pin_free[i].second >= min_bytes) {
        c->pin = g_pin_free[i].first;
        c->pin_size = g_pin_free[i].second;
        g_pin_free.erase(g_pin_free.begin() + (long)i);
        c->pin_used = 0;
        return SILH_OK;
      }
    }
  }
  const size_t bytes = min_bytes > kPinBlock ? min_bytes : kPinBlock;
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SILH_E_NOMEM, "pinned host allocation of %zu bytes failed", bytes);
  }
  c->pin = (unsigned char*)p;
  c->pin_size = bytes;
  c->pin_used = 0;
  return SILH_OK;
}

// A slice of `bytes` for this context's next transfers (synchronises the
// stream first when the block is full).
silh_status stage(silh_ctx* c, size_t bytes, void** out) {
  const size_t span = (bytes + 255) / 256 * 256;
  if (c->pin && c->pin_used + span <= c->pin_size) {
    *out = c->pin + c->pin_used;
    c->pin_used += span;
    return SILH_OK;
  }
  HIPCHK(hipStreamSynchronize(c->st));  // earlier slices are free again
  c->pin_used = 0;
  if (!c->pin || span > c->pin_size) CHK(pin_acquire(c, span));
  *out = c->pin;
  c->pin_used = span;
  return SILH_OK;
}

template <class T>
silh_status h2d(silh_ctx* c, T* dst, const std::vector<T>& src) {
  if (src.empty()) return SILH_OK;
  void* p = nullptr;
  CHK(stage(c, src.size() * sizeof(T), &p));
  std::memcpy(p, src.data(), src.size() * sizeof(T));
  HIPCHK(hipMemcpyAsync(dst, p, src.size() * sizeof(T), hipMemcpyHostToDevice, c->st));
  return SILH_OK;
}

// Two uploads in one copy when dst_b is the next slot of the same carve
// (dst_a's span rounded up to 256 bytes): the padding between them is staged
// as zeros.  Each copy is a transfer of its own on the stream, so adjacent
// small arrays go together.
template <class A, class B>
silh_status h2d_pair(silh_ctx* c, A* dst_a, const std::vector<A>& a, B* dst_b, const std::vector<B>& b) {
  const size_t na = a.size() * sizeof(A), nb = b.size() * sizeof(B);
  const size_t gap = (size_t)((const char*)dst_b - (const char*)dst_a);
  if (na == 0 || nb == 0 || gap != Carve::span(na)) {
    CHK(h2d(c, dst_a, a));
    return h2d(c, dst_b, b);
  }
  void* p = nullptr;
  CHK(stage(c, gap + nb, &p));
  std::memcpy(p, a.data(), na);
  std::memset((char*)p + na, 0, gap - na);
  std::memcpy((char*)p + gap, b.data(), nb);
  HIPCHK(hipMemcpyAsync(dst_a, p, gap + nb, hipMemcpyHostToDevice, c->st));
  return SILH_OK;
}

// Device-to-host read-backs: every part is copied through the staging block,
// then the stream is synchronised and the values land in host memory.  Parts
// that lie within 512 bytes of each other on the device (slots of one carve)
// are copied as one span.
struct Fetch {
  void* host;
  const void* dev;
  size_t bytes;
};
silh_status fetch(silh_ctx* c, std::initializer_list<Fetch> parts) {
  std::vector<Fetch> ps(parts);
  std::sort(ps.begin(), ps.end(), [](const Fetch& x, const Fetch& y) { return x.dev < y.dev; });
  // runs of parts copied together: [first part, last part]
  std::vector<std::pair<size_t, size_t>> runs;
  for (size_t i = 0; i < ps.size(); ++i) {
    if (!runs.empty()) {
      const Fetch& last = ps[runs.back().second];
      const char* end = (const char*)last.dev + last.bytes;
      if ((const char*)ps[i].dev >= end && (const char*)ps[i].dev - end <= 512) {
        runs.back().second = i;
        continue;
      }
    }
    runs.push_back({i, i});
  }
  size_t total = 0;
  for (const auto& r : runs)
    total += ((size_t)((const char*)ps[r.second].dev + ps[r.second].bytes - (const char*)ps[r.first].dev) + 255) / 256 * 256;
  if (!c->pin || c->pin_used + total > c->pin_size) {
    HIPCHK(hipStreamSynchronize(c->st));
    c->pin_used = 0;
    if (!c->pin || total > c->pin_size) CHK(pin_acquire(c, total));
  }
  std::vector<void*> slots;
  for (const auto& r : runs) {
    const char* lo = (const char*)ps[r.first].dev;
    const size_t span = (size_t)((const char*)ps[r.second].dev + ps[r.second].bytes - lo);
    void* p = nullptr;
    CHK(stage(c, span, &p));
    HIPCHK(hipMemcpyAsync(p, lo, span, hipMemcpyDeviceToHost, c->st));
    slots.push_back(p);
  }
  HIPCHK(hipStreamSynchronize(c->st));
  for (size_t ri = 0; ri < runs.size(); ++ri) {
    const char* lo = (const char*)ps[runs[ri].first].dev;
    for (size_t i = runs[ri].first; i <= runs[ri].second; ++i)
      std::memcpy(ps[i].host, (const char*)slots[ri] + ((const char*)ps[i].dev - lo), ps[i].bytes);
  }
  c->pin_used = 0;  // every copy of this context is complete
  return SILH_OK;
}

silh_status check_params(const silh_params* prm, const float* X, const int32_t* labels, bool exact,
                         int64_t* t_out) {
  if (!prm) return fail(SILH_E_ARG, "params is NULL");
  if (!X || !labels) return fail(SILH_E_ARG, "X or labels is NULL");
  if (prm->n < 2 || prm->n > kMaxN) return fail(SILH_E_ARG, "n=%lld outside [2, 2^30]", (long long)prm->n);
  if (prm->d < 1 || prm->d > kMaxD) return fail(SILH_E_ARG, "d=%d outside [1, %d]", prm->d, kMaxD);
  if (prm->k < 2 || prm->k > kMaxK) return fail(SILH_E_ARG, "k=%d outside [2, %d]", prm->k, kMaxK);
  if (prm->metric < 0 || prm->metric > 3) return fail(SILH_E_ARG, "unknown metric %d", prm->metric);
  if (prm->prec < 0 || prm->prec > 3) return fail(SILH_E_ARG, "unknown precision %d", prm->prec);
  if (prm->reserved0 != 0) return fail(SILH_E_ARG, "reserved0 must be 0");
  if ((prm->alloc == nullptr) != (prm->free == nullptr))
    return fail(SILH_E_ARG, "alloc and free must be given together");
  const bool mfma_metric = prm->metric == SILH_EUCL || prm->metric == SILH_COS;
  if ((prm->prec == SILH_FP8 && prm->metric != SILH_COS) || (prm->prec == SILH_BF16 && !mfma_metric))
    return fail(SILH_E_UNSUPPORTED, "precision %d is not built for metric %d", prm->prec, prm->metric);
  if (prm->prec == SILH_FP8 && prm->d < kFp8MinD)
    return fail(SILH_E_UNSUPPORTED, "fp8 operands need d >= %d (d=%d)", kFp8MinD, prm->d);
  if (phase2_valu_dm(prm->d) == 0)
    return fail(SILH_E_UNSUPPORTED, "d=%d has no Phase-2 kernel", prm->d);
  int64_t t = prm->t;
  if (!exact) {
    if (prm->sampler < 0 || prm->sampler > 1) return fail(SILH_E_ARG, "unknown sampler %d", prm->sampler);
    if (!(prm->delta > 0.0 && prm->delta < 1.0)) return fail(SILH_E_ARG, "delta must be in (0, 1)");
    if (t <= 0) {
      if (!(prm->eps > 0.0 && prm->eps < 1.0))
        return fail(SILH_E_ARG, "t <= 0 needs eps in (0, 1)");
      // Lemma 1: t = ceil((3c/eps^2) ln(5nk/delta)), c = 18
      const double v = std::ceil((3.0 * 18.0 / (prm->eps * prm->eps)) *
                                 std::log(5.0 * (double)prm->n * (double)prm->k / prm->delta));
      if (!(v < 9.0e18)) return fail(SILH_E_ARG, "derived t overflows");
      t = (int64_t)v;
    }
  }
  *t_out = t;
  return SILH_OK;
}

// Cluster sizes, offsets and the stable sort by label.
silh_status build_index(silh_ctx* c) {
  const int n = c->n, k = c->k;
  const int seg = sort_seg(n, k);
  const int units = (int)ceil_div(n, seg);
  {
    Carve cv;
    cv.add(&c->csize, (size_t)k).add(&c->off, (size_t)k + 1).add(&c->q, (size_t)k);
    cv.add(&c->uh, (size_t)units * k).add(&c->perm, (size_t)n).add(&c->slab, (size_t)n);
    if (c->prm.metric == SILH_COS) cv.add(&c->rn, (size_t)n);
    CHK(cv.commit(c, c->alloc_init));
  }
  if (c->rn) {
    // cosine rows are made unit length by one float32 factor per row, the
    // same for the element rows of Phase 2 and the packed sample rows
    launch_rnorm(c->st, c->X, n, c->d, c->rn);
    HIPCHK(hipGetLastError());
  }
  // cluster sizes from the sort's per-unit histograms (no separate count pass);
  // a label outside [0, k) is counted nowhere, so the sizes then sum to less
  // than n (no flag word to clear and read)
  {
    Launch L(c, K_SORT_HIST);
    launch_unit_hist(c->st, c->labels, n, k, seg, c->uh, nullptr);
    CHK(L.done());
  }
  {
    Launch L(c, K_SORT_SCAN);
    launch_unit_scan(c->st, c->uh, units, k, c->csize);
    CHK(L.done());
  }
  c->counts_h.assign(k, 0u);
  CHK(fetch(c, {{c->counts_h.data(), c->csize, k * sizeof(uint32_t)}}));
  {
    uint64_t tot = 0;
    for (int j = 0; j < k; ++j) tot += c->counts_h[j];
    if (tot != (uint64_t)n) return fail(SILH_E_LABEL, "a label lies outside [0, %d)", k);
  }
  c->csize_h.assign(k, 0);
  c->off_h.assign(k + 1, 0);
  int nonempty = 0;
  for (int j = 0; j < k; ++j) {
    c->csize_h[j] = (int32_t)c->counts_h[j];
    c->off_h[j + 1] = c->off_h[j] + c->csize_h[j];
    nonempty += c->csize_h[j] > 0;
  }
  if (nonempty < 2) return fail(SILH_E_K, "%d nonempty cluster(s); the silhouette needs at least 2", nonempty);
  // initial-sample rate of Algorithm 1, min(1, (2/|C_j|) ln(5k/delta)), on the host
  c->q_h.assign(k, 0.0);
  const double lnterm = std::log(5.0 * (double)k / c->prm.delta);
  for (int j = 0; j < k; ++j) {
    if (c->csize_h[j] > 0) {
      double qj = 2.0 / (double)c->csize_h[j];
      qj = qj * lnterm;
      c->q_h[j] = qj < 1.0 ? qj : 1.0;
    }
  }
  CHK(h2d_pair(c, c->off, c->off_h, c->q, c->q_h));
  {
    Launch L(c, K_SORT_SCATTER);
    launch_scatter(c->st, c->labels, n, k, seg, c->uh, c->off, c->perm, c->slab);
    CHK(L.done());
  }
  return SILH_OK;
}

silh_status create(const silh_params* prm, const float* X, const int32_t* labels, silh_stream stream,
                   bool exact, silh_ctx** out) {
  int64_t t = 0;
  CHK(check_params(prm, X, labels, exact, &t));
  silh_ctx* c = new (std::nothrow) silh_ctx();
  if (!c) return fail(SILH_E_NOMEM, "host allocation failed");
  c->prm = *prm;
  c->t = t;
  c->st = (hipStream_t)stream;
  c->X = X;
  c->labels = labels;
  c->n = (int)prm->n;
  c->d = prm->d;
  c->k = prm->k;
  c->DM = phase2_valu_dm(prm->d);
  // float32 operands of d > 128 do not fit the MFMA kernel's registers: the
  // vector-ALU kernel takes them
  c->mfma = (prm->metric == SILH_EUCL || prm->metric == SILH_COS) &&
            (prm->prec == SILH_BF16 || prm->prec == SILH_FP8 || (prm->prec == SILH_FP32 && c->DM <= 128));
  c->mprec = prm->prec == SILH_BF16 ? 1 : (prm->prec == SILH_FP8 ? 2 : 0);
  c->p2_rows = c->mfma ? phase2_mfma_rows(c->mprec, c->DM) : phase2_valu_rows(prm->metric, c->DM);
  silh_status s = build_index(c);
  if (s != SILH_OK) {
    std::string msg = g_err;
    silh_destroy(c);
    g_err = msg;
    return s;
  }
  *out = c;
  return SILH_OK;
}

// Scan the selection flags, read the per-cluster sample counts back, and pack
// the selected rows into the padded cluster-blocked layout.
// With *overflow non-null, Phase 1 built its W work items on the device: the
// F0 offsets and the capacity status come back with the sample offsets (one
// read-back), and *overflow reports whether a capacity was exceeded (then
// nothing is packed and the caller runs Phase 1 again with exact sizes).
silh_status compact_and_pack(silh_ctx* c, bool* overflow) {
  const int n = c->n, k = c->k;
  {
    Launch L(c, K_SCAN);
    launch_scan(c->st, c->flag, n, c->pos, c->scan_tmp);
    CHK(L.done());
  }
  launch_gather_at(c->st, c->pos, c->off, k, c->s_off);
  HIPCHK(hipGetLastError());
  c->s_off32_h.assign(k + 1, 0);
  if (overflow) {
    CHK(fetch(c, {{c->s_off32_h.data(), c->s_off, (k + 1) * sizeof(int32_t)},
                  {c->f0_off32_h.data(), c->f0_off, (k + 1) * sizeof(int32_t)},
                  {&c->p1_status_h, c->p1_status, sizeof(int)}}));
    *overflow = (c->p1_status_h & (kStatusF0 | kStatusPartial)) != 0;
    if (*overflow) return SILH_OK;
    for (int j = 0; j <= k; ++j) c->f0_off_h[j] = c->f0_off32_h[j];
    c->F0 = c->f0_off_h[k];
  } else {
    CHK(fetch(c, {{c->s_off32_h.data(), c->s_off, (k + 1) * sizeof(int32_t)}}));
  }
  c->s_off_h.assign(k + 1, 0);
  c->cnt_h.assign(k, 0);
  c->sp_off_h.assign(k + 1, 0);
  for (int j = 0; j <= k; ++j) c->s_off_h[j] = c->s_off32_h[j];
  for (int j = 0; j < k; ++j) {
    c->cnt_h[j] = c->s_off32_h[j + 1] - c->s_off32_h[j];
    c->sp_off_h[j + 1] = c->sp_off_h[j] + (int32_t)(ceil_div(c->cnt_h[j], kSamplePad) * kSamplePad);
  }
  c->S = c->s_off_h[k];
  c->S_pad = c->sp_off_h[k];
  const int prec = c->mprec;
  const int KP = c->mfma ? mfma_kp(prec, c->DM) : 0;
  const bool mfma_pack = c->mfma && c->S_pad > 0;
  {
    Carve cv;
    cv.add(&c->gid_view, (size_t)c->S).add(&c->gid_pk, (size_t)c->S_pad).add(&c->w32, (size_t)c->S_pad);
    cv.add(&c->aux32, (size_t)c->S_pad).add(&c->Y32, (size_t)c->S_pad * c->DM);
    unsigned char* ym = nullptr;
    if (mfma_pack) {
      cv.add(&c->mu, mfma_mu_floats(c->mprec, c->DM, k)).add(&c->bnorm, (size_t)c->S_pad);
      cv.add(&ym, (size_t)c->S_pad * mfma_row_bytes(prec, c->DM));
    }
    CHK(cv.commit(c, c->alloc_sample));
    c->Ym = ym;
  }
  CHK(h2d_pair(c, c->sp_off, c->sp_off_h, c->cnt, c->cnt_h));
  // every packed row, padding included, is written by k_pack (no clears)
  {
    Launch L(c, K_PACK);
    launch_pack(c->st, c->perm, c->slab, c->flag, c->pos, n, k, c->X, c->d, c->DM, c->p_gid, c->s_off,
                c->sp_off, pack_mode(c->prm.metric), c->rn, (int)c->S_pad, c->gid_view, c->gid_pk,
                c->w32, c->aux32, c->Y32);
    CHK(L.done());
  }
  if (mfma_pack) {
    {
      Launch L(c, K_CENTER);
      launch_center(c->st, c->Y32, c->DM, KP, c->sp_off, c->cnt, k, c->mu);
      CHK(L.done());
    }
    {
      Launch L(c, K_PACK_MFMA);
      if (!launch_pack_mfma(c->st, c->prm.metric, prec, c->DM, c->Y32, c->aux32, c->w32, c->gid_pk, c->sp_off,
                            c->cnt, k, c->mu, (int)c->S_pad, c->Ym, c->bnorm))
        return fail(SILH_E_UNSUPPORTED, "no MFMA packing for metric %d, d=%d", c->prm.metric, c->d);
      CHK(L.done());
    }
  }
  c->state = 1;
  return SILH_OK;
}

silh_status sample_stage_buffers(silh_ctx* c) {
  free_list(c, c->alloc_sample);
  c->state = 0;
  c->f0_gid = c->gid_view = nullptr;
  c->f0_cl = c->items = c->citem_first = c->citem_count = c->gid_pk = c->imeta = nullptr;
  c->ibase = c->dbase = nullptr;
  c->dkeep = nullptr;
  c->f0X = c->W0 = c->partial = nullptr;
  c->w32 = c->aux32 = c->Y32 = c->mu = c->bnorm = nullptr;
  c->Ym = nullptr;
  const int n = c->n, k = c->k;
  const int nb = (int)ceil_div(n, c->p2_rows);
  Carve cv;
  cv.add(&c->flag, (size_t)n).add(&c->pos, (size_t)n + 1).add(&c->scan_tmp, (size_t)ceil_div(n, kScanTile) + 1);
  // f0_off, s_off and the Phase-1 status are read back together (one copy)
  cv.add(&c->p_gid, (size_t)n).add(&c->f0_off, (size_t)k + 1).add(&c->s_off, (size_t)k + 1).add(&c->p1_status, 1);
  cv.add(&c->sp_off, (size_t)k + 1).add(&c->cnt, (size_t)k).add(&c->bpart, (size_t)nb).add(&c->mean_d, 1);
  return cv.commit(c, c->alloc_sample);
}

// Phase 1.  PPS builds the W(e_bar) work items on the device from the F0
// offsets (k_f0_items) with the F0 arrays at a capacity of 64k + 1024 rows,
// so nothing is read back between the initial sample and the draw; if F0 (or
// the partial sums) outgrow their capacity, Phase 1 runs again with the F0
// offsets read back and the items built on the host (host_items).
silh_status phase1(silh_ctx* c, bool host_items = false) {
  const int n = c->n, k = c->k, d = c->d;
  CHK(sample_stage_buffers(c));
  c->F0 = 0;
  c->f0_off_h.assign(k + 1, 0);
  c->f0_off32_h.assign(k + 1, 0);
  const bool pps = c->prm.sampler == SILH_PPS;
  // members per work item: one per thread of the W-pass block
  const int chunk = c->DM > 128 ? kWChunkWide : kWChunk;
  if (pps) {
    // initial sample F^0
    {
      Launch L(c, K_F0_FLAG);
      launch_f0_flag(c->st, c->perm, c->slab, n, c->csize, c->q, c->t, c->prm.seed, c->flag);
      CHK(L.done());
    }
    {
      Launch L(c, K_SCAN);
      launch_scan(c->st, c->flag, n, c->pos, c->scan_tmp);
      CHK(L.done());
    }
    launch_gather_at(c->st, c->pos, c->off, k, c->f0_off);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemsetAsync(c->f0_off, 0, (size_t)(k + 1) * sizeof(int32_t), c->st));
  }
  int nitems = 0;
  int64_t f0_rows = 0;
  if (pps && !host_items) {
    const int64_t f0_cap = std::min<int64_t>(n, 64 * (int64_t)k + 1024);
    const int64_t items_cap = ceil_div(n, chunk) + k;
    const int64_t part_cap = std::min<int64_t>((int64_t)1 << 30, items_cap * 64);
    // the W pass keeps its distances for the draw when they fit
    const int64_t dist_cap = dist_capacity(n, std::log(5.0 * (double)k / c->prm.delta));
    {
      Carve cv;
      cv.add(&c->f0_gid, (size_t)f0_cap).add(&c->f0_cl, (size_t)f0_cap).add(&c->f0X, (size_t)f0_cap * c->DM);
      cv.add(&c->W0, (size_t)f0_cap).add(&c->items, (size_t)items_cap * 6).add(&c->citem_first, (size_t)k);
      cv.add(&c->citem_count, (size_t)k).add(&c->partial, (size_t)part_cap).add(&c->ibase, (size_t)k);
      cv.add(&c->imeta, 2);
      if (dist_cap > 0) cv.add(&c->dbase, (size_t)k).add(&c->dkeep, (size_t)dist_cap);
      CHK(cv.commit(c, c->alloc_sample));
    }
    launch_f0_items(c->st, c->csize, c->off, c->f0_off, k, c->t, chunk, (int)f0_cap, part_cap, (int)items_cap,
                    c->citem_first, c->citem_count, c->ibase, c->imeta, c->items, c->p1_status, c->dbase,
                    dist_cap, true);
    HIPCHK(hipGetLastError());
    {
      Launch L(c, K_F0_PACK);
      launch_f0_pack(c->st, c->perm, c->slab, c->flag, c->pos, n, c->X, d, c->DM, (int)f0_cap, c->f0_gid,
                     c->f0_cl, c->f0X);
      CHK(L.done());
    }
    nitems = (int)items_cap;  // the unused item slots are empty
    f0_rows = f0_cap;         // W blocks past F0 return at once
  } else if (pps) {
    CHK(fetch(c, {{c->f0_off32_h.data(), c->f0_off, (k + 1) * sizeof(int32_t)}}));
    for (int j = 0; j <= k; ++j) c->f0_off_h[j] = c->f0_off32_h[j];
    c->F0 = c->f0_off_h[k];
    // work items for W(e_bar), built on the host
    c->items_h.clear();
    c->citem_first_h.assign(k, 0);
    c->citem_count_h.assign(k, 0);
    int64_t pbase = 0;
    if (c->F0 > 0) {
      for (int j = 0; j < k; ++j) {
        const int fj = c->f0_off32_h[j + 1] - c->f0_off32_h[j];
        c->citem_first_h[j] = (int32_t)(c->items_h.size() / 6);
        if ((int64_t)c->csize_h[j] <= c->t || fj == 0) continue;
        for (int b = c->off_h[j]; b < c->off_h[j + 1]; b += chunk) {
          const int e = b + chunk < c->off_h[j + 1] ? b + chunk : c->off_h[j + 1];
          c->items_h.insert(c->items_h.end(), {j, b, e, c->f0_off32_h[j], fj, (int32_t)pbase});
          pbase += fj;
          c->citem_count_h[j] += 1;
        }
        if (pbase > (int64_t)1 << 30) return fail(SILH_E_ARG, "initial sample too large");
      }
    }
    nitems = (int)(c->items_h.size() / 6);
    f0_rows = c->F0;
    {
      Carve cv;
      cv.add(&c->f0_gid, (size_t)c->F0).add(&c->f0_cl, (size_t)c->F0).add(&c->f0X, (size_t)c->F0 * c->DM);
      cv.add(&c->W0, (size_t)c->F0).add(&c->items, c->items_h.size()).add(&c->citem_first, (size_t)k);
      cv.add(&c->citem_count, (size_t)k).add(&c->partial, (size_t)pbase);
      CHK(cv.commit(c, c->alloc_sample));
    }
    if (c->F0 > 0) {
      {
        Launch L(c, K_F0_PACK);
        launch_f0_pack(c->st, c->perm, c->slab, c->flag, c->pos, n, c->X, d, c->DM, (int)c->F0, c->f0_gid,
                       c->f0_cl, c->f0X);
        CHK(L.done());
      }
      CHK(h2d(c, c->items, c->items_h));
      CHK(h2d(c, c->citem_first, c->citem_first_h));
      CHK(h2d(c, c->citem_count, c->citem_count_h));
    }
  }
  DistStore ds;
  if (c->dkeep != nullptr) {
    ds.d = c->dkeep;
    ds.base = c->dbase;
    ds.off = c->off;
    ds.use = c->imeta + 1;
  }
  if (pps && nitems > 0 && f0_rows > 0) {
    {
      Launch L(c, K_W_PARTIAL);
      launch_w_partial(c->st, c->prm.metric, c->DM, c->items, nitems, c->perm, c->X, d, c->f0X, c->partial,
                       ds);
      CHK(L.done());
    }
    {
      Launch L(c, K_W_FINAL);
      launch_w_final(c->st, c->f0_cl, (int)f0_rows, c->f0_off, k, c->citem_first, c->citem_count, c->items,
                     c->partial, c->W0);
      CHK(L.done());
    }
  }
  {
    Launch L(c, K_DRAW);
    launch_draw(c->st, c->prm.metric, c->DM, pps ? 0 : 1, c->perm, c->slab, n, c->X, d, c->csize, c->t,
                c->prm.seed, c->f0_off, c->f0X, c->W0, c->p_gid, c->flag, ds);
    CHK(L.done());
  }
  if (pps && !host_items) {
    bool overflow = false;
    CHK(compact_and_pack(c, &overflow));
    if (overflow) return phase1(c, true);
    return SILH_OK;
  }
  return compact_and_pack(c, nullptr);
}

// ---- autotuning of the MFMA Phase-2 block shape ------------------------------
// Key: (metric, operand type, padded row width, floor(log2(padded sample
// size))).  On the first Phase-2 launch of a key every valid shape (blocks
// per wave, tiles per LDS stage: mfma_shapes) runs twice on the context's
// stream, timed with events, and the fastest is kept for the process.  Every
// shape writes the same values (each element's arithmetic and the
// 128-element partials of the mean do not depend on it).
std::mutex g_tune_mu;
std::map<std::array<int, 4>, int> g_tune;
std::atomic<int> g_tune_mode{1};

int size_bucket(int64_t S_pad) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << (b + 1)) <= S_pad) ++b;
  return b;
}

int pick_pb(silh_ctx* c, const P2Args& A) {
  int ids[3];
  const int m = mfma_shapes(c->mprec, c->DM, ids);
  const int mode = g_tune_mode.load();
  if (mode == 0 || m == 1) return m == 1 ? 1 : pb_builtin(c->prm.metric, c->mprec, c->DM);
  if (mode >= 2) {  // a fixed shape where valid, else the built-in one
    for (int i = 0; i < m; ++i)
      if (ids[i] == mode - 1) return ids[i];
    return pb_builtin(c->prm.metric, c->mprec, c->DM);
  }
  const std::array<int, 4> key{c->prm.metric, c->mprec, c->DM, size_bucket(c->S_pad)};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  // each shape launched twice, in two rounds over the shapes, and the faster
  // launch of each compared (one launch of each mis-picks when they are
  // ~10 % apart)
  hipEvent_t e[7] = {};
  bool ok = true;
  for (int i = 0; i <= 2 * m; ++i) ok = ok && hipEventCreate(&e[i]) == hipSuccess;
  float best_t[3] = {0.f, 0.f, 0.f};
  if (ok) {
    ok = hipEventRecord(e[0], c->st) == hipSuccess;
    for (int r = 0; r < 2 * m && ok; ++r)
      ok = launch_phase2_mfma(c->st, c->prm.metric, c->mprec, c->DM, A, c->mu, c->Ym, c->bnorm, ids[r % m]) &&
           hipEventRecord(e[r + 1], c->st) == hipSuccess;
    ok = ok && hipEventSynchronize(e[2 * m]) == hipSuccess;
    for (int r = 0; r < 2 * m && ok; ++r) {
      float dt = 0.f;
      ok = hipEventElapsedTime(&dt, e[r], e[r + 1]) == hipSuccess;
      if (r < m || dt < best_t[r % m]) best_t[r % m] = dt;
    }
  }
  for (auto& ev : e)
    if (ev) (void)hipEventDestroy(ev);
  if (!ok) {
    (void)hipGetLastError();
    return pb_builtin(c->prm.metric, c->mprec, c->DM);
  }
  int choice = ids[0];
  float tb = best_t[0];
  for (int i = 1; i < m; ++i)
    if (best_t[i] < tb) {
      tb = best_t[i];
      choice = ids[i];
    }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.emplace(key, choice);
  return choice;
}

bool launch_p2(silh_ctx* c, const P2Args& A, int pb) {
  if (!c->mfma) return launch_phase2_valu(c->st, c->prm.metric, c->DM, A);
  return launch_phase2_mfma(c->st, c->prm.metric, c->mprec, c->DM, A, c->mu, c->Ym, c->bnorm, pb);
}

silh_status run_phase2(silh_ctx* c, float* a, float* b, float* s, float* What, double* mean_host) {
  P2Args A;
  A.X = c->X;
  A.n = c->n;
  A.d = c->d;
  A.labels = c->labels;
  A.Y = c->Y32;
  A.w = c->w32;
  A.aux = c->aux32;
  A.gid_pk = c->gid_pk;
  A.sp_off = c->sp_off;
  A.cnt = c->cnt;
  A.csize = c->csize;
  A.k = c->k;
  A.a = a;
  A.b = b;
  A.s = s;
  A.What = What;
  A.bpart = c->bpart;
  A.rn = c->rn;
  free_list(c, c->alloc_p2);
  if (!c->mfma && phase2_valu_split(c->prm.metric, c->DM)) {
    Carve cv;
    cv.add(&A.Wpart, (size_t)c->n * c->k);
    CHK(cv.commit(c, c->alloc_p2));
  }
  {
    const int pb = c->mfma ? pick_pb(c, A) : 0;  // (tuning runs stay outside the timed launch)
    Launch L(c, K_PHASE2);
    const bool ok = launch_p2(c, A, pb);
    if (!ok) return fail(SILH_E_UNSUPPORTED, "no Phase-2 kernel for metric %d, d=%d", c->prm.metric, c->d);
    CHK(L.done());
  }
  if (mean_host) {
    {
      Launch L(c, K_MEAN);
      launch_mean(c->st, c->bpart, (int)ceil_div(c->n, c->p2_rows), c->n, c->mean_d);
      CHK(L.done());
    }
    CHK(fetch(c, {{&c->mean_h, c->mean_d, sizeof(double)}}));
    *mean_host = c->mean_h;
  }
  return SILH_OK;
}

// Phase 2 for the entries of rows[0..m) (duplicates allowed): the distinct
// rows are gathered into a contiguous block and run through the same Phase-2
// kernels, with the sample's ids renumbered into that block so that the
// self-pair test still finds each element's own column.
silh_status rows_phase2(silh_ctx* c, const int32_t* rows, int64_t m, float* a, float* b, float* s,
                        double* mean_host) {
  if (!rows) return fail(SILH_E_ARG, "rows is NULL");
  if (m < 1 || m > kMaxN) return fail(SILH_E_ARG, "m=%lld outside [1, 2^30]", (long long)m);
  free_list(c, c->alloc_rows);
  const int n = c->n, d = c->d;
  const int64_t cap = m < n ? m : n;  // distinct rows
  int32_t *mark = nullptr, *pos = nullptr, *tmp = nullptr, *urows = nullptr, *ls = nullptr, *gsub = nullptr;
  int* bad = nullptr;
  float *Xs = nullptr, *au = nullptr, *bu = nullptr, *su = nullptr, *rnu = nullptr;
  double *bpu = nullptr, *bpm = nullptr, *mean_d = nullptr;
  const int64_t nbm = ceil_div(m, kRowsBlock);
  {
    Carve cv;
    cv.add(&mark, (size_t)n).add(&pos, (size_t)n + 1).add(&tmp, (size_t)ceil_div(n, kScanTile) + 1);
    cv.add(&urows, (size_t)cap).add(&bad, 1).add(&Xs, (size_t)cap * d).add(&ls, (size_t)cap);
    cv.add(&gsub, (size_t)c->S_pad).add(&au, (size_t)cap).add(&bu, (size_t)cap).add(&su, (size_t)cap);
    cv.add(&bpu, (size_t)ceil_div(cap, c->p2_rows)).add(&bpm, (size_t)nbm).add(&mean_d, 1);
    if (c->rn) cv.add(&rnu, (size_t)cap);
    CHK(cv.commit(c, c->alloc_rows));
  }
  HIPCHK(hipMemsetAsync(mark, 0, (size_t)n * sizeof(int32_t), c->st));
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), c->st));
  launch_rows_mark(c->st, rows, m, n, mark, bad);
  HIPCHK(hipGetLastError());
  launch_scan(c->st, mark, n, pos, tmp);
  HIPCHK(hipGetLastError());
  int32_t mu_h = 0;
  int bad_h = 0;
  CHK(fetch(c, {{&mu_h, pos + n, sizeof(int32_t)}, {&bad_h, bad, sizeof(int)}}));
  if (bad_h) return fail(SILH_E_ARG, "a row index lies outside [0, %d)", n);
  const int mu = mu_h;
  launch_rows_compact(c->st, mark, pos, n, urows);
  launch_rows_gather(c->st, c->X, c->labels, d, urows, mu, Xs, ls);
  launch_rows_remap(c->st, c->gid_pk, c->S_pad, urows, mu, gsub);
  if (rnu) launch_rnorm(c->st, Xs, mu, d, rnu);  // the same factors as for the rows of X
  HIPCHK(hipGetLastError());
  P2Args A;
  A.X = Xs;
  A.n = mu;
  A.d = d;
  A.labels = ls;
  A.Y = c->Y32;
  A.w = c->w32;
  A.aux = c->aux32;
  A.gid_pk = gsub;
  A.sp_off = c->sp_off;
  A.cnt = c->cnt;
  A.csize = c->csize;
  A.k = c->k;
  A.a = au;
  A.b = bu;
  A.s = su;
  A.What = nullptr;
  A.bpart = bpu;
  A.rn = rnu;
  if (!c->mfma && phase2_valu_split(c->prm.metric, c->DM)) {
    Carve cv;
    cv.add(&A.Wpart, (size_t)(mu > 0 ? mu : 1) * c->k);
    CHK(cv.commit(c, c->alloc_rows));
  }
  {
    const int pb = c->mfma ? pick_pb(c, A) : 0;  // (tuning runs stay outside the timed launch)
    Launch L(c, K_PHASE2);
    const bool ok = launch_p2(c, A, pb);
    if (!ok) return fail(SILH_E_UNSUPPORTED, "no Phase-2 kernel for metric %d, d=%d", c->prm.metric, c->d);
    CHK(L.done());
  }
  launch_rows_expand(c->st, rows, m, urows, mu, au, bu, su, a, b, s, bpm);
  HIPCHK(hipGetLastError());
  if (mean_host) {
    launch_mean(c->st, bpm, (int)nbm, m, mean_d);
    HIPCHK(hipGetLastError());
    CHK(fetch(c, {{&c->mean_h, mean_d, sizeof(double)}}));
    *mean_host = c->mean_h;
  }
  return SILH_OK;
}

}  // namespace

namespace silh {
silh_status validate_params(const silh_params* prm, const float* X, const int32_t* labels, int64_t* t) {
  return check_params(prm, X, labels, false, t);
}
silh_status validate_exact_params(const silh_params* prm, const float* X, const int32_t* labels) {
  int64_t t = 0;
  return check_params(prm, X, labels, true, &t);
}
int dm_for(int d) { return phase2_valu_dm(d); }
silh_status set_error(silh_status st, const char* msg) { return fail(st, "%s", msg); }
int64_t sample_rows(const silh_ctx* c) { return c && c->state == 1 ? c->S_pad : 0; }

int tuned_shape(silh_ctx* c) {
  if (!c || c->state != 1 || !c->mfma) return 1;
  P2Args A;
  A.X = c->X;
  A.n = c->n;
  A.d = c->d;
  A.labels = c->labels;
  A.Y = c->Y32;
  A.w = c->w32;
  A.aux = c->aux32;
  A.gid_pk = c->gid_pk;
  A.sp_off = c->sp_off;
  A.cnt = c->cnt;
  A.csize = c->csize;
  A.k = c->k;
  A.a = A.b = A.s = A.What = nullptr;
  A.bpart = c->bpart;
  A.rn = c->rn;
  return pick_pb(c, A);
}

bool phase2_job(silh_ctx* c, P2Job* job, P2Class* cls) {
  if (!c || c->state != 1) return false;
  const bool batch = c->mfma || phase2_valu_jobs_ok(c->prm.metric, c->DM);
  if (!batch) return false;
  P2Job J{};
  J.X = c->X;
  J.labels = c->labels;
  J.Ym = c->Ym;
  J.w = c->w32;
  J.gid_pk = c->gid_pk;
  J.sp_off = c->sp_off;
  J.cnt = c->cnt;
  J.csize = c->csize;
  J.mu = c->mu;
  J.a = J.b = J.s = J.What = nullptr;
  J.bpart = c->bpart;
  J.bnorm = c->bnorm;
  J.Y32 = c->Y32;
  J.aux = c->aux32;
  J.rn = c->rn;
  J.n = c->n;
  J.d = c->d;
  J.k = c->k;
  *job = J;
  P2Class K{};
  K.mfma = c->mfma ? 1 : 0;
  K.metric = c->prm.metric;
  K.prec = c->mfma ? c->mprec : -1;
  K.DM = c->DM;
  K.pb = c->mfma ? tuned_shape(c) : 1;
  K.rows = c->mfma ? phase2_mfma_rows(c->mprec, c->DM) * (K.pb == 2 ? 2 : 1) : c->p2_rows;
  K.blocks = ceil_div(c->n, K.rows);
  K.S_pad = c->S_pad;
  *cls = K;
  return true;
}

bool launch_phase2_class(hipStream_t st, const P2Class& cls, const P2Job* jobs, const int2* items, int nitems) {
  if (cls.mfma) return launch_phase2_mfma_jobs(st, cls.metric, cls.prec, cls.DM, cls.pb, jobs, items, nitems);
  return launch_phase2_valu_jobs(st, cls.metric, cls.DM, jobs, items, nitems);
}

silh_status phase2_job_mean(silh_ctx* c, double* mean) {
  if (!c || c->state != 1) return fail(SILH_E_STATE, "no sampled context");
  {
    Launch L(c, K_MEAN);
    launch_mean(c->st, c->bpart, (int)ceil_div(c->n, c->p2_rows), c->n, c->mean_d);
    CHK(L.done());
  }
  CHK(fetch(c, {{&c->mean_h, c->mean_d, sizeof(double)}}));
  *mean = c->mean_h;
  return SILH_OK;
}

int pb_builtin(int metric, int prec, int DM) {
  if (metric == SILH_COS && prec == 1 && DM == 32) return 2;
  return mfma_pb_default(prec, DM);
}

}  // namespace silh

extern "C" {

silh_status silh_sample_init(const silh_params* prm, const float* X, const int32_t* labels,
                             silh_stream stream, silh_ctx** out) {
  if (!out) return fail(SILH_E_ARG, "out is NULL");
  *out = nullptr;
  return create(prm, X, labels, stream, false, out);
}

silh_status silh_pps_sample(silh_ctx* c, int64_t* S_host, int64_t* per_cluster_host) {
  if (!c) return fail(SILH_E_ARG, "ctx is NULL");
  silh_status s = phase1(c);
  if (s != SILH_OK) {
    c->state = 0;
    return s;
  }
  if (S_host) *S_host = c->S;
  if (per_cluster_host)
    for (int j = 0; j < c->k; ++j) per_cluster_host[j] = c->cnt_h[j];
  return SILH_OK;
}

silh_status silh_weighted_sums(silh_ctx* c, float* W_hat) {
  if (!c) return fail(SILH_E_ARG, "ctx is NULL");
  if (!W_hat) return fail(SILH_E_ARG, "W_hat is NULL");
  if (c->state != 1) return fail(SILH_E_STATE, "silh_weighted_sums before a successful silh_pps_sample");
  return run_phase2(c, nullptr, nullptr, nullptr, W_hat, nullptr);
}

silh_status silh_scores(silh_ctx* c, float* a, float* b, float* s, double* s_mean_host) {
  if (!c) return fail(SILH_E_ARG, "ctx is NULL");
  if (c->state != 1) return fail(SILH_E_STATE, "silh_scores before a successful silh_pps_sample");
  return run_phase2(c, a, b, s, nullptr, s_mean_host);
}

silh_status silh_exact(const silh_params* prm, const float* X, const int32_t* labels, silh_stream stream,
                       float* a, float* b, float* s, double* s_mean_host) {
  silh_ctx* c = nullptr;
  CHK(create(prm, X, labels, stream, true, &c));
  silh_status st = sample_stage_buffers(c);
  if (st == SILH_OK) {
    Launch L(c, K_DRAW);
    launch_fill_all(c->st, c->perm, c->n, c->p_gid, c->flag);
    st = L.done();
  }
  if (st == SILH_OK) st = compact_and_pack(c, nullptr);
  if (st == SILH_OK) st = run_phase2(c, a, b, s, nullptr, s_mean_host);
  std::string msg = g_err;
  silh_destroy(c);
  g_err = msg;
  return st;
}

silh_status silh_rows_for(double eps, double delta, int64_t* m) {
  if (!m) return fail(SILH_E_ARG, "m is NULL");
  if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0))
    return fail(SILH_E_ARG, "eps and delta must lie in (0, 1)");
  const double v = std::ceil((2.0 / (eps * eps)) * std::log(2.0 / delta));
  if (!(v <= (double)kMaxN)) return fail(SILH_E_ARG, "m=%g exceeds 2^30", v);
  *m = (int64_t)v;
  return SILH_OK;
}

silh_status silh_draw_rows(uint64_t seed, int64_t n, int64_t m, int32_t* rows, silh_stream stream) {
  if (n < 1 || n > kMaxN) return fail(SILH_E_ARG, "n=%lld outside [1, 2^30]", (long long)n);
  if (m < 0 || m > kMaxN) return fail(SILH_E_ARG, "m=%lld outside [0, 2^30]", (long long)m);
  if (m > 0 && !rows) return fail(SILH_E_ARG, "rows is NULL");
  launch_rows_draw((hipStream_t)stream, seed, n, m, rows);
  HIPCHK(hipGetLastError());
  return SILH_OK;
}

silh_status silh_scores_rows(silh_ctx* c, const int32_t* rows, int64_t m, float* a, float* b, float* s,
                             double* s_mean_host) {
  if (!c) return fail(SILH_E_ARG, "ctx is NULL");
  if (c->state != 1) return fail(SILH_E_STATE, "silh_scores_rows before a successful silh_pps_sample");
  return rows_phase2(c, rows, m, a, b, s, s_mean_host);
}

silh_status silh_exact_rows(const silh_params* prm, const float* X, const int32_t* labels,
                            const int32_t* rows, int64_t m, silh_stream stream, float* a, float* b,
                            float* s, double* s_mean_host) {
  silh_ctx* c = nullptr;
  CHK(create(prm, X, labels, stream, true, &c));
  silh_status st = sample_stage_buffers(c);
  if (st == SILH_OK) {
    Launch L(c, K_DRAW);
    launch_fill_all(c->st, c->perm, c->n, c->p_gid, c->flag);
    st = L.done();
  }
  if (st == SILH_OK) st = compact_and_pack(c, nullptr);
  if (st == SILH_OK) st = rows_phase2(c, rows, m, a, b, s, s_mean_host);
  std::string msg = g_err;
  silh_destroy(c);
  g_err = msg;
  return st;
}

silh_status silh_coh_sep(silh_ctx* c, const float* W_hat, double* coh_host, double* sep_host) {
  if (!c) return fail(SILH_E_ARG, "ctx is NULL");
  if (!coh_host || !sep_host) return fail(SILH_E_ARG, "coh_host or sep_host is NULL");
  if (c->state != 1) return fail(SILH_E_STATE, "silh_coh_sep before a successful silh_pps_sample");
  free_list(c, c->alloc_rows);
  const int n = c->n, k = c->k;
  const int nb = coh_sep_blocks(n);
  float* W = nullptr;
  double *cpart = nullptr, *spart = nullptr, *sums = nullptr;
  {
    Carve cv;
    if (!W_hat) cv.add(&W, (size_t)n * k);
    cv.add(&cpart, (size_t)nb).add(&spart, (size_t)nb).add(&sums, 2);
    CHK(cv.commit(c, c->alloc_rows));
  }
  if (!W_hat) {
    CHK(run_phase2(c, nullptr, nullptr, nullptr, W, nullptr));
    W_hat = W;
  }
  launch_coh_sep(c->st, W_hat, n, k, c->labels, cpart, spart);
  launch_mean(c->st, cpart, nb, 1, sums);
  launch_mean(c->st, spart, nb, 1, sums + 1);
  HIPCHK(hipGetLastError());
  double h[2] = {0.0, 0.0};
  CHK(fetch(c, {{h, sums, sizeof(h)}}));
  // denominators: unordered pairs inside clusters, and across clusters
  int64_t pin = 0, pout = 0, before = 0;
  for (int j = 0; j < k; ++j) {
    const int64_t cj = c->csize_h[j];
    pin += cj * (cj - 1) / 2;
    pout += cj * ((int64_t)n - before - cj);
    before += cj;
  }
  *coh_host = pin > 0 ? 0.5 * h[0] / (double)pin : 0.0;
  *sep_host = pout > 0 ? h[1] / (double)pout : 0.0;
  return SILH_OK;
}

silh_status silh_set_tuning(int mode) {
  if (mode < 0 || mode > 4) return fail(SILH_E_ARG, "tuning mode %d outside [0, 4]", mode);
  g_tune_mode.store(mode);
  if (mode == 1) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
  }
  return SILH_OK;
}

silh_status silh_tuning_choice(int metric, int prec, int d, int64_t S_pad, int* pb) {
  if (!pb) return fail(SILH_E_ARG, "pb is NULL");
  const int DM = phase2_valu_dm(d);
  const int mprec = prec == SILH_BF16 ? 1 : (prec == SILH_FP8 ? 2 : 0);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(std::array<int, 4>{metric, mprec, DM, size_bucket(S_pad)});
  *pb = it == g_tune.end() ? 0 : it->second;
  return SILH_OK;
}

silh_status silh_sample_view(silh_ctx* c, silh_sample_info* out) {
  if (!c || !out) return fail(SILH_E_ARG, "ctx or out is NULL");
  if (c->state != 1) return fail(SILH_E_STATE, "silh_sample_view before a successful silh_pps_sample");
  out->S = c->S;
  out->gid = c->gid_view;
  out->offsets_host = c->s_off_h.data();
  out->p = c->p_gid;
  out->F0 = c->F0;
  out->f0_gid = c->f0_gid;
  out->f0_W = c->W0;
  out->f0_offsets_host = c->f0_off_h.data();
  out->t = c->t;
  return SILH_OK;
}

silh_status silh_philox_uniform(uint64_t seed, int64_t gid0, int64_t count, uint32_t stream_id,
                                double* out, silh_stream stream) {
  if (count < 0 || gid0 < 0) return fail(SILH_E_ARG, "count and gid0 must be >= 0");
  if (count > 0 && !out) return fail(SILH_E_ARG, "out is NULL");
  launch_uniform((hipStream_t)stream, seed, gid0, count, stream_id, out);
  HIPCHK(hipGetLastError());
  return SILH_OK;
}

silh_status silh_prof_enable(silh_ctx* c, int on) {
  if (!c) return fail(SILH_E_ARG, "ctx is NULL");
  if (on < 0 || on > 2) return fail(SILH_E_ARG, "profiling mode %d outside [0, 2]", on);
  c->prof_on = on != 0;
  c->prof_mode = on;
  return SILH_OK;
}

silh_status silh_prof_reset(silh_ctx* c) {
  if (!c) return fail(SILH_E_ARG, "ctx is NULL");
  CHK(drain_prof(c));
  for (int i = 0; i < K_NSLOTS; ++i) {
    c->tot_ms[i] = 0.0;
    c->launches[i] = 0;
  }
  return SILH_OK;
}

int silh_prof_count(void) { return K_NSLOTS; }

silh_status silh_prof_get(silh_ctx* c, int i, const char** name, int64_t* launches, double* total_ms) {
  if (!c) return fail(SILH_E_ARG, "ctx is NULL");
  if (i < 0 || i >= K_NSLOTS) return fail(SILH_E_ARG, "slot %d outside [0, %d)", i, (int)K_NSLOTS);
  CHK(drain_prof(c));
  if (name) *name = kSlotNames[i];
  if (launches) *launches = c->launches[i];
  if (total_ms) *total_ms = c->tot_ms[i];
  return SILH_OK;
}

void silh_destroy(silh_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  for (auto& p : c->pending) {
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
  return_events(c->pool);
  pin_release(c);
  free_list(c, c->alloc_p2);
  free_list(c, c->alloc_rows);
  free_list(c, c->alloc_sample);
  free_list(c, c->alloc_init);
  delete c;
}

const char* silh_last_error(void) { return g_err.c_str(); }

const char* silh_version(void) { return "silh-mi355x 0.1 (gfx950)"; }

}  // extern "C"
