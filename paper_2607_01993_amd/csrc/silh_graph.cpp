// K clusterings of one dataset as one captured HIP graph (include/silh_graph.h).
//
// Each clustering's work is the eager pipeline of silh_api.cpp (cluster
// index, Phase 1 of Algorithm 1, packing, Phase 2, the mean of Eq. 9) with the
// same kernels, except that the sizes the eager path reads back and turns
// into offsets, work items and buffer sizes on the host are computed on the
// device (k_graph.hip) and every buffer is sized by a capacity.  Nothing then
// waits on the host between kernels, and the K pipelines are captured once,
// spread over `chains` streams forked from the capture stream, so the graph
// holds that many independent branches.  A branch reuses its buffers for its
// clusterings one after another.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <new>
#include <vector>

#include "../../include/silh_graph.h"
#include "silh_internal.hpp"

using namespace silh;

namespace {

// one branch's buffers, reused by its clusterings in turn
struct Branch {
  hipStream_t st = nullptr;
  hipEvent_t join = nullptr;
  int* status = nullptr;
  int32_t *uh = nullptr, *csize = nullptr, *off = nullptr, *perm = nullptr, *slab = nullptr;
  double* q = nullptr;
  int32_t *flag = nullptr, *pos = nullptr, *scan_tmp = nullptr;
  int32_t *f0_off = nullptr, *s_off = nullptr, *sp_off = nullptr, *cnt = nullptr;
  double* p_gid = nullptr;
  int64_t* f0_gid = nullptr;
  int32_t* f0_cl = nullptr;
  double *f0X = nullptr, *W0 = nullptr, *partial = nullptr;
  int32_t *items = nullptr, *citem_first = nullptr, *citem_count = nullptr, *meta = nullptr;
  int64_t* ibase = nullptr;
  int64_t* dbase = nullptr;
  double* dkeep = nullptr;
  int64_t* gid_view = nullptr;
  int32_t* gid_pk = nullptr;
  float *w32 = nullptr, *aux32 = nullptr, *Y32 = nullptr, *mu = nullptr, *bnorm = nullptr;
  void* Ym = nullptr;
  double *bpart = nullptr, *Wpart = nullptr;
};

constexpr int kStatusCapacity = kStatusF0 | kStatusPartial | kStatusSample;

}  // namespace

struct silh_graph {
  silh_params base{};
  const float* X = nullptr;
  const int32_t* labels = nullptr;
  std::vector<int32_t> ks;
  std::vector<int64_t> ts;  // Algorithm 1's t of each clustering (k enters it when derived from eps)
  std::vector<int32_t> shape;    // Phase-2 block shape captured for each clustering
  std::vector<int64_t> probe_S;  // padded sample size of the request the shape was tuned on
  int K = 0, n = 0, d = 0, DM = 0, KP = 0, mprec = 0, p2_rows = 0, chunk = 0, kmax = 0;
  bool mfma = false;
  int64_t S_cap = 0, F0_cap = 0, items_cap = 0, part_cap = 0, dist_cap = 0;
  std::vector<Branch> br;
  std::vector<void*> allocs;
  int64_t bytes = 0;
  double* means_d = nullptr;
  int32_t* status_d = nullptr;
  float* rn = nullptr;  // cosine: reciprocal row norms of X, computed once per replay
  double* means_h = nullptr;    // pinned
  int32_t* status_h = nullptr;  // pinned
  hipStream_t cap_st = nullptr;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t nodes = 0;
};

namespace {

void* gmalloc(silh_graph* g, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (g->base.alloc) {
    p = g->base.alloc(bytes, g->base.alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) {
    g->allocs.push_back(p);
    g->bytes += (int64_t)bytes;
  }
  return p;
}

template <class T>
bool take(silh_graph* g, T*& p, int64_t count) {
  p = (T*)gmalloc(g, (size_t)(count > 0 ? count : 1) * sizeof(T));
  return p != nullptr;
}

void release(silh_graph* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (Branch& b : g->br) {
    if (b.join) (void)hipEventDestroy(b.join);
    if (b.st) (void)hipStreamDestroy(b.st);
  }
  if (g->fork) (void)hipEventDestroy(g->fork);
  if (g->cap_st) (void)hipStreamDestroy(g->cap_st);
  for (void* p : g->allocs) {
    if (g->base.alloc) {
      g->base.free(p, g->base.alloc_user);
    } else {
      (void)hipFree(p);
    }
  }
  if (g->means_h) (void)hipHostFree(g->means_h);
  if (g->status_h) (void)hipHostFree(g->status_h);
  delete g;
}

bool alloc_branch(silh_graph* g, Branch& b) {
  const int64_t n = g->n, k = g->kmax;
  int64_t uh = 0;
  for (int32_t kk : g->ks) {
    const int64_t u = ceil_div(n, sort_seg(n, kk)) * kk;
    uh = u > uh ? u : uh;
  }
  const int64_t S = g->S_cap, F0 = g->F0_cap, DM = g->DM;
  bool ok = take(g, b.status, 1) && take(g, b.uh, uh) && take(g, b.csize, k) && take(g, b.off, k + 1) &&
            take(g, b.perm, n) && take(g, b.slab, n) && take(g, b.q, k) && take(g, b.flag, n) &&
            take(g, b.pos, n + 1) && take(g, b.scan_tmp, ceil_div(n, kScanTile) + 1) &&
            take(g, b.f0_off, k + 1) && take(g, b.s_off, k + 1) && take(g, b.sp_off, k + 1) &&
            take(g, b.cnt, k) && take(g, b.p_gid, n) && take(g, b.f0_gid, F0) && take(g, b.f0_cl, F0) &&
            take(g, b.f0X, F0 * DM) && take(g, b.W0, F0) && take(g, b.partial, g->part_cap) &&
            take(g, b.items, g->items_cap * 6) && take(g, b.citem_first, k) && take(g, b.citem_count, k) &&
            take(g, b.meta, 2) && take(g, b.ibase, k) && take(g, b.gid_view, S) && take(g, b.gid_pk, S) &&
            take(g, b.w32, S) && take(g, b.aux32, S) && take(g, b.Y32, S * DM) &&
            take(g, b.bpart, ceil_div(n, g->p2_rows));
  if (ok && g->mfma) {
    unsigned char* ym = nullptr;
    ok = take(g, b.mu, mfma_mu_floats(g->mprec, g->DM, k)) && take(g, b.bnorm, S) && take(g, ym, S * (size_t)mfma_row_bytes(g->mprec, g->DM));
    b.Ym = ym;
  }
  if (ok && !g->mfma && phase2_valu_split(g->base.metric, g->DM)) ok = take(g, b.Wpart, n * k);
  if (ok && g->dist_cap > 0) ok = take(g, b.dbase, k) && take(g, b.dkeep, g->dist_cap);
  return ok;
}

// clustering i's pipeline on branch b's stream: no host synchronisation,
// no allocation, no memset
bool enqueue(silh_graph* g, Branch& b, int i) {
  const int n = g->n, k = g->ks[i], d = g->d, DM = g->DM;
  const int64_t t = g->ts[i];
  const int32_t* lab = g->labels + (size_t)i * (size_t)n;
  const int seg = sort_seg(n, k);
  const int units = (int)ceil_div(n, seg);
  const int metric = g->base.metric;
  const bool pps = g->base.sampler == SILH_PPS;
  const hipStream_t st = b.st;
  DistStore ds;
  if (b.dkeep != nullptr) {
    ds.d = b.dkeep;
    ds.base = b.dbase;
    ds.off = b.off;
    ds.use = b.meta + 1;
  }
  // cluster index (perm and slab start at 0 so that rows a bad label leaves
  // unwritten still name a valid element)
  launch_fill_i32(st, b.status, 1, 0);
  launch_fill_i32(st, b.perm, n, 0);
  launch_fill_i32(st, b.slab, n, 0);
  launch_unit_hist(st, lab, n, k, seg, b.uh, b.status);
  launch_unit_scan(st, b.uh, units, k, b.csize);
  launch_index_sizes(st, b.csize, k, std::log(5.0 * (double)k / g->base.delta), b.off, b.q, b.status);
  launch_scatter(st, lab, n, k, seg, b.uh, b.off, b.perm, b.slab);
  // Phase 1
  if (pps) {
    launch_f0_flag(st, b.perm, b.slab, n, b.csize, b.q, t, g->base.seed, b.flag);
    launch_scan(st, b.flag, n, b.pos, b.scan_tmp);
    launch_gather_at(st, b.pos, b.off, k, b.f0_off);
    launch_f0_items(st, b.csize, b.off, b.f0_off, k, t, g->chunk, (int)g->F0_cap, g->part_cap, (int)g->items_cap,
                    b.citem_first, b.citem_count, b.ibase, b.meta, b.items, b.status, b.dbase, g->dist_cap);
    launch_f0_pack(st, b.perm, b.slab, b.flag, b.pos, n, g->X, d, DM, (int)g->F0_cap, b.f0_gid, b.f0_cl, b.f0X);
    launch_w_partial(st, metric, DM, b.items, (int)g->items_cap, b.perm, g->X, d, b.f0X, b.partial, ds);
    launch_w_final(st, b.f0_cl, (int)g->F0_cap, b.f0_off, k, b.citem_first, b.citem_count, b.items, b.partial,
                   b.W0);
  } else {
    launch_fill_i32(st, b.f0_off, k + 1, 0);
  }
  launch_draw(st, metric, DM, pps ? 0 : 1, b.perm, b.slab, n, g->X, d, b.csize, t, g->base.seed, b.f0_off, b.f0X,
              b.W0, b.p_gid, b.flag, pps ? ds : DistStore{});
  // compaction and packing
  launch_scan(st, b.flag, n, b.pos, b.scan_tmp);
  launch_gather_at(st, b.pos, b.off, k, b.s_off);
  launch_sample_sizes(st, b.s_off, k, (int)g->S_cap, b.cnt, b.sp_off, b.status);
  launch_pack(st, b.perm, b.slab, b.flag, b.pos, n, k, g->X, d, DM, b.p_gid, b.s_off, b.sp_off,
              pack_mode(metric), g->rn, (int)g->S_cap, b.gid_view, b.gid_pk, b.w32, b.aux32, b.Y32);
  // Phase 2 and the mean (the block shape does not change the results)
  P2Args A;
  A.X = g->X;
  A.n = n;
  A.d = d;
  A.labels = lab;
  A.Y = b.Y32;
  A.w = b.w32;
  A.aux = b.aux32;
  A.gid_pk = b.gid_pk;
  A.sp_off = b.sp_off;
  A.cnt = b.cnt;
  A.csize = b.csize;
  A.k = k;
  A.a = A.b = A.s = nullptr;
  A.What = nullptr;
  A.bpart = b.bpart;
  A.Wpart = b.Wpart;
  A.rn = g->rn;
  if (g->mfma) {
    launch_center(st, b.Y32, DM, g->KP, b.sp_off, b.cnt, k, b.mu);
    if (!launch_pack_mfma(st, metric, g->mprec, DM, b.Y32, b.aux32, b.w32, b.gid_pk, b.sp_off, b.cnt, k, b.mu,
                          (int)g->S_cap, b.Ym, b.bnorm))
      return false;
    if (!launch_phase2_mfma(st, metric, g->mprec, DM, A, b.mu, b.Ym, b.bnorm, g->shape[(size_t)i]))
      return false;
  } else if (!launch_phase2_valu(st, metric, DM, A)) {
    return false;
  }
  launch_mean(st, b.bpart, (int)ceil_div(n, g->p2_rows), n, g->means_d + i);
  launch_put_status(st, b.status, g->status_d + i);
  return hipGetLastError() == hipSuccess;
}

// the eager path for one clustering (used when a capacity was exceeded)
silh_status eager_mean(silh_graph* g, int i, hipStream_t st, double* mean) {
  silh_params prm = g->base;
  prm.k = g->ks[i];
  silh_ctx* c = nullptr;
  silh_status s = silh_sample_init(&prm, g->X, g->labels + (size_t)i * (size_t)g->n, st, &c);
  if (s == SILH_OK) s = silh_pps_sample(c, nullptr, nullptr);
  if (s == SILH_OK) s = silh_scores(c, nullptr, nullptr, nullptr, mean);
  silh_destroy(c);
  return s;
}

}  // namespace

extern "C" {

silh_status silh_graph_create(const silh_params* base, const float* X, const int32_t* labels,
                              const int32_t* ks, int32_t K, int32_t chains, double sample_cap,
                              silh_stream stream, silh_graph** out) {
  if (!out) return set_error(SILH_E_ARG, "out is NULL");
  *out = nullptr;
  if (!base || !X || !labels || !ks) return set_error(SILH_E_ARG, "NULL argument");
  if (K < 1) return set_error(SILH_E_ARG, "K must be at least 1");
  if (chains < 1 || chains > 16) return set_error(SILH_E_ARG, "chains outside [1, 16]");
  std::vector<int64_t> ts((size_t)K, 0);
  for (int32_t i = 0; i < K; ++i) {
    silh_params prm = *base;
    prm.k = ks[i];
    const silh_status s = validate_params(&prm, X, labels, &ts[(size_t)i]);
    if (s != SILH_OK) return s;
  }
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return set_error(SILH_E_HIP, "stream failed");
  silh_graph* g = new (std::nothrow) silh_graph();
  if (!g) return set_error(SILH_E_NOMEM, "host allocation failed");
  g->base = *base;
  g->X = X;
  g->labels = labels;
  g->ks.assign(ks, ks + K);
  g->ts = ts;
  g->K = K;
  g->n = (int)base->n;
  g->d = base->d;
  g->DM = dm_for(base->d);
  g->mfma = (base->metric == SILH_EUCL || base->metric == SILH_COS) &&
            (base->prec == SILH_BF16 || base->prec == SILH_FP8 || (base->prec == SILH_FP32 && g->DM <= 128));
  g->mprec = base->prec == SILH_BF16 ? 1 : (base->prec == SILH_FP8 ? 2 : 0);
  g->KP = g->mfma ? mfma_kp(g->mprec, g->DM) : 0;
  g->p2_rows = g->mfma ? phase2_mfma_rows(g->mprec, g->DM) : phase2_valu_rows(base->metric, g->DM);
  g->chunk = g->DM > 128 ? kWChunkWide : kWChunk;
  double kt = 0.0;
  for (int32_t i = 0; i < K; ++i) {
    g->kmax = ks[i] > g->kmax ? ks[i] : g->kmax;
    const double v = (double)ks[i] * (double)ts[(size_t)i];
    kt = v > kt ? v : kt;
  }
  // capacities: the packed sample, the initial sample (E|F0_j| = 2 ln(5k/delta),
  // at most about 24 here), the W work items (exact bound) and their partials
  const double factor = sample_cap > 0.0 ? sample_cap : 4.0;
  const double srows = std::ceil(factor * kt);
  g->S_cap = (srows < (double)g->n ? (int64_t)srows : (int64_t)g->n) + (int64_t)kSamplePad * g->kmax;
  g->F0_cap = std::min<int64_t>(g->n, 64 * (int64_t)g->kmax + 1024);
  g->items_cap = ceil_div(g->n, g->chunk) + g->kmax;
  g->part_cap = std::min<int64_t>((int64_t)1 << 30, g->items_cap * 64);
  // member distances kept by the W pass for the draw (the largest k)
  g->dist_cap = base->sampler == SILH_PPS
                    ? dist_capacity(g->n, std::log(5.0 * (double)g->kmax / base->delta))
                    : 0;
  g->br.resize((size_t)chains);
  bool ok = take(g, g->means_d, K) && take(g, g->status_d, K);
  if (ok && base->metric == SILH_COS) ok = take(g, g->rn, g->n);
  for (Branch& b : g->br) ok = ok && alloc_branch(g, b);
  if (!ok) {
    release(g);
    return set_error(SILH_E_NOMEM, "device allocation failed");
  }
  bool hip = hipHostMalloc((void**)&g->means_h, sizeof(double) * (size_t)K, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&g->status_h, sizeof(int32_t) * (size_t)K, hipHostMallocDefault) == hipSuccess &&
             hipStreamCreateWithFlags(&g->cap_st, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) == hipSuccess;
  for (Branch& b : g->br)
    hip = hip && hipStreamCreateWithFlags(&b.st, hipStreamNonBlocking) == hipSuccess &&
          hipEventCreateWithFlags(&b.join, hipEventDisableTiming) == hipSuccess;
  if (!hip) {
    (void)hipGetLastError();
    release(g);
    return set_error(SILH_E_HIP, "stream, event or pinned allocation failed");
  }
  // Phase-2 block shapes from the autotuner: one eager request per group of
  // clusterings with the same floor(log2(k t)) (the padded sample size is
  // the tuner's key), tuned on its real sample; a probe that fails (bad
  // labels, ...) leaves the built-in shape
  g->shape.assign((size_t)K, 1);
  g->probe_S.assign((size_t)K, 0);
  if (g->mfma) {
    std::map<int, std::pair<int32_t, int64_t>> group;
    for (int32_t i = 0; i < K; ++i) {
      const double kt = (double)ks[i] * (double)ts[(size_t)i];
      const int gk = (int)std::floor(std::log2(kt > 1.0 ? kt : 1.0));
      auto it = group.find(gk);
      if (it == group.end()) {
        silh_params prm = *base;
        prm.k = ks[i];
        silh_ctx* c = nullptr;
        std::pair<int32_t, int64_t> pick{pb_builtin(base->metric, g->mprec, g->DM), 0};
        if (silh_sample_init(&prm, X, labels + (size_t)i * (size_t)g->n, stream, &c) == SILH_OK &&
            silh_pps_sample(c, nullptr, nullptr) == SILH_OK) {
          pick = {tuned_shape(c), sample_rows(c)};
        }
        silh_destroy(c);
        it = group.emplace(gk, pick).first;
      }
      g->shape[(size_t)i] = it->second.first;
      g->probe_S[(size_t)i] = it->second.second;
    }
    (void)hipGetLastError();
  }
  // capture: fork every branch from the capture stream, enqueue, join back
  bool built = hipStreamBeginCapture(g->cap_st, hipStreamCaptureModeThreadLocal) == hipSuccess;
  bool captured = built;
  if (built) {
    if (g->rn) launch_rnorm(g->cap_st, g->X, g->n, g->d, g->rn);  // X is read at every replay
    built = hipEventRecord(g->fork, g->cap_st) == hipSuccess;
    for (Branch& b : g->br) built = built && hipStreamWaitEvent(b.st, g->fork, 0) == hipSuccess;
    for (int32_t i = 0; i < K && built; ++i) built = enqueue(g, g->br[(size_t)i % g->br.size()], i);
    for (Branch& b : g->br) {
      // every forked stream must join back, or the capture cannot end
      const bool j = hipEventRecord(b.join, b.st) == hipSuccess && hipStreamWaitEvent(g->cap_st, b.join, 0) == hipSuccess;
      built = built && j;
    }
    captured = hipStreamEndCapture(g->cap_st, &g->graph) == hipSuccess;
  }
  if (!built || !captured ||
      hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    release(g);
    return set_error(SILH_E_HIP, "graph capture failed");
  }
  size_t nn = 0;
  if (hipGraphGetNodes(g->graph, nullptr, &nn) == hipSuccess) g->nodes = (int64_t)nn;
  *out = g;
  return SILH_OK;
}

silh_status silh_graph_run(silh_graph* g, silh_stream stream, double* means_host, int32_t* status_host,
                           int32_t* best_host, int32_t* reruns_host) {
  if (!g || !means_host) return set_error(SILH_E_ARG, "NULL argument");
  const hipStream_t st = (hipStream_t)stream;
  const size_t K = (size_t)g->K;
  if (hipGraphLaunch(g->exec, st) != hipSuccess ||
      hipMemcpyAsync(g->means_h, g->means_d, K * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(g->status_h, g->status_d, K * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(SILH_E_HIP, "graph launch failed");
  }
  int32_t reruns = 0;
  for (size_t i = 0; i < K; ++i) {
    const int bits = g->status_h[i];
    silh_status s = SILH_OK;
    double m = g->means_h[i];
    if (bits & kStatusLabel) {
      s = SILH_E_LABEL;
    } else if (bits & kStatusEmpty) {
      s = SILH_E_K;
    } else if (bits & kStatusCapacity) {
      s = eager_mean(g, (int)i, st, &m);
      ++reruns;
      if (s != SILH_OK && s != SILH_E_LABEL && s != SILH_E_K) return s;
    }
    means_host[i] = s == SILH_OK ? m : __builtin_nan("");
    if (status_host) status_host[i] = s;
  }
  if (best_host) {
    int32_t best = -1;
    for (size_t i = 0; i < K; ++i)
      if (means_host[i] == means_host[i] && (best < 0 || means_host[i] > means_host[best])) best = (int32_t)i;
    *best_host = best;
  }
  if (reruns_host) *reruns_host = reruns;
  return SILH_OK;
}

silh_status silh_graph_get_info(const silh_graph* g, silh_graph_info* out) {
  if (!g || !out) return set_error(SILH_E_ARG, "NULL argument");
  out->nodes = g->nodes;
  out->sample_cap = g->S_cap;
  out->f0_cap = g->F0_cap;
  out->bytes = g->bytes;
  return SILH_OK;
}

silh_status silh_graph_choice(const silh_graph* g, int32_t i, int32_t* shape, int64_t* probe_S_pad) {
  if (!g || !shape || !probe_S_pad) return set_error(SILH_E_ARG, "NULL argument");
  if (i < 0 || i >= g->K) return set_error(SILH_E_ARG, "clustering index outside [0, K)");
  *shape = g->shape[(size_t)i];
  *probe_S_pad = g->probe_S[(size_t)i];
  return SILH_OK;
}

void silh_graph_destroy(silh_graph* g) {
  if (!g) return;  // silh_graph_run waits for the graph, so nothing of it is in flight here
  release(g);
}

}  // extern "C"
