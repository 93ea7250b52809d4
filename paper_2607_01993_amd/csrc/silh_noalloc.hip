// silh_exact_noalloc: the exact silhouette of silh_exact with every scratch
// buffer carved out of one static device array, for callers that cannot
// allocate device memory.
//
// The work is the pipeline of silh_exact (cluster index, F_j = C_j with
// p = 1, packing, Phase 2, the mean) with every size computed on the device
// (the kernels of the captured-graph path), so nothing is read back before
// the end and nothing is allocated: the library's own buffers are slices of
// `scratch`, a file-scope device array of kScratchBytes.  Each device holds
// its own copy of the array, at its own address, from the first call on it
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).  The array keeps the previous
// call's contents: every slice that must start at a known value is filled by
// a kernel here (no memset, so the sequence is also valid inside a captured
// stream).  Calls on one device share the array: the library serialises the
// calls of one process per device (a lock held until the call has
// synchronised its stream), and calls that overlapped on one device (from
// work the caller enqueued around them on other streams reading the same
// slices) would race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "silh_internal.hpp"

using namespace silh;

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;  // 256 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu[kMaxDevices];
void* g_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch`, looked up once per
// device (with that device current) and kept.
silh_status scratch_for(int dev, unsigned char** out) {
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return set_error(SILH_E_HIP, "hipGetSymbolAddress of the static scratch array failed");
    }
    g_ptr[dev] = p;
  }
  *out = (unsigned char*)g_ptr[dev];
  return SILH_OK;
}

// Slices of the scratch array, each 256-byte aligned.  With base == nullptr
// only the total is counted.
struct Slices {
  unsigned char* base = nullptr;
  size_t used = 0;
  template <class T>
  Slices& add(T** p, int64_t count) {
    const size_t bytes = ((size_t)(count > 0 ? count : 1) * sizeof(T) + 255) & ~(size_t)255;
    if (base) *p = (T*)(base + used);
    used += bytes;
    return *this;
  }
};

struct Bufs {
  int *status = nullptr;
  int32_t *uh = nullptr, *csize = nullptr, *off = nullptr, *perm = nullptr, *slab = nullptr;
  double* q = nullptr;
  int32_t *flag = nullptr, *pos = nullptr, *scan_tmp = nullptr, *s_off = nullptr, *sp_off = nullptr,
          *cnt = nullptr;
  double* p_gid = nullptr;
  int64_t* gid_view = nullptr;
  int32_t* gid_pk = nullptr;
  float *w32 = nullptr, *aux32 = nullptr, *Y32 = nullptr, *mu = nullptr, *bnorm = nullptr;
  unsigned char* Ym = nullptr;
  double *bpart = nullptr, *Wpart = nullptr, *mean = nullptr;
  float* rn = nullptr;
};

struct Shape {
  int n, d, k, DM, KP, mprec, p2_rows, seg, units;
  bool mfma, split, cos;
  int64_t S_cap;
};

void layout(const Shape& s, Slices& sl, Bufs& b) {
  const int64_t n = s.n, k = s.k;
  sl.add(&b.status, 1).add(&b.mean, 1).add(&b.uh, (int64_t)s.units * k).add(&b.csize, k).add(&b.off, k + 1);
  sl.add(&b.perm, n).add(&b.slab, n).add(&b.q, k).add(&b.flag, n).add(&b.pos, n + 1);
  sl.add(&b.scan_tmp, ceil_div(n, kScanTile) + 1).add(&b.s_off, k + 1).add(&b.sp_off, k + 1).add(&b.cnt, k);
  sl.add(&b.p_gid, n).add(&b.gid_view, s.S_cap).add(&b.gid_pk, s.S_cap).add(&b.w32, s.S_cap);
  sl.add(&b.aux32, s.S_cap).add(&b.Y32, s.S_cap * s.DM).add(&b.bpart, ceil_div(n, s.p2_rows));
  if (s.mfma) {
    sl.add(&b.mu, mfma_mu_floats(s.mprec, s.DM, k)).add(&b.bnorm, s.S_cap).add(&b.Ym, s.S_cap * (size_t)mfma_row_bytes(s.mprec, s.DM));
  }
  if (s.split) sl.add(&b.Wpart, n * k);
  if (s.cos) sl.add(&b.rn, n);
}

}  // namespace

extern "C" silh_status silh_exact_noalloc(const silh_params* prm, const float* X, const int32_t* labels,
                                          silh_stream stream, float* a, float* b, float* s,
                                          double* s_mean_host) {
  {
    const silh_status v = validate_exact_params(prm, X, labels);
    if (v != SILH_OK) return v;
  }
  Shape sh;
  sh.n = (int)prm->n;
  sh.d = prm->d;
  sh.k = prm->k;
  sh.DM = dm_for(prm->d);
  sh.mfma = (prm->metric == SILH_EUCL || prm->metric == SILH_COS) &&
            (prm->prec == SILH_BF16 || prm->prec == SILH_FP8 || (prm->prec == SILH_FP32 && sh.DM <= 128));
  sh.mprec = prm->prec == SILH_BF16 ? 1 : (prm->prec == SILH_FP8 ? 2 : 0);
  sh.KP = sh.mfma ? mfma_kp(sh.mprec, sh.DM) : 0;
  sh.p2_rows = sh.mfma ? phase2_mfma_rows(sh.mprec, sh.DM) : phase2_valu_rows(prm->metric, sh.DM);
  sh.split = !sh.mfma && phase2_valu_split(prm->metric, sh.DM);
  sh.cos = prm->metric == SILH_COS;
  sh.seg = sort_seg(sh.n, sh.k);
  sh.units = (int)ceil_div(sh.n, sh.seg);
  sh.S_cap = (int64_t)sh.n + (int64_t)kSamplePad * sh.k;  // every element, each cluster padded
  {
    Slices count;
    Bufs dummy;
    layout(sh, count, dummy);
    if (count.used > kScratchBytes) {
      char msg[200];
      std::snprintf(msg, sizeof msg,
                    "n=%d, d=%d, k=%d needs %zu bytes of scratch; the static array holds %zu", sh.n, sh.d, sh.k,
                    count.used, kScratchBytes);
      return set_error(SILH_E_ARG, msg);
    }
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return set_error(SILH_E_HIP, "no current HIP device");
  }
  std::lock_guard<std::mutex> lk(g_mu[dev]);
  unsigned char* base = nullptr;
  {
    const silh_status v = scratch_for(dev, &base);
    if (v != SILH_OK) return v;
  }
  Slices sl;
  sl.base = base;
  Bufs B;
  layout(sh, sl, B);

  const hipStream_t st = (hipStream_t)stream;
  const int n = sh.n, k = sh.k, d = sh.d, DM = sh.DM;
  const int metric = prm->metric;
  // cluster index (perm and slab start at 0 so that rows a bad label leaves
  // unwritten still name a valid element); the log term of q is unused here
  launch_fill_i32(st, B.status, 1, 0);
  launch_fill_i32(st, B.perm, n, 0);
  launch_fill_i32(st, B.slab, n, 0);
  launch_unit_hist(st, labels, n, k, sh.seg, B.uh, B.status);
  launch_unit_scan(st, B.uh, sh.units, k, B.csize);
  launch_index_sizes(st, B.csize, k, 0.0, B.off, B.q, B.status);
  launch_scatter(st, labels, n, k, sh.seg, B.uh, B.off, B.perm, B.slab);
  if (B.rn) launch_rnorm(st, X, n, d, B.rn);
  // every element sampled with p = 1 (Section 2: the exact sums)
  launch_fill_all(st, B.perm, n, B.p_gid, B.flag);
  launch_scan(st, B.flag, n, B.pos, B.scan_tmp);
  launch_gather_at(st, B.pos, B.off, k, B.s_off);
  launch_sample_sizes(st, B.s_off, k, (int)sh.S_cap, B.cnt, B.sp_off, B.status);
  launch_pack(st, B.perm, B.slab, B.flag, B.pos, n, k, X, d, DM, B.p_gid, B.s_off, B.sp_off, pack_mode(metric),
              B.rn, (int)sh.S_cap, B.gid_view, B.gid_pk, B.w32, B.aux32, B.Y32);
  P2Args A;
  A.X = X;
  A.n = n;
  A.d = d;
  A.labels = labels;
  A.Y = B.Y32;
  A.w = B.w32;
  A.aux = B.aux32;
  A.gid_pk = B.gid_pk;
  A.sp_off = B.sp_off;
  A.cnt = B.cnt;
  A.csize = B.csize;
  A.k = k;
  A.a = a;
  A.b = b;
  A.s = s;
  A.What = nullptr;
  A.bpart = B.bpart;
  A.Wpart = B.Wpart;
  A.rn = B.rn;
  bool ok = true;
  if (sh.mfma) {
    launch_center(st, B.Y32, DM, sh.KP, B.sp_off, B.cnt, k, B.mu);
    ok = launch_pack_mfma(st, metric, sh.mprec, DM, B.Y32, B.aux32, B.w32, B.gid_pk, B.sp_off, B.cnt, k, B.mu,
                          (int)sh.S_cap, B.Ym, B.bnorm) &&
         launch_phase2_mfma(st, metric, sh.mprec, DM, A, B.mu, B.Ym, B.bnorm, pb_builtin(metric, sh.mprec, DM));
  } else {
    ok = launch_phase2_valu(st, metric, DM, A);
  }
  if (!ok) return set_error(SILH_E_UNSUPPORTED, "no Phase-2 kernel for this metric and dimension");
  launch_mean(st, B.bpart, (int)ceil_div(n, sh.p2_rows), n, B.mean);
  // the status word and the mean come back together: B.status and B.mean are
  // the first two 256-byte slices, so one copy of 264 bytes holds both
  struct {
    int status;
    unsigned char pad[252];
    double mean;
  } back;
  static_assert(sizeof(back) == 264, "status / mean read-back layout");
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&back, B.status, sizeof(back), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(SILH_E_HIP, "a kernel launch or the read-back failed");
  }
  if (back.status & kStatusLabel) {
    char msg[96];
    std::snprintf(msg, sizeof msg, "a label lies outside [0, %d)", k);
    return set_error(SILH_E_LABEL, msg);
  }
  if (back.status & kStatusEmpty)
    return set_error(SILH_E_K, "fewer than two nonempty clusters; the silhouette needs at least 2");
  if (back.status != 0) return set_error(SILH_E_HIP, "unexpected capacity status");
  if (s_mean_host) *s_mean_host = back.mean;
  return SILH_OK;
}
