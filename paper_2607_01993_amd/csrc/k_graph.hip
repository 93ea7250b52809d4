// Size bookkeeping on the device for a pipeline whose buffers are sized by
// capacities: the cluster offsets, initial-sample rates, W(e_bar) work items
// and padded sample offsets that the eager path computes on the host after a
// read-back are computed here instead, so that a whole request (cluster
// index, Phase 1, packing, Phase 2, the mean of Eq. 9) is one stream of
// kernels with no size returning to the host, which a HIP graph can capture
// and replay.
//
// Each clustering carries one status word.  A size that exceeds its capacity
// sets a bit and the stage continues on clamped (empty) sizes, so every
// access stays inside its buffer; the host re-runs such a clustering on the
// eager path.  A label outside [0, k) sets a bit too (k_unit_hist).
//
// Every floating-point step below is the host's, in the same order
// (compiled with -ffp-contract=off).
#include "device_common.hpp"
#include "silh_internal.hpp"

#pragma clang fp contract(off)

namespace silh {

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* __restrict__ p, int64_t count, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) p[i] = v;
}

void launch_fill_i32(hipStream_t st, int32_t* p, int64_t count, int32_t v) {
  if (count <= 0) return;
  const int64_t blocks = ceil_div(count, 256);
  hipLaunchKernelGGL(k_fill_i32, dim3((int)(blocks < 2048 ? blocks : 2048)), dim3(256), 0, st, p, count, v);
}

// Inclusive scan of one value per thread over a 1024-thread block; returns
// this thread's exclusive prefix and leaves the total in *total.
__device__ __forceinline__ int64_t block_scan_excl_1024(int64_t v, int64_t* part, int64_t* total) {
  part[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t u = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += u;
    __syncthreads();
  }
  const int64_t incl = part[threadIdx.x];
  *total = part[1023];
  __syncthreads();
  return incl - v;
}

// Cluster offsets (exclusive prefix sums of the sizes) and the initial-sample
// rate of Algorithm 1, q_j = min(1, (2/|C_j|) ln(5k/delta)), with the log term
// computed on the host; fewer than two nonempty clusters sets kStatusEmpty.
// One block of 1024 threads, each over a contiguous run of clusters.
__global__ __launch_bounds__(1024) void k_index_sizes(const int32_t* __restrict__ csize, int k, double lnterm,
                                                      int32_t* __restrict__ off, double* __restrict__ q,
                                                      int* __restrict__ status) {
  __shared__ int64_t part[1024];
  const int per = (k + 1023) / 1024;
  const int j0 = threadIdx.x * per;
  const int j1 = j0 + per < k ? j0 + per : k;
  int64_t s = 0, ne = 0;
  for (int j = j0; j < j1; ++j) {
    s += csize[j];
    ne += csize[j] > 0;
  }
  int64_t tot = 0, ne_tot = 0;
  int64_t run = block_scan_excl_1024(s, part, &tot);
  (void)block_scan_excl_1024(ne, part, &ne_tot);
  for (int j = j0; j < j1; ++j) {
    off[j] = (int32_t)run;
    run += csize[j];
    double qj = 0.0;
    if (csize[j] > 0) {
      qj = 2.0 / (double)csize[j];
      qj = qj * lnterm;
      qj = qj < 1.0 ? qj : 1.0;
    }
    q[j] = qj;
  }
  if (threadIdx.x == 0) {
    off[k] = (int32_t)tot;
    if (ne_tot < 2) *status |= kStatusEmpty;
  }
}

void launch_index_sizes(hipStream_t st, const int32_t* csize, int k, double lnterm, int32_t* off, double* q,
                        int* status) {
  hipLaunchKernelGGL(k_index_sizes, dim3(1), dim3(1024), 0, st, csize, k, lnterm, off, q, status);
}

// W(e_bar) work items from the sizes (the eager path builds the same list on
// the host): clusters with |C_j| > t and a nonempty F0_j are cut into runs of
// `chunk` consecutive sorted positions, in cluster order; item r of cluster j
// writes its |F0_j| partial sums at pbase_j + r |F0_j|.  f0_off is first
// clamped to f0_cap (kStatusF0 when it did not fit); a partial-sum total past
// part_cap sets kStatusPartial and leaves every cluster without items.
// Writes citem_first / citem_count / ibase (first item, count, partial base
// per cluster) and meta[0] = item count; with dbase, the per-cluster bases of
// the kept member distances (|C_j| |F0_j| each, same clusters) and meta[1] = 1
// when their total fits dist_cap.
__global__ __launch_bounds__(1024) void k_f0_items(const int32_t* __restrict__ csize,
                                                   int32_t* __restrict__ f0_off, int k, int64_t t, int chunk,
                                                   int f0_cap, int64_t part_cap,
                                                   int32_t* __restrict__ citem_first,
                                                   int32_t* __restrict__ citem_count,
                                                   int64_t* __restrict__ ibase, int32_t* __restrict__ meta,
                                                   int* __restrict__ status, int64_t* __restrict__ dbase,
                                                   int64_t dist_cap, bool assign) {
  __shared__ int64_t part[1024];
  __shared__ int over;
  if (threadIdx.x == 0) over = f0_off[k] > f0_cap;
  __syncthreads();
  for (int j = threadIdx.x; j <= k; j += 1024) f0_off[j] = f0_off[j] < f0_cap ? f0_off[j] : f0_cap;
  __syncthreads();
  const int per = (k + 1023) / 1024;
  const int j0 = threadIdx.x * per;
  const int j1 = j0 + per < k ? j0 + per : k;
  int64_t ni = 0, np = 0, nd = 0;
  for (int j = j0; j < j1; ++j) {
    const int fj = f0_off[j + 1] - f0_off[j];
    const bool on = (int64_t)csize[j] > t && fj > 0;
    const int64_t items = on ? ((int64_t)csize[j] + chunk - 1) / chunk : 0;
    ni += items;
    np += items * fj;
    nd += on ? (int64_t)csize[j] * fj : 0;
  }
  int64_t ni_tot = 0, np_tot = 0, nd_tot = 0;
  int64_t irun = block_scan_excl_1024(ni, part, &ni_tot);
  int64_t prun = block_scan_excl_1024(np, part, &np_tot);
  int64_t drun = block_scan_excl_1024(nd, part, &nd_tot);
  const bool drop = np_tot > part_cap;
  for (int j = j0; j < j1; ++j) {
    const int fj = f0_off[j + 1] - f0_off[j];
    const bool on = (int64_t)csize[j] > t && fj > 0;
    const int64_t items = (on && !drop) ? ((int64_t)csize[j] + chunk - 1) / chunk : 0;
    citem_first[j] = drop ? 0 : (int32_t)irun;
    citem_count[j] = (int32_t)items;
    ibase[j] = prun;
    if (dbase) dbase[j] = drun;
    irun += items;
    prun += items * fj;
    drun += on ? (int64_t)csize[j] * fj : 0;
  }
  if (threadIdx.x == 0) {
    meta[1] = (dbase != nullptr && !drop && nd_tot <= dist_cap) ? 1 : 0;
    meta[0] = drop ? 0 : (int32_t)ni_tot;
    const int bits = (over ? kStatusF0 : 0) | (drop ? kStatusPartial : 0);
    if (assign)
      *status = bits;
    else if (bits)
      *status |= bits;
  }
}

// items[it] for it < items_cap: the item's cluster by binary search over
// citem_first; slots past the item count get an empty item (no members, no
// F0 rows), so the W pass can run over the full capacity.
// item layout: [cluster, begin, end, f0_begin, f0_count, partial_base]
__global__ __launch_bounds__(256) void k_items_fill(const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ f0_off,
                                                    const int32_t* __restrict__ citem_first,
                                                    const int64_t* __restrict__ ibase,
                                                    const int32_t* __restrict__ meta, int k, int chunk,
                                                    int items_cap, int32_t* __restrict__ items) {
  const int it = blockIdx.x * 256 + threadIdx.x;
  if (it >= items_cap) return;
  int32_t* o = items + (size_t)it * 6;
  if (it >= meta[0]) {
    o[0] = 0;
    o[1] = 0;
    o[2] = 0;
    o[3] = 0;
    o[4] = 0;
    o[5] = 0;
    return;
  }
  // the last cluster whose first item is <= it (citem_first is nondecreasing;
  // a cluster without items shares its first index with the next cluster that
  // has some, and the last such index is taken, so j has items)
  int lo = 0, hi = k;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (citem_first[mid] <= it) lo = mid; else hi = mid;
  }
  const int j = lo;
  const int r = it - citem_first[j];
  const int fj = f0_off[j + 1] - f0_off[j];
  const int b = off[j] + r * chunk;
  const int e = b + chunk < off[j + 1] ? b + chunk : off[j + 1];
  o[0] = j;
  o[1] = b;
  o[2] = e;
  o[3] = f0_off[j];
  o[4] = fj;
  o[5] = (int32_t)(ibase[j] + (int64_t)r * fj);
}

void launch_f0_items(hipStream_t st, const int32_t* csize, const int32_t* off, int32_t* f0_off, int k,
                     int64_t t, int chunk, int f0_cap, int64_t part_cap, int items_cap, int32_t* citem_first,
                     int32_t* citem_count, int64_t* ibase, int32_t* meta, int32_t* items, int* status,
                     int64_t* dbase, int64_t dist_cap, bool assign_status) {
  hipLaunchKernelGGL(k_f0_items, dim3(1), dim3(1024), 0, st, csize, f0_off, k, t, chunk, f0_cap, part_cap,
                     citem_first, citem_count, ibase, meta, status, dbase, dist_cap, assign_status);
  hipLaunchKernelGGL(k_items_fill, dim3((int)ceil_div(items_cap, 256)), dim3(256), 0, st, off, f0_off,
                     citem_first, ibase, meta, k, chunk, items_cap, items);
}

// Per-cluster sample counts and the offsets of the padded sample blocks
// (each cluster padded to kSamplePad rows).  A padded total past s_cap sets
// kStatusSample and leaves every cluster empty.
__global__ __launch_bounds__(1024) void k_sample_sizes(const int32_t* __restrict__ s_off, int k, int s_cap,
                                                       int32_t* __restrict__ cnt, int32_t* __restrict__ sp_off,
                                                       int* __restrict__ status) {
  __shared__ int64_t part[1024];
  const int per = (k + 1023) / 1024;
  const int j0 = threadIdx.x * per;
  const int j1 = j0 + per < k ? j0 + per : k;
  int64_t s = 0;
  for (int j = j0; j < j1; ++j) s += (s_off[j + 1] - s_off[j] + kSamplePad - 1) / kSamplePad * kSamplePad;
  int64_t tot = 0;
  int64_t run = block_scan_excl_1024(s, part, &tot);
  const bool drop = tot > s_cap;
  for (int j = j0; j < j1; ++j) {
    const int32_t c = s_off[j + 1] - s_off[j];
    cnt[j] = drop ? 0 : c;
    sp_off[j] = drop ? 0 : (int32_t)run;
    run += (c + kSamplePad - 1) / kSamplePad * kSamplePad;
  }
  if (threadIdx.x == 0) {
    sp_off[k] = drop ? 0 : (int32_t)tot;
    if (drop) *status |= kStatusSample;
  }
}

void launch_sample_sizes(hipStream_t st, const int32_t* s_off, int k, int s_cap, int32_t* cnt, int32_t* sp_off,
                         int* status) {
  hipLaunchKernelGGL(k_sample_sizes, dim3(1), dim3(1024), 0, st, s_off, k, s_cap, cnt, sp_off, status);
}

__global__ void k_put_status(const int* __restrict__ status, int32_t* __restrict__ out) { *out = *status; }

int64_t dist_capacity(int64_t n, double lnterm) {
  const double v = (double)n * (2.5 * lnterm + 8.0);
  const double cap = (double)((int64_t)1 << 27);
  return (int64_t)(v < cap ? v : cap);
}

void launch_put_status(hipStream_t st, const int* status, int32_t* out) {
  hipLaunchKernelGGL(k_put_status, dim3(1), dim3(1), 0, st, status, out);
}

}  // namespace silh
