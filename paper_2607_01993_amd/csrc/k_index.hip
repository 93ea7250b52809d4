// Cluster index: cluster sizes, and a stable counting sort of the element ids
// by label (ids ascend inside each cluster), plus the int32 exclusive scan used
// for every compaction.  The paper takes the cluster sizes as known to every
// worker (Section 4.3.1); here they are counted once per clustering.
#include "device_common.hpp"
#include "silh_internal.hpp"

namespace silh {

// ----------------------------------------------------------------------------
// stable counting sort by label: per-unit histograms, per-label scan over
// units, then an in-order scatter with one wave per unit
// ----------------------------------------------------------------------------
// Per-unit label histograms; a label outside [0, k) is not counted and sets
// *bad (the cluster sizes are then not used).
__global__ __launch_bounds__(64) void k_unit_hist(const int32_t* __restrict__ labels, int n, int k,
                                                  int32_t* __restrict__ uh, int* __restrict__ bad) {
  extern __shared__ int32_t h[];
  for (int j = threadIdx.x; j < k; j += 64) h[j] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortSeg;
  const int64_t end = base + kSortSeg < n ? base + kSortSeg : n;
  int anybad = 0;
  for (int64_t i = base + threadIdx.x; i < end; i += 64) {
    const int l = labels[i];
    if ((unsigned)l < (unsigned)k)
      atomicAdd(&h[l], 1);
    else
      anybad = 1;
  }
  if (anybad) atomicOr(bad, 1);
  __syncthreads();
  int32_t* row = uh + (size_t)blockIdx.x * k;
  for (int j = threadIdx.x; j < k; j += 64) row[j] = h[j];
}

void launch_unit_hist(hipStream_t st, const int32_t* labels, int n, int k, int32_t* uh, int* bad) {
  const int units = (int)ceil_div(n, kSortSeg);
  hipLaunchKernelGGL(k_unit_hist, dim3(units), dim3(64), k * sizeof(int32_t), st, labels, n, k, uh, bad);
}

// one block per label: uh[u][j] <- sum_{u' < u} uh[u'][j] (the label's rows
// before unit u), and counts[j] = the label's total (the cluster size)
__global__ __launch_bounds__(256) void k_unit_scan(int32_t* __restrict__ uh, int units, int k,
                                                   int32_t* __restrict__ counts) {
  __shared__ int32_t part[256];
  const int j = blockIdx.x;
  const int per = (units + 255) / 256;
  const int u0 = threadIdx.x * per;
  const int u1 = u0 + per < units ? u0 + per : units;
  int32_t s = 0;
  for (int u = u0; u < u1; ++u) s += uh[(size_t)u * k + j];
  part[threadIdx.x] = s;
  __syncthreads();
  // inclusive Hillis-Steele scan over the 256 partial sums
  for (int o = 1; o < 256; o <<= 1) {
    int32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int u = u0; u < u1; ++u) {
    const int32_t v = uh[(size_t)u * k + j];
    uh[(size_t)u * k + j] = run;
    run += v;
  }
  if (threadIdx.x == 255) counts[j] = part[255];
}

void launch_unit_scan(hipStream_t st, int32_t* uh, int units, int k, int32_t* counts) {
  hipLaunchKernelGGL(k_unit_scan, dim3(k), dim3(256), 0, st, uh, units, k, counts);
}

// One wave per unit walks its rows in order, 64 at a time.  Lanes holding the
// same label get consecutive slots in lane order (ballot + popcount), so the
// output is stable: ids ascend inside each cluster.
__global__ __launch_bounds__(64) void k_scatter(const int32_t* __restrict__ labels, int n, int k,
                                                const int32_t* __restrict__ ubase,
                                                const int32_t* __restrict__ off,
                                                int32_t* __restrict__ perm, int32_t* __restrict__ slab) {
  extern __shared__ int32_t run[];
  const int lane = threadIdx.x;
  const int32_t* row = ubase + (size_t)blockIdx.x * k;
  for (int j = lane; j < k; j += 64) run[j] = off[j] + row[j];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortSeg;
  const int64_t end = base + kSortSeg < n ? base + kSortSeg : n;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t c = base; c < end; c += 64) {
    const int64_t i = c + lane;
    const bool valid = i < end;
    const int lab = valid ? labels[i] : -1;
    uint64_t active = __ballot(valid);
    while (active) {
      const int leader = __ffsll((unsigned long long)active) - 1;
      const int L = __shfl(lab, leader, 64);
      const uint64_t mask = __ballot(valid && lab == L);
      int32_t slot = 0;
      if (valid && lab == L) {
        slot = run[L] + __popcll(mask & lt);
        perm[slot] = (int32_t)i;
        slab[slot] = L;
      }
      __syncthreads();
      if (lane == leader) run[L] += __popcll(mask);
      __syncthreads();
      active &= ~mask;
    }
  }
}

void launch_scatter(hipStream_t st, const int32_t* labels, int n, int k, const int32_t* ubase,
                    const int32_t* off, int32_t* perm, int32_t* slab) {
  const int units = (int)ceil_div(n, kSortSeg);
  hipLaunchKernelGGL(k_scatter, dim3(units), dim3(64), k * sizeof(int32_t), st, labels, n, k, ubase, off,
                     perm, slab);
}

// ----------------------------------------------------------------------------
// int32 exclusive scan: per-tile sums, a single-block scan of the tile sums,
// then per-tile scans offset by the tile base.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t* __restrict__ in, int n,
                                                     int32_t* __restrict__ tsum) {
  __shared__ int32_t sh[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (base + i < n) s += in[base + i];
  s = wave_sum_i32(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) tsum[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(1024) void k_scan_tiles(int32_t* __restrict__ tsum, int nt) {
  __shared__ int32_t part[1024];
  const int per = (nt + 1023) / 1024;
  const int t0 = threadIdx.x * per;
  const int t1 = t0 + per < nt ? t0 + per : nt;
  int32_t s = 0;
  for (int t = t0; t < t1; ++t) s += tsum[t];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int t = t0; t < t1; ++t) {
    const int32_t v = tsum[t];
    tsum[t] = run;
    run += v;
  }
  if (threadIdx.x == 1023) tsum[nt] = part[1023];
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* __restrict__ in, int n,
                                                    const int32_t* __restrict__ tsum, int nt,
                                                    int32_t* __restrict__ out) {
  __shared__ int32_t part[256];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  int32_t v[8];
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int32_t u = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += u;
    __syncthreads();
  }
  int32_t run = tsum[blockIdx.x] + (threadIdx.x ? part[threadIdx.x - 1] : 0);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tsum[nt];
}

void launch_scan(hipStream_t st, const int32_t* in, int n, int32_t* out, int32_t* tmp) {
  const int nt = (int)ceil_div(n, kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nt), dim3(256), 0, st, in, n, tmp);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, tmp, nt);
  hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(256), 0, st, in, n, tmp, nt, out);
}

__global__ void k_gather_at(const int32_t* __restrict__ scan, const int32_t* __restrict__ off, int k,
                            int32_t* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j <= k) out[j] = scan[off[j]];
}

void launch_gather_at(hipStream_t st, const int32_t* scan, const int32_t* off, int k, int32_t* out) {
  hipLaunchKernelGGL(k_gather_at, dim3((int)ceil_div(k + 1, 256)), dim3(256), 0, st, scan, off, k, out);
}

}  // namespace silh
