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
__global__ __launch_bounds__(64) void k_unit_hist(const int32_t* __restrict__ labels, int n, int k, int seg,
                                                  int32_t* __restrict__ uh, int* __restrict__ bad) {
  extern __shared__ int32_t h[];
  for (int j = threadIdx.x; j < k; j += 64) h[j] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * seg;
  const int64_t end = base + seg < n ? base + seg : n;
  int anybad = 0;
  for (int64_t i = base + threadIdx.x; i < end; i += 64) {
    const int l = labels[i];
    if ((unsigned)l < (unsigned)k)
      atomicAdd(&h[l], 1);
    else
      anybad = 1;
  }
  if (anybad && bad != nullptr) atomicOr(bad, 1);
  __syncthreads();
  const int units = gridDim.x;  // label-major [k][units]: each label's scan reads one row
  for (int j = threadIdx.x; j < k; j += 64) uh[(size_t)j * units + blockIdx.x] = h[j];
}

void launch_unit_hist(hipStream_t st, const int32_t* labels, int n, int k, int seg, int32_t* uh, int* bad) {
  const int units = (int)ceil_div(n, seg);
  hipLaunchKernelGGL(k_unit_hist, dim3(units), dim3(64), k * sizeof(int32_t), st, labels, n, k, seg, uh, bad);
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
  int32_t* row = uh + (size_t)j * units;
  int32_t s = 0;
  for (int u = u0; u < u1; ++u) s += row[u];
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
    const int32_t v = row[u];
    row[u] = run;
    run += v;
  }
  if (threadIdx.x == 255) counts[j] = part[255];
}

void launch_unit_scan(hipStream_t st, int32_t* uh, int units, int k, int32_t* counts) {
  hipLaunchKernelGGL(k_unit_scan, dim3(k), dim3(256), 0, st, uh, units, k, counts);
}

// One wave per unit walks its rows in order, 64 at a time.  Lanes holding the
// same label (found by one ballot per label bit) get consecutive ranks in lane
// order (popcount of the lower such lanes), so the order is stable: ids ascend
// inside each cluster.  The unit's rows are first
// placed in LDS grouped by label (the unit's own label offsets), then each
// label's run is written to its global range in one contiguous piece.
// LDS: base[k] (global start of the unit's run of label j), loc[k] (next local
// slot of label j), ids[seg], lab[seg].  A label outside [0, k) (already
// flagged by k_unit_hist) is skipped, so no access leaves the arrays.
__global__ __launch_bounds__(64) void k_scatter(const int32_t* __restrict__ labels, int n, int k, int seg,
                                                const int32_t* __restrict__ ubase,
                                                const int32_t* __restrict__ off,
                                                int32_t* __restrict__ perm, int32_t* __restrict__ slab) {
  extern __shared__ int32_t lds[];
  int32_t* base = lds;
  int32_t* loc = lds + k;
  int32_t* ids = lds + 2 * k;
  int32_t* lab = ids + seg;
  const int lane = threadIdx.x;
  const int u = blockIdx.x;
  const int units = (int)(((int64_t)n + seg - 1) / seg);
  const int64_t b0 = (int64_t)u * seg;
  const int64_t end = b0 + seg < n ? b0 + seg : n;
  // the unit's own count of label j: next unit's prefix minus this one's (the
  // last unit: the cluster size, off[j + 1] - off[j], minus its prefix)
  // ubase is label-major: ubase[j * units + u]
  for (int j = lane; j < k; j += 64) {
    const int32_t cur = ubase[(size_t)j * units + u];
    const int32_t nxt = u + 1 < units ? ubase[(size_t)j * units + u + 1] : off[j + 1] - off[j];
    base[j] = off[j] + cur;
    loc[j] = nxt - cur;  // count, turned into the local offset below
  }
  __syncthreads();
  // exclusive scan of the unit's label counts (64 lanes, k / 64 each)
  int nvalid = 0;
  {
    const int per = (k + 63) / 64;
    const int j0 = lane * per;
    const int j1 = j0 + per < k ? j0 + per : k;
    int32_t sum = 0;
    for (int j = j0; j < j1; ++j) sum += loc[j];
    int32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    int32_t run = incl - sum;
    for (int j = j0; j < j1; ++j) {
      const int32_t c = loc[j];
      loc[j] = run;
      run += c;
    }
    nvalid = __shfl(incl, 63, 64);  // rows of the unit with a label in [0, k)
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // bits of a label in [0, k)
  const int kb = k > 1 ? 32 - __clz(k - 1) : 0;
  for (int64_t c = b0; c < end; c += 64) {
    const int64_t i = c + lane;
    const int L = i < end ? labels[i] : -1;
    const bool valid = (unsigned)L < (unsigned)k;
    // the lanes holding this lane's label: one ballot per label bit
    uint64_t same = __ballot(valid);
    for (int bit = 0; bit < kb; ++bit) {
      const bool one = (L >> bit) & 1;
      const uint64_t ones = __ballot(valid && one);
      same &= one ? ones : ~ones;
    }
    if (valid) {
      const int slot = loc[L] + __popcll(same & lt);
      ids[slot] = (int32_t)i;
      lab[slot] = L;
    }
    __syncthreads();
    // the lowest lane of each label advances that label's slot
    if (valid && (same & lt) == 0) loc[L] += __popcll(same);
    __syncthreads();
  }
  __syncthreads();
  // loc[j] is now the end of label j's local run; its start is loc[j] - count.
  // Local slot p of label j goes to base[j] + (p - start_j): runs of one label
  // are consecutive in both places, so the writes are contiguous.
  for (int p = lane; p < nvalid; p += 64) {
    const int Lp = lab[p];
    const int32_t cur = ubase[(size_t)Lp * units + u];
    const int32_t nxt = u + 1 < units ? ubase[(size_t)Lp * units + u + 1] : off[Lp + 1] - off[Lp];
    const int32_t start = loc[Lp] - (nxt - cur);
    const int32_t g = base[Lp] + (p - start);
    perm[g] = ids[p];
    slab[g] = Lp;
  }
}

void launch_scatter(hipStream_t st, const int32_t* labels, int n, int k, int seg, const int32_t* ubase,
                    const int32_t* off, int32_t* perm, int32_t* slab) {
  const int units = (int)ceil_div(n, seg);
  const size_t lds = (size_t)(2 * k + 2 * seg) * sizeof(int32_t);
  hipLaunchKernelGGL(k_scatter, dim3(units), dim3(64), lds, st, labels, n, k, seg, ubase, off, perm, slab);
}

// ----------------------------------------------------------------------------
// int32 exclusive scan: per-tile sums, a single-block scan of the tile sums,
// then per-tile scans offset by the tile base.
// ----------------------------------------------------------------------------
__global__ void k_fill_zero1(int32_t* __restrict__ out) { out[0] = 0; }

// eight consecutive values of a tile (zero past n): two 16-byte loads when
// all eight are in range and the array is 16-byte aligned
__device__ __forceinline__ void scan_load8(const int32_t* __restrict__ in, int64_t base, int n, bool vec,
                                           int32_t (&v)[8]) {
  if (vec && base + 8 <= n) {
    const int4 a = *(const int4*)(in + base);
    const int4 b = *(const int4*)(in + base + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = base + i < n ? in[base + i] : 0;
  }
}

// exclusive prefix of s over the 256 threads of a block (wave scans by
// shuffles, then the four wave totals); *tot receives the block's total
__device__ __forceinline__ int32_t block_excl_256(int32_t s, int32_t* __restrict__ wtot, int32_t* tot) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wtot[wid] = incl;
  __syncthreads();
  int32_t pre = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) pre += w < wid ? wtot[w] : 0;
  *tot = wtot[0] + wtot[1] + wtot[2] + wtot[3];
  return pre + incl - s;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t* __restrict__ in, int n,
                                                     int32_t* __restrict__ tsum) {
  __shared__ int32_t sh[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  const bool vec = ((uintptr_t)in & 15) == 0;
  int32_t v[8];
  scan_load8(in, base, n, vec, v);
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += v[i];
  s = wave_sum_i32(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) tsum[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// exclusive scan of the tile sums in place (one block), tsum[nt] = total
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

// out[i] = tile prefix + the exclusive scan inside the tile.  FUSED: the tile
// prefix is the sum of the raw tile sums before this tile (read by the whole
// block; used while the tiles are few), and the last tile writes out[n];
// otherwise tsum holds the scanned tile sums and tsum[nt] the total.
template <bool FUSED>
__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* __restrict__ in, int n,
                                                    const int32_t* __restrict__ tsum, int nt,
                                                    int32_t* __restrict__ out) {
  __shared__ int32_t wtot[4];
  __shared__ int32_t red[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  const bool vec = ((uintptr_t)in & 15) == 0 && ((uintptr_t)out & 15) == 0;
  int32_t v[8];
  scan_load8(in, base, n, vec, v);
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += v[i];
  int32_t tpre;
  if constexpr (FUSED) {
    int32_t a = 0;
    for (int q = threadIdx.x; q < (int)blockIdx.x; q += 256) a += tsum[q];
    a = wave_sum_i32(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    tpre = red[0] + red[1] + red[2] + red[3];
  } else {
    tpre = tsum[blockIdx.x];
  }
  int32_t btot;
  int32_t run = tpre + block_excl_256(s, wtot, &btot);
  int32_t o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    o[i] = run;
    run += v[i];
  }
  if (vec && base + 8 <= n) {
    *(int4*)(out + base) = int4{o[0], o[1], o[2], o[3]};
    *(int4*)(out + base + 4) = int4{o[4], o[5], o[6], o[7]};
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (base + i < n) out[base + i] = o[i];
  }
  if (threadIdx.x == 0) {
    if constexpr (FUSED) {
      if ((int)blockIdx.x == nt - 1) out[n] = tpre + btot;
    } else {
      if (blockIdx.x == 0) out[n] = tsum[nt];
    }
  }
}

// up to this many tiles the tile prefix is summed inside the apply pass
// (O(nt^2 / 2) L2 reads in all, a few MB at n = 4e6), saving a launch
constexpr int kScanFusedTiles = 2048;

void launch_scan(hipStream_t st, const int32_t* in, int n, int32_t* out, int32_t* tmp) {
  const int nt = (int)ceil_div(n, kScanTile);
  if (nt == 0) {
    hipLaunchKernelGGL(k_fill_zero1, dim3(1), dim3(1), 0, st, out);
    return;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3(nt), dim3(256), 0, st, in, n, tmp);
  if (nt <= kScanFusedTiles) {
    hipLaunchKernelGGL(k_scan_apply<true>, dim3(nt), dim3(256), 0, st, in, n, tmp, nt, out);
  } else {
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, tmp, nt);
    hipLaunchKernelGGL(k_scan_apply<false>, dim3(nt), dim3(256), 0, st, in, n, tmp, nt, out);
  }
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
