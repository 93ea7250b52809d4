// Row subsets for the subsampled global estimators of Section 4.2: the m
// uniform draws of Eq. 8 / Eq. 10 (independent, with replacement), their
// distinct rows gathered into a contiguous block for the Phase-2 kernels, and
// the per-draw results with the float64 block sums of their mean.
#include "device_common.hpp"
#include "silh_internal.hpp"

namespace silh {

__global__ __launch_bounds__(256) void k_rows_draw(uint64_t seed, uint64_t n, int64_t m,
                                                   int32_t* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  // floor(B * n / 2^53) = high 64 bits of (B * 2^11) * n, exactly
  const uint64_t b = bits53(seed, (uint64_t)i, kStreamRows);
  rows[i] = (int32_t)__umul64hi(b << 11, n);
}

void launch_rows_draw(hipStream_t st, uint64_t seed, int64_t n, int64_t m, int32_t* rows) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_rows_draw, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, seed, (uint64_t)n, m,
                     rows);
}

__global__ __launch_bounds__(256) void k_rows_mark(const int32_t* __restrict__ rows, int64_t m, int n,
                                                   int32_t* __restrict__ mark, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int r = rows[i];
  if (r < 0 || r >= n)
    atomicOr(bad, 1);
  else
    mark[r] = 1;  // every writer stores the same value
}

void launch_rows_mark(hipStream_t st, const int32_t* rows, int64_t m, int n, int32_t* mark, int* bad) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_rows_mark, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, rows, m, n, mark, bad);
}

__global__ __launch_bounds__(256) void k_rows_compact(const int32_t* __restrict__ mark,
                                                      const int32_t* __restrict__ pos, int n,
                                                      int32_t* __restrict__ urows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && mark[i]) urows[pos[i]] = i;
}

void launch_rows_compact(hipStream_t st, const int32_t* mark, const int32_t* pos, int n, int32_t* urows) {
  hipLaunchKernelGGL(k_rows_compact, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, mark, pos, n, urows);
}

// one wave per gathered row
__global__ __launch_bounds__(256) void k_rows_gather(const float* __restrict__ X,
                                                     const int32_t* __restrict__ labels, int d,
                                                     const int32_t* __restrict__ urows, int mu,
                                                     float* __restrict__ Xs, int32_t* __restrict__ ls) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= mu) return;
  const int g = urows[r];
  const float* src = X + (size_t)g * d;
  float* dst = Xs + (size_t)r * d;
  for (int c = lane; c < d; c += 64) dst[c] = src[c];
  if (lane == 0) ls[r] = labels[g];
}

void launch_rows_gather(hipStream_t st, const float* X, const int32_t* labels, int d, const int32_t* urows,
                        int mu, float* Xs, int32_t* ls) {
  if (mu <= 0) return;
  hipLaunchKernelGGL(k_rows_gather, dim3((unsigned)ceil_div(mu, 4)), dim3(256), 0, st, X, labels, d, urows,
                     mu, Xs, ls);
}

// index of v in the ascending array a[0..len), or -1
__device__ __forceinline__ int find_sorted(const int32_t* __restrict__ a, int len, int v) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < len && a[lo] == v) ? lo : -1;
}

__global__ __launch_bounds__(256) void k_rows_remap(const int32_t* __restrict__ gid_pk, int64_t S_pad,
                                                    const int32_t* __restrict__ urows, int mu,
                                                    int32_t* __restrict__ gid_sub) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S_pad) return;
  const int g = gid_pk[s];
  gid_sub[s] = g < 0 ? -1 : find_sorted(urows, mu, g);
}

void launch_rows_remap(hipStream_t st, const int32_t* gid_pk, int64_t S_pad, const int32_t* urows, int mu,
                       int32_t* gid_sub) {
  if (S_pad <= 0) return;
  hipLaunchKernelGGL(k_rows_remap, dim3((unsigned)ceil_div(S_pad, 256)), dim3(256), 0, st, gid_pk, S_pad,
                     urows, mu, gid_sub);
}

__global__ __launch_bounds__(kRowsBlock) void k_rows_expand(const int32_t* __restrict__ rows, int64_t m,
                                                            const int32_t* __restrict__ urows, int mu,
                                                            const float* __restrict__ au,
                                                            const float* __restrict__ bu,
                                                            const float* __restrict__ su, float* __restrict__ a,
                                                            float* __restrict__ b, float* __restrict__ s,
                                                            double* __restrict__ bpart) {
  __shared__ double sh[kRowsBlock / kWave];
  const int64_t i = (int64_t)blockIdx.x * kRowsBlock + threadIdx.x;
  double v = 0.0;
  if (i < m) {
    const int u = find_sorted(urows, mu, rows[i]);  // every entry is there
    const float sv = su[u];
    if (a) a[i] = au[u];
    if (b) b[i] = bu[u];
    if (s) s[i] = sv;
    v = (double)sv;
  }
  const double tot = block_sum_f64<kRowsBlock>(v, sh);
  if (threadIdx.x == 0) bpart[blockIdx.x] = tot;
}

void launch_rows_expand(hipStream_t st, const int32_t* rows, int64_t m, const int32_t* urows, int mu,
                        const float* au, const float* bu, const float* su, float* a, float* b, float* s,
                        double* bpart) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_rows_expand, dim3((unsigned)ceil_div(m, kRowsBlock)), dim3(kRowsBlock), 0, st, rows, m,
                     urows, mu, au, bu, su, a, b, s, bpart);
}

}  // namespace silh
