// Cohesion and separation (Appendix B) from the per-element cluster sums
// W_hat [n][k]: per element e in C_own, the own-cluster sum goes to the
// cohesion numerator and the sums over clusters j > own to the separation
// numerator; float64 block partials in a fixed order (deterministic).
#include "device_common.hpp"
#include "silh_internal.hpp"

namespace silh {

__global__ __launch_bounds__(256) void k_coh_sep(const float* __restrict__ W, int n, int k,
                                                 const int32_t* __restrict__ labels,
                                                 double* __restrict__ cpart, double* __restrict__ spart) {
  __shared__ double sh[4];
  double c = 0.0, s = 0.0;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int own = labels[e];
    const float* row = W + (size_t)e * k;
    c += (double)row[own];
    for (int j = own + 1; j < k; ++j) s += (double)row[j];
  }
  const double ct = block_sum_f64<256>(c, sh);
  const double st = block_sum_f64<256>(s, sh);
  if (threadIdx.x == 0) {
    cpart[blockIdx.x] = ct;
    spart[blockIdx.x] = st;
  }
}

int coh_sep_blocks(int n) {
  const int64_t b = ceil_div(n, 256);
  return (int)(b < kCohSepMaxBlocks ? b : kCohSepMaxBlocks);
}

void launch_coh_sep(hipStream_t st, const float* W, int n, int k, const int32_t* labels, double* cpart,
                    double* spart) {
  hipLaunchKernelGGL(k_coh_sep, dim3(coh_sep_blocks(n)), dim3(256), 0, st, W, n, k, labels, cpart, spart);
}

}  // namespace silh
