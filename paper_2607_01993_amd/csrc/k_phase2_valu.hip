// Phase 2 of Algorithm 1 on the vector ALUs (float32 distances; float64 sums
// across tiles): for each element e and cluster C_j,
//   W_hat_{C_j}(e) = sum_{e' in F_j} w_{e'} d(e, e'),  w = 1/p,
// then a_hat, b_hat, s_hat (Eq. 5) and a per-block float64 partial of the sum
// of s_hat (for Eq. 9).
//
// Mapping: one element per lane, its coordinates in registers; the whole wave
// walks the packed sample in the same order, so every sample coordinate and
// weight is wave-uniform and is read by scalar loads into SGPRs, which the
// VALU instructions take as operands directly.  The loop over clusters is
// uniform too, so the per-cluster running sums need no cross-lane traffic.
#include <float.h>

#include <type_traits>

#include "device_common.hpp"
#include "silh_internal.hpp"

namespace silh {

constexpr int kGroup = 32;  // samples summed in float32 before the float64 add

// One coordinate of a float32 distance, and the final step.  Cosine runs as
// half the squared distance of the unit vectors plus u (0.5 for a zero vector,
// else 0): for unit x_hat, y_hat, 1 - x_hat.y_hat = |x_hat - y_hat|^2 / 2, and
// the u terms give 1 whenever either vector is zero; this form does not
// cancel for near-parallel pairs.
// Canberra's guard (G) keeps a 0/0 coordinate at 0 (den >= FLT_MIN).  The
// unguarded form (dist32 with G = false) takes the coordinates in pairs with
// one reciprocal per pair,
//   |x0 - y0| / a + |x1 - y1| / b = (|x0 - y0| b + |x1 - y1| a) / (a b),
// a = |x0| + |y0|, b = |x1| + |y1|: the reciprocal is the costly instruction
// (measured at several times an FMA's issue cost), the pair form has one per
// two coordinates for three more multiplies.  It is valid when every
// coordinate of the element row lies in [2^-62, 2^62] in magnitude and every
// coordinate of the sample row in [0, 2^62]: then a, b lie in [2^-62, 2^63],
// a b is a normal float, the numerator is at most 2 a b, and no 0/0 arises.
template <int M, bool G = true>
__device__ __forceinline__ float dist32_step(float s, float xc, float yc) {
  if (M == kManh) return s + fabsf(xc - yc);
  if (M == kCanb) {
    const float den = G ? fmaxf(fabsf(xc) + fabsf(yc), FLT_MIN) : fabsf(xc) + fabsf(yc);
    return fmaf(fabsf(xc - yc), __builtin_amdgcn_rcpf(den), s);
  }
  const float df = xc - yc;  // Euclidean, cosine
  return fmaf(df, df, s);
}

template <int M>
__device__ __forceinline__ float dist32_final(float s, float ux, float uy) {
  if (M == kEucl) return __builtin_amdgcn_sqrtf(s);
  if (M == kCos) return __builtin_amdgcn_fmed3f(fmaf(0.5f, s, ux + uy), 0.0f, 2.0f);
  return s;
}

// the element's row in registers
template <int M, int DM, bool G = true>
__device__ __forceinline__ float dist32(const float (&x)[DM], const float* __restrict__ y, float ux,
                                      float uy) {
  float s = 0.f;
  if constexpr (M == kCanb && !G) {
    static_assert(DM % 2 == 0, "coordinate pairs");
#pragma unroll
    for (int c = 0; c < DM; c += 2) {
      const float a = fabsf(x[c]) + fabsf(y[c]), b = fabsf(x[c + 1]) + fabsf(y[c + 1]);
      const float num = fmaf(fabsf(x[c] - y[c]), b, fabsf(x[c + 1] - y[c + 1]) * a);
      s = fmaf(num, __builtin_amdgcn_rcpf(a * b), s);
    }
    return s;
  }
#pragma unroll
  for (int c = 0; c < DM; ++c) s = dist32_step<M, G>(s, x[c], y[c]);
  return dist32_final<M>(s, ux, uy);
}

// the element's row in LDS, one column per lane (x[c * 64])
template <int M, int DM>
__device__ __forceinline__ float dist32_col(const float* __restrict__ x, const float* __restrict__ y, float ux,
                                          float uy) {
  float s = 0.f;
#pragma unroll 32
  for (int c = 0; c < DM; ++c) s = dist32_step<M>(s, x[c * kWave], y[c]);
  return dist32_final<M>(s, ux, uy);
}

// PASS 0: the whole row.  Manhattan and Canberra are sums over coordinates,
// so for d > 128 each cluster's weighted sum splits exactly into the sums over
// coordinates [0, 128) and [128, 256): PASS 1 takes the first half and
// stores the per-cluster float64 sums in Wpart [n][k]; PASS 2 takes the second
// half (c0 = 128), adds Wpart and finishes.  ystride is the packed sample's
// row length.
template <int M, int DM, int PASS>
__device__ __forceinline__ void p2_valu_block(
    const int blk, const float* __restrict__ X, int n, int d, const int32_t* __restrict__ labels,
    const float* __restrict__ Y, const float* __restrict__ w, const float* __restrict__ aux,
    const int32_t* __restrict__ sp_off,
    const int32_t* __restrict__ cnt, const int32_t* __restrict__ csize, int k,
    float* __restrict__ a_out, float* __restrict__ b_out, float* __restrict__ s_out,
    float* __restrict__ What, double* __restrict__ bpart, int c0, int ystride,
    double* __restrict__ Wpart, const float* __restrict__ rn) {
  static_assert(PASS == 0 || M == kManh || M == kCanb, "only sums over coordinates split");
  __shared__ double sh[kP2Rows / kWave];
  const int e = blk * kP2Rows + threadIdx.x;
  const bool valid = e < n;
  const int er = valid ? e : n - 1;

  float x[DM];
  const float* xr = X + (size_t)er * d + c0;
#pragma unroll
  for (int c = 0; c < DM; ++c) x[c] = c0 + c < d ? xr[c] : 0.0f;
  float ux = 0.f;
  if (M == kCos) {  // unit vector: the row times its reciprocal norm (zero stays zero, u = 0.5)
    const float rx = rn[er];
    ux = rx > 0.f ? 0.f : 0.5f;
#pragma unroll
    for (int c = 0; c < DM; ++c) x[c] *= rx;
  }
  const int own = (unsigned)labels[er] < (unsigned)k ? labels[er] : 0;  // labels are checked before; stay in bounds

  // Canberra: the pair form (dist32, G = false) when every element row of the
  // wave has its coordinates in [2^-62, 2^62] in magnitude (padding
  // coordinates are 0, so a padded row keeps the guarded form), and for each
  // sample whose row the packing did not flag (aux = 1: a coordinate past
  // 2^62 or not finite)
  bool guard = true;
  if (M == kCanb) {
    bool in = true;
#pragma unroll
    for (int c = 0; c < DM; ++c) in = in && fabsf(x[c]) >= 0x1p-62f && fabsf(x[c]) <= 0x1p62f;
    guard = !__all(in);
  }
  double w_own = 0.0;
  double bmin = __builtin_inf();
  for (int j = 0; j < k; ++j) {
    const int s0 = sp_off[j];
    const int cj = cnt[j];
    double accd = 0.0;
    auto sweep = [&](auto g) {
      constexpr bool G = decltype(g)::value;
      for (int g0 = 0; g0 < cj; g0 += kGroup) {
        const int g1 = g0 + kGroup < cj ? g0 + kGroup : cj;
        float acc = 0.f;
        for (int q = g0; q < g1; ++q) {
          const float* y = Y + (size_t)(s0 + q) * ystride + c0;
          const float uy = M == kCos ? aux[s0 + q] : 0.f;
          if (M == kCanb && !G && aux[s0 + q] != 0.f)  // wave-uniform
            acc = fmaf(w[s0 + q], dist32<M, DM, true>(x, y, ux, uy), acc);
          else
            acc = fmaf(w[s0 + q], dist32<M, DM, G>(x, y, ux, uy), acc);
        }
        accd += (double)acc;
      }
    };
    if (M == kCanb && !guard)
      sweep(std::integral_constant<bool, false>{});
    else
      sweep(std::integral_constant<bool, true>{});
    if (PASS == 1) {
      if (valid) Wpart[(size_t)e * k + j] = accd;
      continue;
    }
    if (PASS == 2) accd += Wpart[(size_t)er * k + j];
    if (What != nullptr && valid) What[(size_t)e * k + j] = (float)accd;
    const int sz = csize[j];
    if (j == own) {
      w_own = accd;
    } else if (sz > 0) {
      const double bj = accd / (double)sz;
      bmin = bj < bmin ? bj : bmin;
    }
  }
  if (PASS == 1) return;
  const int szo = csize[own];
  const double a = szo > 1 ? w_own / (double)(szo - 1) : 0.0;
  const double b = bmin;
  const double mx = a > b ? a : b;
  const double s = (szo > 1 && mx > 0.0) ? (b - a) / mx : 0.0;
  if (valid) {
    if (a_out) a_out[e] = (float)a;
    if (b_out) b_out[e] = (float)b;
    if (s_out) s_out[e] = (float)s;
  }
  const double tot = block_sum_f64<kP2Rows>(valid ? s : 0.0, sh);
  if (threadIdx.x == 0) bpart[blk] = tot;
}

template <int M, int DM, int PASS>
__global__ __launch_bounds__(kP2Rows) void k_p2_valu(
    const float* __restrict__ X, int n, int d, const int32_t* __restrict__ labels,
    const float* __restrict__ Y, const float* __restrict__ w, const float* __restrict__ aux,
    const int32_t* __restrict__ sp_off,
    const int32_t* __restrict__ cnt, const int32_t* __restrict__ csize, int k,
    float* __restrict__ a_out, float* __restrict__ b_out, float* __restrict__ s_out,
    float* __restrict__ What, double* __restrict__ bpart, int c0, int ystride,
    double* __restrict__ Wpart, const float* __restrict__ rn) {
  p2_valu_block<M, DM, PASS>(blockIdx.x, X, n, d, labels, Y, w, aux, sp_off, cnt, csize, k, a_out, b_out, s_out,
                             What, bpart, c0, ystride, Wpart, rn);
}

// Several requests in one launch (one-pass shapes): workgroup i runs work
// item i = (request, block), exactly as that block of the request's own
// launch; job table and items read through the constant address space.
template <int M, int DM>
__global__ __launch_bounds__(kP2Rows) void k_p2_valu_jobs(const P2Job* __restrict__ jobs,
                                                          const int2* __restrict__ items) {
  typedef const __attribute__((address_space(4))) P2Job* cjob_ptr;
  typedef const __attribute__((address_space(4))) int* citem_ptr;
  const int jx = ((citem_ptr)items)[2 * blockIdx.x];
  const int blk = ((citem_ptr)items)[2 * blockIdx.x + 1];
  const auto& J = ((cjob_ptr)jobs)[jx];
  p2_valu_block<M, DM, 0>(blk, J.X, J.n, J.d, J.labels, J.Y32, J.w, J.aux, J.sp_off, J.cnt, J.csize, J.k, J.a, J.b,
                          J.s, J.What, J.bpart, 0, DM, nullptr, J.rn);
}

// d > 128: one wave per block, each lane's row in LDS (column-major, 64 KB);
// otherwise as k_p2_valu
constexpr int kWideDM = 256;
template <int M>
__global__ __launch_bounds__(kWave) void k_p2_valu_wide(
    const float* __restrict__ X, int n, int d, const int32_t* __restrict__ labels,
    const float* __restrict__ Y, const float* __restrict__ w, const float* __restrict__ aux,
    const int32_t* __restrict__ sp_off, const int32_t* __restrict__ cnt, const int32_t* __restrict__ csize, int k,
    float* __restrict__ a_out, float* __restrict__ b_out, float* __restrict__ s_out,
    float* __restrict__ What, double* __restrict__ bpart, const float* __restrict__ rn) {
  __shared__ float xs[kWideDM * kWave];
  __shared__ double sh[1];
  const int e = blockIdx.x * kWave + threadIdx.x;
  const bool valid = e < n;
  const int er = valid ? e : n - 1;
  float* xl = xs + threadIdx.x;
  const float* xr = X + (size_t)er * d;
  // cosine: the row times its reciprocal norm (zero stays zero, u = 0.5)
  const float rx = M == kCos ? rn[er] : 1.0f;
  for (int c = 0; c < kWideDM; ++c) xl[c * kWave] = c < d ? xr[c] * rx : 0.0f;
  const float ux = (M == kCos && !(rx > 0.f)) ? 0.5f : 0.f;
  const int own = (unsigned)labels[er] < (unsigned)k ? labels[er] : 0;  // labels are checked before; stay in bounds
  double w_own = 0.0;
  double bmin = __builtin_inf();
  for (int j = 0; j < k; ++j) {
    const int s0 = sp_off[j];
    const int cj = cnt[j];
    double accd = 0.0;
    for (int g0 = 0; g0 < cj; g0 += kGroup) {
      const int g1 = g0 + kGroup < cj ? g0 + kGroup : cj;
      float acc = 0.f;
      for (int q = g0; q < g1; ++q) {
        const float* y = Y + (size_t)(s0 + q) * kWideDM;
        const float uy = M == kCos ? aux[s0 + q] : 0.f;
        acc = fmaf(w[s0 + q], dist32_col<M, kWideDM>(xl, y, ux, uy), acc);
      }
      accd += (double)acc;
    }
    if (What != nullptr && valid) What[(size_t)e * k + j] = (float)accd;
    const int sz = csize[j];
    if (j == own) {
      w_own = accd;
    } else if (sz > 0) {
      const double bj = accd / (double)sz;
      bmin = bj < bmin ? bj : bmin;
    }
  }
  const int szo = csize[own];
  const double a = szo > 1 ? w_own / (double)(szo - 1) : 0.0;
  const double b = bmin;
  const double mx = a > b ? a : b;
  const double sv = (szo > 1 && mx > 0.0) ? (b - a) / mx : 0.0;
  if (valid) {
    if (a_out) a_out[e] = (float)a;
    if (b_out) b_out[e] = (float)b;
    if (s_out) s_out[e] = (float)sv;
  }
  const double tot = block_sum_f64<kWave>(valid ? sv : 0.0, sh);
  if (threadIdx.x == 0) bpart[blockIdx.x] = tot;
}

int phase2_valu_dm(int d) {
  if (d <= 8) return 8;
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  if (d <= 128) return 128;
  if (d <= kWideDM) return kWideDM;
  return 0;
}

int phase2_valu_rows(int metric, int DM) {
  return (DM == kWideDM && metric != kManh && metric != kCanb) ? kWave : kP2Rows;
}
bool phase2_valu_split(int metric, int DM) { return DM == kWideDM && (metric == kManh || metric == kCanb); }

template <int M, int DM, int PASS = 0>
static void launch_one(hipStream_t st, const P2Args& A, int c0 = 0, int ystride = DM) {
  const int blocks = (int)ceil_div(A.n, kP2Rows);
  hipLaunchKernelGGL((k_p2_valu<M, DM, PASS>), dim3(blocks), dim3(kP2Rows), 0, st, A.X, A.n, A.d, A.labels,
                     A.Y, A.w, A.aux, A.sp_off, A.cnt, A.csize, A.k, A.a, A.b, A.s, A.What, A.bpart, c0,
                     ystride, A.Wpart, A.rn);
}

template <int M>
static bool launch_metric(hipStream_t st, int DM, const P2Args& A) {
  switch (DM) {
    case 8: launch_one<M, 8>(st, A); return true;
    case 16: launch_one<M, 16>(st, A); return true;
    case 32: launch_one<M, 32>(st, A); return true;
    case 64: launch_one<M, 64>(st, A); return true;
    case 128: launch_one<M, 128>(st, A); return true;
    case kWideDM:
      if constexpr (M == kManh || M == kCanb) {
        if (A.Wpart != nullptr) {  // two halves through the register kernel
          launch_one<M, 128, 1>(st, A, 0, kWideDM);
          launch_one<M, 128, 2>(st, A, 128, kWideDM);
          return true;
        }
      }
      hipLaunchKernelGGL(k_p2_valu_wide<M>, dim3((int)ceil_div(A.n, kWave)), dim3(kWave), 0, st, A.X, A.n, A.d,
                         A.labels, A.Y, A.w, A.aux, A.sp_off, A.cnt, A.csize, A.k, A.a, A.b, A.s, A.What,
                         A.bpart, A.rn);
      return true;
    default: return false;
  }
}

template <int M>
static bool launch_jobs_metric(hipStream_t st, int DM, const P2Job* jobs, const int2* items, int nitems) {
  switch (DM) {
    case 8: hipLaunchKernelGGL((k_p2_valu_jobs<M, 8>), dim3(nitems), dim3(kP2Rows), 0, st, jobs, items); return true;
    case 16: hipLaunchKernelGGL((k_p2_valu_jobs<M, 16>), dim3(nitems), dim3(kP2Rows), 0, st, jobs, items); return true;
    case 32: hipLaunchKernelGGL((k_p2_valu_jobs<M, 32>), dim3(nitems), dim3(kP2Rows), 0, st, jobs, items); return true;
    case 64: hipLaunchKernelGGL((k_p2_valu_jobs<M, 64>), dim3(nitems), dim3(kP2Rows), 0, st, jobs, items); return true;
    case 128:
      hipLaunchKernelGGL((k_p2_valu_jobs<M, 128>), dim3(nitems), dim3(kP2Rows), 0, st, jobs, items);
      return true;
    default: return false;
  }
}

bool phase2_valu_jobs_ok(int metric, int DM) { return metric >= 0 && metric <= 3 && DM >= 8 && DM <= 128; }

bool launch_phase2_valu_jobs(hipStream_t st, int metric, int DM, const P2Job* jobs, const int2* items, int nitems) {
  if (nitems <= 0) return true;
  switch (metric) {
    case kEucl: return launch_jobs_metric<kEucl>(st, DM, jobs, items, nitems);
    case kCos: return launch_jobs_metric<kCos>(st, DM, jobs, items, nitems);
    case kManh: return launch_jobs_metric<kManh>(st, DM, jobs, items, nitems);
    case kCanb: return launch_jobs_metric<kCanb>(st, DM, jobs, items, nitems);
    default: return false;
  }
}

bool launch_phase2_valu(hipStream_t st, int metric, int DM, const P2Args& A) {
  switch (metric) {
    case kEucl: return launch_metric<kEucl>(st, DM, A);
    case kCos: return launch_metric<kCos>(st, DM, A);
    case kManh: return launch_metric<kManh>(st, DM, A);
    case kCanb: return launch_metric<kCanb>(st, DM, A);
    default: return false;
  }
}

// ----------------------------------------------------------------------------
// Eq. 9: (1/n) * sum of the per-block partials, float64 with Neumaier
// compensation, fixed order (thread-strided, then a tree over threads).
// ----------------------------------------------------------------------------
__device__ __forceinline__ void neumaier_add(double& s, double& c, double v) {
  const double t = s + v;
  if (fabs(s) >= fabs(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

__global__ __launch_bounds__(256) void k_mean(const double* __restrict__ bpart, int nb, int64_t n,
                                              double* __restrict__ out) {
  __shared__ double ss[256], cc[256];
  double s = 0.0, c = 0.0;
#pragma unroll 8
  for (int i = threadIdx.x; i < nb; i += 256) neumaier_add(s, c, bpart[i]);  // loads issued ahead
  ss[threadIdx.x] = s;
  cc[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      double s1 = ss[threadIdx.x], c1 = cc[threadIdx.x] + cc[threadIdx.x + o];
      neumaier_add(s1, c1, ss[threadIdx.x + o]);
      ss[threadIdx.x] = s1;
      cc[threadIdx.x] = c1;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (ss[0] + cc[0]) / (double)n;
}

void launch_mean(hipStream_t st, const double* bpart, int nb, int64_t n, double* out) {
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, bpart, nb, n, out);
}

}  // namespace silh
