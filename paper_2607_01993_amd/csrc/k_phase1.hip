// Phase 1 of Algorithm 1 (PPS sampling) and the uniform Poisson sampler of
// Section 4.1.3, all decisions in float64.
//
// This file is compiled with -ffp-contract=off: every distance below is one
// rounding per elementary operation, coordinates accumulated in increasing
// order, so its value does not depend on how the compiler schedules it.
#include "device_common.hpp"
#include "silh_internal.hpp"

#pragma clang fp contract(off)

namespace silh {

// Distance from x (float32 row held in registers, promoted exactly; zero
// beyond the true dimension) to one float64 row y (stride DM, zero-padded),
// for the metric M.  Zero coordinates add exact zeros, so the padding does
// not change the value.
// One coordinate of a float64 distance, in coordinate order with one rounding
// per operation (the oracle's order), and the final step.
template <int M>
__device__ __forceinline__ void dist64_step(double& acc, double& dot, double& ny2, double xc, double yc) {
  if (M == kEucl) {
    const double df = xc - yc;
    acc = acc + df * df;
  } else if (M == kManh) {
    acc = acc + fabs(xc - yc);
  } else if (M == kCanb) {
    const double num = fabs(xc - yc);
    const double den = fabs(xc) + fabs(yc);
    const double term = den > 0.0 ? num / den : 0.0;
    acc = acc + term;
  } else {
    dot = dot + xc * yc;
    ny2 = ny2 + yc * yc;
  }
}

template <int M>
__device__ __forceinline__ double dist64_final(double acc, double dot, double ny2, double nx2) {
  if (M == kEucl) return __dsqrt_rn(acc);
  if (M == kCos) {
    const double den = __dsqrt_rn(nx2) * __dsqrt_rn(ny2);
    const double sim = den > 0.0 ? dot / den : 0.0;
    const double v = 1.0 - sim;
    return v < 0.0 ? 0.0 : (v > 2.0 ? 2.0 : v);
  }
  return acc;
}

// the element's row in registers
template <int M, int DM>
__device__ __forceinline__ double dist64(const float (&x)[DM], double nx2, const double* __restrict__ y) {
  double acc = 0.0, dot = 0.0, ny2 = 0.0;
#pragma unroll
  for (int c = 0; c < DM; ++c) dist64_step<M>(acc, dot, ny2, (double)x[c], y[c]);
  return dist64_final<M>(acc, dot, ny2, nx2);
}

// the element's row in LDS, one column per lane (x[c * 64])
template <int M, int DM>
__device__ __forceinline__ double dist64_col(const float* __restrict__ x, double nx2,
                                             const double* __restrict__ y) {
  double acc = 0.0, dot = 0.0, ny2 = 0.0;
#pragma unroll 16
  for (int c = 0; c < DM; ++c) dist64_step<M>(acc, dot, ny2, (double)x[c * kWave], y[c]);
  return dist64_final<M>(acc, dot, ny2, nx2);
}

// x row -> registers (vector loads when the row is 16-byte aligned), and its
// squared norm for the cosine
template <int M, int DM>
__device__ __forceinline__ double load_row(const float* __restrict__ X, int d, int g, float (&x)[DM]) {
  const float* xr = X + (size_t)g * d;
  if ((d & 3) == 0) {
#pragma unroll
    for (int c = 0; c < DM; c += 4) {
      if (c < d) {
        const float4 v = *(const float4*)(xr + c);
        x[c] = v.x;
        x[c + 1] = v.y;
        x[c + 2] = v.z;
        x[c + 3] = v.w;
      } else {
        x[c] = x[c + 1] = x[c + 2] = x[c + 3] = 0.0f;
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < DM; ++c) x[c] = c < d ? xr[c] : 0.0f;
  }
  double nx2 = 0.0;
  if (M == kCos) {
#pragma unroll
    for (int c = 0; c < DM; ++c) nx2 = nx2 + (double)x[c] * (double)x[c];
  }
  return nx2;
}

// Rows too long for registers (d > 128): each thread streams its row from
// memory in chunks of kWideC coordinates and evaluates the distances to a
// group of kWideG rows of the initial sample together (kWideG independent
// float64 chains, so the wave is not held by one chain's latency); the
// group's rows sit in LDS, read by every lane at the same address.  Each
// distance still takes its coordinates in increasing order.
constexpr int kWideDM = 256;
constexpr int kWideC = 32;
constexpr int kWideG = 8;

// coordinates [c0, c0 + kWideC) of row xr (zero from d on)
__device__ __forceinline__ void load_chunk_wide(const float* __restrict__ xr, int d, int c0, bool vec,
                                                float (&x)[kWideC]) {
  if (vec) {
#pragma unroll
    for (int c = 0; c < kWideC; c += 4) {
      const bool in = c0 + c < d;
      const float4 v = *(const float4*)(xr + (in ? c0 + c : 0));
      x[c] = in ? v.x : 0.0f;
      x[c + 1] = in ? v.y : 0.0f;
      x[c + 2] = in ? v.z : 0.0f;
      x[c + 3] = in ? v.w : 0.0f;
    }
  } else {
#pragma unroll
    for (int c = 0; c < kWideC; ++c) {
      const bool in = c0 + c < d;
      const float v = xr[in ? c0 + c : 0];
      x[c] = in ? v : 0.0f;
    }
  }
}

// the squared norm of a streamed row, in coordinate order (cosine; DW is
// the padded width, the coordinates past d add exact zeros)
template <int DW = kWideDM>
__device__ __forceinline__ double row_norm2_wide(const float* __restrict__ xr, int d, bool vec) {
  double nx2 = 0.0;
  for (int c0 = 0; c0 < DW; c0 += kWideC) {
    float x[kWideC];
    load_chunk_wide(xr, d, c0, vec, x);
#pragma unroll
    for (int c = 0; c < kWideC; ++c) nx2 = nx2 + (double)x[c] * (double)x[c];
  }
  return nx2;
}

// distances from row xr to the kWideG rows ys[e][.] (stride kWideDM)
template <int M, int DW = kWideDM>
__device__ __forceinline__ void dist64_group_wide(const float* __restrict__ xr, int d, bool vec, double nx2,
                                                  const double (*__restrict__ ys)[kWideDM],
                                                  double (&dv)[kWideG]) {
  double acc[kWideG], dot[kWideG], ny2[kWideG];
#pragma unroll
  for (int e = 0; e < kWideG; ++e) acc[e] = dot[e] = ny2[e] = 0.0;
  for (int c0 = 0; c0 < DW; c0 += kWideC) {
    float x[kWideC];
    load_chunk_wide(xr, d, c0, vec, x);
#pragma unroll
    for (int c = 0; c < kWideC; ++c) {
      const double xc = (double)x[c];
#pragma unroll
      for (int e = 0; e < kWideG; ++e) dist64_step<M>(acc[e], dot[e], ny2[e], xc, ys[e][c0 + c]);
    }
  }
#pragma unroll
  for (int e = 0; e < kWideG; ++e) dv[e] = dist64_final<M>(acc[e], dot[e], ny2[e], nx2);
}

constexpr int kEB = 4;  // initial-sample rows summed together in the W pass

// ----------------------------------------------------------------------------
// F^0 draw: sorted position i, element g = perm[i] of cluster j; kept when
// |C_j| > t and U(seed, g, 0) < q_j.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_f0_flag(const int32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ slab, int n,
                                                 const int32_t* __restrict__ csize,
                                                 const double* __restrict__ q, int64_t t,
                                                 uint64_t seed, int32_t* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = slab[i];
  int32_t f = 0;
  if ((int64_t)csize[j] > t) f = uniform53(seed, (uint64_t)perm[i], kStreamF0) < q[j] ? 1 : 0;
  flag[i] = f;
}

void launch_f0_flag(hipStream_t st, const int32_t* perm, const int32_t* slab, int n,
                    const int32_t* csize, const double* q, int64_t t, uint64_t seed, int32_t* flag) {
  hipLaunchKernelGGL(k_f0_flag, dim3((int)ceil_div(n, 256)), dim3(256), 0, st, perm, slab, n, csize,
                     q, t, seed, flag);
}

__global__ __launch_bounds__(256) void k_f0_pack(const int32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ slab,
                                                 const int32_t* __restrict__ flag,
                                                 const int32_t* __restrict__ pos, int n,
                                                 const float* __restrict__ X, int d, int DM,
                                                 int cap, int64_t* __restrict__ f0_gid,
                                                 int32_t* __restrict__ f0_cl, double* __restrict__ f0X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const int dst = pos[i];
  if (dst >= cap) return;  // capacity of f0_gid / f0_cl / f0X rows
  const int g = perm[i];
  f0_gid[dst] = g;
  f0_cl[dst] = slab[i];
  const float* xr = X + (size_t)g * d;
  double* yr = f0X + (size_t)dst * DM;
  if ((d & 3) == 0 && ((uintptr_t)X & 15) == 0) {
    // 16-byte row chunks (DM is a multiple of 8, so the float64 row is too)
    for (int c = 0; c < DM; c += 4) {
      const float4 v = c < d ? *(const float4*)(xr + c) : float4{0.f, 0.f, 0.f, 0.f};
      *(double2*)(yr + c) = double2{(double)v.x, (double)v.y};
      *(double2*)(yr + c + 2) = double2{(double)v.z, (double)v.w};
    }
  } else {
    for (int c = 0; c < DM; ++c) yr[c] = c < d ? (double)xr[c] : 0.0;
  }
}

void launch_f0_pack(hipStream_t st, const int32_t* perm, const int32_t* slab, const int32_t* flag,
                    const int32_t* pos, int n, const float* X, int d, int DM, int cap, int64_t* f0_gid,
                    int32_t* f0_cl, double* f0X) {
  hipLaunchKernelGGL(k_f0_pack, dim3((int)ceil_div(n, 256)), dim3(256), 0, st, perm, slab, flag, pos,
                     n, X, d, DM, cap, f0_gid, f0_cl, f0X);
}

// ----------------------------------------------------------------------------
// W(e_bar) = sum_{e' in C_j} d(e_bar, e') (Algorithm 1, Phase 1).  A work item
// covers up to kWChunk consecutive members of one cluster; its block writes
// one partial sum per initial element (per-thread sums in member order, then
// a fixed-order block reduction).
// item layout: [cluster, begin, end, f0_begin, f0_count, partial_base]
// ----------------------------------------------------------------------------
// kEB float64 values per lane summed over the wave: two exchange steps (lane
// distance 32, then 16) leave each lane one of the four values, then a
// butterfly over distances 8, 4, 2, 1.  Every sum pairs the same lanes in the
// same order as a plain butterfly over 32..1 (a + b == b + a), so each total
// equals that butterfly's bit for bit.  Lanes with (lane & 15) == 0 end up
// holding the total of value 2 * ((lane >> 5) & 1) + ((lane >> 4) & 1).
__device__ __forceinline__ double wave_sum4_f64(const double (&v)[kEB], int lane) {
  static_assert(kEB == 4, "four values per exchange");
  const bool b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1;
  const double r0 = __shfl_xor(b5 ? v[0] : v[2], 32, kWave);
  const double r1 = __shfl_xor(b5 ? v[1] : v[3], 32, kWave);
  const double u0 = (b5 ? v[2] : v[0]) + r0;
  const double u1 = (b5 ? v[3] : v[1]) + r1;
  const double r = __shfl_xor(b4 ? u0 : u1, 16, kWave);
  double w = (b4 ? u1 : u0) + r;
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) w += __shfl_xor(w, o, kWave);
  return w;
}

constexpr int kWSlots = 64;  // partial sums gathered in LDS between two barriers

template <int M, int DM>
__global__ __launch_bounds__(256) void k_w_partial(const int32_t* __restrict__ items,
                                                   const int32_t* __restrict__ perm,
                                                   const float* __restrict__ X, int d,
                                                   const double* __restrict__ f0X,
                                                   double* __restrict__ partial, DistStore ds) {
  static_assert(DM <= 64, "longer rows take k_w_partial_wide");
  __shared__ double sh[4][kWSlots];  // per wave, per initial element of the current batch
  const int32_t* it = items + (size_t)blockIdx.x * 6;
  const int begin = it[1], end = it[2], f0b = it[3], f0n = it[4], pb = it[5];
  // the kept distances of this item's members (cluster it[0]): one column
  // per initial element, members contiguous
  double* keep = nullptr;
  int64_t kstride = 0;
  if (ds.d != nullptr && f0n > 0 && *ds.use) {
    const int j = it[0];
    kstride = ds.off[j + 1] - ds.off[j];
    keep = ds.d + ds.base[j] + (begin - ds.off[j]) + threadIdx.x;
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  // one member row per thread (items hold at most 256 members), read once
  const int r = begin + threadIdx.x;
  const bool have = r < end;
  float x[DM];
  double nx2 = 0.0;
  if (have) {
    nx2 = load_row<M, DM>(X, d, perm[r], x);
  } else {
#pragma unroll
    for (int c = 0; c < DM; ++c) x[c] = 0.0f;
  }
  // per initial element: member distances summed over the wave, then the
  // four wave sums in wave order (one thread per element)
  for (int s0 = 0; s0 < f0n; s0 += kWSlots) {
    const int ns = f0n - s0 < kWSlots ? f0n - s0 : kWSlots;
    for (int e0 = 0; e0 < ns; e0 += kEB) {
      double dv[kEB];
#pragma unroll
      for (int e = 0; e < kEB; ++e) {
        const int ee = e0 + e < ns ? e0 + e : ns - 1;   // repeats a row instead of branching
        const double v = dist64<M, DM>(x, nx2, f0X + (size_t)(f0b + s0 + ee) * DM);
        dv[e] = have ? v : 0.0;
        if (keep != nullptr && have && e0 + e < ns) keep[(int64_t)(s0 + e0 + e) * kstride] = v;
      }
      const double w = wave_sum4_f64(dv, lane);
      const int slot = e0 + 2 * ((lane >> 5) & 1) + ((lane >> 4) & 1);
      if ((lane & 15) == 0 && slot < ns) sh[wid][slot] = w;
    }
    __syncthreads();
    if (threadIdx.x < ns) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) t += sh[i][threadIdx.x];
      partial[pb + s0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// d > 64: a 256-thread block per item (one member per thread), each thread
// streaming its row from memory, the item's initial-sample rows (stride DW)
// staged kWideG at a time.  At d <= 128 the row would fit the registers, but
// beside the float64 chains of k_w_partial it leaves one wave per SIMD
template <int M, int DW>
__global__ __launch_bounds__(256) void k_w_partial_wide(const int32_t* __restrict__ items,
                                                        const int32_t* __restrict__ perm,
                                                        const float* __restrict__ X, int d,
                                                        const double* __restrict__ f0X,
                                                        double* __restrict__ partial, DistStore ds) {
  __shared__ double ys[kWideG][kWideDM];
  __shared__ double sh[4];
  const int32_t* it = items + (size_t)blockIdx.x * 6;
  const int begin = it[1], end = it[2], f0b = it[3], f0n = it[4], pb = it[5];
  double* keep = nullptr;
  int64_t kstride = 0;
  if (ds.d != nullptr && f0n > 0 && *ds.use) {
    const int j = it[0];
    kstride = ds.off[j + 1] - ds.off[j];
    keep = ds.d + ds.base[j] + (begin - ds.off[j]) + threadIdx.x;
  }
  const int r = begin + threadIdx.x;
  const bool have = r < end;
  const float* xr = X + (size_t)(have ? perm[r] : 0) * d;
  const bool vec = (d & 3) == 0 && ((uintptr_t)X & 15) == 0;
  const double nx2 = M == kCos ? row_norm2_wide<DW>(xr, d, vec) : 0.0;
  for (int e0 = 0; e0 < f0n; e0 += kWideG) {
    const int ne = f0n - e0 < kWideG ? f0n - e0 : kWideG;  // uniform over the block
    __syncthreads();
    for (int q = threadIdx.x; q < kWideG * DW; q += 256) {
      const int e = q / DW, c = q - e * DW;
      ys[e][c] = f0X[(size_t)(f0b + e0 + (e < ne ? e : ne - 1)) * DW + c];  // past ne: a copy
    }
    __syncthreads();
    double dv[kWideG];
    dist64_group_wide<M, DW>(xr, d, vec, nx2, ys, dv);
#pragma unroll
    for (int e = 0; e < kWideG; ++e) {
      if (e < ne) {
        if (keep != nullptr && have) keep[(int64_t)(e0 + e) * kstride] = dv[e];
        const double tot = block_sum_f64<256>(have ? dv[e] : 0.0, sh);
        if (threadIdx.x == 0) partial[pb + e0 + e] = tot;
      }
    }
  }
}

#define SILH_P1_DISPATCH(KERNEL, GRID, ...)                                                   \
  do {                                                                                        \
    switch (metric * 8 + (DM == 8 ? 0 : DM == 16 ? 1 : DM == 32 ? 2 : DM == 64 ? 3 : 4)) {    \
      case 0: hipLaunchKernelGGL((KERNEL<kEucl, 8>), GRID, dim3(256), 0, st, __VA_ARGS__); break;   \
      case 1: hipLaunchKernelGGL((KERNEL<kEucl, 16>), GRID, dim3(256), 0, st, __VA_ARGS__); break;  \
      case 2: hipLaunchKernelGGL((KERNEL<kEucl, 32>), GRID, dim3(256), 0, st, __VA_ARGS__); break;  \
      case 3: hipLaunchKernelGGL((KERNEL<kEucl, 64>), GRID, dim3(256), 0, st, __VA_ARGS__); break;  \
      case 4: hipLaunchKernelGGL((KERNEL<kEucl, 128>), GRID, dim3(256), 0, st, __VA_ARGS__); break; \
      case 8: hipLaunchKernelGGL((KERNEL<kCos, 8>), GRID, dim3(256), 0, st, __VA_ARGS__); break;    \
      case 9: hipLaunchKernelGGL((KERNEL<kCos, 16>), GRID, dim3(256), 0, st, __VA_ARGS__); break;   \
      case 10: hipLaunchKernelGGL((KERNEL<kCos, 32>), GRID, dim3(256), 0, st, __VA_ARGS__); break;  \
      case 11: hipLaunchKernelGGL((KERNEL<kCos, 64>), GRID, dim3(256), 0, st, __VA_ARGS__); break;  \
      case 12: hipLaunchKernelGGL((KERNEL<kCos, 128>), GRID, dim3(256), 0, st, __VA_ARGS__); break; \
      case 16: hipLaunchKernelGGL((KERNEL<kManh, 8>), GRID, dim3(256), 0, st, __VA_ARGS__); break;  \
      case 17: hipLaunchKernelGGL((KERNEL<kManh, 16>), GRID, dim3(256), 0, st, __VA_ARGS__); break; \
      case 18: hipLaunchKernelGGL((KERNEL<kManh, 32>), GRID, dim3(256), 0, st, __VA_ARGS__); break; \
      case 19: hipLaunchKernelGGL((KERNEL<kManh, 64>), GRID, dim3(256), 0, st, __VA_ARGS__); break; \
      case 20: hipLaunchKernelGGL((KERNEL<kManh, 128>), GRID, dim3(256), 0, st, __VA_ARGS__); break;\
      case 24: hipLaunchKernelGGL((KERNEL<kCanb, 8>), GRID, dim3(256), 0, st, __VA_ARGS__); break;  \
      case 25: hipLaunchKernelGGL((KERNEL<kCanb, 16>), GRID, dim3(256), 0, st, __VA_ARGS__); break; \
      case 26: hipLaunchKernelGGL((KERNEL<kCanb, 32>), GRID, dim3(256), 0, st, __VA_ARGS__); break; \
      case 27: hipLaunchKernelGGL((KERNEL<kCanb, 64>), GRID, dim3(256), 0, st, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL((KERNEL<kCanb, 128>), GRID, dim3(256), 0, st, __VA_ARGS__); break;\
    }                                                                                         \
  } while (0)

void launch_w_partial(hipStream_t st, int metric, int DM, const int32_t* items, int nitems,
                      const int32_t* perm, const float* X, int d, const double* f0X, double* partial,
                      DistStore ds) {
  if (nitems <= 0) return;
  if (DM == kWideDM || DM == 128) {
#define SILH_WP(MM)                                                                                       \
  do {                                                                                                    \
    if (DM == 128)                                                                                        \
      hipLaunchKernelGGL((k_w_partial_wide<MM, 128>), dim3(nitems), dim3(256), 0, st, items, perm, X, d, f0X, \
                         partial, ds);                                                                    \
    else                                                                                                  \
      hipLaunchKernelGGL((k_w_partial_wide<MM, kWideDM>), dim3(nitems), dim3(256), 0, st, items, perm, X, d, \
                         f0X, partial, ds);                                                               \
  } while (0)
    switch (metric) {
      case kEucl: SILH_WP(kEucl); break;
      case kCos: SILH_WP(kCos); break;
      case kManh: SILH_WP(kManh); break;
      default: SILH_WP(kCanb); break;
    }
#undef SILH_WP
    return;
  }
  // DM <= 64 here (the row in registers beside the float64 chains)
  switch (metric * 8 + (DM == 8 ? 0 : DM == 16 ? 1 : DM == 32 ? 2 : 3)) {
#define SILH_WPS(CASE, MM, DD)                                                                            \
  case CASE:                                                                                              \
    hipLaunchKernelGGL((k_w_partial<MM, DD>), dim3(nitems), dim3(256), 0, st, items, perm, X, d, f0X, partial, ds); \
    break;
    SILH_WPS(0, kEucl, 8) SILH_WPS(1, kEucl, 16) SILH_WPS(2, kEucl, 32) SILH_WPS(3, kEucl, 64)
    SILH_WPS(8, kCos, 8) SILH_WPS(9, kCos, 16) SILH_WPS(10, kCos, 32) SILH_WPS(11, kCos, 64)
    SILH_WPS(16, kManh, 8) SILH_WPS(17, kManh, 16) SILH_WPS(18, kManh, 32) SILH_WPS(19, kManh, 64)
    SILH_WPS(24, kCanb, 8) SILH_WPS(25, kCanb, 16) SILH_WPS(26, kCanb, 32)
    default: SILH_WPS(27, kCanb, 64)
#undef SILH_WPS
  }
}

// W(e_bar): sum of its cluster's item partials.  One block per initial
// element (blocks past f0_off[k], the size of F0, return at once); threads
// take items in a fixed stride, then a fixed-order block sum.
__global__ __launch_bounds__(256) void k_w_final(const int32_t* __restrict__ f0_cl,
                                                 const int32_t* __restrict__ f0_off, int k,
                                                 const int32_t* __restrict__ citem_first,
                                                 const int32_t* __restrict__ citem_count,
                                                 const int32_t* __restrict__ items,
                                                 const double* __restrict__ partial,
                                                 double* __restrict__ W) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  if (i >= f0_off[k]) return;
  const int j = f0_cl[i];
  const int local = i - f0_off[j];
  const int first = citem_first[j], cnt = citem_count[j];
  double s = 0.0;
  for (int q = threadIdx.x; q < cnt; q += 256) s = s + partial[items[(size_t)(first + q) * 6 + 5] + local];
  const double tot = block_sum_f64<256>(s, sh);
  if (threadIdx.x == 0) W[i] = tot;
}

void launch_w_final(hipStream_t st, const int32_t* f0_cl, int F0, const int32_t* f0_off, int k,
                    const int32_t* citem_first, const int32_t* citem_count, const int32_t* items,
                    const double* partial, double* W) {
  if (F0 <= 0) return;
  hipLaunchKernelGGL(k_w_final, dim3(F0), dim3(256), 0, st, f0_cl, f0_off, k, citem_first, citem_count,
                     items, partial, W);
}

// ----------------------------------------------------------------------------
// gamma_e, p_e and the final Poisson draw (PPS), or the uniform rate t/|C_j|.
// Clusters with |C_j| <= t are taken whole with p = 1.
// ----------------------------------------------------------------------------
constexpr int kDrawB = 8;  // kept distances loaded together by the draw

// The draw's path for distances the W pass did not keep: the element's row
// read from memory four coordinates at a time as each chain goes (the same
// operations in the same order as dist64 on the row held in registers), so
// that this rarely taken path does not set the draw kernel's register count
// and occupancy for the kept-distance path.
__device__ __forceinline__ void load4_row(const float* __restrict__ xr, int c0, int d, bool vec, float (&x)[4]) {
  if (vec) {
    const bool in = c0 < d;
    const float4 v = *(const float4*)(xr + (in ? c0 : 0));
    x[0] = in ? v.x : 0.0f;
    x[1] = in ? v.y : 0.0f;
    x[2] = in ? v.z : 0.0f;
    x[3] = in ? v.w : 0.0f;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = c0 + e < d ? xr[c0 + e] : 0.0f;
  }
}

template <int M, int DM>
__device__ __forceinline__ double dist64_mem(const float* __restrict__ xr, int d, bool vec, double nx2,
                                             const double* __restrict__ y) {
  double acc = 0.0, dot = 0.0, ny2 = 0.0;
#pragma unroll 2
  for (int c0 = 0; c0 < DM; c0 += 4) {
    float x[4];
    load4_row(xr, c0, d, vec, x);
#pragma unroll
    for (int e = 0; e < 4; ++e) dist64_step<M>(acc, dot, ny2, (double)x[e], y[c0 + e]);
  }
  return dist64_final<M>(acc, dot, ny2, nx2);
}

template <int DM>
__device__ __forceinline__ double row_norm2_mem(const float* __restrict__ xr, int d, bool vec) {
  double nx2 = 0.0;
  for (int c0 = 0; c0 < DM; c0 += 4) {
    float x[4];
    load4_row(xr, c0, d, vec, x);
#pragma unroll
    for (int e = 0; e < 4; ++e) nx2 = nx2 + (double)x[e] * (double)x[e];
  }
  return nx2;
}

template <int M, int DM>
__global__ __launch_bounds__(256) void k_draw(int sampler, const int32_t* __restrict__ perm,
                                              const int32_t* __restrict__ slab, int n,
                                              const float* __restrict__ X, int d,
                                              const int32_t* __restrict__ csize, int64_t t,
                                              uint64_t seed, const int32_t* __restrict__ f0_off,
                                              const double* __restrict__ f0X,
                                              const double* __restrict__ W,
                                              double* __restrict__ p_gid, int32_t* __restrict__ flag,
                                              DistStore ds) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int g = perm[i];
  const int j = slab[i];
  const int64_t m = csize[j];
  double p;
  int32_t sel;
  if (m <= t) {
    p = 1.0;
    sel = 1;
  } else if (sampler == 1) {
    p = (double)t / (double)m;
    p = p < 1.0 ? p : 1.0;
    sel = uniform53(seed, (uint64_t)g, kStreamUNI) < p ? 1 : 0;
  } else if (ds.d != nullptr && *ds.use && i >= ds.off[j] && i < ds.off[j + 1]) {
    // the W pass kept d(e, e_bar) for every initial element of the cluster
    // (the same float64 values the branch below evaluates); a position
    // outside its cluster's range (only where a label was out of range, and
    // the result is discarded) takes the branch below
    double gam = 1.0 / (double)m;
    const int fb = f0_off[j], fn = f0_off[j + 1] - fb;
    const int64_t stride = ds.off[j + 1] - ds.off[j];
    const double* kd = ds.d + ds.base[j] + (i - ds.off[j]);
    // kDrawB weights and distances are loaded before any is used, so their
    // latencies overlap; past the end the last element is repeated, which
    // leaves the maximum unchanged
    for (int e0 = 0; e0 < fn; e0 += kDrawB) {
      double wv[kDrawB], dv[kDrawB];
#pragma unroll
      for (int e = 0; e < kDrawB; ++e) {
        const int ee = e0 + e < fn ? e0 + e : fn - 1;
        wv[e] = W[fb + ee];
        dv[e] = kd[(int64_t)ee * stride];
      }
#pragma unroll
      for (int e = 0; e < kDrawB; ++e) {
        if (wv[e] > 0.0) {
          const double r = dv[e] / wv[e];
          gam = r > gam ? r : gam;
        }
      }
    }
    p = (double)t * gam;
    p = p < 1.0 ? p : 1.0;
    sel = uniform53(seed, (uint64_t)g, kStreamPPS) < p ? 1 : 0;
  } else {
    double gam = 1.0 / (double)m;
    const float* xr = X + (size_t)g * d;
    const bool vec = (d & 3) == 0;
    const double nx2 = M == kCos ? row_norm2_mem<DM>(xr, d, vec) : 0.0;
    // Most waves lie inside one cluster (sorted order): then the initial
    // sample rows and weights are wave-uniform and come in by scalar loads.
    const int jf = __builtin_amdgcn_readfirstlane(j);
    auto scan_f0 = [&](int jj) {
      const int fb = f0_off[jj], fe = f0_off[jj + 1];
      for (int e = fb; e < fe; ++e) {
        const double w = W[e];
        const double dv = dist64_mem<M, DM>(xr, d, vec, nx2, f0X + (size_t)e * DM);
        if (w > 0.0) {
          const double r = dv / w;
          gam = r > gam ? r : gam;
        }
      }
    };
    if (__all(j == jf))
      scan_f0(jf);
    else
      scan_f0(j);
    p = (double)t * gam;
    p = p < 1.0 ? p : 1.0;
    sel = uniform53(seed, (uint64_t)g, kStreamPPS) < p ? 1 : 0;
  }
  p_gid[g] = p;
  flag[i] = sel;
}

// d > 128: the kept distances where the W pass kept them (as k_draw), else
// the element's row streamed against its cluster's initial sample, kWideG
// rows at a time straight from memory
template <int M>
__global__ __launch_bounds__(256) void k_draw_wide(int sampler, const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ slab, int n,
                                                   const float* __restrict__ X, int d,
                                                   const int32_t* __restrict__ csize, int64_t t,
                                                   uint64_t seed, const int32_t* __restrict__ f0_off,
                                                   const double* __restrict__ f0X,
                                                   const double* __restrict__ W,
                                                   double* __restrict__ p_gid, int32_t* __restrict__ flag,
                                                   DistStore ds) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int g = perm[i];
  const int j = slab[i];
  const int64_t m = csize[j];
  double p;
  int32_t sel;
  if (m <= t) {
    p = 1.0;
    sel = 1;
  } else if (sampler == 1) {
    p = (double)t / (double)m;
    p = p < 1.0 ? p : 1.0;
    sel = uniform53(seed, (uint64_t)g, kStreamUNI) < p ? 1 : 0;
  } else {
    double gam = 1.0 / (double)m;
    const int fb = f0_off[j], fn = f0_off[j + 1] - fb;
    if (ds.d != nullptr && *ds.use && i >= ds.off[j] && i < ds.off[j + 1]) {
      const int64_t stride = ds.off[j + 1] - ds.off[j];
      const double* kd = ds.d + ds.base[j] + (i - ds.off[j]);
      for (int e0 = 0; e0 < fn; e0 += kDrawB) {
        double wv[kDrawB], dv[kDrawB];
#pragma unroll
        for (int e = 0; e < kDrawB; ++e) {
          const int ee = e0 + e < fn ? e0 + e : fn - 1;
          wv[e] = W[fb + ee];
          dv[e] = kd[(int64_t)ee * stride];
        }
#pragma unroll
        for (int e = 0; e < kDrawB; ++e) {
          if (wv[e] > 0.0) {
            const double r = dv[e] / wv[e];
            gam = r > gam ? r : gam;
          }
        }
      }
    } else {
      const float* xr = X + (size_t)g * d;
      const bool vec = (d & 3) == 0 && ((uintptr_t)X & 15) == 0;
      const double nx2 = M == kCos ? row_norm2_wide(xr, d, vec) : 0.0;
      for (int e = 0; e < fn; ++e) {
        const double* y = f0X + (size_t)(fb + e) * kWideDM;
        double acc = 0.0, dot = 0.0, ny2 = 0.0;
        for (int c0 = 0; c0 < kWideDM; c0 += kWideC) {
          float x[kWideC];
          load_chunk_wide(xr, d, c0, vec, x);
#pragma unroll
          for (int c = 0; c < kWideC; ++c) dist64_step<M>(acc, dot, ny2, (double)x[c], y[c0 + c]);
        }
        const double dv = dist64_final<M>(acc, dot, ny2, nx2);
        const double w = W[fb + e];
        if (w > 0.0) {
          const double r = dv / w;
          gam = r > gam ? r : gam;
        }
      }
    }
    p = (double)t * gam;
    p = p < 1.0 ? p : 1.0;
    sel = uniform53(seed, (uint64_t)g, kStreamPPS) < p ? 1 : 0;
  }
  p_gid[g] = p;
  flag[i] = sel;
}

void launch_draw(hipStream_t st, int metric, int DM, int sampler, const int32_t* perm,
                 const int32_t* slab, int n, const float* X, int d, const int32_t* csize, int64_t t,
                 uint64_t seed, const int32_t* f0_off, const double* f0X, const double* W,
                 double* p_gid, int32_t* flag, DistStore ds) {
  if (DM == kWideDM) {
#define SILH_DW(MM) hipLaunchKernelGGL(k_draw_wide<MM>, dim3((int)ceil_div(n, 256)), dim3(256), 0, st, sampler, perm, slab, n, X, d, csize, t, seed, f0_off, f0X, W, p_gid, flag, ds)
    switch (metric) {
      case kEucl: SILH_DW(kEucl); break;
      case kCos: SILH_DW(kCos); break;
      case kManh: SILH_DW(kManh); break;
      default: SILH_DW(kCanb); break;
    }
#undef SILH_DW
    return;
  }
  SILH_P1_DISPATCH(k_draw, dim3((int)ceil_div(n, 256)), sampler, perm, slab, n, X, d, csize, t, seed,
                   f0_off, f0X, W, p_gid, flag, ds);
}

// exact silhouette: every element kept with p = 1
__global__ __launch_bounds__(256) void k_fill_all(const int32_t* __restrict__ perm, int n,
                                                  double* __restrict__ p_gid, int32_t* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p_gid[perm[i]] = 1.0;
  flag[i] = 1;
}

void launch_fill_all(hipStream_t st, const int32_t* perm, int n, double* p_gid, int32_t* flag) {
  hipLaunchKernelGGL(k_fill_all, dim3((int)ceil_div(n, 256)), dim3(256), 0, st, perm, n, p_gid, flag);
}

// ----------------------------------------------------------------------------
// Sample packing: cluster-blocked rows padded to kSamplePad (padding rows have
// weight 0 and zero coordinates), weight w = 1/p in float32, and the unpadded
// id list for inspection.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pack(const int32_t* __restrict__ perm,
                                              const int32_t* __restrict__ slab,
                                              const int32_t* __restrict__ flag,
                                              const int32_t* __restrict__ pos, int n, int k,
                                              const float* __restrict__ X, int d, int DM,
                                              const double* __restrict__ p_gid,
                                              const int32_t* __restrict__ s_off,
                                              const int32_t* __restrict__ sp_off, int mode,
                                              const float* __restrict__ rn, int cap,
                                              int64_t* __restrict__ gid_view,
                                              int32_t* __restrict__ gid_pk, float* __restrict__ w32,
                                              float* __restrict__ aux32, float* __restrict__ Y32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) {
    // threads past n: the padding rows of each cluster block (at most 31,
    // slot (i - n) % 32 of cluster (i - n) / 32), id -1 and all zeros, so no
    // clear of the packed arrays is needed
    const int t = i - n, j = t >> 5;
    if (j >= k) return;
    const int dst = sp_off[j] + (s_off[j + 1] - s_off[j]) + (t & 31);
    if (dst >= sp_off[j + 1] || dst >= cap) return;
    gid_pk[dst] = -1;
    w32[dst] = 0.0f;
    aux32[dst] = 0.0f;
    float* yr = Y32 + (size_t)dst * DM;
    for (int c = 0; c < DM; c += 4) *(float4*)(yr + c) = float4{0.f, 0.f, 0.f, 0.f};
    return;
  }
  if (!flag[i]) return;
  const int g = perm[i];
  const int j = slab[i];
  const int ps = pos[i];
  const int dst = sp_off[j] + (ps - s_off[j]);
  if (dst >= cap || ps >= cap) return;  // capacity of the packed rows
  gid_view[ps] = g;
  // the packed row's element id, for the Phase-2 self-pair test (a zero row
  // under cosine gets -1: its distance to itself is 1 by the cosine reading)
  gid_pk[dst] = (mode == 1 && !(rn[g] > 0.0f)) ? -1 : g;
  w32[dst] = (float)(1.0 / p_gid[g]);
  const float* xr = X + (size_t)g * d;
  float* yr = Y32 + (size_t)dst * DM;
  const bool vec = (d & 3) == 0 && ((uintptr_t)X & 15) == 0;
  // cosine: the row times its float32 reciprocal norm, the same product the
  // Phase-2 kernels form for the element side (identical rows stay identical)
  float scale = 1.0f;
  if (mode == 1) scale = rn[g];
  // Canberra (mode 2): whether the row has a coordinate outside [-2^62, 2^62]
  // or not finite (a failed <= test), which keeps the Phase-2 kernel on its
  // per-coordinate form for this sample
  bool big = false;
  if (vec) {
    // 16-byte row chunks (DM is a multiple of 8)
    for (int c = 0; c < DM; c += 4) {
      const float4 v = c < d ? *(const float4*)(xr + c) : float4{0.f, 0.f, 0.f, 0.f};
      *(float4*)(yr + c) = float4{v.x * scale, v.y * scale, v.z * scale, v.w * scale};
      big = big || !(fabsf(v.x) <= 0x1p62f && fabsf(v.y) <= 0x1p62f && fabsf(v.z) <= 0x1p62f &&
                     fabsf(v.w) <= 0x1p62f);
    }
  } else {
    for (int c = 0; c < DM; ++c) {
      const float v = c < d ? xr[c] : 0.0f;
      yr[c] = v * scale;
      big = big || !(fabsf(v) <= 0x1p62f);
    }
  }
  aux32[dst] = (mode == 1 && !(scale > 0.0f)) ? 0.5f : (mode == 2 && big) ? 1.0f : 0.0f;
}

// Reciprocal L2 norm of every row in float32 (one rounding per operation:
// a fused multiply-add chain in coordinate order, then a correctly rounded
// square root and division), 0 for a zero row.  The cosine kernels scale both
// the element rows and the packed sample rows by it.  A block takes
// kRnRows rows: the 256 threads read them kRnCols columns at a time,
// coalesced, into LDS (row stride kRnCols + 1, so the chains below read
// distinct banks), and thread r < kRnRows carries row r's chain.  A row's
// value depends on nothing but its own coordinates.
constexpr int kRnRows = 64, kRnCols = 128;

__global__ __launch_bounds__(256) void k_rnorm(const float* __restrict__ X, int n, int d, float* __restrict__ rn) {
  __shared__ float tile[kRnRows][kRnCols + 1];
  const int64_t row0 = (int64_t)blockIdx.x * kRnRows;
  const int nr = n - row0 < kRnRows ? (int)(n - row0) : kRnRows;
  const bool vec = (d & 3) == 0 && ((uintptr_t)X & 15) == 0;
  float s2 = 0.0f;
  for (int c0 = 0; c0 < d; c0 += kRnCols) {
    const int cw = d - c0 < kRnCols ? d - c0 : kRnCols;
    if (vec) {
      const int q4 = cw >> 2;  // float4 per row of the chunk
      for (int q = threadIdx.x; q < nr * q4; q += 256) {
        const int r = q / q4, c = (q - r * q4) << 2;
        const float4 v = *(const float4*)(X + (row0 + r) * d + c0 + c);
        tile[r][c] = v.x;
        tile[r][c + 1] = v.y;
        tile[r][c + 2] = v.z;
        tile[r][c + 3] = v.w;
      }
    } else {
      for (int q = threadIdx.x; q < nr * cw; q += 256) {
        const int r = q / cw, c = q - r * cw;
        tile[r][c] = X[(row0 + r) * d + c0 + c];
      }
    }
    __syncthreads();
    if (threadIdx.x < nr) {
      for (int c = 0; c < cw; ++c) s2 = fmaf(tile[threadIdx.x][c], tile[threadIdx.x][c], s2);
    }
    __syncthreads();
  }
  if (threadIdx.x < nr) rn[row0 + threadIdx.x] = s2 > 0.0f ? 1.0f / sqrtf(s2) : 0.0f;
}

void launch_rnorm(hipStream_t st, const float* X, int n, int d, float* rn) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_rnorm, dim3((int)ceil_div(n, kRnRows)), dim3(256), 0, st, X, n, d, rn);
}

void launch_pack(hipStream_t st, const int32_t* perm, const int32_t* slab, const int32_t* flag,
                 const int32_t* pos, int n, int k, const float* X, int d, int DM, const double* p_gid,
                 const int32_t* s_off, const int32_t* sp_off, int mode, const float* rn, int cap,
                 int64_t* gid_view,
                 int32_t* gid_pk, float* w32, float* aux32, float* Y32) {
  hipLaunchKernelGGL(k_pack, dim3((int)ceil_div((int64_t)n + 32 * (int64_t)k, 256)), dim3(256), 0, st, perm, slab,
                     flag, pos, n, k, X, d, DM, p_gid, s_off, sp_off, mode, rn, cap, gid_view, gid_pk, w32, aux32,
                     Y32);
}

// ----------------------------------------------------------------------------
// diagnostics: the uniforms themselves
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_uniform(uint64_t seed, int64_t gid0, int64_t count,
                                                 uint32_t stream_id, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = uniform53(seed, (uint64_t)(gid0 + i), stream_id);
}

void launch_uniform(hipStream_t st, uint64_t seed, int64_t gid0, int64_t count, uint32_t stream_id,
                    double* out) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_uniform, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, st, seed, gid0,
                     count, stream_id, out);
}

}  // namespace silh
