// Device helpers shared by the kernels of the silhouette library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace silh {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 bit
// multiplies with the multipliers below, key bumped by the Weyl constants
// between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// 53 random bits for element `gid` in draw `stream`: counter
// (gid_lo, gid_hi, stream, 0), key (seed_lo, seed_hi), first two words as
// w0 * 2^21 + floor(w1 / 2^11).
__device__ __forceinline__ uint64_t bits53(uint64_t seed, uint64_t gid, uint32_t stream) {
  uint32_t c0 = (uint32_t)gid, c1 = (uint32_t)(gid >> 32), c2 = stream, c3 = 0u;
  philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  return ((uint64_t)c0 << 21) | (uint64_t)(c1 >> 11);
}

// the uniform in [0,1) built from those bits
__device__ __forceinline__ double uniform53(uint64_t seed, uint64_t gid, uint32_t stream) {
  return (double)bits53(seed, gid, stream) * 0x1.0p-53;
}

// Draw ids.
constexpr uint32_t kStreamF0 = 0;
constexpr uint32_t kStreamPPS = 1;
constexpr uint32_t kStreamUNI = 2;
constexpr uint32_t kStreamRows = 3;  // row draws of the subsampled global estimators

// Metric ids (same numbering as the C ABI).
constexpr int kEucl = 0, kCos = 1, kManh = 2, kCanb = 3;

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Deterministic block sum of doubles for a 256-thread block (4 waves):
// butterfly inside each wave, then the four wave sums in wave order.
template <int NT>
__device__ __forceinline__ double block_sum_f64(double v, double* sh /* >= NT/64 */) {
  static_assert(NT % kWave == 0, "block size");
  v = wave_sum_f64(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) t += sh[i];
  }
  return t;  // valid in thread 0 only
}

}  // namespace silh
