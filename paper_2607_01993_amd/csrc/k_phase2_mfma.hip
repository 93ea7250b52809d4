// Phase 2 of Algorithm 1 on the matrix cores (gfx950 MFMA), for the
// Euclidean and cosine distances:
//   W_hat_{C_j}(e) = sum_{e' in F_j} w_{e'} d(e, e'),  w = 1/p,
// then a_hat, b_hat, s_hat (Eq. 5) and per-block float64 partials of the sum
// of s_hat (for Eq. 9).
//
// Both distances are evaluated as a squared difference of centred points,
//   |x~ - y~|^2 = |x~|^2 + |y~|^2 - 2 x~.y~ ,   x~ = x - mu_j,  y~ = y - mu_j,
// where mu_j is a centre of cluster j's sample (the mean of its first samples)
// and x, y are the raw rows (Euclidean) or the rows scaled to unit length
// (cosine, where 1 - x^.y^ = |x^ - y^|^2 / 2).  The translation leaves every
// distance unchanged but keeps the operands small near cluster j, so the
// expansion does not cancel for near pairs, in float32 or in bf16.  The dot
// product runs on the MFMA units; the two squared norms ride along as extra
// contraction columns (split into three bf16 pieces in the bf16 path), so the
// accumulator leaves the MFMA holding the squared distance itself:
//   Euclidean:  d = sqrt(|c|)
//   cosine:     d = med3(c, 0, 2) with c = |x~ - y~|^2 / 2 + u_x + u_y
//               (u = 0.5 for a zero vector, else 0, which makes d = 1 there).
//
// Tile mapping (v_mfma_f32_32x32x{2f32,16_bf16}, 32x32x64 f8f6f4): a wave
// owns 32 elements (the B operand columns); each tile is 32 samples of one
// cluster (the A operand rows, cluster blocks padded to 32 with zero-weight
// rows).  Lane l holds element column l%32 of the accumulator and the 16
// sample rows 8g + 4h + r (h = l/32, g, r < 4), so all 16 terms of a tile go
// into the lane's own element: four running float32 sums per lane, each
// term's weight taken from a neighbouring lane by a DPP broadcast inside the
// FMA, and one exchange between the two halves when the cluster ends or
// every kFold tiles, then added in float64.  The pipelined LDS path (long
// rows, bf16 / fp8) keeps the other orientation, elements as the rows (see
// kT in p2_mfma_block).  The contraction order is free,
// so each lane feeds the MFMA a contiguous half of the (augmented) row: half
// h of the row holds logical coordinates [h*HALF, (h+1)*HALF).
#include <utility>

#include "device_common.hpp"
#include "silh_internal.hpp"

namespace silh {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// fp8 (OCP e4m3) path, cosine only: operands are 64 (x~ - y~ components of
// unit vectors lie in [-2, 2], so |64 v| <= 128 < 448) times the centred
// coordinates; the squared norms enter through the accumulator input (with
// elements as rows the sample's through the clamp bounds instead, kF8R).  The
// norms are those of the unrounded float32 coordinates, not of the e4m3
// operands: with c = |x~|^2/2 + |y~|^2/2 - x~_q.y~_q the rounding error of
// each pair is first order in the operand errors (x~.dy + dx.y~), whose sum
// over a cluster's samples averages out, while the exact distance of the
// rounded points |x~_q - y~_q|^2 adds |dx|^2 + |dy|^2 - 2 x~.dx to every pair:
// a bias of one sign that is the same for all samples of the cluster (about
// 0.3 % of W_hat at d = 128, against under 0.02 % this way).
constexpr float kFp8Scale = 64.0f;

// tiles summed in float32 before the float64 add: with samples as the rows
// each of a lane's four sums takes four terms per tile; with elements as the
// rows each of its 16 sums takes one
template <int P, bool T>
constexpr int kFold = T ? (P == 0 ? 8 : 16) : 32;

// Pairs prone to cancellation in the expanded form: with x~, y~ centred on
// mu_j, the squared distance c = |x~|^2 + |y~|^2 - 2 x~.y~ carries
// an absolute error of order eps (|x~|^2 + |y~|^2), so a pair with
// c < tau (|x~|^2 + |y~|^2) loses more than eps/tau of its relative accuracy
// (and the square root halves that).  Such a pair has |y~| < 2|x~| when
// tau < 0.2 (else c >= (|y~| - |x~|)^2 >= |y~|^2/4), hence c < 5 tau |x~|^2:
// every pair with c below 6 tau |x~|^2 (a margin for the error of c itself),
// a threshold of the element alone, is evaluated again as sum (x - y)^2 from
// the float32 rows, which has no cancellation.  tau = 2^-5 for float32 operands (relative error of d below
// 2^-17 for the others) and 2^-8 for bf16 (whose own rounding of x~ and y~
// dominates below that).  The self pair d(e, e) is one of them and comes out
// exactly 0.
template <int P>
constexpr float kRecomputeThr = P == 0 ? 6.0f / 32.0f : 6.0f / 256.0f;

// The test can only flag a pair whose element is near the cluster's sample:
// with R^2 the largest |y~_q|^2 of the sample and |x~_q|^2 >= f R^2, every
// pair has |x~_q - y~_q| >= (1 - 1/sqrt f) |x~_q|, so c >= (1 - 1/sqrt f)^2
// |x~_q|^2 less a float32 rounding error far below that: above the threshold
// 6 tau |x~_q|^2 for f = 2.25 with bf16 (0.111 against 0.023 times
// |x~_q|^2) and f = 4 with float32 (0.25 against 0.19).  A block whose 32
// elements all lie that far out skips the test for the cluster (the same
// results, no test instructions in its tiles).
template <int P>
constexpr float kSkipFactor = P == 0 ? 4.0f : 2.25f;

constexpr int kCenterRows = 256;

__host__ __device__ constexpr int round_up_c(int a, int b) { return (a + b - 1) / b * b; }

// P = 0: float32 operands (32x32x2), P = 1: bf16 (32x32x16), P = 2: fp8 (32x32x64)
template <int P, int DM>
struct MCfg {
  static constexpr int AUG = P == 0 ? 2 : (P == 1 ? 6 : 0);
  static constexpr int KP = P == 0 ? round_up_c(DM + AUG, 4)
                                   : (P == 1 ? round_up_c(DM + AUG, 16) : round_up_c(DM, 64));
  static constexpr int HALF = KP / 2;
  static constexpr int NSTEP = P == 0 ? HALF : (P == 1 ? HALF / 8 : HALF / 32);
  static constexpr int ELEM = P == 0 ? 4 : (P == 1 ? 2 : 1);  // operand bytes
  // long rows go through LDS (the block's waves share each tile)
  static constexpr bool LDS = P == 2 ? HALF > 40 : HALF > 30;
  // bytes per packed row: the operands, and on the LDS path a 16-byte tail
  // with the sample's weight and per-sample value (so that one contiguous
  // copy brings a whole tile into LDS)
  static constexpr int ROWB = KP * ELEM + (LDS ? 16 : 0);
  // bf16: lane half h feeds elements [16 s + 8 h, 16 s + 8 h + 8) of each
  // 16-wide MFMA step s, so both halves hold DM / 2 coordinates and the
  // augmentation sits in step DM / 16 (elements 8 s + e of a lane); the other
  // operand types give each half a contiguous half row [h HALF, (h+1) HALF)
  static constexpr bool IL = P == 1;
  static constexpr int FOFF = IL ? 8 : HALF;   // first element of half h: FOFF h
  static constexpr int FSTEP = IL ? 16 : 8;    // bf16 elements between steps
  // lane elements that can hold coordinates (the rest: augmentation, zeros)
  static constexpr int XR = IL ? 8 * ((DM + 15) / 16) : HALF;
};

int mfma_kp(int prec, int DM) {
  if (prec == 0) return round_up_c(DM + 2, 4);
  if (prec == 1) return round_up_c(DM + 6, 16);
  return round_up_c(DM, 64);
}

bool mfma_lds_path(int prec, int DM) {
  return prec == 2 ? round_up_c(DM, 64) / 2 > 40 : mfma_kp(prec, DM) / 2 > 30;
}

size_t mfma_mu_floats(int prec, int DM, int k) { return (size_t)k * mfma_kp(prec, DM) + k; }

int mfma_row_bytes(int prec, int DM) {
  return mfma_kp(prec, DM) * (prec == 0 ? 4 : (prec == 1 ? 2 : 1)) + (mfma_lds_path(prec, DM) ? 16 : 0);
}

__device__ __forceinline__ int fp8_pack4(float a, float b, float c, float d) {
  int v = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, v, true);
}
__device__ __forceinline__ float q_fp8(float v) {
  return __builtin_amdgcn_cvt_f32_fp8(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false), 0);
}

__device__ __forceinline__ float q_bf16(float v) { return (float)(__bf16)v; }

// split v into three bf16 pieces whose sum is v to about 2^-24 relative
__device__ __forceinline__ void split3(float v, float& h, float& m, float& l) {
  h = q_bf16(v);
  const float r1 = v - h;
  m = q_bf16(r1);
  l = q_bf16(r1 - m);
}

// ----------------------------------------------------------------------------
// centre of each cluster's sample: mean of its first kCenterRows rows of Y32
// (float64 sums; any point of the cluster would do, the mean keeps the
// centred operands smallest); one block per cluster (grid = k)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_center(const float* __restrict__ Y32, int DM, int KP,
                                                const int32_t* __restrict__ sp_off,
                                                const int32_t* __restrict__ cnt,
                                                float* __restrict__ mu) {
  __shared__ double part[256];
  const int j = blockIdx.x;
  // the cluster's squared radius, the packing takes its maximum
  if (threadIdx.x == 0) mu[(size_t)gridDim.x * KP + j] = 0.0f;
  const int m = cnt[j] < kCenterRows ? cnt[j] : kCenterRows;
  const int base = sp_off[j];
  // coordinate chunks of up to 32 columns; 8 row groups per chunk
  const int cc = threadIdx.x & 31, rg = threadIdx.x >> 5;
  for (int c0 = 0; c0 < KP; c0 += 32) {
    const int c = c0 + cc;
    double s = 0.0;
    if (c < DM) {
#pragma unroll 8
      for (int r = rg; r < m; r += 8) s += (double)Y32[(size_t)(base + r) * DM + c];  // loads issued ahead
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (rg == 0 && c < KP) {
      double t = 0.0;
      for (int g = 0; g < 8; ++g) t += part[g * 32 + cc];
      mu[(size_t)j * KP + c] = (m > 0 && c < DM) ? (float)(t / m) : 0.0f;
    }
    __syncthreads();
  }
}

void launch_center(hipStream_t st, const float* Y32, int DM, int KP, const int32_t* sp_off,
                   const int32_t* cnt, int k, float* mu) {
  hipLaunchKernelGGL(k_center, dim3(k), dim3(256), 0, st, Y32, DM, KP, sp_off, cnt, mu);
}

// ----------------------------------------------------------------------------
// Sample operand rows: [ -2 alpha y~_q (DM) | augmentation | 0 ... ] with
// alpha = 1 (Euclidean) or 1/2 (cosine); y~_q = y~ rounded to the input
// precision; the augmentation carries alpha |y~_q|^2 + u_y and the ones that
// take in the element's norm term.  Padding rows keep only those ones, so an
// element meets them at c = its own norm term (never below its recompute
// threshold) with weight 0.  bnorm and, on the LDS path, each row's 16-byte
// tail carry the per-sample value (fp8: the norm term; cosine: the element
// id; Euclidean: the sample's recompute threshold, which the element-row
// layout tests against); the tail also holds the weight w and two zero
// words.
// ----------------------------------------------------------------------------
template <int M, int P, int DM>
__global__ __launch_bounds__(256) void k_pack_mfma(const float* __restrict__ Y32,
                                                   const float* __restrict__ aux,
                                                   const float* __restrict__ w,
                                                   const int32_t* __restrict__ gid_pk,
                                                   const int32_t* __restrict__ sp_off,
                                                   const int32_t* __restrict__ cnt, int k,
                                                   float* __restrict__ mu, int S_pad,
                                                   void* __restrict__ Ym, float* __restrict__ bnorm) {
  using C = MCfg<P, DM>;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  // sp_off[k]: packed rows in use (the Euclidean kernels keep every lane to
  // the end, for the wave-wide radius below)
  const bool valid = s < S_pad && s < sp_off[k];
  if (M != kEucl && !valid) return;
  // cluster of padded row s (binary search over sp_off)
  int lo = 0, hi = k;
  while (valid && hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sp_off[mid] <= s) lo = mid; else hi = mid;
  }
  const int j = lo;
  const bool real = valid && s - sp_off[j] < cnt[j];
  float ny_r = 0.0f;  // Euclidean: the row's squared norm, 0 for padding
  const float alpha = M == kCos ? 0.5f : 1.0f;
  float row[C::KP];
#pragma unroll
  for (int c = 0; c < C::KP; ++c) row[c] = 0.f;
  if (P == 2) {
    // fp8: B = e4m3(-64 y~), the norm term alpha |y~_q|^2 + u_y goes to bnorm
    float bn = 0.0f;
    if (real) {
      const float* y = Y32 + (size_t)s * DM;
      const float* m = mu + (size_t)j * C::KP;
      float ny = 0.f;
#pragma unroll
      for (int c = 0; c < DM; ++c) {
        const float v = y[c] - m[c];
        const float q = q_fp8(kFp8Scale * v);
        ny = fmaf(v, v, ny);  // the norm of the unrounded coordinates
        row[c] = -q;
      }
      bn = fmaf(alpha, ny, M == kCos ? aux[s] : 0.0f);
    }
    bnorm[s] = bn;
    int* out = (int*)((unsigned char*)Ym + (size_t)s * C::ROWB);
#pragma unroll
    for (int c = 0; c < C::KP; c += 4) out[c / 4] = fp8_pack4(row[c], row[c + 1], row[c + 2], row[c + 3]);
    if constexpr (C::LDS)
      *(u32x4*)(out + C::KP / 4) = u32x4{__float_as_uint(w[s]), __float_as_uint(bn), 0u, 0u};
    return;
  }
  // Euclidean, element-row layout: the sample's recompute threshold
  float thr = 0.0f;
  if (real) {
    const float* y = Y32 + (size_t)s * DM;
    const float* m = mu + (size_t)j * C::KP;
    float ny = 0.f;
#pragma unroll
    for (int c = 0; c < DM; ++c) {
      float v = y[c] - m[c];
      if (P == 1) v = q_bf16(v);
      ny = fmaf(v, v, ny);
      row[c] = -2.0f * alpha * v;
    }
    const float bn = fmaf(alpha, ny, M == kCos ? aux[s] : 0.0f);
    thr = M == kEucl ? kRecomputeThr<P> * ny : 0.0f;
    ny_r = ny;
    if (P == 0) {
      row[DM + 1] = bn;
    } else {
      split3(bn, row[DM + 3], row[DM + 4], row[DM + 5]);
    }
  }
  if (P == 0) {
    row[DM] = 1.0f;
  } else {
    row[DM] = row[DM + 1] = row[DM + 2] = 1.0f;
  }
  if (valid) {
    bnorm[s] = thr;
    unsigned char* rowp = (unsigned char*)Ym + (size_t)s * C::ROWB;
    if constexpr (P == 0) {
      float* out = (float*)rowp;
#pragma unroll
      for (int c = 0; c < C::KP; ++c) out[c] = row[c];
    } else {
      __bf16* out = (__bf16*)rowp;
#pragma unroll
      for (int c = 0; c < C::KP; ++c) out[c] = (__bf16)row[c];
    }
    if constexpr (C::LDS) {
      const unsigned g = M == kCos ? (unsigned)gid_pk[s] : __float_as_uint(thr);
      *(u32x4*)(rowp + C::KP * C::ELEM) = u32x4{__float_as_uint(w[s]), g, 0u, 0u};
    }
  }
  if constexpr (M == kEucl) {
    // the cluster's squared radius, the largest ny (>= 0, so its bits order
    // like the values): one atomic per wave where all its rows belong to one
    // cluster (rows of a cluster are contiguous), else one per row
    int* rad = (int*)(mu + (size_t)k * C::KP);
    const int jv = valid ? j : -1;
    const int j0 = __builtin_amdgcn_readfirstlane(jv);
    if (__builtin_amdgcn_ballot_w64(jv != j0) == 0 && j0 >= 0) {
      int m = __float_as_int(ny_r);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
      if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(rad + j0, m);
    } else if (real) {
      atomicMax(rad + j, __float_as_int(ny_r));
    }
  }
}

// ----------------------------------------------------------------------------
// The weighted sums of a tile: accumulator row r of lane l is sample row
// 8 (r >> 2) + 4 h + (r & 3) of the tile (h = l >> 5).  A lane holds two
// weights, wv[0] = w[(l & 11) + 4h] and wv[1] = w[16 + (l & 11) + 4h], so
// within each 16-lane row, lane (r & 3) + 8 ((r >> 2) & 1) of wv[r >> 3]
// holds the weight of row r for every lane of that 16-lane row: a DPP
// broadcast (row_newbcast) inside the FMA reads it.  The compiler does not
// fuse a DPP move into v_fmac_f32, so the FMAs are written as asm; a DPP
// source written by the vector ALU needs two wait states, a square root's
// result one before a non-transcendental use.
// ----------------------------------------------------------------------------
__host__ __device__ constexpr int wsrc_lane(int r) { return (r & 3) + 8 * ((r >> 2) & 1); }

// f(std::integral_constant<int, i>) for i = 0 .. N-1 (indices the DPP
// controls and asm operands need as constants)
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// lane l's index into its tile's weights (and other per-row values): the
// two loads take rows wrow(l) and 16 + wrow(l)
__device__ __forceinline__ int wrow(int lane) { return (lane & 11) + 4 * (lane >> 5); }

// acc[r & 3] += w(row r) * dv[r] for the 16 rows, after two wait states
__device__ __forceinline__ void wsum16(float (&acc)[4], float w0, float w1, const float (&dv)[16]) {
#define SILH_FMAC(A, W, V, Q) "v_fmac_f32_dpp %" #A ", %" #W ", %" #V " row_newbcast:" #Q " row_mask:0xf bank_mask:0xf\n\t"
  asm("s_nop 1\n\t"
      SILH_FMAC(0, 4, 6, 0) SILH_FMAC(1, 4, 7, 1) SILH_FMAC(2, 4, 8, 2) SILH_FMAC(3, 4, 9, 3)
      SILH_FMAC(0, 4, 10, 8) SILH_FMAC(1, 4, 11, 9) SILH_FMAC(2, 4, 12, 10) SILH_FMAC(3, 4, 13, 11)
      SILH_FMAC(0, 5, 14, 0) SILH_FMAC(1, 5, 15, 1) SILH_FMAC(2, 5, 16, 2) SILH_FMAC(3, 5, 17, 3)
      SILH_FMAC(0, 5, 18, 8) SILH_FMAC(1, 5, 19, 9) SILH_FMAC(2, 5, 20, 10) SILH_FMAC(3, 5, 21, 11)
      : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])
      : "v"(w0), "v"(w1), "v"(dv[0]), "v"(dv[1]), "v"(dv[2]), "v"(dv[3]), "v"(dv[4]), "v"(dv[5]), "v"(dv[6]),
        "v"(dv[7]), "v"(dv[8]), "v"(dv[9]), "v"(dv[10]), "v"(dv[11]), "v"(dv[12]), "v"(dv[13]), "v"(dv[14]),
        "v"(dv[15]));
#undef SILH_FMAC
}

// per-row value v of row r (the same broadcast, for the compiler's own
// DPP-combined adds)
template <int R>
__device__ __forceinline__ float row_val(float v0, float v1) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(R < 8 ? v0 : v1), 0x150 + wsrc_lane(R), 0xF, 0xF, true));
}

// the sum of a lane's four running sums and its partner's in the other half
// (lanes l and l ^ 32 hold the same element)
__device__ __forceinline__ float lane_sum(const float (&acc)[4]) {
  const float v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// ----------------------------------------------------------------------------
// Element-row layout: 16 per-lane row sums, each over the lane's column: five exchange steps, each
// pairing lanes that differ in one bit of the column index and halving the
// number of live values (the partner receives the half it keeps).  Partners:
// lane ^ 16 by a row swap between two registers, then within 16-lane rows by
// DPP (rotate by 8, mirror inside 8, quad permutations), which pair lanes
// that differ in bit 3, bit 2, bit 1 and bit 0 respectively.  Afterwards lane
// l holds the sum over all 32 columns for row r = (l >> 1) & 15 of its half
// (lanes l and l^1 agree).
// ----------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppRor8 = 0x128;        // row_ror:8      -> lane ^ 8 inside 16
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror: 7 - (lane & 7)
constexpr int kDppQuad2301 = 0x4E;     // quad_perm [2,3,0,1] -> lane ^ 2
constexpr int kDppQuad1032 = 0xB1;     // quad_perm [1,0,3,2] -> lane ^ 1

__device__ __forceinline__ float transpose_reduce16(float (&v)[16], int lane) {
  {
    // lane ^ 16: v_permlane16_swap exchanges the odd 16-lane rows of v[i]
    // with the even rows of v[i + 8], leaving every lane both copies of the
    // value it keeps (v[i] below lane 16 of each half, v[i + 8] above)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 8]), false, false);
      v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
  }
  {
    const bool up = lane & 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float send = up ? v[i] : v[i + 4];
      const float keep = up ? v[i + 4] : v[i];
      v[i] = keep + dpp_f<kDppRor8>(send);
    }
  }
  {
    const bool up = lane & 4;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float send = up ? v[i] : v[i + 2];
      const float keep = up ? v[i + 2] : v[i];
      v[i] = keep + dpp_f<kDppHalfMirror>(send);
    }
  }
  {
    const bool up = lane & 2;
    const float send = up ? v[0] : v[1];
    const float keep = up ? v[1] : v[0];
    v[0] = keep + dpp_f<kDppQuad2301>(send);
  }
  return v[0] + dpp_f<kDppQuad1032>(v[0]);
}

template <int P, int DM>
struct AFrag;
template <int DM>
struct AFrag<0, DM> {
  float v[MCfg<0, DM>::NSTEP];
};
template <int DM>
struct AFrag<1, DM> {
  bf16x8 v[MCfg<1, DM>::NSTEP];
};
template <int DM>
struct AFrag<2, DM> {
  i32x8 v[MCfg<2, DM>::NSTEP];
};

template <int P, int DM>
struct BFrag;
template <int DM>
struct BFrag<0, DM> {
  float2 v[MCfg<0, DM>::NSTEP / 2];
};
template <int DM>
struct BFrag<1, DM> {
  bf16x8 v[MCfg<1, DM>::NSTEP];
};
template <int DM>
struct BFrag<2, DM> {
  i32x8 v[MCfg<2, DM>::NSTEP];
};

// A raw buffer resource over `bytes` bytes at p (gfx9 descriptor: stride 0,
// offsets are byte offsets, reads past `bytes` return 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_at(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}

// 16 bytes per lane at byte voff + soff of the buffer straight into LDS:
// lane l's bytes land at LDS byte address la + 16 l (la, the descriptor and
// soff wave-uniform).  Written as one asm statement (M0, the LDS address, saved
// and restored around it) because the compiler, unable to tell the slot being
// filled from the slots being read, would otherwise wait for every such load
// before the next LDS read; the kernel orders them itself (a vmcnt wait and a
// barrier before a slot is read, no load into a slot read in the same stage).
// It has no register results, so nothing the compiler allocates is written
// late.
__device__ __forceinline__ void lds_load16(u32x4 rsrc, unsigned la, unsigned voff, unsigned soff) {
  // all wave-uniform; made explicit for the scalar operands of the asm
  la = (unsigned)__builtin_amdgcn_readfirstlane((int)la);
  rsrc = u32x4{(unsigned)__builtin_amdgcn_readfirstlane((int)rsrc.x), (unsigned)__builtin_amdgcn_readfirstlane((int)rsrc.y),
               (unsigned)__builtin_amdgcn_readfirstlane((int)rsrc.z), (unsigned)__builtin_amdgcn_readfirstlane((int)rsrc.w)};
  unsigned saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "buffer_load_dwordx4 %2, %3, 0 offen lds\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "s"(la), "v"(voff + soff), "s"(rsrc)
      : "memory");
}

// the buffer descriptor of lds_load16: `bytes` bytes from p (stride 0; reads
// past the end give 0)
__device__ __forceinline__ u32x4 rsrc_words(const void* p, unsigned bytes) {
  const unsigned long long a = (unsigned long long)(uintptr_t)p;
  return u32x4{(unsigned)a, (unsigned)(a >> 32) & 0xffffu, bytes, 0x00020000u};
}

// V consecutive row elements from c on, zero from lim on.  With vec (rows
// V-float aligned and c a multiple of V) the chunk is one vector load and lies
// wholly inside or outside [0, lim); otherwise element by element.  Loads go
// to a clamped address and the value is selected, so no load is predicated.
template <int V>
__device__ __forceinline__ void load_chunk(const float* __restrict__ xp, int c, int lim, bool vec,
                                           float (&out)[V]) {
  typedef float fvec __attribute__((ext_vector_type(V)));
  if (vec) {
    const bool in = c < lim;
    const fvec t = *(const fvec*)(xp + (in ? c : 0));
#pragma unroll
    for (int e = 0; e < V; ++e) out[e] = in ? t[e] : 0.0f;
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const bool in = c + e < lim;
      const float t = xp[in ? c + e : 0];
      out[e] = in ? t : 0.0f;
    }
  }
}

// one tile's sample operand (this lane's half row), the weights of rows
// wrow(lane) and 16 + wrow(lane), and per-row values: fp8 the norm terms of
// those two rows (bnorm), cosine the element id of row lane % 32 (gid_pk)
template <int M, int P, int DM>
__device__ __forceinline__ void load_tile(const void* __restrict__ Ym, const float* __restrict__ w,
                                          const int32_t* __restrict__ gid_pk,
                                          const float* __restrict__ bnorm, int row0, uint32_t lane_off,
                                          uint32_t col, uint32_t wr, BFrag<P, DM>& b, float (&wv)[2],
                                          int (&gv)[2]) {
  using C = MCfg<P, DM>;
  // row0 is wave-uniform: each 32-row tile gets buffer descriptors built on
  // the scalar unit, and a lane reads at a fixed byte offset (no per-tile
  // vector address arithmetic)
  const auto rb = rsrc_at((const unsigned char*)Ym + (size_t)row0 * (size_t)(C::KP * C::ELEM),
                          32 * C::KP * C::ELEM);
  const auto rw = rsrc_at(w + row0, 32 * 4);
  const auto rg = rsrc_at(P != 2 ? (const void*)(gid_pk + row0) : (const void*)(bnorm + row0), 32 * 4);
  if constexpr (P == 2) {
#pragma unroll
    for (int s = 0; s < C::NSTEP; ++s) {
      const u32x4 lo = __builtin_amdgcn_raw_buffer_load_b128(rb, lane_off + 32u * s, 0, 0);
      const u32x4 hi = __builtin_amdgcn_raw_buffer_load_b128(rb, lane_off + 32u * s + 16u, 0, 0);
      b.v[s] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
  } else if constexpr (P == 0) {
#pragma unroll
    for (int s2 = 0; s2 < C::NSTEP / 2; ++s2)
      b.v[s2] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rb, lane_off + 8u * s2, 0, 0));
  } else {
#pragma unroll
    for (int s = 0; s < C::NSTEP; ++s)
      b.v[s] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rb, lane_off + 2u * C::FSTEP * s, 0, 0));
  }
  wv[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rw, 4u * wr, 0, 0));
  wv[1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rw, 4u * (wr + 16u), 0, 0));
  if constexpr (P == 2) {
    gv[0] = (int)__builtin_amdgcn_raw_buffer_load_b32(rg, 4u * wr, 0, 0);
    gv[1] = (int)__builtin_amdgcn_raw_buffer_load_b32(rg, 4u * (wr + 16u), 0, 0);
  } else if constexpr (M == kCos) {
    gv[0] = (int)__builtin_amdgcn_raw_buffer_load_b32(rg, 4u * col, 0, 0);
  }
}

// waves per SIMD the one-block shapes from d = 32 on keep (their occupancy
// without the recompute path, which must not lower it)
// (two tiles per LDS stage hold enough LDS to set the occupancy themselves)
template <int M, int P, int DM, int PB, int TBX>
constexpr int kMinWaves = (P == 2 && DM == 128) ? 2
                          : (M != kEucl || P == 2 || PB == 2 || DM < 32 || (TBX == 2 && MCfg<P, DM>::LDS)) ? 1
                          : DM == 32 ? (P == 1 ? 4 : 1) : DM == 64 ? 3 : DM == 128 ? 2 : 1;

// One block of the Phase-2 launch: 4 waves x PB x 32 elements, from element
// blk * 128 * PB on.  The kernels below run it for blockIdx.x (one request)
// or for the (request, block) work items of a multi-request launch.

// tiles per LDS stage of the one-block shape by default: two where measured
// faster (bf16 from d = 64 on, fp8), else one; the autotuner may try the other
template <int P, int DM>
constexpr int kTBDefault = (P == 2 || (P == 1 && DM >= 64)) ? 2 : 1;

template <int M, int P, int DM, int PB, int TBX>
__device__ __forceinline__ void p2_mfma_block(
    const int blk, const float* __restrict__ X, int n, int d, const int32_t* __restrict__ labels,
    const void* __restrict__ Ym, const float* __restrict__ w, const int32_t* __restrict__ gid_pk,
    const int32_t* __restrict__ sp_off, const int32_t* __restrict__ cnt,
    const int32_t* __restrict__ csize, int k, const float* __restrict__ mu,
    float* __restrict__ a_out, float* __restrict__ b_out, float* __restrict__ s_out,
    float* __restrict__ What, double* __restrict__ bpart, const float* __restrict__ bnorm,
    const float* __restrict__ Y32, int DMY, const float* __restrict__ aux, const float* __restrict__ rn) {
  using C = MCfg<P, DM>;
  // contiguous halves: the augmentation columns always fall in the upper half
  // of the row
  constexpr int AUG0 = DM - C::HALF;
  static_assert(C::IL || C::AUG == 0 || (AUG0 >= 0 && AUG0 + C::AUG <= C::HALF), "augmentation placement");
  constexpr float S2 = kFp8Scale * kFp8Scale;
  __shared__ double sh32[4 * PB];  // 32-element partials of the block, in element order
  // Long rows (bf16 / float32 with d >= 64, fp8 with d >= 128): the block's
  // four waves sweep the same tiles, so each is loaded once per block into
  // LDS and every wave reads its sample fragment from there.  Tiles go in stages
  // of kTB; a stage's slot holds its tiles (32 packed rows each, whose
  // 16-byte tails with the weight and per-sample value also shift the rows
  // so that the lanes' 16-byte reads fall in different banks; the tile
  // padded to whole kilobytes) and the centre mu_j of the stage's cluster.  Slots are filled by direct
  // global-to-LDS loads (16 bytes per lane, placed at the slot offset plus
  // 16 x lane) two stages ahead in a ring of three, so a stage's loads have
  // two stages of compute to arrive; one wait and one barrier per stage.
  constexpr int kRowB = C::KP * C::ELEM;
  constexpr int kLRow = C::ROWB;                    // operands + tail (weight, value)
  constexpr int kTileCh = round_up_c(32 * kLRow / 16, 64);
  constexpr int kTileI = kTileCh / 64;              // loads (one per wave) per tile
  constexpr bool kLds = C::LDS;
  // tiles per LDS stage (one barrier per stage; kTBDefault or the other)
  constexpr int kTB = (kLds && PB == 1) ? TBX : 1;
  constexpr int kMuOff = kTB * kTileCh * 16;
  constexpr int kMuI = (C::KP * 4 + 1023) / 1024;   // loads for mu (its region: whole kilobytes)
  constexpr int kSlotB = kMuOff + kMuI * 1024;
  static_assert(!kLds || (kTileI >= 4 && kMuI <= 4), "every wave loads part of each tile; mu takes at most four loads");
  constexpr int kDw = (kTileI + 3) / 4;             // loads per wave per tile
  constexpr int kNIw = kTB * kDw;                   // per wave per stage, without mu
  // LDS path with bf16 / fp8 operands: one tile's epilogue runs beside the
  // next tile's MFMAs (float32 operands are bound by the MFMA rate)
  constexpr bool kPipe = kLds && P != 0 && DM >= 128;
  // Accumulator layout.  kT (every path but the pipelined one): samples are
  // the MFMA rows, a lane's 16 accumulator rows all belong to its element
  // column, weighted through DPP broadcasts, combined across the two halves.
  // Pipelined path: elements are the rows and a lane holds one sample column
  // (its weight a single register), so the tile's sums need no broadcast in
  // the steps woven around the MFMAs, and are combined across the 32
  // columns by a transpose-reduction when a cluster ends (over many tiles
  // at these widths).
  constexpr bool kT = !kPipe;
  __shared__ __attribute__((aligned(16))) unsigned char ldsS[kLds ? 3 * kSlotB : 16];
  // the LDS byte address of ldsS (the direct loads take LDS addresses)
  const unsigned lds_base = (unsigned)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)ldsS;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int col = lane & 31;
  // PB blocks of 32 elements per wave share every sample tile
  const int P0 = __builtin_amdgcn_readfirstlane((blk * 4 + (threadIdx.x >> 6)) * 32 * PB);
  const float alpha = M == kCos ? 0.5f : 1.0f;
  const uint32_t lane_off = (uint32_t)((col * C::KP + h * C::FOFF) * C::ELEM);  // bytes
  // kT: this lane's rows of a tile's per-row values (weights)
  const int wr = wrow(lane);
  // element-row layout: the element whose sums this lane ends up holding
  // (twice: lanes l, l^1)
  const int rr = (lane >> 1) & 15;
  const int prow = 8 * (rr >> 2) + 4 * h + (rr & 3);

  // this lane's half of its A rows (raw or unit-scaled), zero outside [0, d),
  // resident for the whole cluster loop (at d = 256 partly in AGPRs, which
  // the one wave per SIMD that the tile registers allow leaves free);
  // re-reading it per cluster would stream X k times through L2.
  // Rows and centres are read in V-float chunks (h * HALF is a multiple of V).
  constexpr int V = C::HALF % 4 == 0 ? 4 : 2;
  typedef float fvec __attribute__((ext_vector_type(V)));
  const bool vec = d % V == 0 && ((uintptr_t)X & (4 * V - 1)) == 0;
  float xr[PB][C::HALF];
  // d = 256: the rows wait in the AGPRs, so the vector registers serve the
  // tile pipeline (deeper B-operand reads ahead of the MFMAs)
  constexpr bool kXA = kLds && C::HALF >= 128;
  auto xget = [&](int b, int i) {
    if constexpr (kXA) {
      float r;
      asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(r) : "a"(xr[b][i]));
      return r;
    } else {
      return xr[b][i];
    }
  };
  float ux[PB];
  int pout[PB], own[PB];
  // b_hat as the fraction bnum / bden of the smallest W_hat_j / |C_j| so far
  // (candidates compared by cross-multiplication, one division at the end;
  // bden = 0: none yet)
  double w_own[PB], bnum[PB], bden[PB];
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    const int pb = P0 + 32 * b + col;
    const int pa = pb < n ? pb : n - 1;
    const float* xp = X + (size_t)pa * d;
#pragma unroll
    for (int i0 = 0; i0 < C::XR; i0 += V) {
      float xc[V];
      // lane element i0 is coordinate 16 (i0 / 8) + 8 h + i0 % 8 (bf16)
      load_chunk<V>(xp, C::IL ? 16 * (i0 / 8) + 8 * h + i0 % 8 : h * C::HALF + i0, d, vec, xc);
#pragma unroll
      for (int e = 0; e < V; ++e) xr[b][i0 + e] = xc[e];
    }
    ux[b] = 0.f;
    if (M == kCos) {
      // unit vector: the row times its float32 reciprocal norm, the product
      // the packing forms for the sample rows (u = 0.5 for a zero row)
      const float rx = rn[pa];
      ux[b] = rx > 0.f ? 0.f : 0.5f;
#pragma unroll
      for (int i = 0; i < C::XR; ++i) xr[b][i] *= rx;
    }
    if constexpr (kXA) {
      // kept in accumulation registers (AGPRs) until the A operands of each
      // cluster read them back
#pragma unroll
      for (int i = 0; i < C::XR; ++i) asm volatile("v_accvgpr_write_b32 %0, %1" : "=a"(xr[b][i]) : "v"(xr[b][i]));
    }
    pout[b] = P0 + 32 * b + (kT ? col : prow);
    own[b] = labels[pout[b] < n ? pout[b] : n - 1];
    own[b] = (unsigned)own[b] < (unsigned)k ? own[b] : 0;  // labels are checked before; stay in bounds
    w_own[b] = 0.0;
    bnum[b] = 1.0;
    bden[b] = 0.0;
  }

  AFrag<P, DM> A[PB];
  // fp8: 64^2 (alpha |x~_q|^2 + u_x) of this lane's element (kT), of its
  // 16 accumulator rows (element-row layout)
  float nxc[PB][kT ? 1 : 16];
  // fp8 with element rows (the pipelined path): the element terms as the
  // MFMA's accumulator input (the same every tile of a cluster); the sample
  // term 64^2 |y~|^2 / 2 of column col shifts the clamp instead,
  //   med3(c + v, 0, 2 S2) = med3(c, -v, 2 S2 - v) + v,
  // and its weighted sum, the same for every element, goes into tcol (per
  // lane column, added to every element's sum at the fold)
  constexpr bool kF8R = P == 2 && !kT;
  f32x16 nxv[PB];
  float tcol[PB];
  int thrx[PB];   // Euclidean: the element's recompute threshold (float bits, >= 0)
  int chk[PB];    // Euclidean: some element of the block may meet the threshold (wave-uniform, 0 / 1)
  // The packed cluster blocks are contiguous, so the tile after a cluster's
  // last one is the first tile of the next cluster with samples: it is
  // prefetched there, and a cluster normally starts with its first tile
  // already loaded while its A operands are built.  Past the sample's end the
  // last tile is re-read.  `pre` is the first row of the tile held in b0 (the
  // register path) or in LDS buffer `cb` (the LDS path).
  const int last_row = sp_off[k] - 32;
  auto clamp_row = [&](int row) { return row <= last_row ? row : last_row; };
  int pre = -1;
  BFrag<P, DM> b0, b1;
  float w0[2] = {0.f, 0.f}, w1[2] = {0.f, 0.f};
  int g0[2] = {-1, -1}, g1[2] = {-1, -1};

  // ---- LDS path: the stage ring.  (cj, cm) is the next stage to load
  // (cluster, stage within it; cj = k past the end, where the last tile is
  // loaded again and never read); rs the slot of the next stage to compute.
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int cj = 0, cm = 0, rs = 0;
  int cnt_c = 0, row_c = 0;  // samples and first packed row of cluster cj
  auto seek = [&](int j0) {  // cj: the first cluster from j0 on with samples
    while (j0 < k && cnt[j0] <= 0) ++j0;
    cj = j0;
    if (j0 < k) {
      cnt_c = cnt[j0];
      row_c = sp_off[j0];
    }
  };
  auto advance = [&]() {
    if (cj >= k) return;
    if (++cm * kTB * 32 >= cnt_c) {
      cm = 0;
      seek(cj + 1);
    }
  };
  // Wave w loads kilobytes w, w + 4, ... of each tile (kDw loads; where the
  // tile ends first the last one repeats its final kilobyte, the same bytes
  // to the same place, so every wave issues the same count) and kilobyte w
  // of mu.  stage_begin fixes the stage to load next and loads its mu;
  // tile_load(tt, mi) issues load mi of its tile tt.
  const unsigned voff0 = 16u * (unsigned)lane;
  int st_row0 = 0;
  unsigned st_sb = lds_base;
  auto stage_begin = [&](int slot) {
    const bool past = cj >= k;
    st_row0 = past ? last_row : row_c + cm * kTB * 32;
    st_sb = lds_base + (unsigned)(slot * kSlotB);
    if (cm == 0 && !past && wave < kMuI) {
      // mu of the stage's cluster, with its first stage (reads past KP
      // floats give 0 and stay inside the region)
      const u32x4 rm = rsrc_words(mu + (size_t)cj * C::KP, C::KP * 4);
      lds_load16(rm, st_sb + (unsigned)(kMuOff + 1024 * wave), voff0, 1024u * (unsigned)wave);
    }
  };
  auto tile_load = [&](int tt, int mi) {
    const int u0 = wave + 4 * mi;
    const int u = u0 < kTileI ? u0 : kTileI - 1;  // wave-uniform
    const int r0 = clamp_row(st_row0 + 32 * tt);
    const u32x4 rb = rsrc_words((const unsigned char*)Ym + (size_t)r0 * (size_t)kLRow, 32 * kLRow);
    // zeros past the tile's 32 rows
    lds_load16(rb, st_sb + (unsigned)(tt * kTileCh * 16 + 1024 * u), voff0, 1024u * (unsigned)u);
  };
  auto issue = [&](int slot) {
    stage_begin(slot);
#pragma unroll
    for (int tt = 0; tt < kTB; ++tt)
#pragma unroll
      for (int mi = 0; mi < kDw; ++mi) tile_load(tt, mi);
  };
  if constexpr (kLds) {
    if (last_row >= 0) {  // block-uniform; an empty sample loads nothing
      seek(0);
      issue(0);
      advance();
      issue(1);
      advance();
    }
  }

  for (int j = 0; j < k; ++j) {
    // ---- A operands for cluster j: x~ = x - mu_j (mu zero-padded to KP),
    // rounded to the input precision, plus the augmentation; m is this
    // lane's half of mu_j (in memory, or in the LDS slot of the cluster's
    // first stage)
    // Euclidean: the squared radius of the cluster's packed sample
    const float R2 = (M == kEucl && P != 2) ? mu[(size_t)k * C::KP + j] : 0.0f;
    auto buildA = [&](const float* m) {
    float mv[C::HALF];
#pragma unroll
    for (int i0 = 0; i0 < C::XR; i0 += V) {
      const fvec t = *(const fvec*)(m + (C::IL ? 16 * (i0 / 8) + i0 % 8 : i0));
#pragma unroll
      for (int e = 0; e < V; ++e) mv[i0 + e] = t[e];
    }
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      float xq[C::HALF];
      float part = 0.f;
      if constexpr (P == 2) {
#pragma unroll
        for (int i = 0; i < C::HALF; ++i) {
          const float v = xget(b, i) - mv[i];
          xq[i] = q_fp8(kFp8Scale * v);
          part = fmaf(v, v, part);  // the norm of the unrounded coordinates
        }
        const float rowv = S2 * fmaf(alpha, part + __shfl_xor(part, 32, kWave), ux[b]);
        if constexpr (kT) {
          nxc[b][0] = rowv;  // the lane's element is its accumulator column
        } else {
          // the C rows of this lane are elements 8(r/4) + 4h + r%4 of the block
#pragma unroll
          for (int r = 0; r < 16; ++r) nxv[b][r] = __shfl(rowv, 8 * (r >> 2) + 4 * h + (r & 3), kWave);
        }
#pragma unroll
        for (int s = 0; s < C::NSTEP; ++s)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            A[b].v[s][e] = fp8_pack4(xq[32 * s + 4 * e], xq[32 * s + 4 * e + 1], xq[32 * s + 4 * e + 2],
                                     xq[32 * s + 4 * e + 3]);
        continue;
      }
      if constexpr (P == 1) {
        // bf16: each pair of centred coordinates is rounded into one packed
        // register (the fragment's layout) and its squares are added to the
        // norm by one bf16 dot product (the products are exact in float32).
        // Only the lane elements that can hold coordinates (C::XR) are
        // formed; the step at DM / 16 carries the augmentation in half
        // (DM / 8) & 1 (DM = 8 shares step 0: coordinates in half 0)
        constexpr int kSA = DM / 16, kHA = (DM / 8) & 1;
        bf16x2 pk[C::HALF / 2];
#pragma unroll
        for (int i2 = 0; i2 < C::HALF / 2; ++i2) {
          if (2 * i2 < C::XR) {
            const f32x2 v = {xget(b, 2 * i2) - mv[2 * i2], xget(b, 2 * i2 + 1) - mv[2 * i2 + 1]};
            pk[i2] = __builtin_convertvector(v, bf16x2);
            part = __builtin_amdgcn_fdot2_f32_bf16(pk[i2], pk[i2], part, false);
          } else {
            pk[i2] = bf16x2{};
          }
        }
        const float an = fmaf(alpha, part + __shfl_xor(part, 32, kWave), ux[b]);
        thrx[b] = __float_as_int(kRecomputeThr<P> * an);
        chk[b] = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_ballot_w64(an < kSkipFactor<P> * R2) != 0 ? 1 : 0);
        float aug[6];
        split3(an, aug[0], aug[1], aug[2]);
        aug[3] = aug[4] = aug[5] = 1.0f;
        // the augmentation columns hold zeros in the other half's pairs
#pragma unroll
        for (int q = 0; q < C::AUG; q += 2)
          pk[(8 * kSA + q) / 2] =
              h == kHA ? __builtin_convertvector((f32x2{aug[q], aug[q + 1]}), bf16x2) : pk[(8 * kSA + q) / 2];
#pragma unroll
        for (int s = 0; s < C::NSTEP; ++s)
#pragma unroll
          for (int e = 0; e < 8; ++e) A[b].v[s][e] = pk[4 * s + e / 2][e % 2];
        continue;
      }
#pragma unroll
      for (int i = 0; i < C::HALF; ++i) {
        const float v = xget(b, i) - mv[i];
        xq[i] = v;
        part = fmaf(v, v, part);
      }
      // float32: the norm and a 1 ride along as two extra columns
      const float nx = part + __shfl_xor(part, 32, kWave);
      const float an = fmaf(alpha, nx, ux[b]);
      thrx[b] = __float_as_int(kRecomputeThr<P> * an);
      chk[b] = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_ballot_w64(an < kSkipFactor<P> * R2) != 0 ? 1 : 0);
      xq[AUG0] = h ? an : xq[AUG0];
      xq[AUG0 + 1] = h ? 1.0f : xq[AUG0 + 1];
#pragma unroll
      for (int s = 0; s < C::NSTEP; ++s) A[b].v[s] = xq[s];
    }
    };
    if constexpr (!kLds) buildA(mu + (size_t)j * C::KP + h * C::FOFF);

    // ---- sweep the cluster's sample tiles (sample operand double-buffered:
    // the next tile's loads are issued before this tile's MFMAs)
    const int base = sp_off[j];
    const int ntile = (cnt[j] + 31) >> 5;
    double wsum[PB];
    constexpr int kNA = kT ? 4 : 16;  // running float32 sums per lane and block
    float acc[PB][kNA];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      wsum[b] = 0.0;
      tcol[b] = 0.f;
#pragma unroll
      for (int r = 0; r < kNA; ++r) acc[b][r] = 0.f;
    }
    int g = 0;
    // One tile, in four parts: chain (the MFMAs; getB(q) gives step q of
    // this lane's sample fragment, a float2 of two steps for float32, from
    // registers or read from LDS just in time), fixup (pairs prone to
    // cancellation, the cosine self pair), wsum_add (distances and the
    // weighted sums) and fold (the float64 add every kFold tiles and at the
    // cluster's end).  The LDS path overlaps the wsum_add of one tile with
    // the chain of the next; the arithmetic per pair is the same.  wv, gv:
    // the tile's weights and per-row values as load_tile gives them.
    auto dist = [&](float c) {
      if constexpr (M == kEucl)
        return __builtin_amdgcn_sqrtf(fabsf(c));
      else
        return __builtin_amdgcn_fmed3f(c, 0.0f, P == 2 ? 2.0f * S2 : 2.0f);
    };
    // fp8: the accumulator starts at 64^2 (element term + sample term), the
    // MFMA adds -64^2 x~_q . y~_q (unscaled f8f6f4 form, e4m3 operands)
    auto fp8_init = [&](f32x16& c, int b, const int (&gv)[2]) {
      if constexpr (kT) {
        const float v0 = S2 * __int_as_float(gv[0]), v1 = S2 * __int_as_float(gv[1]);
        static_for<16>([&](auto RC) {
          constexpr int r = decltype(RC)::value;
          c[r] = nxc[b][0] + row_val<r>(v0, v1);
        });
      } else {
        c = nxv[b];  // the sample term is in the clamp bounds (kF8R)
      }
    };
    auto chain = [&](auto&& getB, const int (&gv)[2], f32x16 (&cc)[PB]) {
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        f32x16 c;
        if constexpr (P == 0) {
          const float2 b0 = getB(0);
          c = __builtin_amdgcn_mfma_f32_32x32x2f32(b0.x, A[b].v[0], f32x16{}, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_32x32x2f32(b0.y, A[b].v[1], c, 0, 0, 0);
#pragma unroll
          for (int s2 = 1; s2 < C::NSTEP / 2; ++s2) {
            const float2 bq = getB(s2);
            c = __builtin_amdgcn_mfma_f32_32x32x2f32(bq.x, A[b].v[2 * s2], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_32x32x2f32(bq.y, A[b].v[2 * s2 + 1], c, 0, 0, 0);
          }
        } else if constexpr (P == 1) {
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(getB(0), A[b].v[0], f32x16{}, 0, 0, 0);
#pragma unroll
          for (int s = 1; s < C::NSTEP; ++s)
            c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(getB(s), A[b].v[s], c, 0, 0, 0);
        } else {
          fp8_init(c, b, gv);
#pragma unroll
          for (int s = 0; s < C::NSTEP; ++s)
            c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(getB(s), A[b].v[s], c, 0, 0, 0, 0, 0, 0);
        }
        cc[b] = c;
      }
    };
    auto fixup = [&](f32x16 (&cc)[PB], const int (&gv)[2], int srow) {
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        f32x16& c = cc[b];
        if constexpr (P != 2 && M == kEucl) {
          // pairs prone to cancellation (kRecomputeThr) get their squared
          // distance again from the float32 rows; rare outside the self pair.
          // The threshold is >= 0, so comparing bit patterns as signed
          // integers orders c like the values (every negative c, -0 included,
          // compares below it): min3 on integers needs no NaN quieting.
          // kT: the element's threshold, skipped where no pair can meet it;
          // element rows: the sample's (the lane's column, 6 tau |y~_q|^2,
          // the same argument with the roles of x~ and y~ exchanged).
          if constexpr (kT) {
            if (__builtin_amdgcn_readfirstlane(chk[b]) == 0) continue;  // wave-uniform: no pair of the block can be flagged
          }
          const int tx = kT ? thrx[b] : gv[0];
          int mn = __float_as_int(c[0]);
#pragma unroll
          for (int r = 1; r < 16; ++r) mn = min(mn, __float_as_int(c[r]));
          if (__builtin_expect(mn < tx, 0)) {
            // one code copy for the flagged rows, taken in turn
            unsigned flagged = 0;
#pragma unroll
            for (int r = 0; r < 16; ++r) flagged |= (__float_as_int(c[r]) < tx ? 1u : 0u) << r;
            const int e0 = P0 + 32 * b + col;
            const float* xc = X + (size_t)(e0 < n ? e0 : n - 1) * d;
            const float* yc = Y32 + (size_t)(srow + col) * DMY;
            while (flagged) {
              const int r = __builtin_ctz(flagged);
              flagged &= flagged - 1;
              // the row's partner: a sample (kT) or an element
              const int rw = 8 * (r >> 2) + 4 * h + (r & 3);
              const int er = P0 + 32 * b + rw;
              const float* xp = kT ? xc : X + (size_t)(er < n ? er : n - 1) * d;
              const float* yr = kT ? Y32 + (size_t)(srow + rw) * DMY : yc;
              float acc2 = 0.0f;
              for (int q = 0; q < d; ++q) {
                const float t = xp[q] - yr[q];
                acc2 = fmaf(t, t, acc2);
              }
#pragma unroll
              for (int q = 0; q < 16; ++q) c[q] = q == r ? acc2 : c[q];
            }
          }
        } else if constexpr (P != 2 && !kT) {
          // cosine, element rows: a column holding one of this block's own
          // 32 elements (in this lane's half of the rows) zeroes that row
          // (the self pair, as below)
          const int self = gv[0] - (P0 + 32 * b);
          if ((unsigned)self < 32u && ((self >> 2) & 1) == h) {
            const int rh = ((self >> 3) << 2) | (self & 3);
#pragma unroll
            for (int r = 0; r < 16; ++r)
              if (r == rh) c[r] = 0.0f;
          }
        } else if constexpr (P != 2) {
          // cosine: no square root amplifies the expansion's absolute error
          // (of order 2^-22 here), so only the self pair d(e, e) = 0 is
          // forced: a sample row holding one of this block's own 32 elements
          // (lane l reads the id of row l % 32) zeroes that row in the
          // element's column.  The unit rows of both sides are the same
          // product x * rn, so the pair's operands are identical; zero rows
          // carry id -1 and keep their d = 1.
          const int self = gv[0] - (P0 + 32 * b);
          unsigned hit = (unsigned)__builtin_amdgcn_ballot_w64((unsigned)self < 32u);  // rows 0..31
          while (__builtin_expect(hit != 0u, 0)) {  // wave-uniform
            const int sr = __builtin_ctz(hit);
            hit &= hit - 1u;
            const int e = __builtin_amdgcn_readlane(self, sr);
            const int rs = 4 * (sr >> 3) + (sr & 3);
            const bool mine = col == e && h == ((sr >> 2) & 1);
#pragma unroll
            for (int q = 0; q < 16; ++q) c[q] = (mine && q == rs) ? 0.0f : c[q];
          }
        }
      }
    };
    // (element rows: wv[0] is the weight of the lane's sample column)
    auto wsum_add = [&](const f32x16 (&cc)[PB], const float (&wv)[2]) {
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        float dv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) dv[r] = dist(cc[b][r]);
        if constexpr (kT) {
          wsum16(acc[b], wv[0], wv[1], dv);
        } else if constexpr (kF8R) {
#pragma unroll
          for (int r = 0; r < 16; ++r)
            acc[b][r] = fmaf(wv[0], __builtin_amdgcn_fmed3f(cc[b][r], -wv[1], 2.0f * S2 - wv[1]), acc[b][r]);
          tcol[b] = fmaf(wv[0], wv[1], tcol[b]);
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[b][r] = fmaf(wv[0], dv[r], acc[b][r]);
        }
      }
    };
    auto fold = [&](bool last, int tiles = 1) {
      g += tiles;
      if (__builtin_expect(g >= kFold<P, kT> || last, 0)) {
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          float v;
          if constexpr (kT)
            v = lane_sum(acc[b]);
          else
            v = transpose_reduce16(acc[b], lane);
          if constexpr (kF8R) {
            // the sample terms' sum over the 32 columns (the same in both halves)
            float t = tcol[b];
#pragma unroll
            for (int o = 16; o > 0; o >>= 1) t += __shfl_xor(t, o, kWave);
            wsum[b] += ((double)v + (double)t) * (1.0 / S2);
            tcol[b] = 0.f;
          } else {
            // fp8: the distances came scaled by 64^2 (a power of two)
            wsum[b] += P == 2 ? (double)v * (1.0 / S2) : (double)v;
          }
#pragma unroll
          for (int r = 0; r < kNA; ++r) acc[b][r] = 0.f;
        }
        g = 0;
      }
    };
    // The LDS path's chain with the pending tile's sums woven in (one block
    // of 32 elements per wave there, element rows): the sample operand is
    // read kAhead steps ahead of its MFMA, and each step carries a share of
    // the pending tile's distances and FMAs and of the loads of tile tt of
    // the stage two ahead, issued while the MFMA runs.  Scheduling barriers
    // keep the steps in this
    // order (left to itself the compiler reads each step's operand right
    // before its MFMA, which then waits for the whole LDS latency).  Same
    // arithmetic per accumulator as chain + wsum_add.
    auto chain_pipe = [&](auto&& getB, const int (&gv)[2], f32x16 (&cn)[PB], const f32x16 (&cp)[PB],
                          const float (&wp)[2], int tt) {
      static_assert(PB == 1 && !kT, "the pipelined LDS path runs one block of 32 elements per wave, element rows");
      constexpr int NS = C::NSTEP;
      constexpr int kAhead = NS < 4 ? NS : 4;
      using BT = decltype(getB(0));
      BT bq[kAhead];
#pragma unroll
      for (int q = 0; q < kAhead; ++q) bq[q] = getB(q);
      f32x16 c;
      if constexpr (P == 2) {
        fp8_init(c, 0, gv);
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) c[r] = 0.0f;
      }
      // fp8: the pending tile's clamp bounds and its sample-term sum
      const float plo = -wp[1], phi = 2.0f * S2 - wp[1];
      if constexpr (kF8R) tcol[0] = fmaf(wp[0], wp[1], tcol[0]);
      __builtin_amdgcn_sched_barrier(0);
      static_for<NS>([&](auto QC) {
        constexpr int q = decltype(QC)::value;
        const BT cur = bq[q % kAhead];
        if constexpr (P == 1)
          c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0].v[q], cur, c, 0, 0, 0);
        else
          c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[0].v[q], cur, c, 0, 0, 0, 0, 0, 0);
        if constexpr (q + kAhead < NS) bq[q % kAhead] = getB(q + kAhead);
        // the next-but-one stage's loads of tile tt, spread over the steps
#pragma unroll
        for (int mi = 0; mi < kDw; ++mi)
          if (q == (2 * mi + 1) * NS / (2 * kDw)) tile_load(tt, mi);
#pragma unroll
        for (int r = 16 * q / NS; r < 16 * (q + 1) / NS; ++r)
          acc[0][r] = fmaf(wp[0], kF8R ? __builtin_amdgcn_fmed3f(cp[0][r], plo, phi) : dist(cp[0][r]), acc[0][r]);
        __builtin_amdgcn_sched_barrier(0);
      });
      cn[0] = c;
    };
    auto tile = [&](auto&& getB, const float (&wv)[2], const int (&gv)[2], int srow, bool last) {
      f32x16 cc[PB];
      chain(getB, gv, cc);
      fixup(cc, gv, srow);
      wsum_add(cc, wv);
      fold(last);
    };
    if constexpr (kLds) {
      // pipelined: ca holds the tile whose sums are pending (zeros before
      // the cluster's first); with two tiles per stage the two accumulator
      // sets swap roles from tile to tile
      f32x16 ca[PB], cb[PB];
      float wa[2] = {0.0f, 0.0f}, wb[2] = {0.0f, 0.0f};
      if constexpr (kPipe) {
#pragma unroll
        for (int b = 0; b < PB; ++b)
#pragma unroll
          for (int r = 0; r < 16; ++r) ca[b][r] = 0.0f;
      }
      for (int t = 0; t < ntile; t += kTB) {
        // this wave's loads of the stage are done once at most the next
        // stage's remain in flight; the barrier makes every wave's visible
        // and frees the slot the new loads go to (read two stages ago)
        asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(kNIw) : "memory");
        // the stage two ahead goes to the slot read two stages ago; its tile
        // loads ride on this stage's MFMA steps (all at once off that path)
        if constexpr (kPipe)
          stage_begin(rs == 0 ? 2 : rs - 1);
        else
          issue(rs == 0 ? 2 : rs - 1);
        advance();
        const unsigned char* sb = ldsS + rs * kSlotB;
        if (t == 0) buildA((const float*)(sb + kMuOff) + h * C::FOFF);
        auto fromLds = [&](int tt) {
          const unsigned char* tl = sb + tt * kTileCh * 16 + col * kLRow + h * C::FOFF * C::ELEM;
          return [tl](int q) {
            if constexpr (P == 0) {
              return *(const float2*)(tl + 8 * q);
            } else if constexpr (P == 1) {
              return *(const bf16x8*)(tl + 2 * C::FSTEP * q);
            } else {
              const u32x4 lo = *(const u32x4*)(tl + 32 * q), hi = *(const u32x4*)(tl + 32 * q + 16);
              return i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            }
          };
        };
        // the row tails: weights of rows wr and 16 + wr, per-row values
        // (element rows: the weight and value of the lane's sample column)
        auto wval = [&](int tt, float (&wv)[2]) {
          const unsigned char* tb = sb + tt * kTileCh * 16 + kRowB;
          if constexpr (kT) {
            wv[0] = *(const float*)(tb + wr * kLRow);
            wv[1] = *(const float*)(tb + (wr + 16) * kLRow);
          } else {
            wv[0] = *(const float*)(tb + col * kLRow);
            // fp8: the sample term 64^2 |y~|^2 / 2 of the lane's column
            if constexpr (kF8R) wv[1] = S2 * *(const float*)(tb + 4 + col * kLRow);
          }
        };
        auto gval = [&](int tt, int (&gv)[2]) {
          const unsigned char* tb = sb + tt * kTileCh * 16 + kRowB + 4;
          if constexpr (!kT) {
            gv[0] = *(const int*)(tb + col * kLRow);
          } else if constexpr (P == 2) {
            gv[0] = *(const int*)(tb + wr * kLRow);
            gv[1] = *(const int*)(tb + (wr + 16) * kLRow);
          } else if constexpr (M == kCos) {
            gv[0] = *(const int*)(tb + col * kLRow);
          }
        };
        if constexpr (kPipe) {
          // a tile's MFMAs and the pending tile's square roots and sums in one
          // stretch of code, so the vector ALU works while the matrix core runs
          {
            int gv[2];
            gval(0, gv);
            chain_pipe(fromLds(0), gv, cb, ca, wa, 0);
            if (t > 0) fold(false);
            fixup(cb, gv, base + t * 32);
            wval(0, wb);
          }
          if (kTB == 2 && t + 1 < ntile) {  // block-uniform
            int gv[2];
            gval(1, gv);
            chain_pipe(fromLds(1), gv, ca, cb, wb, 1);
            fold(false);
            fixup(ca, gv, base + (t + 1) * 32);
            wval(1, wa);
          } else {
            // one tile in the stage: the pending tile is in cb (and the
            // second tile of the stage two ahead is loaded here)
            if constexpr (kTB == 2) {
#pragma unroll
              for (int mi = 0; mi < kDw; ++mi) tile_load(1, mi);
            }
#pragma unroll
            for (int b = 0; b < PB; ++b) ca[b] = cb[b];
            wa[0] = wb[0];
            wa[1] = wb[1];
          }
        } else {
#pragma unroll
          for (int tt = 0; tt < kTB; ++tt)
            if (t + tt < ntile) {  // block-uniform
              float wv[2];
              int gv[2];
              wval(tt, wv);
              gval(tt, gv);
              tile(fromLds(tt), wv, gv, base + (t + tt) * 32, t + tt + 1 == ntile);
            }
        }
        rs = rs == 2 ? 0 : rs + 1;
      }
      if constexpr (kPipe) {
        if (ntile > 0) {
          wsum_add(ca, wa);
          fold(true);
        }
      }
    } else {
      // Tiles go in pairs with unconditional prefetches, so the wait before
      // each tile covers only that tile's loads; an odd last tile runs after
      // the loop from the buffer already loaded, and its successor is loaded
      // into the same buffer once its MFMAs are issued.
      if (ntile > 0 && pre != base) load_tile<M, P, DM>(Ym, w, gid_pk, bnorm, base, lane_off, col, wr, b0, w0, g0);
      int t = 0;
      for (; t + 2 <= ntile; t += 2) {
        load_tile<M, P, DM>(Ym, w, gid_pk, bnorm, base + (t + 1) * 32, lane_off, col, wr, b1, w1, g1);
        tile([&](int q) { return b0.v[q]; }, w0, g0, base + t * 32, false);
        pre = clamp_row(base + (t + 2) * 32);
        load_tile<M, P, DM>(Ym, w, gid_pk, bnorm, pre, lane_off, col, wr, b0, w0, g0);
        tile([&](int q) { return b1.v[q]; }, w1, g1, base + (t + 1) * 32, t + 2 == ntile);
      }
      if (t < ntile) {
        tile([&](int q) { return b0.v[q]; }, w0, g0, base + t * 32, true);
        pre = clamp_row(base + ntile * 32);
        load_tile<M, P, DM>(Ym, w, gid_pk, bnorm, pre, lane_off, col, wr, b0, w0, g0);
      }
    }
    const int sz = csize[j];
    const double dsz = (double)sz;
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      if (What != nullptr && pout[b] < n && (kT ? h == 0 : (lane & 1) == 0)) What[(size_t)pout[b] * k + j] = (float)wsum[b];
      if (j == own[b]) {
        w_own[b] = wsum[b];
      } else if (sz > 0 && wsum[b] * bden[b] < bnum[b] * dsz) {
        bnum[b] = wsum[b];
        bden[b] = dsz;
      }
    }
  }
  // the loads issued ahead of the last stages land in LDS before the block
  // may end (its LDS can then go to another block)
  if constexpr (kLds) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    const int szo = csize[own[b]];
    const double a = szo > 1 ? w_own[b] / (double)(szo - 1) : 0.0;
    const double bb = bden[b] > 0.0 ? bnum[b] / bden[b] : __builtin_inf();
    const double mx = a > bb ? a : bb;
    const double s = (szo > 1 && mx > 0.0) ? (bb - a) / mx : 0.0;
    const bool writer = pout[b] < n && (kT ? h == 0 : (lane & 1) == 0);
    if (writer) {
      if (a_out) a_out[pout[b]] = (float)a;
      if (b_out) b_out[pout[b]] = (float)bb;
      if (s_out) s_out[pout[b]] = (float)s;
    }
    // a float64 partial per 32 elements (fixed tree over the wave) ...
    const double part = wave_sum_f64(writer ? s : 0.0);
    if (lane == 0) sh32[(threadIdx.x >> 6) * PB + b] = part;
  }
  // ... and per 128 elements the four of them added in element order, so the
  // partials, and the mean, do not depend on the block shape PB
  __syncthreads();
  if (threadIdx.x < PB) {
    const int g = threadIdx.x;
    const int row0 = blk * 128 * PB + 128 * g;
    const double v = ((sh32[4 * g] + sh32[4 * g + 1]) + sh32[4 * g + 2]) + sh32[4 * g + 3];
    if (row0 < n) bpart[row0 >> 7] = v;
  }
}

template <int M, int P, int DM, int PB, int TBX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMinWaves<M, P, DM, PB, TBX>))) void k_p2_mfma(
    const float* __restrict__ X, int n, int d, const int32_t* __restrict__ labels,
    const void* __restrict__ Ym, const float* __restrict__ w, const int32_t* __restrict__ gid_pk,
    const int32_t* __restrict__ sp_off, const int32_t* __restrict__ cnt,
    const int32_t* __restrict__ csize, int k, const float* __restrict__ mu,
    float* __restrict__ a_out, float* __restrict__ b_out, float* __restrict__ s_out,
    float* __restrict__ What, double* __restrict__ bpart, const float* __restrict__ bnorm,
    const float* __restrict__ Y32, int DMY, const float* __restrict__ aux, const float* __restrict__ rn) {
  p2_mfma_block<M, P, DM, PB, TBX>(blockIdx.x, X, n, d, labels, Ym, w, gid_pk, sp_off, cnt, csize, k, mu, a_out, b_out,
                              s_out, What, bpart, bnorm, Y32, DMY, aux, rn);
}

// Several requests in one launch: workgroup i runs work item i = (request,
// block), doing exactly what that block of the request's own launch does, so
// results do not depend on which requests share the launch.  The hardware
// dispatcher hands the workgroups to the CUs in order as slots free up, which
// is the schedule a software work queue would give; a loop over items inside
// one workgroup kept the block's state across iterations and spilled 15-47
// registers in the shapes from d = 32 on.  The job table and the items are
// read through the constant address space, so their values sit in scalar
// registers like kernel arguments.
template <int M, int P, int DM, int PB, int TBX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMinWaves<M, P, DM, PB, TBX>))) void k_p2_mfma_jobs(
    const P2Job* __restrict__ jobs, const int2* __restrict__ items) {
  typedef const __attribute__((address_space(4))) P2Job* cjob_ptr;
  typedef const __attribute__((address_space(4))) int* citem_ptr;
  const int jx = ((citem_ptr)items)[2 * blockIdx.x];
  const int blk = ((citem_ptr)items)[2 * blockIdx.x + 1];
  const auto& J = ((cjob_ptr)jobs)[jx];
  p2_mfma_block<M, P, DM, PB, TBX>(blk, J.X, J.n, J.d, J.labels, J.Ym, J.w, J.gid_pk, J.sp_off, J.cnt, J.csize, J.k, J.mu,
                              J.a, J.b, J.s, J.What, J.bpart, J.bnorm, J.Y32, DM, J.aux, J.rn);
}

// Block shapes of the matrix-core kernel (ids used by the autotuner):
//  1  one 32-element block per wave (on the LDS path with kTBDefault tiles
//     per stage);
//  2  two blocks per wave: half the B-operand loads per pair (the float32
//     path is bound by the MFMA rate and gains) but twice the accumulator
//     and A-operand registers (fewer waves per SIMD); d <= 64, not fp8;
//  3  one block per wave with the other number of tiles per LDS stage (the
//     LDS path only).
// The arithmetic of every element, and the 128-element partials of the
// mean, are the same in every shape.
int mfma_pb_default(int prec, int DM) { return (prec == 0 && DM <= 32) ? 2 : 1; }
int mfma_pb_max(int prec, int DM) { return (prec == 2 || DM > 64) ? 1 : 2; }
int mfma_shapes(int prec, int DM, int* ids) {
  int m = 0;
  ids[m++] = 1;
  if (mfma_pb_max(prec, DM) == 2) ids[m++] = 2;
  if (mfma_lds_path(prec, DM)) ids[m++] = 3;
  return m;
}

template <int M, int P, int DM, int PB, int TBX>
static void launch_mfma_pb(hipStream_t st, const P2Args& A, const float* mu, const void* Ym,
                           const float* bnorm) {
  const int blocks = (int)ceil_div(A.n, 128 * PB);
  hipLaunchKernelGGL((k_p2_mfma<M, P, DM, PB, TBX>), dim3(blocks), dim3(256), 0, st, A.X, A.n, A.d, A.labels, Ym,
                     A.w, A.gid_pk, A.sp_off, A.cnt, A.csize, A.k, mu, A.a, A.b, A.s, A.What, A.bpart,
                     bnorm, A.Y, DM, A.aux, A.rn);
}

template <int M, int P, int DM>
static void launch_mfma_one(hipStream_t st, const P2Args& A, const float* mu, const void* Ym,
                            const float* bnorm, int shape) {
  constexpr int TB0 = kTBDefault<P, DM>;
  if constexpr (P != 2 && DM <= 64) {  // two blocks per wave would not fit the registers beyond
    if (shape == 2) {
      launch_mfma_pb<M, P, DM, 2, 1>(st, A, mu, Ym, bnorm);
      return;
    }
  }
  if (shape == 3 && mfma_lds_path(P, DM)) {
    launch_mfma_pb<M, P, DM, 1, 3 - TB0>(st, A, mu, Ym, bnorm);
    return;
  }
  launch_mfma_pb<M, P, DM, 1, TB0>(st, A, mu, Ym, bnorm);
}

template <int M, int P, int DM>
static void launch_jobs_one(hipStream_t st, const P2Job* jobs, const int2* items, int nitems, int shape) {
  constexpr int TB0 = kTBDefault<P, DM>;
  if constexpr (P != 2 && DM <= 64) {
    if (shape == 2) {
      hipLaunchKernelGGL((k_p2_mfma_jobs<M, P, DM, 2, 1>), dim3(nitems), dim3(256), 0, st, jobs, items);
      return;
    }
  }
  if (shape == 3 && mfma_lds_path(P, DM)) {
    hipLaunchKernelGGL((k_p2_mfma_jobs<M, P, DM, 1, 3 - TB0>), dim3(nitems), dim3(256), 0, st, jobs, items);
    return;
  }
  hipLaunchKernelGGL((k_p2_mfma_jobs<M, P, DM, 1, TB0>), dim3(nitems), dim3(256), 0, st, jobs, items);
}

template <int M, int P, int DM>
static void launch_pack_one(hipStream_t st, const float* Y32, const float* aux, const float* w,
                            const int32_t* gid_pk, const int32_t* sp_off, const int32_t* cnt, int k,
                            float* mu, int S_pad, void* Ym, float* bnorm) {
  hipLaunchKernelGGL((k_pack_mfma<M, P, DM>), dim3((int)ceil_div(S_pad, 256)), dim3(256), 0, st, Y32,
                     aux, w, gid_pk, sp_off, cnt, k, mu, S_pad, Ym, bnorm);
}

#define SILH_MFMA_DISPATCH(FN, ...)                                     \
  do {                                                                  \
    if (metric == kEucl && prec == 0) {                                 \
      switch (DM) {                                                     \
        case 8: FN<kEucl, 0, 8>(__VA_ARGS__); return true;              \
        case 16: FN<kEucl, 0, 16>(__VA_ARGS__); return true;            \
        case 32: FN<kEucl, 0, 32>(__VA_ARGS__); return true;            \
        case 64: FN<kEucl, 0, 64>(__VA_ARGS__); return true;            \
        case 128: FN<kEucl, 0, 128>(__VA_ARGS__); return true;          \
      }                                                                 \
    } else if (metric == kEucl && prec == 1) {                          \
      switch (DM) {                                                     \
        case 8: FN<kEucl, 1, 8>(__VA_ARGS__); return true;              \
        case 16: FN<kEucl, 1, 16>(__VA_ARGS__); return true;            \
        case 32: FN<kEucl, 1, 32>(__VA_ARGS__); return true;            \
        case 64: FN<kEucl, 1, 64>(__VA_ARGS__); return true;            \
        case 128: FN<kEucl, 1, 128>(__VA_ARGS__); return true;          \
        case 256: FN<kEucl, 1, 256>(__VA_ARGS__); return true;          \
      }                                                                 \
    } else if (metric == kCos && prec == 0) {                           \
      switch (DM) {                                                     \
        case 8: FN<kCos, 0, 8>(__VA_ARGS__); return true;               \
        case 16: FN<kCos, 0, 16>(__VA_ARGS__); return true;             \
        case 32: FN<kCos, 0, 32>(__VA_ARGS__); return true;             \
        case 64: FN<kCos, 0, 64>(__VA_ARGS__); return true;             \
        case 128: FN<kCos, 0, 128>(__VA_ARGS__); return true;           \
      }                                                                 \
    } else if (metric == kCos && prec == 1) {                           \
      switch (DM) {                                                     \
        case 8: FN<kCos, 1, 8>(__VA_ARGS__); return true;               \
        case 16: FN<kCos, 1, 16>(__VA_ARGS__); return true;             \
        case 32: FN<kCos, 1, 32>(__VA_ARGS__); return true;             \
        case 64: FN<kCos, 1, 64>(__VA_ARGS__); return true;             \
        case 128: FN<kCos, 1, 128>(__VA_ARGS__); return true;           \
        case 256: FN<kCos, 1, 256>(__VA_ARGS__); return true;           \
      }                                                                 \
    } else if (metric == kCos && prec == 2) {                           \
      switch (DM) {                                                     \
        case 8: FN<kCos, 2, 8>(__VA_ARGS__); return true;               \
        case 16: FN<kCos, 2, 16>(__VA_ARGS__); return true;             \
        case 32: FN<kCos, 2, 32>(__VA_ARGS__); return true;             \
        case 64: FN<kCos, 2, 64>(__VA_ARGS__); return true;             \
        case 128: FN<kCos, 2, 128>(__VA_ARGS__); return true;           \
        case 256: FN<kCos, 2, 256>(__VA_ARGS__); return true;           \
      }                                                                 \
    }                                                                   \
    return false;                                                       \
  } while (0)

bool launch_pack_mfma(hipStream_t st, int metric, int prec, int DM, const float* Y32, const float* aux,
                      const float* w, const int32_t* gid_pk, const int32_t* sp_off, const int32_t* cnt, int k,
                      float* mu, int S_pad, void* Ym, float* bnorm) {
  SILH_MFMA_DISPATCH(launch_pack_one, st, Y32, aux, w, gid_pk, sp_off, cnt, k, mu, S_pad, Ym, bnorm);
}

bool launch_phase2_mfma(hipStream_t st, int metric, int prec, int DM, const P2Args& A, const float* mu,
                        const void* Ym, const float* bnorm, int shape) {
  SILH_MFMA_DISPATCH(launch_mfma_one, st, A, mu, Ym, bnorm, shape);
}

bool launch_phase2_mfma_jobs(hipStream_t st, int metric, int prec, int DM, int shape, const P2Job* jobs,
                             const int2* items, int nitems) {
  if (nitems <= 0) return true;
  SILH_MFMA_DISPATCH(launch_jobs_one, st, jobs, items, nitems, shape);
}

int phase2_mfma_rows(int, int) { return 128; }

}  // namespace silh
