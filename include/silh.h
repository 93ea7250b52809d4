/*
 * silh.h - C ABI of the MI355X (gfx950) silhouette library.
 *
 * The library computes, on one AMD Instinct MI355X, the sampled silhouette
 * estimator of "Scalable and Distributed Silhouette Approximation"
 * (arxiv 2607.01993): Phase 1 (PPS sampling, Algorithm 1; or uniform Poisson
 * sampling, Section 4.1.3), Phase 2 (for every element e and cluster C_j the
 * weighted sum W_hat_{C_j}(e) = sum_{e' in F_j} d(e,e')/p_{e'}, then a_hat,
 * b_hat and s_hat, Algorithm 1 / Eq. 5) and the global mean (Eq. 9); and the
 * exact silhouette (Section 2, Eqs. 1-3).
 *
 * Conventions for every call:
 *  - Pointers are DEVICE pointers (memory of the current HIP device) unless
 *    the argument name ends in _host.
 *  - All GPU work is enqueued on the stream given at creation (a hipStream_t
 *    passed as silh_stream; NULL is the legacy default stream).  A call with
 *    a *_host output synchronises that stream before it returns; other calls
 *    return as soon as the work is enqueued.
 *  - Element ids ("gid") are row indices of X, 0 .. n-1.  Labels are cluster
 *    ids in [0, k); clusters may be empty.
 *  - Every call returns a silh_status.  On anything but SILH_OK,
 *    silh_last_error() returns a message for the calling thread.  No C++
 *    exception crosses this interface.
 *  - Calls on one context must not run concurrently from several threads.
 */
#ifndef SILH_H
#define SILH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SILH_OK = 0,
  SILH_E_ARG = 1,          /* invalid argument or parameter combination          */
  SILH_E_LABEL = 2,        /* a label outside [0, k)                              */
  SILH_E_K = 3,            /* fewer than two nonempty clusters: b is undefined    */
  SILH_E_STATE = 4,        /* call out of order (see silh_pps_sample)             */
  SILH_E_NOMEM = 5,        /* the allocator returned NULL                         */
  SILH_E_HIP = 6,          /* a HIP runtime error                                 */
  SILH_E_UNSUPPORTED = 7   /* metric / precision / size combination not built     */
} silh_status;

/* The four distances of the paper's experiments (Section 5.1.2).
 * SILH_COS reads the garbled printed formula as 1 - x.y/(|x||y|) (0 similarity
 * for a zero vector), clamped to [0, 2]; SILH_CANB takes a 0/0 coordinate as 0. */
typedef enum { SILH_EUCL = 0, SILH_COS = 1, SILH_MANH = 2, SILH_CANB = 3 } silh_metric;

/* Arithmetic of the Phase-2 distance tiles.  Accumulation is float32 inside
 * a tile and float64 across tiles; Phase 1 always runs in float64.
 *  SILH_FP32       float32.  Euclidean and cosine run on the matrix cores
 *                  (v_mfma_f32_32x32x2_f32), Manhattan and Canberra on the
 *                  vector ALUs.
 *  SILH_BF16       bf16 operands, float32 accumulation (v_mfma_f32_32x32x16_bf16);
 *                  Euclidean and cosine only.
 *  SILH_FP8        OCP e4m3 operands, float32 accumulation
 *                  (v_mfma_f32_32x32x64_f8f6f4); cosine with d >= 64 only
 *                  (the K step is 64 wide, and at smaller d the 3-bit
 *                  mantissa's error per coordinate no longer averages out).
 *                  Operands are the centred unit vectors times 64.
 *  SILH_FP32_VALU  float32 on the vector ALUs for every metric. */
typedef enum { SILH_FP32 = 0, SILH_BF16 = 1, SILH_FP8 = 2, SILH_FP32_VALU = 3 } silh_prec;

/* SILH_PPS: Algorithm 1, Phase 1.  SILH_UNI: uniform Poisson sampling with
 * rate t/|C_j| (Section 4.1.3). */
typedef enum { SILH_PPS = 0, SILH_UNI = 1 } silh_sampler;

/* Device-memory allocator hooks.  alloc must return device memory of at least
 * `bytes` bytes, usable on the context's stream, or NULL on failure (the call
 * then fails with SILH_E_NOMEM).  free receives every pointer alloc returned,
 * exactly once.  If alloc is NULL the library takes blocks from a cache it
 * keeps per (device, stream) until the process ends (new blocks by
 * hipMalloc; a freed block is reused only by later allocations on the same
 * stream, so no call synchronises the device once the cache is warm). */
typedef void* (*silh_alloc_fn)(size_t bytes, void* user);
typedef void (*silh_free_fn)(void* ptr, void* user);

typedef void* silh_stream; /* a hipStream_t */

typedef struct {
  int64_t n;         /* number of elements (rows of X); n >= 2                         */
  int32_t d;         /* dimension (columns of X); 1 <= d <= 256                         */
  int32_t k;         /* number of cluster ids; 2 <= k <= 4096                           */
  int32_t metric;    /* silh_metric                                                     */
  int32_t prec;      /* silh_prec                                                       */
  int32_t sampler;   /* silh_sampler                                                    */
  int32_t reserved0; /* must be 0                                                       */
  int64_t t;         /* expected sample size per cluster (Algorithm 1's t).  t <= 0:
                        derived from eps and delta as ceil((3*18/eps^2) ln(5nk/delta)),
                        the form of Lemma 1                                            */
  double eps;        /* accuracy parameter, used only when t <= 0; in (0, 1)            */
  double delta;      /* confidence parameter in (0, 1); enters the initial-sample rate
                        (2/|C_j|) ln(5k/delta) of Algorithm 1 (the paper uses 0.01)     */
  uint64_t seed;     /* key of the Philox4x32-10 generator behind every Poisson draw    */
  silh_alloc_fn alloc;
  silh_free_fn free;
  void* alloc_user;
} silh_params;

typedef struct silh_ctx silh_ctx;

/*
 * silh_sample_init - create a context for one dataset and one clustering.
 * Problem 1 / Problem 2 (Section 4.1, Section 4.2): the input is a dataset V
 * of n elements and a k-clustering of it.
 *
 *  X       [n][d] float32, row-major, device.  Owned by the caller; must stay
 *          valid and unchanged until silh_destroy.
 *  labels  [n] int32 in [0, k), device.  Owned by the caller, same lifetime.
 *  stream  the stream all of this context's work runs on.
 *  out     receives the new context (NULL on failure).
 *
 * Counts the clusters and builds the cluster index (a stable counting sort of
 * the ids by label).  Synchronises the stream once (the k cluster sizes are
 * read back to the host).
 * Errors: SILH_E_ARG (bad n, d, k, t/eps, delta, metric, prec, sampler, NULL
 * pointer), SILH_E_UNSUPPORTED (prec not built for the metric), SILH_E_LABEL,
 * SILH_E_K, SILH_E_NOMEM, SILH_E_HIP.
 */
silh_status silh_sample_init(const silh_params* prm, const float* X, const int32_t* labels,
                             silh_stream stream, silh_ctx** out);

/*
 * silh_pps_sample - Phase 1 (Algorithm 1; the uniform variant of Section 4.1.3
 * when prm->sampler == SILH_UNI).  For every cluster with |C_j| <= t the
 * sample is the whole cluster (p = 1).  Otherwise (PPS): the initial sample
 * F^0_j keeps each element with probability min(1, (2/|C_j|) ln(5k/delta));
 * W(e_bar) = sum_{e' in C_j} d(e_bar, e') for e_bar in F^0_j;
 * gamma_e = max{1/|C_j|, max_{e_bar, W(e_bar) > 0} d(e, e_bar)/W(e_bar)};
 * p_e = min{1, t gamma_e}; F_j keeps e with probability p_e.  All of this is
 * float64.  Each draw compares U < p with the 53-bit uniform
 * U = (w0*2^21 + (w1 >> 11)) * 2^-53, where (w0, w1) are the first two words of
 * Philox4x32-10 with key (seed_lo, seed_hi) and counter (gid_lo, gid_hi,
 * stream, 0), stream 0 for F^0, 1 for F (PPS), 2 for F (uniform).
 * Can be called again: it redraws from the same seed (same result).
 *
 *  S_host            receives |F| = sum_j |F_j| (nullable).
 *  per_cluster_host  [k] receives |F_j| (nullable).
 * Synchronises the stream.  Errors: SILH_E_ARG (ctx NULL), SILH_E_NOMEM,
 * SILH_E_HIP.
 */
silh_status silh_pps_sample(silh_ctx* ctx, int64_t* S_host, int64_t* per_cluster_host);

/*
 * silh_weighted_sums - Phase 2 weights, Algorithm 1 (loop over e and C_j):
 * W_hat[e][j] = sum_{e' in F_j} d(e, e') / p_{e'}, for every element e and
 * every cluster j (0 for an empty cluster).
 *
 *  W_hat  [n][k] float32, row-major, device, written by the call.
 * Requires a successful silh_pps_sample on ctx (else SILH_E_STATE).
 */
silh_status silh_weighted_sums(silh_ctx* ctx, float* W_hat);

/*
 * silh_scores - Phase 2 scores, Algorithm 1 / Eq. 5, and the global mean
 * s_hat_2 = (1/n) sum_e s_hat(e) (Eq. 9):
 *   a_hat(e) = W_hat_C(e) / (|C| - 1)                (0 for a singleton),
 *   b_hat(e) = min over nonempty C_j != C of W_hat_{C_j}(e) / |C_j|,
 *   s_hat(e) = (b_hat - a_hat) / max(a_hat, b_hat)   (0 for a singleton or when
 *              the max is 0).
 *
 *  a, b, s       [n] float32, device, each nullable.
 *  s_mean_host   receives the mean (float64; summed in float64 with
 *                compensation), nullable; when given, the stream is synchronised.
 * Requires a successful silh_pps_sample on ctx (else SILH_E_STATE).
 */
silh_status silh_scores(silh_ctx* ctx, float* a, float* b, float* s, double* s_mean_host);

/*
 * silh_exact - exact silhouette (Section 2, Eqs. 1-3): a(e), b(e), s(e) with
 * every cluster used whole (F_j = C_j, p = 1), and s(C).  Uses prm->n, d, k,
 * metric, prec, alloc/free/alloc_user; ignores t, eps, delta, sampler, seed.
 * Arguments as in silh_sample_init and silh_scores.  Synchronises the stream
 * (cluster sizes are read back).  Errors as silh_sample_init.
 */
silh_status silh_exact(const silh_params* prm, const float* X, const int32_t* labels,
                       silh_stream stream, float* a, float* b, float* s, double* s_mean_host);

/*
 * silh_exact_noalloc - silh_exact without any device allocation, for callers
 * that cannot allocate device memory (code under stream capture, serving
 * loops that must not call hipMalloc, harnesses that forbid it).  Arguments,
 * results and errors as silh_exact; prm->alloc, free and alloc_user are
 * ignored.  The library's buffers (cluster index, packed rows, partial sums)
 * are slices of one static device array of 256 MiB that each device holds
 * from the first call on it until the process ends; a problem whose buffers
 * do not fit it (about 270 bytes per element at d = 32 with bf16 operands,
 * so n up to about 10^6) is rejected with SILH_E_ARG before anything is
 * enqueued.  The caller still passes X, labels and the outputs.  The array
 * keeps the last call's contents (the call refills what must start at a known
 * value).  Calls on one device share it, so calls that overlapped on one
 * device would race: the library runs the calls of one process on one device
 * one at a time (each returns after its stream has synchronised).
 * Synchronises the stream once, at the end.  On SILH_E_LABEL or SILH_E_K the
 * contents of a, b, s are unspecified.
 */
silh_status silh_exact_noalloc(const silh_params* prm, const float* X, const int32_t* labels,
                               silh_stream stream, float* a, float* b, float* s, double* s_mean_host);

/*
 * Subsampled estimates of s(C) (Section 4.2).  The m rows are drawn
 * independently and uniformly from {0..n-1}, with replacement (Eqs. 8 and 10;
 * the Hoeffding bounds after them need independent draws).
 *
 * silh_rows_for - the sample size of those bounds, m = ceil((2/eps^2)
 * ln(2/delta)), into *m.  SILH_E_ARG unless eps, delta lie in (0, 1) and m
 * fits 2^30.
 */
silh_status silh_rows_for(double eps, double delta, int64_t* m);

/*
 * silh_draw_rows - rows[i] = floor(B_i * n / 2^53) for i in [0, m), B_i the
 * 53 bits of the Philox4x32-10 draw of counter i in draw stream 3 (the same
 * generator and bit layout as the Poisson draws), computed in integers.
 *  rows   [m] int32, device, caller-owned.  Enqueued on stream; no sync.
 * SILH_E_ARG for n outside [1, 2^30], m outside [0, 2^30], NULL rows (m > 0).
 */
silh_status silh_draw_rows(uint64_t seed, int64_t n, int64_t m, int32_t* rows, silh_stream stream);

/*
 * silh_scores_rows - gl-pps-s (PPS context) or gl-uni-s (uniform context),
 * Eq. 10: a_hat, b_hat, s_hat of Algorithm 1, Phase 2, for the m entries of
 * rows (duplicates allowed; entry i gets the values of element rows[i]) and
 * their mean (1/m) sum_i s_hat(rows[i]).  Only the distinct rows are
 * evaluated.
 *  rows          [m] int32, device, each in [0, n); unchanged.
 *  a, b, s       [m] float32, device, each nullable.
 *  s_mean_host   the mean (float64 with compensation), nullable.
 * Synchronises the stream (the number of distinct rows is read back).
 * SILH_E_STATE before a successful silh_pps_sample; SILH_E_ARG for NULL rows,
 * m outside [1, 2^30] or an entry outside [0, n) (then nothing is written).
 */
silh_status silh_scores_rows(silh_ctx* ctx, const int32_t* rows, int64_t m, float* a, float* b,
                             float* s, double* s_mean_host);

/*
 * silh_exact_rows - gl-s, Eq. 8: the exact a(e), b(e), s(e) (Eqs. 1-2) of
 * the m entries of rows and their mean.  Arguments as silh_exact and
 * silh_scores_rows; the cost is m' * n distance evaluations for m' distinct
 * rows.
 */
silh_status silh_exact_rows(const silh_params* prm, const float* X, const int32_t* labels,
                            const int32_t* rows, int64_t m, silh_stream stream, float* a, float* b,
                            float* s, double* s_mean_host);

/*
 * silh_coh_sep - estimates of the cohesion and separation of the clustering
 * (Appendix B) with W_hat of Algorithm 1, Phase 2, in place of W:
 *   Coh = (1/2) sum_j sum_{e in C_j} W_hat_{C_j}(e) / sum_j C(|C_j|, 2),
 *   Sep = sum_{j1<j2} sum_{e in C_j1} W_hat_{C_j2}(e) / sum_{j1<j2} |C_j1||C_j2|
 * (the printed |C_{j-1}| in the separation denominator read as |C_j1|).
 * With t >= max |C_j| every p is 1 and these are the exact measures.
 *  W_hat      [n][k] float32, device, as written by silh_weighted_sums for
 *             this context; NULL: the call computes it into context memory.
 *  coh_host, sep_host   the two values (float64 sums); 0 when a denominator
 *             is 0.  Synchronises the stream.
 * SILH_E_STATE before a successful silh_pps_sample; SILH_E_ARG for NULL ctx
 * or outputs.
 */
silh_status silh_coh_sep(silh_ctx* ctx, const float* W_hat, double* coh_host, double* sep_host);

/*
 * Autotuning of the matrix-core Phase-2 kernel's block shape, process-wide.
 * Shapes: 1 one 32-element block per wave; 2 two blocks per wave (d <= 64,
 * not fp8); 3 one block per wave with the other number of tiles per stage
 * (one or two 32-row sample tiles between block barriers) on the shapes that
 * stage sample tiles in LDS (bf16 / float32 with d >= 64, fp8 with d >= 128).
 *  mode 0  the built-in choice (two blocks for float32 operands with
 *          d <= 32 and for cosine bf16 at d = 32, else one);
 *  mode 1  (default) on the first launch for a key (metric, operand type, d
 *          rounded up as in the kernels, floor(log2) of the padded sample
 *          size) time every valid shape twice, keep the fastest; setting
 *          mode 1 again forgets the measurements;
 *  mode 2 / 3 / 4  always shape 1 / 2 / 3 where valid (else the built-in).
 * Results do not depend on the shape (the partial sums of the mean are per
 * 128 elements, added in the same order, in every shape).  SILH_E_ARG for a
 * mode outside [0, 4].
 */
silh_status silh_set_tuning(int mode);

/* *pb = the measured shape id for that key (1, 2 or 3), 0 if none yet. */
silh_status silh_tuning_choice(int metric, int prec, int d, int64_t S_pad, int* pb);

/* Read-only view of a context's Phase-1 result (for inspection and tests). */
typedef struct {
  int64_t S;                  /* sum_j |F_j|                                              */
  const int64_t* gid;         /* device [S]: ids of the sampled elements, grouped by
                                 cluster (cluster 0 first), ascending inside a cluster   */
  const int64_t* offsets_host;/* host [k+1]: cluster j's ids are gid[offsets[j]..offsets[j+1]) */
  const double* p;            /* device [n]: inclusion probability of each element by id  */
  int64_t F0;                 /* sum_j |F^0_j| (0 for the uniform sampler)                */
  const int64_t* f0_gid;      /* device [F0]: ids of the initial sample, grouped by cluster */
  const double* f0_W;         /* device [F0]: W(e_bar) of each initial element            */
  const int64_t* f0_offsets_host; /* host [k+1]                                           */
  int64_t t;                  /* the t in use (after derivation from eps when t <= 0)     */
} silh_sample_info;

/*
 * silh_sample_view - fill *out with views of ctx-owned storage, valid until
 * the next silh_pps_sample or silh_destroy on ctx.  Requires a successful
 * silh_pps_sample (else SILH_E_STATE).
 */
silh_status silh_sample_view(silh_ctx* ctx, silh_sample_info* out);

/*
 * silh_philox_uniform - diagnostic: out[i] = U(seed, gid0 + i, stream) for
 * i in [0, count), the same uniform the samplers draw (see silh_pps_sample).
 *  out  [count] float64, device.  Enqueued on `stream`; does not synchronise.
 * Errors: SILH_E_ARG (count < 0, gid0 < 0, out NULL when count > 0), SILH_E_HIP.
 */
silh_status silh_philox_uniform(uint64_t seed, int64_t gid0, int64_t count, uint32_t stream_id,
                                double* out, silh_stream stream);

/*
 * Kernel timing.  on = 1: every kernel launch of the context is bracketed by
 * HIP events recorded on its stream; on = 2: only the Phase-2 launches; 0:
 * off (SILH_E_ARG outside [0, 2]).  silh_prof_get
 * returns, for kernel slot i (0 <= i < silh_prof_count), its name, the number
 * of timed launches and their total duration in milliseconds (this call
 * synchronises the stream).  silh_prof_reset clears the totals.
 */
silh_status silh_prof_enable(silh_ctx* ctx, int on);
silh_status silh_prof_reset(silh_ctx* ctx);
int silh_prof_count(void);
silh_status silh_prof_get(silh_ctx* ctx, int i, const char** name, int64_t* launches,
                          double* total_ms);

/* Synchronise the context's stream, then free every buffer the context
 * allocated, through its allocator.  NULL is a no-op. */
void silh_destroy(silh_ctx* ctx);

/* Message of the last failed call on this thread ("" if none). */
const char* silh_last_error(void);

/* Library version string. */
const char* silh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SILH_H */
