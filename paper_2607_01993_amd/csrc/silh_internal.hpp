// Internal interface between the C ABI (silh_api.cpp) and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace silh {

// Rows per unit of the stable counting sort (one wave per unit): 256 while the
// per-unit histograms (units x k ints) stay small, else 1024.
inline int sort_seg(int64_t n, int k) {
  return (n + 255) / 256 * (int64_t)k <= ((int64_t)1 << 26) ? 256 : 1024;
}
// Elements per block of the int32 exclusive scan (256 threads x 8).
constexpr int kScanTile = 2048;
// Members per work item of the W(e_bar) partial sums.
constexpr int kWChunk = 256;   // one member per thread of a 256-thread block
constexpr int kWChunkWide = 256;  // d > 128: one member per thread as well
// Sample rows of each cluster are padded to a multiple of this.
constexpr int kSamplePad = 32;
// Rows per Phase-2 block in the VALU kernel.
constexpr int kP2Rows = 256;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---- cluster index -------------------------------------------------------
// per-unit label histograms uh [k][units] (label-major); *bad = 1 if a label
// is outside [0, k) (bad may be null: such a label is counted nowhere)
void launch_unit_hist(hipStream_t st, const int32_t* labels, int n, int k, int seg, int32_t* uh, int* bad);
// uh[u][j] <- label j's rows before unit u; counts[j] = |C_j|
void launch_unit_scan(hipStream_t st, int32_t* uh, int units, int k, int32_t* counts);
// stable scatter: rows of label j go to off[j] + uh[u][j] + (rank inside the unit)
void launch_scatter(hipStream_t st, const int32_t* labels, int n, int k, int seg, const int32_t* ubase,
                    const int32_t* off, int32_t* perm, int32_t* slab);
// out[0..n] = exclusive prefix sums of in[0..n), out[n] = total.  tmp holds
// ceil_div(n, kScanTile) + 1 ints.
void launch_scan(hipStream_t st, const int32_t* in, int n, int32_t* out, int32_t* tmp);
// out[j] = scan[off[j]] for j in [0, k]
void launch_gather_at(hipStream_t st, const int32_t* scan, const int32_t* off, int k, int32_t* out);

// ---- Phase 1 -----------------------------------------------------------------
void launch_f0_flag(hipStream_t st, const int32_t* perm, const int32_t* slab, int n,
                    const int32_t* csize, const double* q, int64_t t, uint64_t seed, int32_t* flag);
// rows past `cap` (the capacity of f0_gid / f0_cl / f0X) are not written
void launch_f0_pack(hipStream_t st, const int32_t* perm, const int32_t* slab, const int32_t* flag,
                    const int32_t* pos, int n, const float* X, int d, int DM, int cap, int64_t* f0_gid,
                    int32_t* f0_cl, double* f0X);
// float64 distances from the members of each cluster to its initial-sample
// rows, kept by the W pass for the draw (which then reads them instead of
// evaluating them again): the distance of the member at sorted position i of
// cluster j to F0_j's e-th row is at d[base[j] + e |C_j| + (i - off[j])].
// With d null, or *use == 0 (set on the device when the distances did not fit
// their capacity), nothing is kept and the draw evaluates the distances.
struct DistStore {
  double* d = nullptr;
  const int64_t* base = nullptr;  // [k]
  const int32_t* off = nullptr;   // [k + 1] cluster offsets
  const int32_t* use = nullptr;   // device flag
};
// one block per work item: item = (cluster, first sorted pos, end sorted pos,
// first F0 index of the cluster, |F0_j|, base in `partial`)
// f0X rows have stride DM (zero-padded)
void launch_w_partial(hipStream_t st, int metric, int DM, const int32_t* items, int nitems,
                      const int32_t* perm, const float* X, int d, const double* f0X, double* partial,
                      DistStore ds = {});
// F0 blocks at most; those at or past f0_off[k] return at once
void launch_w_final(hipStream_t st, const int32_t* f0_cl, int F0, const int32_t* f0_off, int k,
                    const int32_t* citem_first, const int32_t* citem_count, const int32_t* items,
                    const double* partial, double* W);
void launch_draw(hipStream_t st, int metric, int DM, int sampler, const int32_t* perm,
                 const int32_t* slab, int n, const float* X, int d, const int32_t* csize, int64_t t,
                 uint64_t seed, const int32_t* f0_off, const double* f0X, const double* W,
                 double* p_gid, int32_t* flag, DistStore ds = {});
void launch_fill_all(hipStream_t st, const int32_t* perm, int n, double* p_gid, int32_t* flag);
// rn[i] = 1 / |X_i| in float32 (fused chain in coordinate order, correctly
// rounded square root and division), 0 for a zero row
void launch_rnorm(hipStream_t st, const float* X, int n, int d, float* rn);
// the launch_pack mode of a metric (metric ids as in silh_metric: 1 cosine,
// 3 Canberra)
inline int pack_mode(int metric) { return metric == 1 ? 1 : (metric == 3 ? 2 : 0); }
// Scatter the selected elements into the cluster-blocked, padded sample.
// mode 0: raw coordinates; 1: rows times rn (unit L2 norm, cosine); 2: raw
// coordinates with aux32 = 1 for a row holding a coordinate of magnitude
// above 2^62 (or not finite), else 0 (Canberra; see k_phase2_valu.hip).  Rows at
// or past `cap` (the capacity of the packed arrays) are not written.  Every
// other row in [0, sp_off[k]) is written, the padding rows of each cluster
// block as id -1 with zero weight, aux and coordinates: no prior clear.
void launch_pack(hipStream_t st, const int32_t* perm, const int32_t* slab, const int32_t* flag,
                 const int32_t* pos, int n, int k, const float* X, int d, int DM, const double* p_gid,
                 const int32_t* s_off, const int32_t* sp_off, int mode, const float* rn, int cap,
                 int64_t* gid_view, int32_t* gid_pk, float* w32, float* aux32, float* Y32);

// ---- Phase 2 -----------------------------------------------------------------
struct P2Args {
  const float* X;
  int n, d;
  const int32_t* labels;
  const float* Y;      // [S_pad][DM]
  const float* w;      // [S_pad]
  const float* aux;    // [S_pad] cosine: 0.5 for a zero sample vector, else 0
  const int32_t* gid_pk;  // [S_pad] element id of each packed sample row, -1 for padding
  const int32_t* sp_off;  // [k+1] padded sample offsets
  const int32_t* cnt;     // [k] |F_j|
  const int32_t* csize;   // [k] |C_j|
  int k;
  float* a;
  float* b;
  float* s;
  float* What;          // [n][k] or null
  double* bpart;        // [ceil(n / rows per partial)]
  double* Wpart = nullptr;  // [n][k] float64, for the split vector-ALU pass (d > 128)
  const float* rn = nullptr;  // [n] cosine: reciprocal row norms (launch_rnorm) of X's rows
};
// One request's Phase-2 launch as a work source of a multi-request launch
// (the arguments of P2Args and of the matrix-core operands, in device memory).
struct P2Job {
  const float* X;
  const int32_t* labels;
  const void* Ym;        // matrix-core operands (null on the vector-ALU path)
  const float* w;
  const int32_t* gid_pk;
  const int32_t* sp_off;
  const int32_t* cnt;
  const int32_t* csize;
  const float* mu;
  float* a;
  float* b;
  float* s;
  float* What;
  double* bpart;
  const float* bnorm;
  const float* Y32;
  const float* aux;
  const float* rn;
  int n, d, k, pad0;
};
// returns false if (metric, d) has no VALU kernel
bool launch_phase2_valu(hipStream_t st, int metric, int DM, const P2Args& a);
// Multi-request launches: workgroup i runs work item items[i] = (index into
// jobs, block of that job's own launch).  The vector-ALU form covers the
// one-pass shapes with the row in registers (phase2_valu_jobs_ok); blocks
// are phase2_valu_rows / phase2_mfma_rows * pb elements.
bool launch_phase2_valu_jobs(hipStream_t st, int metric, int DM, const P2Job* jobs, const int2* items, int nitems);
bool phase2_valu_jobs_ok(int metric, int DM);
bool launch_phase2_mfma_jobs(hipStream_t st, int metric, int prec, int DM, int shape, const P2Job* jobs,
                             const int2* items, int nitems);
int phase2_valu_dm(int d);   // padded dimension used by the VALU kernel, 0 if unsupported
// elements per block (and per partial of the mean) of the VALU kernel
int phase2_valu_rows(int metric, int DM);
// d > 128 Manhattan / Canberra run as two coordinate halves and need
// P2Args::Wpart ([n][k] float64 scratch)
bool phase2_valu_split(int metric, int DM);

// MFMA path (Euclidean and cosine with float32 or bf16 operands; cosine with
// fp8 operands).  prec: 0 float32, 1 bf16, 2 fp8.
int mfma_kp(int prec, int DM);   // contraction length of a packed row
int mfma_row_bytes(int prec, int DM);  // bytes per packed row (operands, LDS-path tail)
// mu: [k][KP] centres, zero beyond DM, then [k] squared radii of the
// clusters' packed samples (Euclidean; the largest |y~_q|^2), mfma_mu_floats
// floats in all
size_t mfma_mu_floats(int prec, int DM, int k);
void launch_center(hipStream_t st, const float* Y32, int DM, int KP, const int32_t* sp_off,
                   const int32_t* cnt, int k, float* mu);
// packs rows [0, min(S_pad, sp_off[k])) (w: weights, gid_pk: element ids of
// the packed rows, copied into the rows' tails on the LDS path)
bool launch_pack_mfma(hipStream_t st, int metric, int prec, int DM, const float* Y32, const float* aux,
                      const float* w, const int32_t* gid_pk, const int32_t* sp_off, const int32_t* cnt, int k,
                      float* mu, int S_pad, void* Ym, float* bnorm);
// elements per float64 partial of the sum of s_hat written by the MFMA
// Phase-2 kernel (independent of its block shape)
int phase2_mfma_rows(int prec, int DM);
// Block shapes (ids): 1 one 32-element block per wave, 2 two blocks per wave
// (d <= 64, not fp8), 3 one block with the other number of tiles per LDS
// stage (the LDS-staged shapes only).  The default choice of blocks per wave:
int mfma_pb_default(int prec, int DM);
// the built-in shape with the metric taken into account (cosine bf16 at
// d = 32 measures faster with two blocks per wave, Euclidean with one)
int pb_builtin(int metric, int prec, int DM);
int mfma_pb_max(int prec, int DM);
bool mfma_lds_path(int prec, int DM);
// the shape ids valid for (prec, DM) into ids[0..2]; returns their count
int mfma_shapes(int prec, int DM, int* ids);
bool launch_phase2_mfma(hipStream_t st, int metric, int prec, int DM, const P2Args& A, const float* mu,
                        const void* Ym, const float* bnorm, int shape);

// ---- global mean -------------------------------------------------------------
void launch_mean(hipStream_t st, const double* bpart, int nb, int64_t n, double* out);

// ---- device-side sizes for the capturable pipeline (k_graph.hip) ------------
// bits of a clustering's status word
constexpr int kStatusLabel = 1;    // a label outside [0, k) (set by k_unit_hist)
constexpr int kStatusEmpty = 2;    // fewer than two nonempty clusters
constexpr int kStatusF0 = 4;       // F0 larger than its capacity
constexpr int kStatusPartial = 8;  // W(e_bar) partial sums larger than their capacity
constexpr int kStatusSample = 16;  // padded sample larger than its capacity
void launch_fill_i32(hipStream_t st, int32_t* p, int64_t count, int32_t v);
// off[0..k] = exclusive prefix sums of csize; q[j] = min(1, (2/|C_j|) lnterm)
void launch_index_sizes(hipStream_t st, const int32_t* csize, int k, double lnterm, int32_t* off, double* q,
                        int* status);
// clamps f0_off to f0_cap and writes the W work items (items_cap slots, the
// unused ones empty), per-cluster first item / count and partial bases;
// with dbase non-null also the bases of the kept distances (DistStore) and
// meta[1] = 1 when they fit dist_cap doubles.  The capacity bits go into
// *status: ORed in, or with assign_status the word is set to them (a status
// word of its own, which then needs no clear before the launch)
void launch_f0_items(hipStream_t st, const int32_t* csize, const int32_t* off, int32_t* f0_off, int k,
                     int64_t t, int chunk, int f0_cap, int64_t part_cap, int items_cap, int32_t* citem_first,
                     int32_t* citem_count, int64_t* ibase, int32_t* meta, int32_t* items, int* status,
                     int64_t* dbase = nullptr, int64_t dist_cap = 0, bool assign_status = false);
// capacity (doubles) of the kept distances for n elements, k clusters and
// ln(5k/delta): about 1.25 times their expected count, at most 2^27
int64_t dist_capacity(int64_t n, double lnterm);
// cnt[j] = |F_j|, sp_off = offsets of the blocks padded to kSamplePad rows
void launch_sample_sizes(hipStream_t st, const int32_t* s_off, int k, int s_cap, int32_t* cnt, int32_t* sp_off,
                         int* status);
void launch_put_status(hipStream_t st, const int* status, int32_t* out);

// ---- host-side helpers shared by the C-ABI files ----------------------------
}  // namespace silh
#include "../../include/silh.h"
namespace silh {
// the argument checks of silh_sample_init; *t receives the sample size used
silh_status validate_params(const silh_params* prm, const float* X, const int32_t* labels, int64_t* t);
// the argument checks of silh_exact (t, eps, delta, sampler and seed unused)
silh_status validate_exact_params(const silh_params* prm, const float* X, const int32_t* labels);
// padded row width of the packed sample for dimension d (0 if unsupported)
int dm_for(int d);
// sets the thread's silh_last_error message and returns st
silh_status set_error(silh_status st, const char* msg);

// ---- one request's Phase 2 inside a multi-request launch (serving) ---------
// The kernel class of a request's Phase 2 (requests of one class share a
// launch) and its work: `blocks` work items of `rows` elements, each against
// the S_pad packed sample rows.
struct P2Class {
  int mfma, metric, prec, DM, pb, rows;  // prec: 0 float32, 1 bf16, 2 fp8 operands, -1 vector ALU; pb: shape id
  int64_t blocks, S_pad;
};
// After a successful silh_pps_sample: ctx's Phase 2 (no per-element outputs;
// the block partials of the mean stay in the context) as a job of the
// multi-request launch.  False when its shape has no multi-request kernel
// (vector ALU with d > 128): then silh_scores runs it alone.
bool phase2_job(silh_ctx* c, P2Job* job, P2Class* cls);
// the autotuner's shape for ctx's Phase 2 (timing the shapes on ctx's data
// when its key is new; the built-in shape on the vector ALUs or in mode 0)
int tuned_shape(silh_ctx* c);
// padded sample rows of a sampled context (the tuner's size key), else 0
int64_t sample_rows(const silh_ctx* c);
// launch work items of requests of one class (workgroup i runs items[i])
bool launch_phase2_class(hipStream_t st, const P2Class& cls, const P2Job* jobs, const int2* items, int nitems);
// after the job's items have all run: the Eq. 9 mean from its block partials
// (on the context's stream; synchronises it)
silh_status phase2_job_mean(silh_ctx* c, double* mean);

// ---- cohesion / separation numerators from W_hat [n][k] ---------------------
constexpr int kCohSepMaxBlocks = 1024;
int coh_sep_blocks(int n);
// cpart/spart[block] = float64 partial sums of W_hat[e][own(e)] and of
// W_hat[e][j] over j > own(e)
void launch_coh_sep(hipStream_t st, const float* W, int n, int k, const int32_t* labels, double* cpart,
                    double* spart);

// ---- subsampled global estimators (row subsets) ------------------------------
// rows[i] = floor(B_i * n / 2^53), B_i the 53 Philox bits of counter i in the
// row stream
void launch_rows_draw(hipStream_t st, uint64_t seed, int64_t n, int64_t m, int32_t* rows);
// mark[rows[i]] = 1 for every valid entry; *bad = 1 if any entry lies outside [0, n)
void launch_rows_mark(hipStream_t st, const int32_t* rows, int64_t m, int n, int32_t* mark, int* bad);
// urows[pos[i]] = i for every marked i (ascending, distinct)
void launch_rows_compact(hipStream_t st, const int32_t* mark, const int32_t* pos, int n, int32_t* urows);
// Xs[i] = X[urows[i]], ls[i] = labels[urows[i]]
void launch_rows_gather(hipStream_t st, const float* X, const int32_t* labels, int d,
                        const int32_t* urows, int mu, float* Xs, int32_t* ls);
// gid_sub[s] = index of gid_pk[s] in urows, or -1 when it is not there
void launch_rows_remap(hipStream_t st, const int32_t* gid_pk, int64_t S_pad, const int32_t* urows,
                       int mu, int32_t* gid_sub);
// a/b/s[i] = a/b/s_u[index of rows[i] in urows]; bpart[block] = float64 sum
// of the block's s (blocks of kRowsBlock entries)
constexpr int kRowsBlock = 256;
void launch_rows_expand(hipStream_t st, const int32_t* rows, int64_t m, const int32_t* urows, int mu,
                        const float* au, const float* bu, const float* su, float* a, float* b, float* s,
                        double* bpart);

// ---- diagnostics -------------------------------------------------------------
void launch_uniform(hipStream_t st, uint64_t seed, int64_t gid0, int64_t count, uint32_t stream_id,
                    double* out);

}  // namespace silh
