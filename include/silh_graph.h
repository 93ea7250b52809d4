/*
 * silh_graph.h - the sampled silhouette of many clusterings of one dataset
 * (a sweep over k) as one captured HIP graph.
 *
 * Each clustering runs the whole path of include/silh.h: the cluster index,
 * Phase 1 of Algorithm 1 (PPS; or the uniform sampler of Section 4.1.3),
 * packing, Phase 2 and the mean s_hat_2 of Eq. 9.  The kernels and results are
 * those of silh_sample_init / silh_pps_sample / silh_scores, but every size
 * stays on the device: buffers are sized by capacities fixed at creation, so
 * no size returns to the host between kernels and the K pipelines can be
 * captured once and replayed.  The clusterings form `chains` independent
 * branches of the graph (clustering i on branch i % chains), so that several
 * run on the device at once.
 *
 * A clustering whose sample (or initial sample, or W(e_bar) partial sums)
 * outgrows its capacity is flagged on the device, its pipeline runs on
 * clamped sizes (every access stays inside its buffer), and silh_graph_run
 * computes it again on the eager path: its mean is the eager path's, bit for
 * bit, like every other clustering's.  The choice of k by the largest global
 * silhouette follows Section 5 ("Selection of the best value of k").
 */
#ifndef SILH_GRAPH_H
#define SILH_GRAPH_H

#include <stdint.h>

#include "silh.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct silh_graph silh_graph;

/*
 * silh_graph_create - allocate the buffers of `chains` pipelines and capture
 * the K clusterings' work into one graph (nothing runs yet).
 *  base        metric, prec, sampler, t (or eps), delta, seed, and the
 *              allocator hooks (used for every buffer); base->k is ignored
 *  X           [n][d] float32, device, n = base->n, d = base->d
 *  labels      [K][n] int32, device; clustering i reads labels[i*n .. i*n+n).
 *              X and labels are caller-owned and must stay allocated until
 *              silh_graph_destroy; their contents are read at every run, so
 *              a caller may write new labels between runs.
 *  ks          [K] int32, host: clustering i has labels in [0, ks[i])
 *  chains      parallel branches, 1..16
 *  sample_cap  capacity of the packed sample as a multiple of k * t
 *              (rows: min(n, ceil(sample_cap * kmax * t)) + 32 kmax); <= 0
 *              selects 4.  PPS samples average about 1.0-1.5 t per cluster.
 *  stream      the stream the capture is made from is the library's own; this
 *              stream is synchronised first (X and labels ready)
 * Errors: SILH_E_ARG (NULL pointer, K < 1, chains outside [1, 16], any
 * clustering's parameters as silh_sample_init checks them),
 * SILH_E_UNSUPPORTED, SILH_E_NOMEM, SILH_E_HIP.
 */
silh_status silh_graph_create(const silh_params* base, const float* X, const int32_t* labels,
                              const int32_t* ks, int32_t K, int32_t chains, double sample_cap,
                              silh_stream stream, silh_graph** out);

/*
 * silh_graph_run - launch the graph on `stream`, wait for it, and report.
 *  means_host   [K] float64: s_hat_2 of each clustering (NaN where the
 *               status is not SILH_OK)
 *  status_host  [K] int32, nullable: SILH_OK, SILH_E_LABEL (a label outside
 *               [0, k)) or SILH_E_K (fewer than two nonempty clusters) per
 *               clustering
 *  best_host    nullable: index of the largest mean (lowest index among
 *               equal ones; -1 if none is SILH_OK)
 *  reruns_host  nullable: clusterings recomputed on the eager path because
 *               a capacity was exceeded
 * Returns SILH_OK when the graph ran (per-clustering outcomes are in
 * status_host), else SILH_E_ARG / SILH_E_HIP or the eager path's error.
 * Runs of one graph must not overlap (they share its buffers).
 */
silh_status silh_graph_run(silh_graph* g, silh_stream stream, double* means_host, int32_t* status_host,
                           int32_t* best_host, int32_t* reruns_host);

/* Graph nodes and the capacities chosen (for inspection). */
typedef struct {
  int64_t nodes;       /* kernel nodes in the graph */
  int64_t sample_cap;  /* packed-sample rows per branch */
  int64_t f0_cap;      /* initial-sample rows per branch */
  int64_t bytes;       /* device memory held */
} silh_graph_info;
silh_status silh_graph_get_info(const silh_graph* g, silh_graph_info* out);

/*
 * silh_graph_choice - the Phase-2 block shape captured for clustering i (the
 * ids of silh_tuning_choice: 1 one 32-element block per wave, 2 two, 3 one
 * with the other number of tiles per LDS stage) and the padded sample size
 * of the request it was tuned on.  Before capture, silh_graph_create runs one
 * eager request per group of clusterings with equal floor(log2(k t)) and
 * takes the autotuner's shape for it (silh_set_tuning's mode applies; with
 * the float32 vector-ALU kernels the shape is 1 and the size 0).
 * SILH_E_ARG for NULL arguments or i outside [0, K).
 */
silh_status silh_graph_choice(const silh_graph* g, int32_t i, int32_t* shape, int64_t* probe_S_pad);

/* Free the graph and every buffer (through the allocator hooks).  NULL is a
 * no-op. */
void silh_graph_destroy(silh_graph* g);

#ifdef __cplusplus
}
#endif

#endif /* SILH_GRAPH_H */
