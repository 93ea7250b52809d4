/*
 * silh_server.h - a request-serving runtime around the sampled-silhouette
 * path of include/silh.h, on one GPU.
 *
 * Datasets stay resident in device memory (caller-owned).  Each request asks
 * for the silhouette estimate s_hat_2 of one clustering of one dataset
 * (Algorithm 1, Phases 1 and 2, and Eq. 9: the sequence silh_sample_init,
 * silh_pps_sample, silh_scores of silh.h, with the same kernels and results).
 * A request may instead ask for the subsampled estimate of Eq. 10 (silh.h's
 * silh_draw_rows and silh_scores_rows).
 * Requests are admitted in arrival order while the device memory they are
 * estimated to need fits the configured budget (a request that does not fit
 * lets later ones that do go first, up to 8 times, then holds the queue until
 * it fits).  Worker threads, each with its own HIP stream and its own cache
 * of device blocks (trimmed after every request to budget / (2 workers)
 * bytes of free blocks), run the cluster index and Phase 1 of admitted
 * requests.  In mode 0 a batcher thread then runs the Phase 2 of every
 * request whose Phase 1 is done in shared launches: each launch takes about
 * 4 ms of (request, block-of-rows) work items of one kernel class (metric,
 * operands, width), the request with the least remaining work first and at
 * least a quarter for the oldest one, so a request arriving while others are
 * on the device joins the next launch and a small request does not wait for
 * a large one to end.  Each work item computes exactly what that block of
 * the request's own launch computes, so results equal a direct call's.
 * Requests with the row draws of Eq. 10, and vector-ALU shapes with d > 128,
 * run their own Phase-2 launch on their worker.
 *
 * All calls are thread-safe.  Timestamps are nanoseconds of one steady clock
 * (silh_server_now_ns), so callers can schedule arrivals on the same clock.
 */
#ifndef SILH_SERVER_H
#define SILH_SERVER_H

#include <stdint.h>

#include "silh.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct silh_server silh_server;

typedef struct {
  int32_t workers;           /* worker threads (each with its own stream) running the
                                cluster index and Phase 1 of admitted requests, 1..64 */
  int32_t mode;              /* 0: the Phase 2 of every request whose Phase 1 is done runs
                                in shared launches over (request, row-block) work items;
                                1: each request launches its own Phase 2 on its worker */
  uint64_t hbm_budget_bytes; /* device memory the admitted requests may use (estimate) */
} silh_server_cfg;

typedef struct {
  int32_t dataset;        /* id from silh_server_add_dataset */
  int32_t k;              /* number of cluster ids, 2..4096 */
  const int32_t* labels;  /* [n] int32 in [0, k), device; caller-owned and unchanged
                             until the request has completed */
  int32_t metric;         /* silh_metric */
  int32_t prec;           /* silh_prec (as silh_params.prec) */
  int32_t sampler;        /* silh_sampler */
  int32_t reserved0;      /* must be 0 */
  int64_t t;              /* expected samples per cluster (>= 1) */
  double delta;           /* in (0, 1) */
  uint64_t seed;          /* Philox key */
  int64_t m;              /* 0: the mean over every element (Eq. 9, gl-pps-f);
                             m > 0: the mean over m uniform row draws with the
                             same seed (Eq. 10, gl-pps-s / gl-uni-s) */
} silh_request;

typedef struct {
  int32_t status;         /* silh_status of the request */
  int32_t reserved0;
  double s_mean;          /* s_hat_2 (Eq. 9) when status is SILH_OK */
  int64_t S;              /* sampled elements */
  int64_t submit_ns;      /* silh_server_submit returned the ticket */
  int64_t start_ns;       /* a worker began the request */
  int64_t done_ns;        /* the result was ready */
  char message[160];      /* silh_last_error text of a failed request */
} silh_result;

/* Steady-clock time in nanoseconds (the clock of every silh_result). */
int64_t silh_server_now_ns(void);

/* Create a server on the calling thread's current device.  SILH_E_ARG for
 * NULL arguments, workers outside [1, 64], mode outside [0, 1] or a zero budget. */
silh_status silh_server_create(const silh_server_cfg* cfg, silh_server** out);

/* Register a resident dataset: X [n][d] float32 row-major, device,
 * caller-owned and unchanged while any request on it may run.  *id receives
 * its id.  SILH_E_ARG for NULL X or id, n outside [2, 2^30], d outside
 * [1, 256]. */
silh_status silh_server_add_dataset(silh_server* srv, const float* X, int64_t n, int32_t d, int32_t* id);

/* Queue a request; *ticket receives its id.  Arguments are checked as
 * silh_sample_init checks them (SILH_E_ARG / SILH_E_UNSUPPORTED; also m
 * outside [0, 2^30]) before the request is queued; SILH_E_NOMEM if its
 * estimate alone exceeds the budget. */
silh_status silh_server_submit(silh_server* srv, const silh_request* req, int64_t* ticket);

/* Block until the request has completed, copy its result to *out and retire
 * the ticket.  SILH_E_ARG for an unknown (or already retired) ticket. */
silh_status silh_server_wait(silh_server* srv, int64_t ticket, silh_result* out);

/* Block until every queued request has completed (results stay available to
 * silh_server_wait). */
silh_status silh_server_drain(silh_server* srv);

/* Drain, stop the workers, free their cached device blocks and streams.
 * NULL is a no-op. */
void silh_server_destroy(silh_server* srv);

/* Number of shared Phase-2 launches the batcher has issued so far (-1 for a
 * NULL server). */
int64_t silh_server_launches(silh_server* srv);

/*
 * silh_sweep - s_hat_2 (Algorithm 1 and Eq. 9; with m > 0 the subsampled
 * mean of Eq. 10 over m row draws) of K clusterings of one dataset, and the
 * clustering with the largest value (the choice of k by the global
 * silhouette, Section 5, "Selection of the best value of k").  Clustering i has labels[i*n .. i*n + n) in
 * [0, ks[i]); every other setting (metric, prec, sampler, t, delta, seed, the
 * allocator hooks are ignored) comes from *base, whose k is ignored.  The
 * clusterings run concurrently on `workers` worker streams (1..64) through
 * the serving runtime, within hbm_budget_bytes of estimated device memory.
 *  X        [n][d] float32, device;  labels  [K][n] int32, device (caller-owned)
 *  ks       [K] int32, host;  means_host  [K] float64, host
 *  best_host  index of the largest mean (the lowest index among equal ones),
 *           nullable
 * The caller's stream is synchronised first (X and labels must be ready on
 * it); the call returns when every clustering is done.  The first failing
 * clustering's status is returned (its mean is NaN); the others still run.
 */
silh_status silh_sweep(const silh_params* base, const float* X, const int32_t* labels, const int32_t* ks,
                       int32_t K, int64_t m, int32_t workers, uint64_t hbm_budget_bytes, silh_stream stream,
                       double* means_host, int32_t* best_host);

#ifdef __cplusplus
}
#endif

#endif /* SILH_SERVER_H */
