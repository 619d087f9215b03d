/* damf_serve.h -- continuous-batching update server on one DAMF context.
 *
 * Clients submit edge-update requests (batches of edits, up to
 * max_request_ops each) from any thread; a server thread admits them by
 * memory (host staging, and the device memory their graph edits may claim),
 * coalesces every admitted request that fits into the next update step, and
 * runs the steps back to back.  A request longer than max_step_ops runs alone
 * as consecutive parts of max_step_ops ops (its ops in order: the graph ends
 * as after one batch; the factorisation follows the parts' chunks).  The result equals applying the requests one by one in
 * admission order with damf_update (Algorithm 2's per-event loop with one
 * request as the event): within a step, each request's net change is taken
 * against the graph the earlier requests leave and no chunk mixes two
 * requests (see damf_update_requests).  Step 4 of a step runs on a second HIP
 * stream while the chunks of the next step run (overlap_push), so PPR work of
 * one step hides behind the core SVDs of the next.
 *
 * A request is complete ("visible") once Steps 1-3 of its step are applied
 * and, with Step 4 on (alpha < 1 and auto_enhance), that step's push has
 * brought max |R| <= eps.  While a server runs, the context belongs to it:
 * call no other damf_* function on the context until damf_server_destroy.
 */
#ifndef DAMF_SERVE_H
#define DAMF_SERVE_H

#include "damf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct damf_server damf_server;

typedef struct {
  int64_t admit_bytes;       /* admission cap: host staging bytes held by requests
                                admitted and not yet complete, 9 per op + 64 per
                                request (default 64 MiB)                       */
  int32_t max_step_ops;      /* ops coalesced into one step, 1..8192 (8192)    */
  int32_t max_step_requests; /* requests coalesced into one step, 1..256 (256) */
  int32_t overlap_push;      /* 1: a step's Step 4 overlaps the next step (1)  */
  int32_t start_paused;      /* 1: admit but do not start steps until
                                damf_server_resume (0)                         */
  int64_t admit_device_bytes;/* admission cap on the device memory admitted,
                                incomplete requests may claim: 24 bytes per op
                                (a CSR entry in the out- and in-pools, with a
                                moved row's reservation and the copy compaction
                                frees later); 0 (default): half the device
                                memory free when the server starts           */
  int32_t max_request_ops;   /* largest request, 1..2^20 (65536)               */
  int32_t autotune;          /* 1: pick the chunk rank r (max_core_rank) among
                                16, 32, 48, 64 (those <= max_side and
                                d + r <= 192): 4 steps at each, the rank with
                                the least Steps 1-3 time per net entry is kept
                                and appended to tune_cache; a cache entry for
                                the same device architecture, n, d, precision
                                and log2(m) is used without tuning (0)       */
  const char *tune_cache;    /* tuner cache file path, or NULL (NULL)          */
} damf_server_config;

/* Per-request result, filled by damf_wait. */
typedef struct {
  int64_t ticket;
  int64_t ops;
  int64_t step;              /* index of the update step that carried it       */
  int32_t step_requests;     /* requests coalesced in that step                */
  int32_t status;            /* damf_status of the request                     */
  int64_t net_entries;       /* the request's own net change                   */
  int64_t chunks;            /* chunks of the request                          */
  double submit_us;          /* server clock: microseconds since creation      */
  double start_us;           /* its step started                               */
  double done_us;            /* visible                                        */
  double latency_ms;         /* done - submit                                  */
  int32_t parts;             /* steps that carried it (> 1 above max_step_ops) */
  int32_t chunk_rank;        /* r of its (last) step, for an exact replay      */
} damf_request_info;

typedef struct {
  int64_t requests_done;
  int64_t ops_done;
  int64_t steps;
  int64_t busy_rejects;      /* submits refused by admission                   */
  int64_t admitted_bytes_peak;
  double elapsed_s;          /* first submit -> last completion                */
  double ops_per_s;          /* ops_done / elapsed_s                           */
  double latency_p50_ms;
  double latency_p99_ms;
  double latency_mean_ms;
  double latency_max_ms;
  double mean_requests_per_step;
  double mean_ops_per_step;
  double push_overlapped_ms; /* Step 4 time that ran beside a chain kernel     */
  int64_t admitted_device_bytes_peak;
  int64_t device_cap_bytes;  /* the device admission cap in force               */
  int32_t tuned_chunk_rank;  /* the tuner's choice (0: not tuned)               */
  int32_t pad_;
  int64_t tuner_steps;       /* steps the tuner measured                        */
} damf_server_stats;

void damf_server_config_default(damf_server_config *cfg);

/* Starts the server thread on ctx.  Errors: DAMF_E_INVALID_ARG (null ctx or
 * out-of-range config), DAMF_E_STATE (poisoned context), DAMF_E_DEVICE. */
damf_status damf_server_create(damf_ctx *ctx, const damf_server_config *cfg,
                               damf_server **out);

/* Admits one request: k ops (host arrays, read during the call; ids in
 * [0, n), op +1 insert / -1 delete), 1 <= k <= max_request_ops.  On success
 * *ticket identifies it.  DAMF_E_BUSY: admitting it would exceed admit_bytes
 * or the device cap (nothing is kept; retry after requests complete).  DAMF_E_OUT_OF_RANGE /
 * DAMF_E_INVALID_ARG: bad ops or size (nothing is kept).  DAMF_E_STATE: the
 * server stopped after a device error. */
damf_status damf_submit(damf_server *srv, int64_t k, const int32_t *src, const int32_t *dst,
                        const int8_t *op, int64_t *ticket);

/* Waits until the request is complete, at most timeout_us microseconds
 * (< 0: no limit), then fills *info (nullable) and releases the ticket.
 * Returns the request's status, DAMF_E_TIMEOUT (ticket kept), or
 * DAMF_E_INVALID_ARG for an unknown ticket.  A step whose core comes out
 * non-finite fails each of its requests with DAMF_E_NUMERIC: the step is
 * undone (bases, P, Sigma; its graph edits had not run yet) and the PPR state
 * is seeded again from the restored basis (its previous push ran beside the
 * chain), and the server goes on with the next requests. */
damf_status damf_wait(damf_server *srv, int64_t ticket, int64_t timeout_us,
                      damf_request_info *info);

/* Starts steps after start_paused. */
damf_status damf_server_resume(damf_server *srv);

/* Latency percentiles over completed requests, throughput, step shape. */
damf_status damf_server_get_stats(damf_server *srv, damf_server_stats *out);

/* Finishes every admitted request, stops the thread and frees the server (not
 * the context).  Unwaited tickets are dropped. */
void damf_server_destroy(damf_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* DAMF_SERVE_H */
