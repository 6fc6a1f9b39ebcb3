/*
 * paco_server.h -- batching request server of libpaco.
 *
 * Requests are independent semiring products C = A (x) B (section "PACO MM"
 * problem statement) of arbitrary shapes and mixed semirings whose operands
 * are already resident in device memory.  A dispatcher thread admits queued
 * requests while the bytes of their operands stay within an HBM budget,
 * takes every admitted request as one batch, splits the processors over the
 * batch in proportion to each request's work (the throughput-ratio split of
 * section "Extension to Heterogeneous Computing System", here applied to
 * requests), partitions each request over its processors with MM-1-Piece,
 * and runs one persistent launch per semiring group, the groups concurrently
 * on their own streams.  Completion times are stamped per request.
 *
 * Conventions are those of paco.h (layouts, semiring constants, device
 * pointers owned by the caller).  The caller keeps A, B and C of a request
 * alive and unmodified from submit until the request is reported done.
 * A server owns its own context and streams on the device of the context it
 * is created from; server calls are thread-safe.
 */
#ifndef PACO_SERVER_H
#define PACO_SERVER_H

#include <stdint.h>

#include "paco.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct paco_server_s* paco_server;

typedef struct paco_request {
  int64_t n, m, k;
  paco_semiring sr;
  const void* A; int64_t lda;   /* 0 = dense default */
  const void* B; int64_t ldb;
  void* C;       int64_t ldc;
  paco_precision precision;     /* ring only; AUTO picks per request */
  double arrival_s;             /* caller's arrival time on paco_server_clock();
                                   <= 0 means "now" (submission time) */
} paco_request;

typedef struct paco_request_result {
  paco_status status;
  paco_precision precision;     /* ring precision used */
  double arrival_s, launch_s, done_s;   /* paco_server_clock() seconds */
  int32_t batch_id, batch_size;
} paco_request_result;

typedef struct paco_server_opts {
  uint64_t hbm_budget_bytes;    /* admission budget: sum of A, B, C bytes of
                                   requests in flight (0 = 64 GiB) */
  int32_t max_batch;            /* requests per launch (0 = 8192) */
  int32_t per_request;          /* 1: baseline mode, every request is its own
                                   library call on all compute units */
  int32_t p;                    /* processors per batch (0 = compute units) */
  double batch_window_s;        /* after the first arrival, wait this long
                                   for more before launching (0 = none) */
  double spin_s;                /* an idle dispatcher polls for new requests
                                   (and completions) this long before it
                                   sleeps; waking a sleeping thread costs
                                   microseconds of scheduler latency.  For a
                                   server with a CPU core to spare (0 = sleep
                                   at once; negative: PACO_ERR_INVALID_ARG) */
} paco_server_opts;

typedef struct paco_server_stats {
  int64_t submitted, completed, failed, batches;
  double mean_batch;            /* requests per launch */
  double p50_s, p99_s, max_s;   /* latency done - arrival over completed
                                   requests: p50 and p99 from a histogram of
                                   256 bins per octave (within 0.3% of the
                                   exact order statistic), max exact */
  double span_s;                /* first arrival to last completion */
  double ops;                   /* 2 n m k summed over completed requests */
  int64_t retained;             /* requests the server holds (queued, in
                                   flight, or finished and not yet polled) */
  uint64_t bytes_in_flight;     /* admitted operand bytes not yet released */
} paco_server_stats;

/* Monotonic clock the server stamps times with (seconds). */
double paco_server_clock(void);

paco_status paco_server_create(paco_ctx ctx, const paco_server_opts* opts, paco_server* out);
/* Queue a request; *ticket identifies it.  Returns PACO_ERR_BUDGET when the
 * request alone exceeds the admission budget, PACO_ERR_INVALID_ARG for bad
 * shapes or pointers, PACO_ERR_UNSUPPORTED for a leading dimension of 2^22
 * elements or more (nothing is queued then). */
paco_status paco_server_submit(paco_server s, const paco_request* r, uint64_t* ticket);
/* *done = 1 and *out filled once the request has completed (or failed).
 * A request reported done is forgotten: polling its ticket again returns
 * PACO_ERR_NOT_FOUND.  Finished requests that are never polled are kept up
 * to 65536; beyond that the oldest are forgotten, so a long-running server
 * holds bounded memory. */
paco_status paco_server_poll(paco_server s, uint64_t ticket, int* done, paco_request_result* out);
/* Block until every submitted request has completed. */
paco_status paco_server_drain(paco_server s);
paco_status paco_server_stats_get(paco_server s, paco_server_stats* out);
paco_status paco_server_destroy(paco_server s);

/* Testing hook for the failure path: the next `count` batches fail before
 * any of their kernels is launched (nothing touches the device).  Their
 * requests finish with PACO_ERR_INTERNAL and their bytes return to the
 * admission budget; later requests run normally. */
paco_status paco_server_fail_batches(paco_server s, int32_t count);

/* Host-only: the processor split and pieces the server would launch for a
 * batch of `nreq` requests on p processors.  Pieces are written like
 * paco_partition's, with the request index of each piece in req_of_piece;
 * call with cap = 0 to size the arrays. */
paco_status paco_batch_partition(const paco_request* reqs, int32_t nreq, int32_t p, paco_piece* out,
                                 int32_t* req_of_piece, int64_t cap, int64_t* n_out);

#ifdef __cplusplus
}
#endif

#endif /* PACO_SERVER_H */
