/*
 * cdc_serve.h: a request loop around cdc_chunk_batch (continuous batching).
 *
 * Not part of the paper's method, which chunks one stream on one CPU core:
 * this is the serving layer of the library.  Chunking requests arrive
 * open-loop at given times; the loop admits them while their device bytes
 * fit a memory budget and a batch slot (a HIP stream) is free, launches each
 * slot's admitted requests as one cdc_chunk_batch, and lets requests that
 * arrive meanwhile join the next batch on another slot, so batches overlap
 * on the device.  Every request's offsets equal cdc_chunk on that request's
 * bytes alone.
 */
#ifndef CDC_SERVE_H
#define CDC_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "cdc.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * One request.  Its bytes are pool[offset, offset + n) (pool is the device
 * buffer passed to cdc_serve); its offsets go to cuts[cut_base, cut_base +
 * cdc_max_cuts(n)) and its count to n_cuts[i], i being its index in the
 * request array.  arrival is in seconds after the loop starts; arrivals are
 * nondecreasing along the array.  reserved must be 0.
 */
typedef struct {
    uint64_t offset;
    uint64_t n;
    uint64_t cut_base;
    uint32_t algo;
    uint32_t window;
    uint32_t max_chunk;
    uint32_t reserved;
    double arrival;
} cdc_request;

/*
 * budget_bytes: device bytes admitted requests may hold at once; a request
 *   holds its payload plus its offset array (n + 8 * cdc_max_cuts bytes).
 *   0: half of the device memory free when the loop starts.
 * max_batch: requests per launch (1 .. 65536).
 * slots: batches in flight, one HIP stream each (1 .. 16).
 * min_window / max_chunk: bounds over every request's parameters (used to
 *   pre-size each slot's workspace; a request outside them is rejected).
 */
typedef struct {
    uint64_t budget_bytes;
    uint32_t max_batch;
    uint32_t slots;
    uint32_t min_window;
    uint32_t max_chunk;
} cdc_serve_config;

typedef struct {
    double elapsed;          /* seconds from the start to the last completion */
    uint64_t launches;       /* batches launched */
    uint64_t rejected;       /* requests refused at arrival */
    uint64_t bytes_done;     /* payload bytes of requests completed with CDC_OK */
    uint64_t budget_bytes;   /* the budget used */
    uint32_t max_queue;      /* longest wait queue seen */
    uint32_t max_inflight;   /* most batches in flight at once */
} cdc_serve_stats;

/*
 * Serve the requests; returns when every request has completed or was
 * rejected.
 *   pool, pool_bytes  device buffer holding every request's bytes.
 *   cuts, n_cuts      device output arrays (see cdc_request).
 *   reqs, n_req       HOST request array.
 *   latency           HOST, n_req doubles: completion time minus arrival, in
 *                     seconds (queueing included); -1 for a rejected request.
 *   status            HOST, n_req: CDC_OK, CDC_EINVAL (request invalid, out
 *                     of the pool, or its parameters outside the config),
 *                     CDC_ENOMEM (larger than the whole budget), or the
 *                     status its batch produced.
 *   stats             HOST, filled on return (may be null).
 * The loop runs on the calling thread and busy-polls for completions.  It
 * creates its streams and pinned descriptor buffers on the current device at
 * the start and frees them at the end.  Returns CDC_OK, CDC_EINVAL for bad
 * arguments (nothing launched), CDC_ENOMEM or CDC_EHIP.
 */
int cdc_serve(const uint8_t* pool, uint64_t pool_bytes, uint64_t* cuts,
              uint64_t* n_cuts, const cdc_request* reqs, uint32_t n_req,
              const cdc_serve_config* cfg, double* latency, int32_t* status,
              cdc_serve_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* CDC_SERVE_H */
