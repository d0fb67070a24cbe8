/*
 * cdc_fingerprint.h: the deduplication step after chunking, on the device.
 * C ABI of libcdc.so (with cdc.h).
 *
 * A deduplication pipeline chunks the data, fingerprints every chunk with a
 * collision-resistant hash and keeps one copy of each distinct chunk
 * (Section 2; Section 6.2 measures the fingerprinting step beside chunking,
 * with xxHash3 and SHA-256).  These calls take the cut list a chunking call
 * wrote (device memory, as cdc_chunk writes it) and, without a round trip
 * to the host, compute each chunk's SHA-256 (FIPS 180-4) and count the
 * distinct chunks and their bytes over any number of lists.
 */
#ifndef CDC_FINGERPRINT_H
#define CDC_FINGERPRINT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * SHA-256 of every chunk of a cut list.
 *   data         device, n bytes (the buffer that was chunked); read only.
 *   cut_offsets  device, the exclusive chunk ends (increasing, last = n);
 *   n_cuts       device, one uint64: their number K (as written by
 *                cdc_chunk; at most max_cuts are used).
 *   digests      device, room for max_cuts * 32 bytes; digest k (the 32
 *                bytes of SHA-256 of data[cut[k-1], cut[k]), cut[-1] = 0)
 *                is written at digests + 32 k.
 * Enqueued on `stream` after whatever wrote the cut list there.  Returns
 * CDC_OK, CDC_EINVAL (null pointer with max_cuts > 0) or CDC_EHIP.
 */
int cdc_fingerprint(const uint8_t* data, size_t n, const uint64_t* cut_offsets,
                    const uint64_t* n_cuts, size_t max_cuts, uint8_t* digests,
                    hipStream_t stream);

/* A device table of the distinct chunks seen so far (opaque). */
typedef struct cdc_dedup cdc_dedup;

typedef struct {
    uint64_t total_bytes;     /* bytes of every chunk added              */
    uint64_t chunks;          /* chunks added                            */
    uint64_t unique_bytes;    /* bytes of the distinct chunks            */
    uint64_t unique_chunks;   /* distinct chunks                         */
    uint64_t collisions;      /* chunks whose first 64 digest bits matched a
                                 different chunk's (counted as distinct) */
    uint64_t flags;           /* bit 0: the table filled up; chunks past
                                 that point were not counted             */
} cdc_dedup_stats;

/*
 * Create a table for up to max_chunks chunks in all, on the current device
 * (2^k slots with 2^k >= 2 max_chunks, 40 bytes each, allocated here).  The
 * table starts empty (cleared on `stream`).  Returns CDC_OK, CDC_EINVAL,
 * CDC_ENOMEM or CDC_EHIP.
 */
int cdc_dedup_create(uint64_t max_chunks, hipStream_t stream, cdc_dedup** out);

/*
 * Add the chunks of one cut list: digests as cdc_fingerprint wrote them,
 * and the same cut_offsets / n_cuts / max_cuts (the chunk lengths come from
 * the cut list).  Two chunks are the same when their SHA-256 digests and
 * lengths are equal.  Asynchronous on `stream`; lists added on one stream
 * are counted in order, and a list may repeat chunks of earlier lists or
 * of itself.  Returns CDC_OK, CDC_EINVAL or CDC_EHIP.
 */
int cdc_dedup_add(cdc_dedup* d, const uint8_t* digests,
                  const uint64_t* cut_offsets, const uint64_t* n_cuts,
                  size_t max_cuts, hipStream_t stream);

/* Synchronise `stream` and read the counts.  CDC_OK, CDC_EINVAL, CDC_EHIP. */
int cdc_dedup_stats_get(cdc_dedup* d, hipStream_t stream, cdc_dedup_stats* out);

/* Empty the table (on `stream`).  CDC_OK, CDC_EINVAL or CDC_EHIP. */
int cdc_dedup_reset(cdc_dedup* d, hipStream_t stream);

/* Free the table (after its work completed). */
void cdc_dedup_destroy(cdc_dedup* d);

#ifdef __cplusplus
}
#endif

#endif /* CDC_FINGERPRINT_H */
