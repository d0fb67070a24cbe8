// Host side of the fingerprint and distinct-chunk calls
// (include/cdc_fingerprint.h).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "cdc.h"
#include "cdc_fingerprint.h"
#include "fingerprint.h"

struct cdc_dedup {
    void* mem = nullptr;
    cdc::DedupDev dev{};
};

extern "C" {

int cdc_fingerprint(const uint8_t* data, size_t n, const uint64_t* cut_offsets,
                    const uint64_t* n_cuts, size_t max_cuts, uint8_t* digests,
                    hipStream_t stream) {
    if (max_cuts == 0) return CDC_OK;
    if (!data || !cut_offsets || !n_cuts || !digests) return CDC_EINVAL;
    const hipError_t e = cdc::launch_fingerprint(data, n, cut_offsets, n_cuts,
                                                 max_cuts, digests, stream);
    return e == hipSuccess ? CDC_OK : CDC_EHIP;
}

int cdc_dedup_create(uint64_t max_chunks, hipStream_t stream, cdc_dedup** out) {
    if (!out || max_chunks == 0 || max_chunks > (1ull << 40)) return CDC_EINVAL;
    *out = nullptr;
    uint64_t slots = 1024;
    while (slots < 2 * max_chunks) slots <<= 1;
    cdc_dedup* d = new (std::nothrow) cdc_dedup;
    if (!d) return CDC_ENOMEM;
    const size_t keys = slots * sizeof(uint64_t);
    const size_t side = slots * sizeof(cdc::DedupSlot);
    const size_t ctr = cdc::kDedupCounters * sizeof(uint64_t);
    if (hipMalloc(&d->mem, keys + side + ctr) != hipSuccess) {
        delete d;
        return CDC_ENOMEM;
    }
    char* b = static_cast<char*>(d->mem);
    d->dev.keys = reinterpret_cast<uint64_t*>(b);
    d->dev.slots = reinterpret_cast<cdc::DedupSlot*>(b + keys);
    d->dev.ctr = reinterpret_cast<uint64_t*>(b + keys + side);
    d->dev.mask = slots - 1;
    if (cdc::launch_dedup_clear(d->dev, stream) != hipSuccess) {
        (void)hipFree(d->mem);
        delete d;
        return CDC_EHIP;
    }
    *out = d;
    return CDC_OK;
}

int cdc_dedup_add(cdc_dedup* d, const uint8_t* digests,
                  const uint64_t* cut_offsets, const uint64_t* n_cuts,
                  size_t max_cuts, hipStream_t stream) {
    if (!d) return CDC_EINVAL;
    if (max_cuts == 0) return CDC_OK;
    if (!digests || !cut_offsets || !n_cuts) return CDC_EINVAL;
    const hipError_t e = cdc::launch_dedup_add(d->dev, digests, cut_offsets,
                                               n_cuts, max_cuts, stream);
    return e == hipSuccess ? CDC_OK : CDC_EHIP;
}

int cdc_dedup_stats_get(cdc_dedup* d, hipStream_t stream, cdc_dedup_stats* out) {
    if (!d || !out) return CDC_EINVAL;
    uint64_t c[cdc::kDedupCounters] = {};
    hipError_t e = hipMemcpyAsync(c, d->dev.ctr, sizeof c, hipMemcpyDeviceToHost,
                                  stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return CDC_EHIP;
    out->total_bytes = c[cdc::kDedupTotalBytes];
    out->chunks = c[cdc::kDedupChunks];
    out->unique_bytes = c[cdc::kDedupUniqueBytes];
    out->unique_chunks = c[cdc::kDedupUniqueChunks];
    out->collisions = c[cdc::kDedupCollisions];
    out->flags = c[cdc::kDedupFlags];
    return CDC_OK;
}

int cdc_dedup_reset(cdc_dedup* d, hipStream_t stream) {
    if (!d) return CDC_EINVAL;
    return cdc::launch_dedup_clear(d->dev, stream) == hipSuccess ? CDC_OK : CDC_EHIP;
}

void cdc_dedup_destroy(cdc_dedup* d) {
    if (!d) return;
    if (d->mem) (void)hipFree(d->mem);
    delete d;
}

}  // extern "C"
