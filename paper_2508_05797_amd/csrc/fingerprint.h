// Internal structures of the fingerprint and distinct-chunk passes, shared
// by their kernels and the host runtime (include/cdc.h is the public ABI).
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>

namespace cdc {

// Rest of a stored digest (bytes 8..31) and the chunk's length.
struct DedupSlot {
    uint64_t d1, d2, d3;
    uint64_t len;
};

enum : int {
    kDedupTotalBytes = 0,
    kDedupChunks = 1,
    kDedupUniqueBytes = 2,
    kDedupUniqueChunks = 3,
    kDedupCollisions = 4,
    kDedupFlags = 5,        // bit 0: the table filled up (some chunks not counted)
    kDedupCounters = 8
};

// Device view of a distinct-chunk table: 2^k slots (mask = 2^k - 1).
struct DedupDev {
    uint64_t* keys;
    DedupSlot* slots;
    uint64_t* ctr;
    uint64_t mask;
};

hipError_t launch_fingerprint(const uint8_t* data, uint64_t n,
                              const uint64_t* cuts, const uint64_t* n_cuts,
                              uint64_t max_cuts, uint8_t* digests,
                              hipStream_t st);
hipError_t launch_dedup_add(const DedupDev& D, const uint8_t* digests,
                            const uint64_t* cuts, const uint64_t* n_cuts,
                            uint64_t max_cuts, hipStream_t st);
hipError_t launch_dedup_clear(const DedupDev& D, hipStream_t st);

}  // namespace cdc
