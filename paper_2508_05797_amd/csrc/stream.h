// Internal structures of resumable stream chunking (cdc_stream_*), shared by
// its kernels and the host runtime.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>

#include "cdc.h"

namespace cdc {

// Device state of one stream.  tail_abs: absolute stream offset of the
// tail's first byte (the start of the open chunk); tail_len: its length.
struct StreamState {
    uint64_t tail_abs;
    uint64_t tail_len;
    uint64_t n_stage;        // count written by the current job
    uint64_t emitted;        // cuts of job 1 already emitted by this push
    uint64_t split;          // job 1's cut (relative to the tail) job 2 starts at
    uint64_t pad[3];
};

struct StreamDev {
    StreamState* st;
    uint8_t* tail;           // tail_cap bytes
    uint8_t* joined;         // 2 * tail_cap bytes: tail + the piece's head
    uint64_t* stage;         // job 1's cuts
    uint64_t stage_cap;
    cdc_job* job;            // the one descriptor of the batch calls
    uint64_t tail_cap;
    uint32_t algo, w, M, lambda;
};

hipError_t launch_stream_join(const StreamDev& S, const uint8_t* piece,
                              uint64_t jp, hipStream_t st);
hipError_t launch_stream_mid(const StreamDev& S, const uint8_t* piece,
                             uint64_t L, uint64_t jp, int last, uint64_t* out,
                             hipStream_t st);
hipError_t launch_stream_fin(const StreamDev& S, const uint8_t* piece,
                             uint64_t L, uint64_t jp, int last, uint64_t* out,
                             uint64_t* n_out, hipStream_t st);
hipError_t launch_stream_reset(const StreamDev& S, hipStream_t st);

}  // namespace cdc
