// Resumable chunking of a stream that arrives in pieces (the upload path:
// chunking sits on the critical path of data that is still arriving,
// Section 1).  The device side of cdc_stream_push.
//
// Why a piece can be chunked on its own.  next(s) depends only on the bytes
// from s on (and, for MAXP, on w bytes past the candidate), so the chain
// from a chunk start over a prefix of the stream agrees with the chain over
// the whole stream for every cut c with c + lambda <= the prefix length,
// where lambda = 1 for RAM / AE (a cut before the prefix end was decided
// inside it) and lambda = w for MAXP (a candidate's right window must be
// complete, and a forced cut stands only when every candidate before it had
// a complete window).  Those cuts are final; the bytes from the last final
// cut on (fewer than max_chunk + lambda) are kept as the stream's tail.
//
// A push joins the tail with the piece's first max_chunk + w + 64 bytes in
// a staging buffer and chunks that (job 1).  When the piece is longer, the
// first cut of job 1 that lies in the piece is final (it is less than
// max_chunk past the piece start), and the chain continues from there over
// the piece itself, in place (job 2).  The kernels below stage job 1, pick
// job 1's final cuts and set up job 2, and finish: job 2's final cuts, the
// count, and the new tail.  Both jobs run through the batch path, whose
// descriptors live in device memory, so no value crosses to the host.
#include "cdc.h"
#include "stream.h"
#include "wave.h"

namespace cdc {

// Job 1: tail (t bytes) followed by the piece's first jp bytes, in `joined`.
__global__ __launch_bounds__(256) void k_stream_join(StreamDev S,
                                                     const uint8_t* piece,
                                                     uint64_t jp) {
    const uint64_t t = S.st->tail_len;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < t + jp;
         i += (uint64_t)gridDim.x * blockDim.x)
        S.joined[i] = i < t ? S.tail[i] : piece[i - t];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cdc_job& j = *S.job;
        j.data = S.joined;
        j.n = t + jp;
        j.cut_offsets = S.stage;
        j.n_cuts = &S.st->n_stage;
        j.algo = S.algo;
        j.window = S.w;
        j.max_chunk = S.M;
        j.status = 0;
    }
}

// Job 1's cuts (relative to the tail start).  Whole piece staged (jp == L):
// every final cut is emitted, and the new tail is cut from `joined`.
// Otherwise the cuts up to and including the first one at or past the piece
// start are emitted, and job 2 chunks the piece from that cut on.
__global__ __launch_bounds__(256) void k_stream_mid(StreamDev S,
                                                    const uint8_t* piece,
                                                    uint64_t L, uint64_t jp,
                                                    int last, uint64_t* out) {
    StreamState& st = *S.st;
    const uint64_t t = st.tail_len;
    const uint64_t base = st.tail_abs;
    const uint64_t k = min(st.n_stage, S.stage_cap);
    const uint64_t lam = S.lambda;
    __shared__ uint64_t s_emit, s_cut;
    if (threadIdx.x == 0) {
        uint64_t e = 0, cut = 0;
        if (jp == L) {
            // final: c + lambda <= t + L (all of them for the last piece)
            while (e < k && (last || S.stage[e] + lam <= t + L)) e++;
            cut = e ? S.stage[e - 1] : 0;
        } else {
            while (e < k && S.stage[e] < t) e++;
            cut = S.stage[e];           // exists: it is below t + max_chunk
            e++;
        }
        s_emit = e;
        s_cut = cut;
        st.emitted = e;
        st.split = cut;
        cdc_job& j = *S.job;
        if (jp == L) {
            j.n = 0;                     // no job 2
            j.data = piece;
        } else {
            j.data = piece + (cut - t);
            j.n = L - (cut - t);
        }
        j.cut_offsets = out + e;
        j.n_cuts = &st.n_stage;
        j.status = 0;
    }
    __syncthreads();
    const uint64_t e = s_emit, cut = s_cut;
    for (uint64_t i = threadIdx.x; i < e; i += blockDim.x) out[i] = base + S.stage[i];
    if (jp == L) {
        // new tail: joined[cut, t + L)
        const uint64_t nt = t + L - cut;
        __syncthreads();
        for (uint64_t i = threadIdx.x; i < nt; i += blockDim.x)
            S.tail[i] = S.joined[cut + i];
    }
}

// Job 2's cuts (relative to the split point, written in place after job 1's
// emitted ones): final ones are made absolute, the rest dropped; the count
// goes to *n_out and the tail / its absolute start are updated.
__global__ __launch_bounds__(256) void k_stream_fin(StreamDev S,
                                                    const uint8_t* piece,
                                                    uint64_t L, uint64_t jp,
                                                    int last, uint64_t* out,
                                                    uint64_t* n_out) {
    StreamState& st = *S.st;
    const uint64_t t = st.tail_len;
    const uint64_t e1 = st.emitted;
    const uint64_t cut = st.split;
    const uint64_t lam = S.lambda;
    __shared__ uint64_t s_fin, s_last;
    if (jp == L) {
        // everything was settled by k_stream_mid
        if (threadIdx.x == 0) {
            *n_out = e1;
            st.tail_abs += cut;
            st.tail_len = last ? 0 : t + L - cut;
        }
        return;
    }
    const uint64_t r = cut - t;                  // split point in the piece
    const uint64_t k2 = st.n_stage;
    uint64_t* o2 = out + e1;
    if (threadIdx.x == 0) {
        uint64_t f = 0;
        while (f < k2 && (last || o2[f] + lam <= L - r)) f++;
        s_fin = f;
        s_last = f ? o2[f - 1] : 0;
    }
    __syncthreads();
    const uint64_t f = s_fin, lastc = s_last;
    const uint64_t abs0 = st.tail_abs + cut;     // absolute position of the split
    for (uint64_t i = threadIdx.x; i < f; i += blockDim.x) o2[i] += abs0;
    // new tail: piece[r + lastc, L)
    const uint64_t from = r + lastc;
    const uint64_t nt = last ? 0 : L - from;
    for (uint64_t i = threadIdx.x; i < nt; i += blockDim.x) S.tail[i] = piece[from + i];
    __syncthreads();
    if (threadIdx.x == 0) {
        *n_out = e1 + f;
        st.tail_abs = abs0 + lastc;
        st.tail_len = nt;
    }
}

__global__ void k_stream_reset(StreamDev S) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        S.st->tail_len = 0;
        S.st->tail_abs = 0;
        S.st->n_stage = 0;
        S.st->emitted = 0;
        S.st->split = 0;
    }
}

hipError_t launch_stream_join(const StreamDev& S, const uint8_t* piece,
                              uint64_t jp, hipStream_t st) {
    const uint64_t most = S.tail_cap + jp;
    const uint32_t grid = (uint32_t)max((uint64_t)1, min((most + 4095) / 4096, (uint64_t)256));
    hipLaunchKernelGGL(k_stream_join, dim3(grid), dim3(256), 0, st, S, piece, jp);
    return hipGetLastError();
}

hipError_t launch_stream_mid(const StreamDev& S, const uint8_t* piece,
                             uint64_t L, uint64_t jp, int last, uint64_t* out,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_stream_mid, dim3(1), dim3(256), 0, st, S, piece, L, jp,
                       last, out);
    return hipGetLastError();
}

hipError_t launch_stream_fin(const StreamDev& S, const uint8_t* piece,
                             uint64_t L, uint64_t jp, int last, uint64_t* out,
                             uint64_t* n_out, hipStream_t st) {
    hipLaunchKernelGGL(k_stream_fin, dim3(1), dim3(256), 0, st, S, piece, L, jp,
                       last, out, n_out);
    return hipGetLastError();
}

hipError_t launch_stream_reset(const StreamDev& S, hipStream_t st) {
    hipLaunchKernelGGL(k_stream_reset, dim3(1), dim3(64), 0, st, S);
    return hipGetLastError();
}

}  // namespace cdc
