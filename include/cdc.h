/*
 * cdc.h: chunk-boundary finding for hashless content-defined chunking on
 * AMD Instinct MI355X (gfx950).  C ABI of libcdc.so.
 *
 * The library computes, for a byte buffer, the exclusive end offsets of the
 * chunks produced by one of the hashless chunkers the paper accelerates:
 *
 *   CDC_RAM     RAM (Section 2.1 "RAM"; Section 4.3): the maximum T of the
 *               first w bytes of a chunk, then the chunk ends right after the
 *               first later byte >= T.
 *   CDC_AE      AE-Max (Section 2.1 "AE"; Section 4.3): a target is a byte
 *               greater than all bytes before it in the chunk; when none of
 *               the w bytes after a target is greater than it, the chunk ends
 *               right after those w bytes.
 *   CDC_MAXP    MAXP (Section 2.1 "MAXP"; Section 4.3): the chunk ends right
 *               after a byte that is strictly greater than the w bytes before
 *               it and the w bytes after it.
 *   CDC_AE_MIN  AE-Min: AE-Max with minima (Section 2.1 "AE").
 *
 * Common rules (identical for every chunker): bytes compare as unsigned
 * values; every chunk is at most max_chunk bytes (a forced cut at
 * start + max_chunk); every chunk except the last is at least window+1
 * bytes; the offsets are strictly increasing and the last one is n.
 * The chunk boundaries are exactly those of the plain byte-by-byte
 * definition (the paper's accelerated versions generate identical chunks,
 * Section 6.1).
 *
 * Memory and asynchrony.  Every pointer marked "device" is device memory of
 * the current HIP device (or host memory mapped for device access).  Calls
 * only validate their scalar arguments, enqueue work on `stream` and return;
 * results (offsets, counts, per-job status) are written on the device in
 * stream order and are valid after the caller synchronises the stream.  The
 * library owns a workspace per (device, stream); it grows only outside
 * stream capture.  A workspace that grows is replaced, not freed: a HIP
 * graph captured before the growth keeps using the old buffer, which stays
 * allocated until cdc_release.  Calls on different streams may run
 * concurrently.
 */
#ifndef CDC_H
#define CDC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CDC_RAM = 0,
    CDC_AE = 1,       /* AE-Max */
    CDC_MAXP = 2,
    CDC_AE_MIN = 3
} cdc_algo;

/* Chunker parameters.  window (w) >= 1; window + 1 <= max_chunk <= 2^28
 * (268,435,456); flags and reserved must be 0. */
typedef struct {
    uint32_t window;
    uint32_t max_chunk;
    uint32_t flags;
    uint32_t reserved;
} cdc_params;

/* Status codes: 0 on success, negative on error. */
enum {
    CDC_OK = 0,
    CDC_EINVAL = -1,   /* bad argument (null pointer, bad parameters)      */
    CDC_ENOMEM = -2,   /* workspace too small and cannot grow (capture)    */
    CDC_EHIP = -3,     /* a HIP call failed; see cdc_last_error()          */
    CDC_ENOTSUP = -4   /* unsupported device or request                    */
};

/*
 * Upper bound on the number of chunk boundaries of an n-byte buffer:
 * 0 if n == 0, else (n-1)/(window+1) + 1, since every chunk but the last is
 * at least window+1 bytes.  Returns 0 for invalid parameters.
 */
size_t cdc_max_cuts(const cdc_params* p, size_t n);

/*
 * Chunk one buffer.
 *   data         device, n bytes, any alignment; read only.
 *   cut_offsets  device, room for cdc_max_cuts(p, n) uint64 values; receives
 *                the exclusive chunk ends in increasing order.
 *   n_cuts       device, one uint64; receives the number of offsets written.
 *   stream       HIP stream the work is enqueued on (0 = null stream).
 * Returns CDC_OK once the work is enqueued; CDC_EINVAL for a null pointer
 * (data may be null when n == 0), bad algo or parameters; CDC_ENOMEM when
 * the workspace would have to grow during stream capture (call cdc_reserve
 * first); CDC_EHIP when a launch fails.  Nothing is written on error.
 * All buffers are owned by the caller.
 */
int cdc_chunk(cdc_algo algo, const cdc_params* p, const uint8_t* data,
              size_t n, uint64_t* cut_offsets, uint64_t* n_cuts,
              hipStream_t stream);

/*
 * cdc_chunk for callers that cannot allocate device memory: code under HIP
 * graph capture that has no reservation, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, semantics and results as
 * cdc_chunk, but the library's working memory is a fixed 64 MiB array per
 * device inside the library (held from load until the process ends)
 * instead of a per-stream workspace: nothing is allocated, no workspace is
 * created, and no event is recorded (profiling does not apply).
 * Limit: the call's workspace (for RAM / AE, 48 bytes of tile summaries and
 * successor words per KiB of input, and per segment of the chain search a
 * record and three cut lists of about (segment + max_chunk) / (window + 1)
 * slots; for MAXP, block summaries of the input and a candidate list) must
 * fit the 64 MiB; with the built-in tuning that covers, for example, about
 * 1.2 GiB for RAM or AE at window 4096 and about 5.5 GiB for MAXP at
 * window 2048.
 * Larger requests are refused with CDC_ENOMEM before anything is enqueued,
 * cdc_last_error() stating the bytes needed.  All calls on one device share
 * the array: calls that can overlap on the device (on different streams,
 * or from different host threads) race and must not be issued; calls in
 * one stream's order are safe.  Returns as cdc_chunk.
 */
int cdc_chunk_noalloc(cdc_algo algo, const cdc_params* p, const uint8_t* data,
                      size_t n, uint64_t* cut_offsets, uint64_t* n_cuts,
                      hipStream_t stream);

/*
 * One job of a batch.  data (device, n bytes), cut_offsets (device, room for
 * cdc_max_cuts entries) and n_cuts (device, one uint64) are owned by the
 * caller; algo/window/max_chunk as for cdc_chunk.  status is written by the
 * library: CDC_OK, or CDC_EINVAL for an invalid job (whose *n_cuts is then
 * set to 0 and whose offsets are not written), or CDC_ENOMEM when the
 * reserved workspace cannot hold the batch (every job gets it).
 */
typedef struct {
    const uint8_t* data;
    uint64_t n;
    uint64_t* cut_offsets;
    uint64_t* n_cuts;
    uint32_t algo;
    uint32_t window;
    uint32_t max_chunk;
    int32_t status;
} cdc_job;

/*
 * Chunk many independent buffers with one planned set of launches (the
 * many-file case).  jobs is a DEVICE array of n_jobs descriptors that stays
 * valid until the work completes; each job's result equals cdc_chunk on that
 * job alone, with offsets relative to its own data.  The work is sized on
 * the device from the descriptors, so the sequence can be captured into a
 * HIP graph and replayed with new descriptor contents, provided
 * cdc_reserve(stream, ...) reserved room for the largest batch first.
 * Without a reservation and outside capture, the call reads the
 * descriptors back (a synchronous copy) to size the workspace.  The RAM,
 * AE, AE-Min and MAXP jobs of a batch run side by side: RAM on `stream`, AE
 * and AE-Min on one and MAXP on another of two library-owned streams per
 * `stream` (default priority), forked from and joined back into `stream` by
 * events; they are made by the first batch outside capture (before that,
 * the algorithms run in order).
 * Returns CDC_OK once enqueued, CDC_EINVAL (jobs null, n_jobs 0),
 * CDC_ENOMEM (capture without enough reservation) or CDC_EHIP.
 */
int cdc_chunk_batch(const cdc_job* jobs, uint32_t n_jobs, hipStream_t stream);

/*
 * Pre-size the workspace of `stream` for batches of at most max_jobs jobs
 * holding at most max_total_bytes bytes in total, with windows >= min_window
 * and max_chunk <= max_chunk.  Also covers single-buffer calls of up to
 * max_total_bytes bytes with such parameters.  Call it outside stream
 * capture.  Returns CDC_OK, CDC_EINVAL, CDC_ENOMEM or CDC_EHIP.
 */
int cdc_reserve(hipStream_t stream, size_t max_total_bytes, uint32_t max_jobs,
                uint32_t min_window, uint32_t max_chunk);

/*
 * The plain alternative to cdc_chunk_batch: one cdc_chunk call per job, in
 * order, on `stream`.  host_jobs is a HOST array; each job's status field
 * receives the return code of its call.  Returns CDC_OK, the first error of
 * a job, or CDC_EHIP (then the remaining jobs are not enqueued).
 */
int cdc_chunk_each(cdc_job* host_jobs, uint32_t n_jobs, hipStream_t stream);

/* Free every workspace owned by the library, including buffers replaced by
 * growth (after all work completed; graphs captured with library calls must
 * not be replayed afterwards). */
void cdc_release(void);

/* Static text for a status code. */
const char* cdc_status_string(int status);

/* Detail of the last error on the calling thread ("" if none). */
const char* cdc_last_error(void);

/*
 * Resumable chunking of a stream that arrives in pieces (an upload: the
 * paper places chunking on the critical path of incoming data, Section 1).
 * The pieces, pushed in order, are chunked as one stream: the offsets all
 * pushes return, concatenated, equal cdc_chunk's offsets on the
 * concatenated bytes.  A push returns the cuts that the bytes seen so far
 * decide (for RAM and AE a cut c once c < bytes seen; for MAXP once
 * c + window <= bytes seen, since a candidate needs its right window); the
 * open chunk and its bytes (fewer than max_chunk + window) stay in the
 * object, on the device.  Offsets are absolute positions in the stream.
 *
 * cdc_stream_open: a stream object for one chunker and its parameters,
 *   pieces of at most max_piece bytes, used on `stream` only (every push
 *   and reset names the same stream).  Allocates its buffers and a
 *   workspace of its own here (about 3 x (max_chunk + window) bytes plus
 *   the workspace of a cdc_chunk of max_piece bytes); pushes allocate
 *   nothing.  Returns CDC_OK, CDC_EINVAL, CDC_ENOMEM or CDC_EHIP.
 * cdc_stream_max_cuts: room (uint64 entries) a push of len bytes needs in
 *   cut_offsets.
 * cdc_stream_push: chunk the next piece (device, len <= max_piece bytes,
 *   any alignment; read during the push's work only, so it may be reused
 *   once that work completes).  last != 0 ends the stream: every remaining
 *   cut is returned (the last one is the stream's length) and further
 *   pushes are refused until cdc_stream_reset.  cut_offsets (device,
 *   cdc_stream_max_cuts(len) entries) receives the newly decided offsets,
 *   n_cuts (device, one uint64) their number.  Asynchronous; nothing is
 *   read back to the host.  Returns CDC_OK, CDC_EINVAL (bad argument, a
 *   piece longer than max_piece, another stream, an ended stream) or
 *   CDC_EHIP.
 * cdc_stream_reset: start a new stream at offset 0 (on `stream`).
 * cdc_stream_close: wait for the stream's work and free the object.
 */
typedef struct cdc_stream cdc_stream;
int cdc_stream_open(cdc_algo algo, const cdc_params* p, size_t max_piece,
                    hipStream_t stream, cdc_stream** out);
size_t cdc_stream_max_cuts(const cdc_stream* s, size_t len);
int cdc_stream_push(cdc_stream* s, const uint8_t* piece, size_t len, int last,
                    uint64_t* cut_offsets, uint64_t* n_cuts, hipStream_t stream);
int cdc_stream_reset(cdc_stream* s, hipStream_t stream);
void cdc_stream_close(cdc_stream* s);

/*
 * Tuning knobs.  They change only speed, never the offsets.
 *   chain_segment    bytes per segment of the segment-parallel chain search
 *                    of RAM / AE / AE-Min (16 .. 2^28; 0: 512 KiB);
 *   maxp_segment     bytes per MAXP work item (16 .. 2^28; 0: 256 KiB);
 *   waves_per_block  waves per workgroup of the MAXP and output passes (1 .. 4;
 *                    0: 4);
 *   reserved         must be 0.
 * A reservation (cdc_reserve) keeps the segment lengths it was made with.
 */
typedef struct {
    uint64_t chain_segment;
    uint64_t maxp_segment;
    uint32_t waves_per_block;
    uint32_t reserved;
} cdc_tuning;

/* Set the process-wide tuning (null: the built-in choice).  Returns CDC_OK
 * or CDC_EINVAL. */
int cdc_set_tuning(const cdc_tuning* t);

/* The tuning in effect, with built-in choices filled in.  CDC_OK or
 * CDC_EINVAL (null). */
int cdc_get_tuning(cdc_tuning* t);

/*
 * Autotune for a batch: time the batch (jobs: DEVICE descriptors as for
 * cdc_chunk_batch) under a grid of segment lengths and waves per workgroup,
 * one knob at a time, `reps` timed runs per candidate on `stream`, then set
 * the fastest tuning and reserve the stream's workspace for this batch
 * (so it can be captured next).  The batch's outputs are written (with the
 * same values) by the trial runs.  Results are remembered per (device,
 * job count, total bytes, windows, algorithms) in the process: tuning the
 * same shape again only applies the remembered choice.  Synchronises;
 * not for use under capture.  chosen (host, may be null) receives the
 * choice.  Every trial's job statuses are read back: a trial in which a job
 * ends with a status other than CDC_OK or CDC_EINVAL fails the call with
 * that status.  Returns CDC_OK, CDC_EINVAL, CDC_ENOMEM or CDC_EHIP.
 */
int cdc_autotune(const cdc_job* jobs, uint32_t n_jobs, hipStream_t stream,
                 uint32_t reps, cdc_tuning* chosen);

/*
 * Kernel timing (tracing).  level 0: off; 1: HIP events around the main
 * kernel of each call (the speculation pass of RAM / AE, the block-summary
 * pass of MAXP); 2: around every kernel.  Events are recorded on the stream
 * of the call.  Returns CDC_OK or CDC_EINVAL.
 */
int cdc_set_profiling(int level);

/*
 * Synchronise `stream` and report the kernels timed on it since the last
 * report: for up to max_kernels distinct kernel names, names[i] (static
 * strings), calls[i] and total_ms[i].  Returns the number of names filled,
 * or a negative status.  Clears the records.
 */
int cdc_kernel_times(hipStream_t stream, const char** names, uint32_t* calls,
                     double* total_ms, int max_kernels);

/*
 * Diagnostic: synchronise `stream`, return and clear the sticky flags the
 * kernels raised on it, and those raised by cdc_chunk_noalloc calls on the
 * current device (bit 0: a chain exceeded its planned slot bound, which
 * indicates a library bug; 0 when nothing was flagged), or CDC_EHIP.
 */
int cdc_check_device_errors(hipStream_t stream);

/*
 * How the last cdc_chunk call on `stream` (RAM, AE or AE-Min) decided its
 * chunks: the speculation pass walks every segment once, and each of its
 * chunks was decided by a successor word, by the fast step from the tile
 * summaries, as a chunk of w + 1 inside a run of one byte value, or by the
 * exact patterns (Section 4.1's extreme byte search and Section 4.2's range
 * scan, reading a tile's bytes where its summary cannot decide).
 * tiles_read_* count the tiles whose bytes each pattern read in all passes
 * of the call (saturated at 65,535 per segment and pass).  A diagnostic:
 * synchronises `stream`; all counts are 0 when the last call was MAXP, a
 * batch, or absent.  Returns CDC_OK, CDC_EINVAL (out is null) or CDC_EHIP.
 */
typedef struct {
    uint64_t segments;
    uint64_t steps_successor, steps_fast, steps_run, steps_exact;
    uint64_t tiles_read_ebs, tiles_read_rs;
} cdc_walk_stats_t;
int cdc_walk_stats(hipStream_t stream, cdc_walk_stats_t* out);

#ifdef __cplusplus
}
#endif

#endif /* CDC_H */
