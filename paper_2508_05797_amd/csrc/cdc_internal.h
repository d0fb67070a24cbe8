// Internal structures shared by the HIP kernels and the host runtime of
// libcdc.  Not part of the public ABI (include/cdc.h is).
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>

#include "cdc.h"

namespace cdc {

constexpr int kWave = 64;          // lanes per wavefront on CDNA
constexpr int kTile = 1024;        // bytes one wave stages per step (64 x 16 B)

enum Algo : uint32_t { kRam = 0, kAe = 1, kMaxp = 2, kAeMin = 3 };

// One job as the kernels see it: the caller's descriptor plus the plan
// (segmentation and workspace slots) computed for it.
struct JobDesc {
    const uint8_t* data;
    uint64_t n;
    uint64_t* cuts;          // caller's output offsets
    uint64_t* n_cuts;        // caller's output count
    int32_t* status;         // caller's status word (batch) or nullptr
    uint32_t algo;
    uint32_t w;
    uint32_t M;
    uint32_t nseg;           // number of segments (work items) of this job
    uint64_t seg;            // segment length S in bytes
    uint32_t item0;          // index of the first work item of this job
    uint32_t cap;            // cut (or candidate) slots per segment and list
    uint64_t slot0;          // first slot of this job in the slot arrays
    uint64_t blk0;           // first block-summary entry (MAXP)
    uint64_t idx0;           // first tile-index entry (RAM / AE / AE-Min)
    uint32_t blog;           // log2 of the MAXP block length (0: direct path)
    int32_t ok;              // 1 if the job passed validation
};

// Cut lists of a RAM / AE segment (positions relative to the segment
// start, increasing): the speculative chain from the segment start, the
// fix-up chain from the previous segment's speculative exit, and a re-walk
// chain from a later-known entry.
enum : uint32_t { kListSpec = 0, kListFix = 1, kListRewalk = 2 };
constexpr uint32_t kNone = 0xFFFFFFFFu;

// A run [lo, hi) of one list that belongs to the resolved chain.
struct Piece {
    uint32_t list, lo, hi;
};

// Per-segment record of the speculate / fix-up / round / resolve passes.
// Absolute positions are job offsets.
struct SegMeta {
    uint64_t exit;           // speculative chain: first cut at or past the segment end
    uint64_t fexit;          // fix-up chain: where it leaves (if it never met the speculative one)
    uint64_t entry;          // entry the current resolution starts from
    uint64_t rexit;          // current resolution: first cut at or past the segment end
    uint64_t xo[2];          // resolved exits of the parallel rounds (double buffer)
    uint64_t out;            // offset of this segment's cuts in the output
    uint32_t nspec;          // speculative cuts stored (MAXP: candidates)
    uint32_t nfix;           // fix-up cuts stored before it met the speculative chain
    uint32_t fms;            // speculative index the fix-up chain continues from, or kNone
    uint32_t count;          // cuts of the current resolution
    uint32_t npieces;
    uint32_t reads;          // tiles whose bytes the walkers of this item read
                             // (extreme byte search: low half; range scan: high half)
    uint32_t steps[4];       // the speculation walk's chunks by how each was
                             // decided: successor word, fast step, run of one
                             // value, exact patterns
    uint32_t claim;          // settling pass that holds this segment
    Piece pieces[3];
};

struct Item {
    uint32_t job;
    uint32_t seg;
};

// Where a kernel finds its work: a device job table with an item table
// (batch), or one job passed by value.
struct Plan {
    const JobDesc* jobs;     // device job table, or nullptr for one job
    const Item* items;       // device item table (with jobs)
    const uint32_t* n_items; // device item count and per-algorithm item ranges (with jobs)
    JobDesc one;             // the single job (jobs == nullptr)
    uint32_t one_items;      // its item count
};

// Flags raised on the device (workspace word) when a bound was violated.
enum : uint32_t { kErrOverflow = 1u };

// Capacity of a batch workspace and the planning constants.
struct BatchCaps {
    uint64_t items, slots, blocks, tiles;
    uint64_t items_chain;    // items of RAM / AE jobs (chain segments + jobs)
    uint64_t seg_chain, seg_maxp;
    uint64_t max_chunk_limit;
};

// Host-side event marks around kernels (tracing); nullptr when off.
struct Marks {
    virtual void begin(const char* name, int level, hipStream_t st) = 0;
    virtual void end(int level, hipStream_t st) = 0;
};

// Host-side launch sequences (defined with the kernels).
// Workspace of the RAM / AE passes.
struct ChainWs {
    uint4* idx;              // tile index entries (job's idx0 on)
    uint32_t* succ;          // successor words, kSuccSlots per tile (same numbering)
    SegMeta* meta;           // per item
    uint32_t* spec;          // speculative cuts, cap per item (job slots)
    uint32_t* fix;           // fix-up cuts, cap per item
    uint32_t* rew;           // re-walk cuts, cap per item
    uint32_t* err;
};

// Successor words per tile: one per stored position of the tile's maximum
// (seven) and one unused, so that a tile's words are two 16-byte loads.
constexpr uint32_t kSuccSlots = 8;

// Parallel resolution rounds after the fix-up before the ordered pass.
constexpr int kRounds = 2;

// Parts of a RAM / AE launch sequence: the index pass (streaming over the
// bytes), the successor and speculation passes, the fix-up pass, and the
// rounds with the settling pass.
enum : int { kPartIndex = 8, kPartSpec = 1, kPartFix = 2, kPartRest = 4, kPartGates = 16,
             kPartAll = 31 };

// RAM jobs of fewer segments are settled by the fix-up and the two rounds
// alone; the gate pass (kPartGates, with the rounds) only serves longer ones.
constexpr uint32_t kGateMinSeg = 2 + kRounds + 1;

// A batch whose RAM / AE items can exceed this count runs AE and AE-Min
// without successor words: their walkers then hold half the registers, and
// with many short jobs in flight that occupancy is worth more than the
// words (launch_chain's ae_succ).
constexpr uint64_t kAeSuccItems = 8192;

hipError_t launch_ram_ae(const Plan& P, uint32_t items_upper,
                         uint32_t jobs_upper, const uint32_t* n_jobs_d,
                         const ChainWs& ws, int waves_per_block,
                         hipStream_t st, Marks* marks, int part = kPartAll);
// The passes of one algorithm (kRam, kAe or kAeMin), and the output copy of
// all RAM / AE items (launch_ram_ae is the three and the copy in order).
hipError_t launch_chain(const Plan& P, uint32_t algo, uint32_t items_upper,
                        uint32_t jobs_upper, const uint32_t* n_jobs_d,
                        const ChainWs& ws, hipStream_t st, Marks* marks,
                        int part = kPartAll, bool ae_succ = true);
hipError_t launch_emit(const Plan& P, uint32_t items_upper, const ChainWs& ws,
                       int waves_per_block, hipStream_t st, Marks* marks);
hipError_t launch_maxp(const Plan& P, uint32_t items_upper, uint32_t jobs_upper,
                       const uint32_t* n_jobs_d, SegMeta* meta,
                       uint32_t* cand, uint8_t* bmax, int64_t* bpos,
                       uint32_t* err, int waves_per_block, bool any_blocks,
                       hipStream_t st, Marks* marks);
hipError_t launch_set_u64(uint64_t* p, uint64_t v, hipStream_t st);
// Batch planning: ctl[0] receives the item count, ctl[1] the overflow flag,
// ctl[2 + a] / ctl[6 + a] the first / end item of algorithm a (each
// algorithm's items are contiguous); bsum holds the per-block totals.
hipError_t launch_plan(cdc_job* jobs, uint32_t n_jobs, const BatchCaps& caps,
                       JobDesc* jd, Item* items, uint32_t* ctl, void* bsum,
                       hipStream_t st);
constexpr size_t plan_bsum_bytes(uint64_t n_jobs) {
    return (size_t)((n_jobs + 1023) / 1024) * 64;   // one Counts (7 words) per block
}
hipError_t launch_clear_u32(uint32_t* p, size_t count, hipStream_t st);

// Free the workspace of a stream the caller is about to destroy (the
// stream must be idle).
void drop_workspace(hipStream_t st);

// cdc_chunk_batch with the batch's total length known to the caller (0: not
// known; the length only sizes the launch grids), the choice of running
// the algorithms side by side on the workspace's own streams (side) or in
// order on `stream`, the algorithms the batch can contain (bit a of
// algo_mask for algorithm a; the passes of the others are not enqueued),
// and the length of its longest RAM job when the caller knows it (the gate
// pass is enqueued only where a RAM job can have kGateMinSeg segments).
int batch_run(const cdc_job* jobs, uint32_t n_jobs, uint64_t bytes_hint,
              bool side, hipStream_t stream, uint32_t algo_mask = 0xFu,
              uint64_t ram_max_n = ~0ull);

}  // namespace cdc
