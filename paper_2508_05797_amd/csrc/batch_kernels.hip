// Batch planning on the device: many independent buffers (the many-file
// case) chunked by one set of launches.
//
// The planner reads the caller's job descriptors, validates each job,
// splits it into segments (work items), and lays out every job's slots in
// the shared workspace with exclusive scans over the jobs (per block, then
// over the blocks).  Sizes are only known on the
// device, so the launches that follow are sized by the reserved upper bound
// and walk the real item count grid-stride; the whole sequence can be
// captured into a HIP graph and replayed with new descriptor contents.
#include "cdc.h"
#include "wave.h"

namespace cdc {

static_assert(sizeof(cdc_job) == 48, "cdc_job layout");

__device__ __forceinline__ uint32_t blog_for(uint32_t w) {
    const uint64_t b = min((uint64_t)w + 1, (uint64_t)kTile);
    uint32_t lg = 0;
    while ((2ull << lg) <= b) lg++;
    return lg >= 4 ? lg : 0;
}

// Counts per job, scanned together: work items per algorithm (so that each
// algorithm's items are contiguous), cut slots, MAXP blocks.
constexpr int kNumCounts = 7;
constexpr int kSlots = 4, kBlocks = 5, kTiles = 6;

struct Counts {
    uint64_t v[kNumCounts];
};
static_assert(sizeof(Counts) <= 64, "plan_bsum_bytes reserves 64 bytes per block");

__device__ __forceinline__ Counts zero_counts() {
    Counts c;
#pragma unroll
    for (int i = 0; i < kNumCounts; i++) c.v[i] = 0;
    return c;
}

__device__ __forceinline__ Counts add(const Counts& x, const Counts& y) {
    Counts c;
#pragma unroll
    for (int i = 0; i < kNumCounts; i++) c.v[i] = x.v[i] + y.v[i];
    return c;
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int o) {
    return (uint64_t)__shfl_up((long long)v, (unsigned)o, kWave);
}

// Exclusive scan over the block of one Counts per thread (blockDim a
// multiple of 64, at most 1024): inclusive scans inside each wave by
// shuffles, then the waves' totals from LDS.  Two barriers.
__device__ Counts plan_exscan(const Counts& v, Counts* wsum, Counts& total) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t nw = blockDim.x / kWave;
    Counts inc = v;
    for (int o = 1; o < kWave; o <<= 1) {
        Counts u;
#pragma unroll
        for (int i = 0; i < kNumCounts; i++) u.v[i] = shfl_up64(inc.v[i], o);
        if ((int)lane >= o) inc = add(inc, u);
    }
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    Counts pre = zero_counts(), tot = zero_counts();
    for (uint32_t k = 0; k < nw; k++) {
        if (k < wave) pre = add(pre, wsum[k]);
        tot = add(tot, wsum[k]);
    }
    __syncthreads();                     // wsum is reused by the next call
    total = tot;
    Counts ex;
#pragma unroll
    for (int i = 0; i < kNumCounts; i++) ex.v[i] = pre.v[i] + inc.v[i] - v.v[i];
    return ex;
}

// One job's descriptor (without its offsets) and its counts.
__device__ JobDesc plan_job(cdc_job* jobs, uint32_t j, const BatchCaps& caps,
                            Counts& c) {
    JobDesc d{};
    c = zero_counts();
    const cdc_job q = jobs[j];
    const bool ok = q.algo <= 3 && q.window >= 1 &&
                    (uint64_t)q.max_chunk >= (uint64_t)q.window + 1 &&
                    (uint64_t)q.max_chunk <= caps.max_chunk_limit &&
                    q.n_cuts != nullptr && (q.n == 0 || (q.data && q.cut_offsets));
    d.data = q.data;
    d.n = q.n;
    d.cuts = q.cut_offsets;
    d.n_cuts = q.n_cuts;
    d.status = &jobs[j].status;
    d.algo = q.algo;
    d.w = q.window;
    d.M = q.max_chunk;
    d.ok = ok ? 1 : 0;
    uint64_t nseg = 0;
    if (ok && q.n > 0) {
        const bool maxp = q.algo == kMaxp;
        d.seg = maxp ? caps.seg_maxp : caps.seg_chain;
        nseg = (q.n + d.seg - 1) / d.seg;
        // cuts (MAXP: candidates) of a segment lie in (a, a + S + M)
        // (MAXP: [a, a + S + 1 KiB)) and inside the job, spaced >= w + 1
        const uint64_t span = min(maxp ? d.seg + kTile : d.seg + q.max_chunk, q.n);
        d.cap = (uint32_t)(span / ((uint64_t)q.window + 1) + 2);
        c.v[kSlots] = nseg * d.cap;
        d.blog = maxp ? blog_for(q.window) : 0;
        const uint64_t shift = (uintptr_t)q.data & 15;
        if (maxp && d.blog)
            c.v[kBlocks] = (q.n + shift + kTile - 1) / kTile * ((uint64_t)kTile >> d.blog);
        if (!maxp) c.v[kTiles] = (q.n + shift + kTile - 1) / kTile;
        c.v[q.algo] = nseg;
    }
    d.nseg = (uint32_t)nseg;
    return d;
}

constexpr uint32_t kPlanThreads = 1024;

// Planning in three launches.  (1) Every block validates its 1,024 jobs,
// counts their items, slots and MAXP blocks, stores the descriptors with
// offsets inside the block, and the block's totals.
__global__ __launch_bounds__(kPlanThreads) void k_plan_count(
    cdc_job* jobs, uint32_t n_jobs, BatchCaps caps, JobDesc* jd, Counts* bsum) {
    __shared__ Counts wsum[kPlanThreads / kWave];
    const uint32_t j = blockIdx.x * kPlanThreads + threadIdx.x;
    Counts c = zero_counts();
    JobDesc d{};
    if (j < n_jobs) d = plan_job(jobs, j, caps, c);
    Counts t;
    const Counts e = plan_exscan(c, wsum, t);
    if (j < n_jobs) {
        d.item0 = d.ok ? (uint32_t)e.v[d.algo] : 0u;
        d.slot0 = e.v[kSlots];
        d.blk0 = e.v[kBlocks];
        d.idx0 = e.v[kTiles];
        jd[j] = d;
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

// (2) One block turns the block totals into block offsets, places each
// algorithm's items after the previous algorithm's, and checks the totals
// against the workspace capacity.  ctl: [0] items, [1] overflow flag,
// [2 + a] and [6 + a] the first and end item of algorithm a.
__global__ __launch_bounds__(kPlanThreads) void k_plan_scan(
    uint32_t n_blocks, BatchCaps caps, Counts* bsum, uint32_t* ctl) {
    __shared__ Counts wsum[kPlanThreads / kWave];
    Counts carry = zero_counts();
    for (uint32_t base = 0; base < n_blocks; base += kPlanThreads) {
        const uint32_t k = base + threadIdx.x;
        const Counts v = k < n_blocks ? bsum[k] : zero_counts();
        Counts t;
        const Counts e = plan_exscan(v, wsum, t);
        if (k < n_blocks) bsum[k] = add(carry, e);
        carry = add(carry, t);
    }
    if (threadIdx.x == 0) {
        const uint64_t items = carry.v[0] + carry.v[1] + carry.v[2] + carry.v[3];
        const bool over = items > caps.items || carry.v[kSlots] > caps.slots ||
                          carry.v[kBlocks] > caps.blocks || carry.v[kTiles] > caps.tiles;
        ctl[1] = over ? 1u : 0u;
        ctl[0] = over ? 0u : (uint32_t)items;
        uint64_t first = 0;
        for (int a = 0; a < 4; a++) {
            ctl[2 + a] = over ? 0u : (uint32_t)first;
            first += carry.v[a];
            ctl[6 + a] = over ? 0u : (uint32_t)first;
        }
    }
}

// (3) Every job gets its final offsets and status; empty or rejected jobs
// get zero cuts; the item table lists (job, segment) for every segment.  A
// thread writes the first kOwnItems items of its job; the items of larger
// jobs past those are written by the whole block.
constexpr uint32_t kOwnItems = 64;

__global__ __launch_bounds__(kPlanThreads) void k_plan_items(
    cdc_job* jobs, uint32_t n_jobs, JobDesc* jd, Item* items,
    const Counts* bsum, const uint32_t* ctl) {
    __shared__ uint32_t big_job[kPlanThreads], big_n[kPlanThreads], big_first[kPlanThreads];
    __shared__ uint32_t n_big;
    const uint32_t j = blockIdx.x * kPlanThreads + threadIdx.x;
    if (threadIdx.x == 0) n_big = 0;
    __syncthreads();
    if (j < n_jobs) {
        const bool over = ctl[1] != 0;
        JobDesc d = jd[j];
        const Counts o = bsum[blockIdx.x];
        const bool valid = d.ok != 0;
        if (valid) d.item0 += ctl[2 + d.algo] + (uint32_t)o.v[d.algo];
        d.slot0 += o.v[kSlots];
        d.blk0 += o.v[kBlocks];
        d.idx0 += o.v[kTiles];
        if (over) d.ok = 0;
        jd[j] = d;
        jobs[j].status = over ? CDC_ENOMEM : (valid ? CDC_OK : CDC_EINVAL);
        if (!d.ok || d.n == 0) {
            if (d.n_cuts) *d.n_cuts = 0;
        } else {
            Item* it = items + d.item0;
            const uint32_t own = min(d.nseg, kOwnItems);
            for (uint32_t sg = 0; sg < own; sg++) it[sg] = Item{j, sg};
            if (d.nseg > kOwnItems) {
                const uint32_t k = atomicAdd(&n_big, 1u);
                big_job[k] = j;
                big_n[k] = d.nseg;
                big_first[k] = d.item0;
            }
        }
    }
    __syncthreads();
    const uint32_t nb = n_big;
    for (uint32_t k = 0; k < nb; k++) {
        const uint32_t jj = big_job[k], ns = big_n[k], i0 = big_first[k];
        for (uint32_t sg = kOwnItems + threadIdx.x; sg < ns; sg += blockDim.x)
            items[i0 + sg] = Item{jj, sg};
    }
}

hipError_t launch_plan(cdc_job* jobs, uint32_t n_jobs, const BatchCaps& caps,
                       JobDesc* jd, Item* items, uint32_t* ctl, void* bsum,
                       hipStream_t st) {
    const uint32_t nb = (n_jobs + kPlanThreads - 1) / kPlanThreads;
    Counts* bs = (Counts*)bsum;
    hipLaunchKernelGGL(k_plan_count, dim3(nb), dim3(kPlanThreads), 0, st, jobs,
                       n_jobs, caps, jd, bs);
    hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(kPlanThreads), 0, st, nb, caps,
                       bs, ctl);
    hipLaunchKernelGGL(k_plan_items, dim3(nb), dim3(kPlanThreads), 0, st, jobs,
                       n_jobs, jd, items, (const Counts*)bs, (const uint32_t*)ctl);
    return hipGetLastError();
}

}  // namespace cdc
