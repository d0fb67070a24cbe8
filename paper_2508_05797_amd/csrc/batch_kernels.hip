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

// Three counts per job (work items, cut slots, MAXP blocks), scanned
// together.
struct Counts {
    uint64_t items, slots, blocks;
};

__device__ __forceinline__ Counts add(const Counts& x, const Counts& y) {
    return Counts{x.items + y.items, x.slots + y.slots, x.blocks + y.blocks};
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
        const Counts u{shfl_up64(inc.items, o), shfl_up64(inc.slots, o),
                       shfl_up64(inc.blocks, o)};
        if ((int)lane >= o) inc = add(inc, u);
    }
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    Counts pre{0, 0, 0}, tot{0, 0, 0};
    for (uint32_t k = 0; k < nw; k++) {
        if (k < wave) pre = add(pre, wsum[k]);
        tot = add(tot, wsum[k]);
    }
    __syncthreads();                     // wsum is reused by the next call
    total = tot;
    return Counts{pre.items + inc.items - v.items, pre.slots + inc.slots - v.slots,
                  pre.blocks + inc.blocks - v.blocks};
}

// One job's descriptor (without its offsets) and its counts.
__device__ JobDesc plan_job(cdc_job* jobs, uint32_t j, const BatchCaps& caps,
                            Counts& c) {
    JobDesc d{};
    c = Counts{0, 0, 0};
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
        const uint64_t span = maxp ? d.seg + kTile : d.seg + q.max_chunk;
        uint64_t cap = span / ((uint64_t)q.window + 1) + 2;
        // a job's chains never hold more cuts than the job has
        cap = min(cap, (q.n + kTile) / ((uint64_t)q.window + 1) + 2);
        d.cap = (uint32_t)cap;
        c.slots = nseg * cap;
        d.blog = maxp ? blog_for(q.window) : 0;
        if (maxp && d.blog) {
            const uint64_t shift = (uintptr_t)q.data & 15;
            c.blocks = (q.n + shift + kTile - 1) / kTile * ((uint64_t)kTile >> d.blog);
        }
    }
    c.items = nseg;
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
    Counts c{0, 0, 0};
    JobDesc d{};
    if (j < n_jobs) d = plan_job(jobs, j, caps, c);
    Counts t;
    const Counts e = plan_exscan(c, wsum, t);
    if (j < n_jobs) {
        d.item0 = (uint32_t)e.items;
        d.slot0 = e.slots;
        d.blk0 = e.blocks;
        jd[j] = d;
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

// (2) One block turns the block totals into block offsets and checks the
// totals against the workspace capacity (ctl[0] = items, ctl[1] = overflow).
__global__ __launch_bounds__(kPlanThreads) void k_plan_scan(
    uint32_t n_blocks, BatchCaps caps, Counts* bsum, uint32_t* ctl) {
    __shared__ Counts wsum[kPlanThreads / kWave];
    Counts carry{0, 0, 0};
    for (uint32_t base = 0; base < n_blocks; base += kPlanThreads) {
        const uint32_t k = base + threadIdx.x;
        const Counts v = k < n_blocks ? bsum[k] : Counts{0, 0, 0};
        Counts t;
        const Counts e = plan_exscan(v, wsum, t);
        if (k < n_blocks) bsum[k] = add(carry, e);
        carry = add(carry, t);
    }
    if (threadIdx.x == 0) {
        const bool over = carry.items > caps.items || carry.slots > caps.slots ||
                          carry.blocks > caps.blocks;
        ctl[1] = over ? 1u : 0u;
        ctl[0] = over ? 0u : (uint32_t)carry.items;
    }
}

// (3) Every job gets its final offsets and status; empty or rejected jobs
// get zero cuts; the item table lists (job, segment) for every segment.
__global__ __launch_bounds__(kPlanThreads) void k_plan_items(
    cdc_job* jobs, uint32_t n_jobs, JobDesc* jd, Item* items,
    const Counts* bsum, const uint32_t* ctl) {
    const uint32_t j = blockIdx.x * kPlanThreads + threadIdx.x;
    if (j >= n_jobs) return;
    const bool over = ctl[1] != 0;
    JobDesc d = jd[j];
    const Counts o = bsum[blockIdx.x];
    const bool valid = d.ok != 0;
    d.item0 += (uint32_t)o.items;
    d.slot0 += o.slots;
    d.blk0 += o.blocks;
    if (over) d.ok = 0;
    jd[j] = d;
    jobs[j].status = over ? CDC_ENOMEM : (valid ? CDC_OK : CDC_EINVAL);
    if (!d.ok || d.n == 0) {
        if (d.n_cuts) *d.n_cuts = 0;
        return;
    }
    Item* it = items + d.item0;
    for (uint32_t s = 0; s < d.nseg; s++) it[s] = Item{j, s};
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
